"""The allocation-free entry point mbbp_run_static against mbbp_run.

Two calls in a row on one decoder, the second with a smaller batch at another
shot offset: the counters equal those of mbbp_run on the same arguments bit for
bit; a batch beyond the static scratch is rejected with MBBP_EINVAL.
"""

import sys

import numpy as np
import pytest

import oracle
from workloads.configs import WORKLOADS

from .common import bases_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_14170_amd as m
    return m


@pytest.mark.parametrize("key,calls", [
    ("bb144_L16_T50", [(1, 0.06, 0, 40000), (2, 0.08, 123457, 9001)]),
    ("qc882_L64_T100", [(1, 0.03, 5, 2000), (3, 0.02, 10**6, 333)]),
])
def test_run_static_equals_run(pk, key, calls):
    wl = WORKLOADS[key]
    code = wl.code()
    bx = bases_for(code.hx, wl, oracle.build_bases)
    bz = bases_for(code.hz, wl, oracle.build_bases)
    dec = pk.Decoder(code.hx, code.hz, bx, bz, wl.T, alpha=wl.alpha, max_batch=max(c[3] for c in calls))
    for seed, p, shot0, shots in calls:
        say(f"run_static {key} seed={seed} p={p} shot0={shot0} shots={shots}")
        ref = dec.run(seed, p, shot0, shots).cpu().numpy()
        got = torch.zeros(pk.NUM_COUNTERS, dtype=torch.int64, device="cuda")
        dec.run_static(seed, p, shot0, shots, got)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        say(f"  counters {got.tolist()}")
        np.testing.assert_array_equal(got, ref)
        assert got[pk.CNT_EDGE_UPDATES] > 0
    dec.close()


def test_run_static_rejects_oversized_batch(pk):
    wl = WORKLOADS["bb144_L16_T50"]
    code = wl.code()
    bx = bases_for(code.hx, wl, oracle.build_bases)
    bz = bases_for(code.hz, wl, oracle.build_bases)
    dec = pk.Decoder(code.hx, code.hz, bx, bz, wl.T, alpha=wl.alpha, max_batch=10)
    c = torch.zeros(pk.NUM_COUNTERS, dtype=torch.int64, device="cuda")
    with pytest.raises(pk.MbbpError) as ei:
        dec.run_static(1, 0.05, 0, 200000, c)
    assert ei.value.status == -1 and "static scratch" in str(ei.value)
    say(f"  rejected: {ei.value}")
    dec.run_static(1, 0.05, 0, 20000, c)   # beyond max_batch, within the scratch
    torch.cuda.synchronize()
    assert int(c[pk.CNT_EDGE_UPDATES].item()) > 0
    dec.close()
