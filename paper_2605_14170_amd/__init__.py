"""MI355X (gfx950) multiple-bases BP list decoding (MBBP-LD) for CSS QLDPC codes.

Python binding of libmbbp.so.  Every step of the decoding path (noise sampling,
syndromes, BP on every representation, the list decision, the failure test)
runs in the library's HIP kernels; this module only marshals arguments.  PyTorch
provides device memory and the current HIP stream.

Bit vectors are int64 tensors holding the uint64 words of the C ABI (bit i of a
vector is bit i % 64 of word i // 64).
"""

from __future__ import annotations

import ctypes
from typing import Optional, Sequence, Tuple

import numpy as np

from . import _lib
from ._lib import MbbpError, NUM_COUNTERS  # noqa: F401

FLOODING, LAYERED = 0, 1
NMS, SPA, WEIGHTED = 0, 1, 2
MIN_WEIGHT, FWS = 0, 1
DEPOLARIZING, X_ONLY = 0, 1  # noise models (mbbp_set_noise)
PART_X, PART_Z = 0, 1
SERIAL_AUTO, SERIAL_SLOTS, SERIAL_LANES, SERIAL_LEVELS = 0, 1, 2, 3  # mbbp_set_serial_kernel

CNT_FAIL, CNT_FAIL_X, CNT_FAIL_Z, CNT_SUM_KMAX, CNT_SUM_K, CNT_EDGE_UPDATES, CNT_NOCONV, CNT_TIES = range(8)


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _need(t, name: str, shape, dtype) -> None:
    """The C ABI cannot see buffer sizes: check them here before any call."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: must be device memory")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")


def _prior_shape(prior, shots: int, n: int):
    return (shots, n) if prior.dim() == 2 else (n,)


def _stream(stream) -> Optional[int]:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class _SparseKeep:
    """Keeps the numpy arrays of an mbbp_sparse alive."""

    def __init__(self, h: np.ndarray):
        h = np.asarray(h, dtype=np.uint8)
        rows, cols = np.nonzero(h)
        ptr = np.zeros(h.shape[0] + 1, dtype=np.int32)
        np.add.at(ptr, rows + 1, 1)
        self.ptr = np.ascontiguousarray(np.cumsum(ptr), dtype=np.int32)
        self.idx = np.ascontiguousarray(cols, dtype=np.int32)
        self.s = _lib.Sparse(h.shape[0], h.shape[1], self.ptr.ctypes.data, self.idx.ctypes.data)


def subtrees(h: np.ndarray, perm: Sequence[int]) -> Tuple[np.ndarray, np.ndarray, int]:
    """Algorithm 2 (host): (check_sets 1-based, acceptance order, number of subtrees)."""
    sp = _SparseKeep(h)
    m = h.shape[0]
    pm = np.ascontiguousarray(perm, dtype=np.int32)
    cs = np.zeros(m, np.int32)
    order = np.zeros(m, np.int32)
    ns = np.zeros(1, np.int32)
    _lib.check(_lib.lib().mbbp_subtrees(ctypes.byref(sp.s), pm.ctypes.data, cs.ctypes.data,
                                        order.ctypes.data, ns.ctypes.data), "mbbp_subtrees")
    return cs, order, int(ns[0])


BASIS_MODES = {"subtrees": 0, "ramp": 1}


def build_bases(h: np.ndarray, mode: str, L: int, perms: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Representations from subtrees (host): (basis_ptr int32[L+1], rows int32[])."""
    sp = _SparseKeep(h)
    pm = np.ascontiguousarray(perms, dtype=np.int32)
    cap = L * h.shape[0]
    bp = np.zeros(L + 1, np.int32)
    rows = np.zeros(max(cap, 1), np.int32)
    _lib.check(_lib.lib().mbbp_build_bases(ctypes.byref(sp.s), BASIS_MODES[mode], L, pm.shape[0],
                                           pm.ctypes.data, bp.ctypes.data, rows.ctypes.data, cap),
               "mbbp_build_bases")
    return bp, rows[: bp[-1]].copy()


class Decoder:
    """An MBBP-LD decoder context (mbbp_create) bound to the current HIP device."""

    def __init__(self, hx: np.ndarray, hz: np.ndarray, bases_hx, bases_hz, T: int,
                 schedule: int = FLOODING, rule: int = NMS, alpha: float = 0.875,
                 r_max: float = 65536.0, select: int = MIN_WEIGHT, max_batch: int = 1 << 20,
                 fixed_T: bool = False, extra_hx: Optional[np.ndarray] = None,
                 extra_hz: Optional[np.ndarray] = None, one_per_wave: bool = False):
        L_ = _lib.lib()
        self.n = int(hx.shape[1])
        self.mx, self.mz = int(hx.shape[0]), int(hz.shape[0])
        self.W = (self.n + 63) // 64
        self.T = int(T)
        self.L = int(len(bases_hx[0]) - 1)
        self.max_batch = int(max_batch)
        spx, spz = _SparseKeep(hx), _SparseKeep(hz)
        keep = [spx, spz]
        bl = []
        for (bp, rows), extra in ((bases_hx, extra_hx), (bases_hz, extra_hz)):
            bp = np.ascontiguousarray(bp, dtype=np.int32)
            rows = np.ascontiguousarray(rows if len(rows) else np.zeros(1, np.int32), dtype=np.int32)
            ex = None
            if extra is not None:
                ek = _SparseKeep(extra)
                keep.append(ek)
                ex = ctypes.pointer(ek.s)
            keep += [bp, rows]
            bl.append(_lib.BasisList(int(bp.shape[0] - 1), bp.ctypes.data, rows.ctypes.data, ex))
        bases = _lib.Bases(bl[0], bl[1])
        prm = _lib.Params()
        L_.mbbp_params_default(ctypes.byref(prm))
        prm.rule, prm.alpha, prm.r_max, prm.select = int(rule), float(alpha), float(r_max), int(select)
        prm.max_batch = int(max_batch)
        prm.flags = (_lib.MBBP_FLAG_FIXED_T if fixed_T else 0) | \
            (_lib.MBBP_FLAG_ONE_PER_WAVE if one_per_wave else 0)
        ctx = ctypes.c_void_p()
        _lib.check(L_.mbbp_create(ctypes.byref(spx.s), ctypes.byref(spz.s), ctypes.byref(bases), int(T),
                                  int(schedule), ctypes.byref(prm), ctypes.byref(ctx)), "mbbp_create")
        self._ctx = ctx
        del keep

    def close(self) -> None:
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            _lib.lib().mbbp_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ helpers
    def _dev(self, shape, dtype):
        torch = _torch()
        return torch.empty(shape, dtype=dtype, device="cuda")

    def edge_counts(self, part: int) -> np.ndarray:
        out = np.zeros(self.L, np.int64)
        _lib.check(_lib.lib().mbbp_edge_counts(self._ctx, int(part), out.ctypes.data), "mbbp_edge_counts")
        return out

    def logicals(self) -> Tuple[np.ndarray, np.ndarray]:
        k = np.zeros(1, np.int32)
        _lib.check(_lib.lib().mbbp_logicals(self._ctx, None, None, k.ctypes.data), "mbbp_logicals")
        lx = np.zeros((int(k[0]), self.W), np.uint64)
        lz = np.zeros((int(k[0]), self.W), np.uint64)
        _lib.check(_lib.lib().mbbp_logicals(self._ctx, lx.ctypes.data, lz.ctypes.data, k.ctypes.data),
                   "mbbp_logicals")
        return lx, lz

    # ------------------------------------------------------------------ entry points
    def sample(self, seed: int, p: float, shot0: int, shots: int, stream=None):
        """(err_x, err_z, syn_x, syn_z) device int64 tensors."""
        torch = _torch()
        ex = self._dev((shots, self.W), torch.int64)
        ez = self._dev((shots, self.W), torch.int64)
        sx = self._dev((shots, (self.mz + 63) // 64), torch.int64)
        sz = self._dev((shots, (self.mx + 63) // 64), torch.int64)
        _lib.check(_lib.lib().mbbp_sample(self._ctx, int(seed) & (2**64 - 1), float(p), int(shot0), int(shots),
                                          _ptr(ex), _ptr(ez), _ptr(sx), _ptr(sz), _stream(stream)),
                   "mbbp_sample")
        return ex, ez, sx, sz

    def _decode(self, fn, syn_x, syn_z, prior_x, prior_z, stream, out=None):
        torch = _torch()
        shots = int(syn_x.shape[0])
        pps = 1 if prior_x.dim() == 2 else 0
        _need(syn_x, "syn_x", (shots, (self.mz + 63) // 64), torch.int64)
        _need(syn_z, "syn_z", (shots, (self.mx + 63) // 64), torch.int64)
        _need(prior_x, "prior_x", _prior_shape(prior_x, shots, self.n), torch.float32)
        _need(prior_z, "prior_z", _prior_shape(prior_z, shots, self.n), torch.float32)
        if prior_x.dim() != prior_z.dim():
            raise ValueError("prior_x and prior_z: both per shot or both one vector")
        if out is None:
            out = dict(corr_x=self._dev((shots, self.W), torch.int64),
                       corr_z=self._dev((shots, self.W), torch.int64),
                       conv_x=self._dev((shots,), torch.int64), conv_z=self._dev((shots,), torch.int64),
                       basis_x=self._dev((shots,), torch.int16), basis_z=self._dev((shots,), torch.int16))
        for k, shape, dt in (("corr_x", (shots, self.W), torch.int64), ("corr_z", (shots, self.W), torch.int64),
                             ("conv_x", (shots,), torch.int64), ("conv_z", (shots,), torch.int64),
                             ("basis_x", (shots,), torch.int16), ("basis_z", (shots,), torch.int16)):
            _need(out[k], k, shape, dt)
        _lib.check(fn(self._ctx, shots, _ptr(syn_x), _ptr(syn_z), _ptr(prior_x), _ptr(prior_z), pps,
                      _ptr(out["corr_x"]), _ptr(out["corr_z"]), _ptr(out["conv_x"]), _ptr(out["conv_z"]),
                      _ptr(out["basis_x"]), _ptr(out["basis_z"]), _stream(stream)), fn.__name__)
        return out

    def decode(self, syn_x, syn_z, prior_x, prior_z, stream=None, out=None):
        return self._decode(_lib.lib().mbbp_decode, syn_x, syn_z, prior_x, prior_z, stream, out)

    def decode_batched(self, syn_x, syn_z, prior_x, prior_z, stream=None, out=None):
        return self._decode(_lib.lib().mbbp_decode_batched, syn_x, syn_z, prior_x, prior_z, stream, out)

    def decode_detail(self, part: int, syn, prior, want_llr: bool = False, stream=None):
        """Per-representation results of one part: (cand [shots, L, W], kstat [shots, L], llr)."""
        torch = _torch()
        shots = int(syn.shape[0])
        cand = self._dev((shots, self.L, self.W), torch.int64)
        kstat = self._dev((shots, self.L), torch.int16)
        llr = self._dev((shots, self.L, self.n), torch.float32) if want_llr else None
        pps = 1 if prior.dim() == 2 else 0
        m = self.mz if int(part) == 0 else self.mx
        _need(syn, "syn", (shots, (m + 63) // 64), torch.int64)
        _need(prior, "prior", _prior_shape(prior, shots, self.n), torch.float32)
        _lib.check(_lib.lib().mbbp_decode_detail(self._ctx, int(part), shots, _ptr(syn), _ptr(prior), pps,
                                                 _ptr(cand), _ptr(kstat), _ptr(llr), _stream(stream)),
                   "mbbp_decode_detail")
        return cand, kstat, llr

    def failures(self, err_x, err_z, corr_x, corr_z, stream=None):
        torch = _torch()
        shots = int(err_x.shape[0])
        for name, t in (("err_x", err_x), ("err_z", err_z), ("corr_x", corr_x), ("corr_z", corr_z)):
            _need(t, name, (shots, self.W), torch.int64)
        fail = self._dev((shots,), torch.uint8)
        _lib.check(_lib.lib().mbbp_failures(self._ctx, shots, _ptr(err_x), _ptr(err_z), _ptr(corr_x),
                                            _ptr(corr_z), _ptr(fail), _stream(stream)), "mbbp_failures")
        return fail

    def set_config(self, form: int, lanes_per_instance: int, waves_per_block: int = 4, chunk: int = 8,
                   blocks: int = 0) -> None:
        """BP launch shape for form 0 (plain) or 1 (batched); outputs do not depend on it."""
        cfg = _lib.LaunchConfig(int(lanes_per_instance), int(waves_per_block), int(chunk), int(blocks))
        _lib.check(_lib.lib().mbbp_set_config(self._ctx, int(form), ctypes.byref(cfg)), "mbbp_set_config")

    def get_config(self, form: int) -> dict:
        cfg = _lib.LaunchConfig()
        _lib.check(_lib.lib().mbbp_get_config(self._ctx, int(form), ctypes.byref(cfg)), "mbbp_get_config")
        return dict(lanes_per_instance=cfg.lanes_per_instance, waves_per_block=cfg.waves_per_block,
                    chunk=cfg.chunk, blocks=cfg.blocks)

    def autotune(self, form: int, seed: int = 12345, p: float = 0.05, shots: int = 65536) -> dict:
        """Time the candidate launch shapes of `form` and keep the fastest."""
        cfg = _lib.LaunchConfig()
        _lib.check(_lib.lib().mbbp_autotune(self._ctx, int(form), int(seed), float(p), int(shots),
                                            ctypes.byref(cfg)), "mbbp_autotune")
        return dict(lanes_per_instance=cfg.lanes_per_instance, waves_per_block=cfg.waves_per_block,
                    chunk=cfg.chunk, blocks=cfg.blocks)

    def set_noise(self, model: int) -> None:
        """Noise model of sample(), run() and autotune(): DEPOLARIZING or X_ONLY."""
        _lib.check(_lib.lib().mbbp_set_noise(self._ctx, int(model)), "mbbp_set_noise")

    def set_stats(self, counters=None) -> None:
        """decode() / decode_batched() add SUM_K, EDGE_UPDATES, NOCONV and TIES to
        `counters` (device int64 [NUM_COUNTERS], kept alive by the caller); None stops."""
        if counters is not None:
            _need(counters, "counters", (NUM_COUNTERS,), _torch().int64)
        self._stats = counters
        _lib.check(_lib.lib().mbbp_set_stats(self._ctx, _ptr(counters) if counters is not None else None),
                   "mbbp_set_stats")

    def set_serial_kernel(self, kernel: int) -> None:
        """Serial schedule kernel: SERIAL_AUTO, SERIAL_SLOTS (eight lanes per shot,
        normalized min-sum), SERIAL_LANES (one shot per lane) or SERIAL_LEVELS."""
        _lib.check(_lib.lib().mbbp_set_serial_kernel(self._ctx, int(kernel)), "mbbp_set_serial_kernel")

    def set_serial_lanes(self, lanes: int) -> None:
        """Serial schedule: shots per wavefront (0 = chosen from the LDS size)."""
        _lib.check(_lib.lib().mbbp_set_serial_lanes(self._ctx, int(lanes)), "mbbp_set_serial_lanes")

    def set_per_basis(self, enable: bool) -> None:
        """decode() as one BP launch per (part, representation): the naive form."""
        _lib.check(_lib.lib().mbbp_set_per_basis(self._ctx, 1 if enable else 0), "mbbp_set_per_basis")

    def run_graph_config(self, shots: int) -> dict:
        """Launch shape held by the BP kernel node of run()'s graph for `shots`."""
        cfg = _lib.LaunchConfig()
        _lib.check(_lib.lib().mbbp_run_graph_config(self._ctx, int(shots), ctypes.byref(cfg)),
                   "mbbp_run_graph_config")
        return dict(lanes_per_instance=cfg.lanes_per_instance, waves_per_block=cfg.waves_per_block,
                    chunk=cfg.chunk, blocks=cfg.blocks)

    def set_graph(self, enable: bool) -> None:
        _lib.check(_lib.lib().mbbp_set_graph(self._ctx, 1 if enable else 0), "mbbp_set_graph")

    def set_timing(self, enable: bool) -> None:
        _lib.check(_lib.lib().mbbp_set_timing(self._ctx, 1 if enable else 0), "mbbp_set_timing")

    def bp_time(self, reset: bool = True) -> Tuple[float, int]:
        """(summed BP kernel milliseconds from HIP events, launches) since the last reset."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _lib.check(_lib.lib().mbbp_bp_time(self._ctx, ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0),
                   "mbbp_bp_time")
        return ms.value, n.value

    # ------------------------------------------------------------------ weighted form
    def set_weights(self, alpha, beta) -> None:
        """Weights [T, L] (device float32) for decoding with rule WEIGHTED; None, None
        clears.  The tensors are kept referenced while set."""
        torch = _torch()
        if alpha is None and beta is None:
            _lib.check(_lib.lib().mbbp_set_weights(self._ctx, None, None), "mbbp_set_weights")
            self._weights = None
            return
        _need(alpha, "alpha", (self.T, self.L), torch.float32)
        _need(beta, "beta", (self.T, self.L), torch.float32)
        _lib.check(_lib.lib().mbbp_set_weights(self._ctx, _ptr(alpha), _ptr(beta)), "mbbp_set_weights")
        self._weights = (alpha, beta)

    def _wbp_check(self, part, syn, prior, alpha, beta):
        torch = _torch()
        shots = int(syn.shape[0])
        m = self.mz if int(part) == 0 else self.mx
        _need(syn, "syn", (shots, (m + 63) // 64), torch.int64)
        _need(prior, "prior", _prior_shape(prior, shots, self.n), torch.float32)
        _need(alpha, "alpha", (self.T, self.L), torch.float32)
        _need(beta, "beta", (self.T, self.L), torch.float32)
        return shots, (1 if prior.dim() == 2 else 0)

    def wbp_ckpt_floats(self, part: int, shots: int, ckpt_every: int) -> int:
        n = ctypes.c_int64()
        _lib.check(_lib.lib().mbbp_wbp_ckpt_floats(self._ctx, int(part), int(shots), int(ckpt_every),
                                                   ctypes.byref(n)), "mbbp_wbp_ckpt_floats")
        return int(n.value)

    def wbp_forward(self, part: int, syn, prior, alpha, beta, ckpt_every: int = 5, stream=None):
        """Weighted min-sum for exactly T iterations on every representation of one
        part: (P^(T) [shots, L, n] float32, checkpoint buffer for wbp_backward)."""
        torch = _torch()
        shots, pps = self._wbp_check(part, syn, prior, alpha, beta)
        llr = self._dev((shots, self.L, self.n), torch.float32)
        nck = self.wbp_ckpt_floats(part, shots, ckpt_every)
        ckpt = self._dev((max(nck, 1),), torch.float32)
        _lib.check(_lib.lib().mbbp_wbp_forward(self._ctx, int(part), shots, _ptr(syn), _ptr(prior), pps,
                                               _ptr(alpha), _ptr(beta), int(ckpt_every), _ptr(ckpt), _ptr(llr),
                                               _stream(stream)), "mbbp_wbp_forward")
        return llr, ckpt

    def wbp_backward(self, part: int, syn, prior, alpha, beta, ckpt_every: int, ckpt, grad_llr,
                     grad_alpha=None, grad_beta=None, stream=None):
        """Adds dL/dalpha, dL/dbeta ([T, L] float32) of one part, given dL/dP^(T)."""
        torch = _torch()
        shots, pps = self._wbp_check(part, syn, prior, alpha, beta)
        _need(grad_llr, "grad_llr", (shots, self.L, self.n), torch.float32)
        if grad_alpha is None:
            grad_alpha = torch.zeros((self.T, self.L), dtype=torch.float32, device="cuda")
        if grad_beta is None:
            grad_beta = torch.zeros((self.T, self.L), dtype=torch.float32, device="cuda")
        _need(grad_alpha, "grad_alpha", (self.T, self.L), torch.float32)
        _need(grad_beta, "grad_beta", (self.T, self.L), torch.float32)
        _need(ckpt, "ckpt", (max(self.wbp_ckpt_floats(part, shots, ckpt_every), 1),), torch.float32)
        _lib.check(_lib.lib().mbbp_wbp_backward(self._ctx, int(part), shots, _ptr(syn), _ptr(prior), pps,
                                                _ptr(alpha), _ptr(beta), int(ckpt_every), _ptr(ckpt),
                                                _ptr(grad_llr), _ptr(grad_alpha), _ptr(grad_beta),
                                                _stream(stream)), "mbbp_wbp_backward")
        return grad_alpha, grad_beta

    def run_static(self, seed: int, p: float, shot0: int, shots: int, counters=None, stream=None):
        """run() through mbbp_run_static: no device allocation inside the library (its
        buffers live in one static device array; `counters` must be given by callers
        that cannot allocate)."""
        torch = _torch()
        if counters is None:
            counters = torch.zeros(NUM_COUNTERS, dtype=torch.int64, device="cuda")
        _need(counters, "counters", (NUM_COUNTERS,), torch.int64)
        _lib.check(_lib.lib().mbbp_run_static(self._ctx, int(seed) & (2**64 - 1), float(p), int(shot0),
                                              int(shots), _ptr(counters), _stream(stream)), "mbbp_run_static")
        return counters

    def run(self, seed: int, p: float, shot0: int, shots: int, counters=None, stream=None):
        torch = _torch()
        if counters is None:
            counters = torch.zeros(NUM_COUNTERS, dtype=torch.int64, device="cuda")
        _need(counters, "counters", (NUM_COUNTERS,), torch.int64)
        _lib.check(_lib.lib().mbbp_run(self._ctx, int(seed) & (2**64 - 1), float(p), int(shot0), int(shots),
                                       _ptr(counters), _stream(stream)), "mbbp_run")
        return counters


def prior_llr(p: float, noise: int = DEPOLARIZING) -> float:
    """The library's uniform prior LLR of one part (Section II-B initialisation) at
    error rate p under `noise`, as a float32 value (mbbp_prior_llr)."""
    mu = ctypes.c_float()
    _lib.check(_lib.lib().mbbp_prior_llr(int(noise), float(p), ctypes.byref(mu)), "mbbp_prior_llr")
    return float(mu.value)


def words_to_numpy(t) -> np.ndarray:
    """int64 device tensor of uint64 words -> numpy uint64."""
    return t.detach().cpu().numpy().view(np.uint64)
