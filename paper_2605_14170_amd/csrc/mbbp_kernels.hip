// HIP kernels of the MBBP-LD library for gfx950 (CDNA4, wave64), apart from BP.
//
//  sample_kernel  : counter-based depolarizing noise and syndromes
//  select_kernel  : list decision per shot (Algorithm 1 decision phase, Section III-B)
//  fail_kernel    : logical-failure test of the residual (Section II-A)
//  small kernels  : run descriptor set-up, counter reset and accumulation
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mbbp_device.h"
#include "mbbp_wave.h"

namespace mbbp {

constexpr int MBBP_NUM_COUNTERS_DEV = 8;

// ----------------------------------------------------------------------------- Philox4x64-10

// Philox4x64 with 10 rounds (Salmon et al., SC'11): per round two 64x64->128
// products with multipliers M0, M1, XOR with the neighbouring words and the round
// key; the key advances by the Weyl constants W0, W1 between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                uint64_t k0, uint64_t k1, uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
        const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// ----------------------------------------------------------------------------- sampler

constexpr int kSampleBlock = 64;
constexpr int kMaxWords = kMaxN / 64;

// One thread per shot.  Error words are staged in LDS as [word][thread] so the
// syndrome loop (rows are wave-uniform) reads them without bank conflicts.
__global__ __launch_bounds__(kSampleBlock) void sample_kernel(SampleArgs a) {
    __shared__ uint64_t sh_e[2][kMaxWords][kSampleBlock];
    const int t = threadIdx.x;
    uint64_t seed = a.seed;
    int64_t shot0 = a.shot0;
    uint64_t t1 = a.t1, t2 = a.t2, t3 = a.t3;
    if (a.desc) {
        seed = a.desc->seed;
        shot0 = a.desc->shot0;
        t1 = a.desc->t1;
        t2 = a.desc->t2;
        t3 = a.desc->t3;
    }
    const int64_t s = (int64_t)blockIdx.x * kSampleBlock + t;
    const bool live = s < a.shots;
    const int n = a.n;
    const int W = (n + 63) >> 6;
    for (int w = 0; w < W; ++w) {
        uint64_t bx = 0, bz = 0;
        for (int b8 = 0; b8 < 8; ++b8) {
            const int q0 = w * 64 + b8 * 8;
            if (q0 >= n) break;
            uint64_t o[4];
            philox4x64_10((uint64_t)(shot0 + s), (uint64_t)(q0 >> 3), 0, 0, seed, 0, o);
#pragma unroll
            for (int sub = 0; sub < 8; ++sub) {
                const uint64_t u = (o[sub >> 1] >> (32 * (sub & 1))) & 0xffffffffull;
                const int bit = b8 * 8 + sub;
                if (q0 + sub < n) {
                    const uint64_t xb = (u < t2) ? 1ull : 0ull;            // X or Y
                    const uint64_t zb = (u >= t1 && u < t3) ? 1ull : 0ull;  // Y or Z
                    bx |= xb << bit;
                    bz |= zb << bit;
                }
            }
        }
        sh_e[0][w][t] = bx;
        sh_e[1][w][t] = bz;
        if (live) {
            a.err[0][s * W + w] = bx;
            a.err[1][s * W + w] = bz;
        }
    }
    __syncthreads();
    // part 0: s_X = H_Z e_X (H_Z is part[0]'s matrix); part 1: s_Z = H_X e_Z
#pragma unroll
    for (int pt = 0; pt < 2; ++pt) {
        const DevPart &P = a.part[pt];
        const int m = P.m, Ws = P.Ws;
        for (int w = 0; w < Ws; ++w) {
            uint64_t sw = 0;
            const int jend = min(m, (w + 1) * 64);
            for (int j = w * 64; j < jend; ++j) {
                const int k0 = P.hrow_ptr[j], k1 = P.hrow_ptr[j + 1];
                uint64_t par = 0;
                for (int k = k0; k < k1; ++k) {
                    const int col = P.hrow_idx[k];
                    par ^= sh_e[pt][col >> 6][t] >> (col & 63);
                }
                sw |= (par & 1ull) << (j - w * 64);
            }
            if (live) a.syn[pt][s * Ws + w] = sw;
        }
    }
}

// ----------------------------------------------------------------------------- select

// A group of G lanes (G = the smallest power of two >= L) per (part, shot): lane
// l of the group reads representation l's iteration word and candidate; the
// groups of a wave take consecutive shots, so each representation's loads of a
// wave are contiguous (the records are representation-major).  Items
// are (part, shot) pairs, part-major; each wave walks them in grid-stride rounds
// (the round count is wave-uniform, so every group of a wave takes part in the
// shuffles) and the counters are reduced per block before one atomic each.
// WM >= W bounds the unrolled word loops so the candidate words stay in registers.
template <int WM>
__global__ __launch_bounds__(256) void select_kernel(SelectArgs a) {
    const int G = a.group;
    const int lane = threadIdx.x & 63;
    const int lg = lane & (G - 1);
    const int gbase = lane & ~(G - 1);
    const int64_t total = a.shots * a.nparts;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x / G;
    long long c_sumk = 0, c_edges = 0, c_noconv = 0, c_ties = 0;
    for (int64_t base = ((int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63)) / G; base < total;
         base += stride) {
        const int64_t idx = base + lane / G;
        const bool live = idx < total;
        const int part = a.part0 + (live ? (int)(idx / a.shots) : 0);
        const int64_t shot = live ? idx - (int64_t)(part - a.part0) * a.shots : 0;
        const DevPart &pt = a.part[part];
        const int L = pt.L, W = pt.W;
        const bool mine = live && lg < L;
        // candidates and iteration words are representation-major: [L][shots][W], [L][shots]
        const uint64_t *cand = a.cand[part] + (size_t)shot * W;
        const size_t rstride = (size_t)a.shots * W;
        uint64_t words[WM];
        int st = 0, w = 0;
#pragma unroll
        for (int i = 0; i < WM; ++i) words[i] = 0;
        if (mine) {
            st = a.kstat[part][(size_t)lg * a.shots + shot];
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                if (i < W) words[i] = cand[(size_t)lg * rstride + i];
                w += __popcll(words[i]);
            }
            const int K = st & 0x7fff;
            c_sumk += K;
            c_edges += (long long)K * pt.E[lg];
        }
        const bool conv = mine && (st & 0x8000);
        const uint64_t ball = __ballot(conv);
        const uint64_t convm = G == 64 ? ball : (ball >> gbase) & ((1ull << G) - 1ull);
        int kmax = st & 0x7fff;
        for (int o = 1; o < G; o <<= 1) kmax = max(kmax, __shfl_xor(kmax, o, 64));
        int best = -1;
        if (a.rule == 0) {
            // least weight, ties to the smaller representation index
            int key = conv ? (w << 7) | lg : 0x7fffffff;
            for (int o = 1; o < G; o <<= 1) key = min(key, __shfl_xor(key, o, 64));
            best = key == 0x7fffffff ? -1 : (key & 127);
            // a tie: another converged candidate of the same weight that differs
            const int bw = key >> 7;
            bool differs = false;
#pragma unroll
            for (int i = 0; i < WM; ++i) differs |= __shfl(words[i], gbase + max(best, 0), 64) != words[i];
            const bool tie = best >= 0 && conv && lg > best && w == bw && differs;
            const uint64_t tb = __ballot(tie);
            if (lg == 0 && ((G == 64 ? tb : (tb >> gbase) & ((1ull << G) - 1ull)) != 0)) ++c_ties;
        } else {
            // FWS: argmax count(e) / (w(e) + 1) over distinct converged candidates, exact
            // cross-multiplied comparison, ties to the smaller index of first occurrence
            bool first = conv;
            long long cnt = 0;
            for (int k = 0; k < G; ++k) {
                bool eq = true;
#pragma unroll
                for (int i = 0; i < WM; ++i) eq &= __shfl(words[i], gbase + k, 64) == words[i];
                eq = eq && conv && ((convm >> k) & 1ull);
                if (eq && k < lg) first = false;
                if (eq && k >= lg) ++cnt;
            }
            const long long my_c = first ? cnt : -1, my_w1 = w + 1;
            long long bc = my_c, bw1 = my_w1;
            int bl = first ? lg : 0x7fff;
            for (int o = 1; o < G; o <<= 1) {
                const long long oc = __shfl_xor(bc, o, 64), ow1 = __shfl_xor(bw1, o, 64);
                const int ol = __shfl_xor(bl, o, 64);
                bool take;
                if (oc < 0 || bc < 0) take = bc < 0 && (oc >= 0 || ol < bl);
                else {
                    const long long lhs = oc * bw1, rhs = bc * ow1;
                    take = lhs > rhs || (lhs == rhs && ol < bl);
                }
                if (take) { bc = oc; bw1 = ow1; bl = ol; }
            }
            best = bc < 0 ? -1 : bl;
            // a tie: another distinct candidate (first occurrence) with the same score
            const bool tie = best >= 0 && my_c >= 0 && lg != best && my_c * bw1 == bc * my_w1;
            const uint64_t tb = __ballot(tie);
            if (lg == 0 && ((G == 64 ? tb : (tb >> gbase) & ((1ull << G) - 1ull)) != 0)) ++c_ties;
        }
        if (live) {
            if (lg == 0) {
                if (best < 0) ++c_noconv;
                if (a.counters && a.kmax_shot) atomicMax(&a.kmax_shot[shot], kmax);
                a.conv[part][shot] = convm;
                a.basis[part][shot] = (int16_t)best;
            }
            uint64_t *co = a.corr[part] + (size_t)shot * W;
            for (int i = lg; i < W; i += G) co[i] = best >= 0 ? cand[(size_t)best * rstride + i] : 0ull;
        }
    }
    if (a.counters) {
        __shared__ long long red[4][4];
        c_sumk = wave_sum_i64(c_sumk);
        c_edges = wave_sum_i64(c_edges);
        c_noconv = wave_sum_i64(c_noconv);
        c_ties = wave_sum_i64(c_ties);
        const int wv = threadIdx.x >> 6;
        if (lane == 0) {
            red[wv][0] = c_sumk; red[wv][1] = c_edges; red[wv][2] = c_noconv; red[wv][3] = c_ties;
        }
        __syncthreads();
        if (threadIdx.x < 4) {
            long long v = 0;
            for (int k = 0; k < (int)(blockDim.x >> 6); ++k) v += red[k][threadIdx.x];
            atomicAdd((unsigned long long *)&a.counters[4 + threadIdx.x], (unsigned long long)v);
        }
    }
}

// ----------------------------------------------------------------------------- failures

// One thread per shot.  Part X: residual r = e_X ^ corr_x fails iff H_Z r != 0 or
// L_Z r != 0 (it is then not a product of X stabilizers); part Z symmetric.
// part[0] holds H_Z and L_Z, part[1] holds H_X and L_X.  The residual words are
// read from memory once and staged in LDS as [word][thread] (the row loop's
// column indices are block-uniform, so the reads are conflict-free).
constexpr int kFailBlock = 256;
__global__ __launch_bounds__(kFailBlock) void fail_kernel(FailArgs a) {
    __shared__ uint64_t sh_r[kMaxWords][kFailBlock];
    const int t = threadIdx.x;
    const int64_t shot = (int64_t)blockIdx.x * blockDim.x + t;
    long long c_fail = 0, c_fx = 0, c_fz = 0, c_kmax = 0;
    const bool live = shot < a.shots;
    uint32_t flags = 0;
    for (int pt = 0; pt < 2; ++pt) {
        const DevPart &P = a.part[pt];
        const int W = P.W;
        __syncthreads();
        if (live) {
            const uint64_t *e = a.err[pt] + (size_t)shot * W;
            const uint64_t *c = a.corr[pt] + (size_t)shot * W;
            for (int w = 0; w < W; ++w) sh_r[w][t] = e[w] ^ c[w];
        }
        __syncthreads();
        if (live) {
            bool bad = false;
            for (int j = 0; j < P.m && !bad; ++j) {
                uint32_t par = 0;
                for (int k = P.hrow_ptr[j]; k < P.hrow_ptr[j + 1]; ++k) {
                    const int col = P.hrow_idx[k];
                    par ^= (uint32_t)(sh_r[col >> 6][t] >> (col & 63)) & 1u;
                }
                bad = par != 0;
            }
            for (int r = 0; r < P.k && !bad; ++r) {
                int cnt = 0;
                for (int w = 0; w < W; ++w) cnt += __popcll(sh_r[w][t] & P.logical[(size_t)r * W + w]);
                bad = (cnt & 1) != 0;
            }
            if (bad) flags |= 1u << pt;
        }
    }
    if (live) {
        if (a.fail) a.fail[shot] = (uint8_t)flags;
        c_fail = flags != 0;
        c_fx = flags & 1u;
        c_fz = (flags >> 1) & 1u;
        if (a.kmax_shot) c_kmax = a.kmax_shot[shot];
    }
    if (a.counters) {
        c_fail = wave_sum_i64(c_fail);
        c_fx = wave_sum_i64(c_fx);
        c_fz = wave_sum_i64(c_fz);
        c_kmax = wave_sum_i64(c_kmax);
        if ((threadIdx.x & 63) == 0) {
            atomicAdd((unsigned long long *)&a.counters[0], (unsigned long long)c_fail);
            atomicAdd((unsigned long long *)&a.counters[1], (unsigned long long)c_fx);
            atomicAdd((unsigned long long *)&a.counters[2], (unsigned long long)c_fz);
            atomicAdd((unsigned long long *)&a.counters[3], (unsigned long long)c_kmax);
        }
    }
}

__global__ void reset_kernel(unsigned long long *queue, int64_t *counters, int nc) {
    const int t = threadIdx.x;
    if (queue && t == 0) *queue = 0ull;
    if (counters && t < nc) counters[t] = 0;
}

__global__ void run_prep_kernel(RunPrepArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.n) {
        a.prior0[i] = a.mu;
        a.prior1[i] = a.mu;
    }
    if (i < a.shots) a.kmax[i] = 0;
    if (i == 0) {
        *a.desc = a.d;
        if (a.queue) *a.queue = 0ull;
    }
    if (a.counters && i < MBBP_NUM_COUNTERS_DEV) a.counters[i] = 0;
}

__global__ void accumulate_kernel(const int64_t *src, const RunDesc *desc, int nc) {
    const int t = threadIdx.x;
    if (t < nc && desc->counters) atomicAdd((unsigned long long *)&desc->counters[t], (unsigned long long)src[t]);
}

const void *run_prep_kernel_ptr() { return reinterpret_cast<const void *>(&run_prep_kernel); }

// ----------------------------------------------------------------------------- launchers

hipError_t launch_run_prep(const RunPrepArgs &a, hipStream_t s) {
    int64_t total = a.shots > a.n ? a.shots : a.n;
    if (total < MBBP_NUM_COUNTERS_DEV) total = MBBP_NUM_COUNTERS_DEV;
    hipLaunchKernelGGL(run_prep_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_accumulate(const int64_t *src, const RunDesc *desc, int nc, hipStream_t s) {
    hipLaunchKernelGGL(accumulate_kernel, dim3(1), dim3(64), 0, s, src, desc, nc);
    return hipGetLastError();
}

hipError_t launch_sample(const SampleArgs &a, hipStream_t s) {
    const int64_t blocks = (a.shots + kSampleBlock - 1) / kSampleBlock;
    hipLaunchKernelGGL(sample_kernel, dim3((unsigned)blocks), dim3(kSampleBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_select(SelectArgs a, hipStream_t s) {
    int lmax = 1;
    for (int p = a.part0; p < a.part0 + a.nparts; ++p) lmax = max(lmax, a.part[p].L);
    a.group = 1;
    while (a.group < lmax) a.group <<= 1;
    const int64_t threads = a.shots * a.nparts * a.group;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>((threads + 255) / 256, (int64_t)cus * 8)));
    int wmax = 1;
    for (int p = a.part0; p < a.part0 + a.nparts; ++p) wmax = max(wmax, a.part[p].W);
    if (wmax <= 2) hipLaunchKernelGGL((select_kernel<2>), grid, dim3(256), 0, s, a);
    else if (wmax <= 4) hipLaunchKernelGGL((select_kernel<4>), grid, dim3(256), 0, s, a);
    else if (wmax <= 8) hipLaunchKernelGGL((select_kernel<8>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((select_kernel<kMaxWords>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fail(const FailArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(fail_kernel, dim3((unsigned)((a.shots + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reset(unsigned long long *queue, int64_t *counters, int ncounters, hipStream_t s) {
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, queue, counters, ncounters);
    return hipGetLastError();
}

}  // namespace mbbp
