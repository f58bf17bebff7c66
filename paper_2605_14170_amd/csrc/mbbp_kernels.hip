// HIP kernels of the MBBP-LD library for gfx950 (CDNA4, wave64).
//
//  sample_kernel  : counter-based depolarizing noise and syndromes
//  bp_kernel      : BP on the L representations [H; H_t] (eqs. (1)-(2), Section II-B),
//                   flooding schedule, normalized min-sum or sum-product; plain
//                   (one work item per wave) and persistent (atomic work queue with
//                   per-instance refill) forms share this one kernel
//  select_kernel  : list decision per shot (Algorithm 1 decision phase, Section III-B)
//  fail_kernel    : logical-failure test of the residual (Section II-A)
//
// Work decomposition of bp_kernel: a wavefront owns G = 64 / LPI instances
// (shots) of ONE representation; each instance uses LPI lanes.  Lane `lig` of an
// instance handles checks j = c * LPI + lig and variable slots s = v * LPI + lig
// (c, v < P, compile-time), so per-lane graph tables and priors live in VGPRs.
// Per-edge messages live in LDS, one float per edge, in place: the check phase
// reads v->c messages of its row and overwrites them with c->v messages, the
// variable phase reads c->v messages and overwrites them with v->c messages.
// The variable phase also writes its hard decision as a byte at every edge so a
// check reads its row's decisions with one 8-byte LDS load (syndrome test).
// Phases are wave-synchronous: no workgroup barrier is ever needed.
#include <hip/hip_runtime.h>

#include "mbbp_device.h"

namespace mbbp {

constexpr int MBBP_NUM_COUNTERS_DEV = 8;

// ----------------------------------------------------------------------------- helpers

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ long long uniform_i64(long long v) {
    unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v & 0xffffffffu));
    unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ long long wave_sum_i64(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t fbits(float x) { return __float_as_uint(x); }
__device__ __forceinline__ float bitsf(uint32_t x) { return __uint_as_float(x); }

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

// ----------------------------------------------------------------------------- BP

template <int RULE>
struct CheckRule;

// Normalized min-sum (eq. (1)) with syndrome sign and clamp: the message to slot k
// is (-1)^{s_j} * prod_{k' != k} sgn(q_k') * min(alpha * min_{k' != k} |q_k'|, rmax).
// min over the others is min2 for the (first) minimum and min1 for every other slot.
template <>
struct CheckRule<0> {
    template <int DC>
    __device__ __forceinline__ static void apply(float (&q)[DC], int sbit, float alpha, float rmax) {
        float m1 = fminf(fabsf(q[0]), fabsf(q[1]));
        float m2 = fmaxf(fabsf(q[0]), fabsf(q[1]));
        uint32_t sx = fbits(q[0]) ^ fbits(q[1]);
#pragma unroll
        for (int k = 2; k < DC; ++k) {
            const float a = fabsf(q[k]);
            m2 = __builtin_amdgcn_fmed3f(m1, m2, a);
            m1 = fminf(m1, a);
            sx ^= fbits(q[k]);
        }
        const float A1 = fminf(alpha * m1, rmax);
        const float A2 = fminf(alpha * m2, rmax);
        const uint32_t sgn = (sx & 0x80000000u) ^ ((uint32_t)sbit << 31);
#pragma unroll
        for (int k = 0; k < DC; ++k) {
            const float mag = (fabsf(q[k]) == m1) ? A2 : A1;
            q[k] = bitsf(fbits(mag) | ((fbits(q[k]) ^ sgn) & 0x80000000u));
        }
    }
};

// Sum-product: pairwise box-plus x [+] y = sgn(x) sgn(y) min(|x|,|y|)
//   + log(1 + e^{-|x+y|}) - log(1 + e^{-|x-y|}), forward/backward over the row so
// slot k gets the box-plus of all other slots; syndrome sign; clamp.
template <>
struct CheckRule<1> {
    __device__ __forceinline__ static float boxplus(float x, float y) {
        const float ax = fabsf(x), ay = fabsf(y);
        const float mn = fminf(ax, ay);
        const float s = (fbits(x) ^ fbits(y)) & 0x80000000u ? -1.0f : 1.0f;
        const float c1 = __logf(1.0f + __expf(-fabsf(x + y)));
        const float c2 = __logf(1.0f + __expf(-fabsf(x - y)));
        return s * mn + c1 - c2;
    }
    template <int DC>
    __device__ __forceinline__ static void apply(float (&q)[DC], int sbit, float, float rmax) {
        float f[DC], b[DC];
        f[0] = q[0];
#pragma unroll
        for (int k = 1; k < DC; ++k) f[k] = boxplus(f[k - 1], q[k]);
        b[DC - 1] = q[DC - 1];
#pragma unroll
        for (int k = DC - 2; k >= 0; --k) b[k] = boxplus(b[k + 1], q[k]);
        const uint32_t sgn = (uint32_t)sbit << 31;
#pragma unroll
        for (int k = 0; k < DC; ++k) {
            float r = (k == 0) ? b[1] : (k == DC - 1) ? f[DC - 2] : boxplus(f[k - 1], b[k + 1]);
            r = fminf(fmaxf(r, -rmax), rmax);
            q[k] = bitsf(fbits(r) ^ sgn);
        }
    }
};

struct ItemPos {
    int part, l;
    int64_t begin, end;
};

__device__ __forceinline__ ItemPos decode_item(const BPArgs &a, int64_t item) {
    const int64_t rank = item / a.n_chunks;
    const int64_t ch = item - rank * a.n_chunks;
    const int pl = a.item_order ? a.item_order[rank] : (int)rank;
    ItemPos p;
    p.part = a.part0 + pl / a.L;
    p.l = pl - (pl / a.L) * a.L;
    p.begin = ch * a.chunk;
    p.end = min(p.begin + (int64_t)a.chunk, a.shots);
    return p;
}

template <typename T>
__device__ __forceinline__ T pick(const T (&v)[2], int part) { return part == 0 ? v[0] : v[1]; }

typedef __attribute__((address_space(3))) float lds_f32;
typedef __attribute__((address_space(3))) unsigned char lds_u8;

__device__ __forceinline__ lds_f32 *lds_ptr_f32(uint32_t byte_addr) { return (lds_f32 *)(size_t)byte_addr; }
__device__ __forceinline__ lds_u8 *lds_ptr_u8(uint32_t byte_addr) { return (lds_u8 *)(size_t)byte_addr; }

// LDS layout of one BP instance, 64 * PC rows (Mpad) of at most 8 edge slots:
//   messages  float [8][Mpad]  slot-major: edge (j, k) at k * Mpad + j
//   decisions u8    [8][Mpad]  stored as 32-bit cells at the message offset + 32 * Mpad,
//                              so one table address serves both arrays
//   syndrome words, output staging words, per-shot priors.
// Rows >= M_l are unused by representation l; row Mmax (of the part) is the sink
// of absent edges.  Every table entry is a byte address in LDS.
template <int PC>
struct Layout {
    static constexpr int Mpad = 64 * PC;
    static constexpr uint32_t kDecOff = 32u * Mpad;       // decisions after the messages
    static constexpr uint32_t kTail = 64u * Mpad;         // syndrome words start here
};

// Variable rule (eq. (2) and the posterior of Section II-B) for a variable of
// degree deg <= D (edges k >= deg point at the sink and read as 0):
// P = mu + sum r,  q_k = mu + sum_{k' != k} r_k'  accumulated in ascending check
// order (never P - r_k); every q_k and the hard decision are written back.
template <int D, uint32_t DECOFF>
__device__ __forceinline__ void var_rule(const uint32_t *ea, int deg, float mu, float &P, bool &dec) {
    float r[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const float x = *lds_ptr_f32(ea[k]);
        r[k] = k < deg ? x : 0.0f;
    }
    float q[D];
    float pre = mu;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        float acc = pre;
#pragma unroll
        for (int k2 = k + 1; k2 < D; ++k2) acc += r[k2];
        q[k] = acc;
        pre += r[k];
    }
    dec = pre < 0.0f;
    P = pre;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        *lds_ptr_f32(ea[k]) = q[k];
        *lds_ptr_u8(ea[k] + DECOFF) = (unsigned char)dec;
    }
}

// Posterior only (serial schedule): P = mu + sum r in ascending check order and the
// hard decision written to every edge's decision cell; messages are left alone.
template <int D, uint32_t DECOFF>
__device__ __forceinline__ void var_post(const uint32_t *ea, int deg, float mu, float &P, bool &dec) {
    float pre = mu;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const float x = *lds_ptr_f32(ea[k]);
        pre += k < deg ? x : 0.0f;
    }
    dec = pre < 0.0f;
    P = pre;
#pragma unroll
    for (int k = 0; k < D; ++k) *lds_ptr_u8(ea[k] + DECOFF) = (unsigned char)dec;
}

// One instance per wavefront.  Every per-instance quantity (shot, iteration,
// halting) is wave-uniform; per lane live only the variable slots' edge addresses,
// priors and the check slots' syndrome bits.  Variable slots: s = v * 64 + lane,
// v < PV (slots sorted by degree, so a pass has one degree almost everywhere);
// checks: j = c * 64 + lane, c < PC.  The shots of a work item are decoded one
// after another by the same wave.
// DC: 6 = every row has weight 6; 8 = rows of weight 2..8 with unused slots read
// as +FLT_MAX (never a minimum, neutral for box-plus).
// SCHED 0: flooding (variable phase, then check phase with the syndrome test).
// SCHED 1: serial (Section II-B): posterior phase, syndrome test, then a sweep
// over the conflict-free levels of the checks in which every check computes its
// incoming messages from the latest check messages.
template <int PV, int PC, int DC, int RULE, int SCHED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PV <= 3 ? 4 : 1)))
void bp_wave_kernel(BPArgs a) {
    using LY = Layout<PC>;
    constexpr int Mpad = LY::Mpad;
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char *ibase = smem + (size_t)wib * a.inst_bytes;
    const uint32_t ibase_addr = (uint32_t)(size_t)(lds_u8 *)ibase;
    uint64_t *synl = reinterpret_cast<uint64_t *>(ibase + LY::kTail);
    uint32_t *stage = reinterpret_cast<uint32_t *>(synl + a.ws_max);
    float *mul = reinterpret_cast<float *>(stage + 2 * a.w_max);
    unsigned char *sbl = reinterpret_cast<unsigned char *>(mul + a.n_max);  // serial: syndrome byte per check
    constexpr bool kMuLds = SCHED == 1;  // the serial sweep reads priors from LDS

    int64_t item;
    if (a.persistent) {
        unsigned long long v = 0;
        if (lane == 0) v = atomicAdd(a.queue, 1ull);
        item = uniform_i64((long long)v);
    } else {
        item = (int64_t)blockIdx.x * (blockDim.x >> 6) + wib;
    }
    const float alpha = a.alpha, rmax = a.rmax;
    const int T = a.T;
    int cur_key = -1;
    int dmax_rep = 0;  // largest variable degree of the representation (wave-uniform)

    uint32_t ea[PV][kMaxVarDegree];  // LDS byte address of every edge of the lane's variables
    uint32_t vinfo[PV];              // variable id | degree << 16
    int dmaxp[PV];                   // max degree of pass v (wave-uniform)
    uint32_t cwp[PC];                // row weights (DC == 8 only)
    float mu[PV];

    while (item < a.n_items) {
        const ItemPos ip = decode_item(a, item);
        const DevPart *pt = a.dparts + ip.part;
        const int n = pt->n, m = pt->m, Mmax = pt->Mmax, W = pt->W, Ws = pt->Ws, L = pt->L;
        const int l = ip.l;
        const int Ml = pt->M[l];
        const int vp = (n + 63) >> 6;
        const int key = ip.part * 256 + l;
        if (key != cur_key) {
            cur_key = key;
            // edge ids e = j * 8 + k  ->  address of (j, k) in the slot-major layout
            const uint4 *vo4 = reinterpret_cast<const uint4 *>(pt->voff) + (size_t)l * n;
            const uint16_t *vid = pt->vid + (size_t)l * n;
            const uint8_t *vdg = pt->vdeg + (size_t)l * n;
            const float *pr0 = pick(a.prior, ip.part);
            const uint32_t sink = (uint32_t)Mmax * 8u;
#pragma unroll
            for (int v = 0; v < PV; ++v) {
                const int s = v * 64 + lane;
                const bool valid = v < vp && s < n;
                const uint32_t sk2 = sink | (sink << 16);
                uint4 o = make_uint4(sk2, sk2, sk2, sk2);
                int deg = 0;
                uint32_t id = 0;
                if (valid) {
                    o = vo4[s];
                    deg = vdg[s];
                    id = vid[s];
                }
                const uint32_t w4[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
                for (int k = 0; k < kMaxVarDegree; ++k) {
                    const uint32_t e = (w4[k >> 1] >> (16 * (k & 1))) & 0xffffu;
                    ea[v][k] = ibase_addr + 4u * ((e & 7u) * (uint32_t)Mpad + (e >> 3));
                }
                vinfo[v] = id | ((uint32_t)deg << 16);
                dmaxp[v] = uniform_i32(wave_max_i32(deg));
                if (!a.prior_per_shot) mu[v] = valid ? pr0[id] + 0.0f : 0.0f;
            }
            dmax_rep = 0;
#pragma unroll
            for (int v = 0; v < PV; ++v) dmax_rep = max(dmax_rep, dmaxp[v]);
            if (DC == 8) {
#pragma unroll
                for (int c = 0; c < PC; ++c) {
                    const int j = c * 64 + lane;
                    cwp[c] = j < Ml ? (uint32_t)pt->cw[(size_t)l * Mmax + j] : 8u;
                }
            }
        }
        const float *prior = pick(a.prior, ip.part);
        const uint64_t *syn = pick(a.syn, ip.part);
        uint64_t *cand = pick(a.cand, ip.part);
        uint16_t *kstat = pick(a.kstat, ip.part);
        float *llr = pick(a.llr, ip.part);
        const int32_t *csrc = pt->csrc + (size_t)l * Mmax;

        for (int64_t shot = ip.begin; shot < ip.end; ++shot) {
            // ---------------- fill: clear messages and decisions, stage syndrome (and priors)
            {
                uint4 *z = reinterpret_cast<uint4 *>(ibase);
                constexpr int nz = (int)(LY::kTail / 16);
                for (int i = lane; i < nz; i += 64) z[i] = make_uint4(0u, 0u, 0u, 0u);
                if (lane < Ws) synl[lane] = syn[shot * Ws + lane];
                if (a.prior_per_shot || kMuLds) {
                    const float *pr = prior + (a.prior_per_shot ? shot * n : 0);
                    for (int i = lane; i < n; i += 64) mul[i] = pr[i] + 0.0f;
                }
            }
            wave_sync();
            if (a.prior_per_shot) {
#pragma unroll
                for (int v = 0; v < PV; ++v) {
                    const int s = v * 64 + lane;
                    mu[v] = (v < vp && s < n) ? mul[vinfo[v] & 0xffffu] + 0.0f : 0.0f;
                }
            }
            uint32_t sbits = 0;
#pragma unroll
            for (int c = 0; c < PC; ++c) {
                const int j = c * 64 + lane;
                if (j < Ml) {
                    const int src = j < m ? j : csrc[j];
                    uint32_t bit = 0;
                    if (src >= 0) {
                        bit = (uint32_t)(synl[src >> 6] >> (src & 63)) & 1u;
                    } else {
                        for (int t = pt->comb_ptr[-src - 1]; t < pt->comb_ptr[-src]; ++t) {
                            const int r = pt->comb_idx[t];
                            bit ^= (uint32_t)(synl[r >> 6] >> (r & 63)) & 1u;
                        }
                    }
                    sbits |= bit << c;
                    if (SCHED == 1) sbl[j] = (unsigned char)bit;
                }
            }
            int it = 0, kfix = -1, K = T;
            bool conv = false;
            uint32_t decb = 0;
            if constexpr (SCHED == 1) {
                const int32_t *lp = pt->lev_ptr + pt->lev_off[l];
                const int nlev = pt->lev_off[l + 1] - pt->lev_off[l] - 1;
                const uint16_t *lc = pt->lev_chk + (size_t)l * Mmax;
                const uint4 *lt = pt->ltab + (size_t)l * Mmax * 8;
                while (true) {
                    // ---------------- posterior phase (r = 0 at iteration 0)
#pragma unroll
                    for (int v = 0; v < PV; ++v) {
                        if (v < vp) {
                            const int deg = (int)(vinfo[v] >> 16);
                            float Pv = 0.0f;
                            bool d = false;
                            switch (uniform_i32(dmaxp[v])) {
                            case 1: var_post<1, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            case 2: var_post<2, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            case 3: var_post<3, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            case 4: var_post<4, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            case 5: var_post<5, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            case 6: var_post<6, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            case 7: var_post<7, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            case 8: var_post<8, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            default: Pv = mu[v]; d = Pv < 0.0f; break;
                            }
                            decb = (decb & ~(1u << v)) | ((uint32_t)d << v);
                            if (llr) {
                                const int s = v * 64 + lane;
                                if (s < n) llr[((size_t)shot * L + l) * n + (vinfo[v] & 0xffffu)] = Pv;
                            }
                        }
                    }
                    wave_sync();
                    // ---------------- syndrome test
                    uint32_t unsat = 0;
#pragma unroll
                    for (int c = 0; c < PC; ++c) {
                        const int j = c * 64 + lane;
                        const lds_u8 *drow = lds_ptr_u8(ibase_addr + LY::kDecOff + 4u * (uint32_t)j);
                        uint32_t par = (sbits >> c) & 1u;
#pragma unroll
                        for (int k = 0; k < DC; ++k) par ^= drow[4 * k * Mpad];
                        unsat |= par & (j < Ml ? 1u : 0u);
                    }
                    const bool sat = __ballot(unsat != 0u) == 0ull;
                    if (!a.fixed_T) {
                        if (sat) { conv = true; K = it; break; }
                        if (it == T) { K = T; break; }
                    } else {
                        if (sat && kfix < 0) kfix = it;
                        if (it == T) { conv = kfix >= 0; K = conv ? kfix : T; break; }
                    }
                    // ---------------- sweep: levels in order, checks of a level in parallel
                    for (int lev = 0; lev < nlev; ++lev) {
                        const int b = lp[lev], e = lp[lev + 1];
                        for (int base = b; base < e; base += 64) {
                            const int idx = base + lane;
                            if (idx < e) {
                                const int j = lc[idx];
                                const uint32_t sb = sbl[j];
                                float q[DC];
#pragma unroll
                                for (int k = 0; k < DC; ++k) {
                                    const uint4 t = lt[j * 8 + k];
                                    const int vid = (int)(t.x & 0x3ffu);
                                    const int deg = (int)((t.x >> 12) & 0xfu);
                                    const uint32_t oth[7] = {t.x >> 16, t.y & 0xffffu, t.y >> 16, t.z & 0xffffu,
                                                             t.z >> 16, t.w & 0xffffu, t.w >> 16};
                                    float acc = mul[vid];
#pragma unroll
                                    for (int u = 0; u < kMaxVarDegree - 1; ++u) {
                                        if (u < dmax_rep - 1) {
                                            const uint32_t eo = oth[u];
                                            const float x = *lds_ptr_f32(ibase_addr +
                                                                         4u * ((eo & 7u) * (uint32_t)Mpad + (eo >> 3)));
                                            acc += u < deg - 1 ? x : 0.0f;
                                        }
                                    }
                                    q[k] = deg == 0 ? 3.402823466e38f : acc;
                                }
                                CheckRule<RULE>::template apply<DC>(q, (int)sb, alpha, rmax);
                                lds_f32 *row = lds_ptr_f32(ibase_addr + 4u * (uint32_t)j);
#pragma unroll
                                for (int k = 0; k < DC; ++k) row[k * Mpad] = q[k];
                            }
                            wave_sync();
                        }
                    }
                    ++it;
                }
            } else {
                while (true) {
                    // ---------------- variable phase
    #pragma unroll
                    for (int v = 0; v < PV; ++v) {
                        if (v < vp) {
                            const int deg = (int)(vinfo[v] >> 16);
                            float Pv = 0.0f;
                            bool d = false;
                            switch (uniform_i32(dmaxp[v])) {
                            case 1: var_rule<1, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            case 2: var_rule<2, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            case 3: var_rule<3, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            case 4: var_rule<4, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            case 5: var_rule<5, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            case 6: var_rule<6, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            case 7: var_rule<7, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            case 8: var_rule<8, LY::kDecOff>(ea[v], deg, mu[v], Pv, d); break;
                            default: Pv = mu[v]; d = Pv < 0.0f; break;
                            }
                            decb = (decb & ~(1u << v)) | ((uint32_t)d << v);
                            if (llr) {
                                const int s = v * 64 + lane;
                                if (s < n) llr[((size_t)shot * L + l) * n + (vinfo[v] & 0xffffu)] = Pv;
                            }
                        }
                    }
                    wave_sync();
                    // ---------------- check phase: syndrome test of the decisions, c->v messages.
                    // Rows beyond the representation's checks are junk rows (unused by it).
                    uint32_t unsat = 0;
    #pragma unroll
                    for (int c = 0; c < PC; ++c) {
                        const int j = c * 64 + lane;
                        lds_f32 *row = lds_ptr_f32(ibase_addr + 4u * (uint32_t)j);
                        const lds_u8 *drow = lds_ptr_u8(ibase_addr + LY::kDecOff + 4u * (uint32_t)j);
                        float q[DC];
                        uint32_t par = (sbits >> c) & 1u;
    #pragma unroll
                        for (int k = 0; k < DC; ++k) {
                            q[k] = row[k * Mpad];
                            par ^= drow[4 * k * Mpad];
                        }
                        if constexpr (DC == 8) {
                            const int w = (int)cwp[c];
    #pragma unroll
                            for (int k = 2; k < DC; ++k)
                                if (k >= w) q[k] = 3.402823466e38f;
                        }
                        unsat |= par & (j < Ml ? 1u : 0u);
                        CheckRule<RULE>::template apply<DC>(q, (int)((sbits >> c) & 1u), alpha, rmax);
    #pragma unroll
                        for (int k = 0; k < DC; ++k) row[k * Mpad] = q[k];
                    }
                    const bool sat = __ballot(unsat != 0u) == 0ull;
                    // ---------------- halting (Section II-B)
                    if (!a.fixed_T) {
                        if (sat) { conv = true; K = it; break; }
                        if (it == T) { K = T; break; }
                    } else {
                        if (sat && kfix < 0) kfix = it;
                        if (it == T) { conv = kfix >= 0; K = conv ? kfix : T; break; }
                    }
                    ++it;
                    wave_sync();
                }
            }
            // ---------------- output: bit-packed hard decisions via the staging words
            if (lane < 2 * W) stage[lane] = 0u;
            wave_sync();
#pragma unroll
            for (int v = 0; v < PV; ++v) {
                const int s = v * 64 + lane;
                if (v < vp && s < n && ((decb >> v) & 1u)) {
                    const uint32_t id = vinfo[v] & 0xffffu;
                    atomicOr(&stage[id >> 5], 1u << (id & 31));
                }
            }
            wave_sync();
            const size_t inst = (size_t)shot * L + l;
            if (lane < W) cand[inst * W + lane] = reinterpret_cast<const uint64_t *>(stage)[lane];
            if (lane == 0) kstat[inst] = (uint16_t)(K | (conv ? 0x8000 : 0));
            wave_sync();
        }

        if (a.persistent) {
            unsigned long long v = 0;
            if (lane == 0) v = atomicAdd(a.queue, 1ull);
            item = uniform_i64((long long)v);
        } else {
            item = a.n_items;
        }
    }
}

// ----------------------------------------------------------------------------- select

__device__ __forceinline__ int popc_words(const uint64_t *w, int W) {
    int c = 0;
    for (int i = 0; i < W; ++i) c += __popcll(w[i]);
    return c;
}

__device__ __forceinline__ bool words_equal(const uint64_t *x, const uint64_t *y, int W) {
    for (int i = 0; i < W; ++i)
        if (x[i] != y[i]) return false;
    return true;
}

// One thread per (part, shot): decision over the converged representations.
__global__ __launch_bounds__(256) void select_kernel(SelectArgs a) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = a.shots * a.nparts;
    long long c_sumk = 0, c_edges = 0, c_noconv = 0, c_ties = 0;
    if (idx < total) {
        const int part = a.part0 + (int)(idx / a.shots);
        const int64_t shot = idx - (int64_t)(part - a.part0) * a.shots;
        const DevPart &pt = a.part[part];
        const int L = pt.L, W = pt.W;
        const uint64_t *cand = a.cand[part] + (size_t)shot * L * W;
        const uint16_t *ks = a.kstat[part] + (size_t)shot * L;
        uint64_t convm = 0;
        int best = -1, bw = 0x7fffffff, kmax = 0;
        for (int l = 0; l < L; ++l) {
            const int st = ks[l];
            const int K = st & 0x7fff;
            c_sumk += K;
            c_edges += (long long)K * pt.E[l];
            kmax = max(kmax, K);
            if (st & 0x8000) {
                convm |= 1ull << l;
                if (a.rule == 0) {
                    const int w = popc_words(cand + (size_t)l * W, W);
                    if (w < bw) { bw = w; best = l; }
                }
            }
        }
        if (a.rule == 1) {
            // FWS: argmax count(e) / (w(e) + 1), exact cross-multiplied comparison,
            // ties to the smaller index of first occurrence
            long long bc = 0, bw1 = 1;
            for (int l = 0; l < L; ++l) {
                if (!((convm >> l) & 1ull)) continue;
                const uint64_t *cl = cand + (size_t)l * W;
                bool first = true;
                for (int k = 0; k < l && first; ++k)
                    if (((convm >> k) & 1ull) && words_equal(cand + (size_t)k * W, cl, W)) first = false;
                if (!first) continue;
                long long cnt = 0;
                for (int k = l; k < L; ++k)
                    if (((convm >> k) & 1ull) && words_equal(cand + (size_t)k * W, cl, W)) ++cnt;
                const long long w1 = popc_words(cl, W) + 1;
                if (best < 0 || cnt * bw1 > bc * w1) { best = l; bc = cnt; bw1 = w1; }
            }
        }
        if (a.counters) {
            if (best < 0) {
                c_noconv = 1;
            } else if (a.rule == 0) {
                const uint64_t *cb = cand + (size_t)best * W;
                for (int l = best + 1; l < L; ++l) {
                    if (((convm >> l) & 1ull) && popc_words(cand + (size_t)l * W, W) == bw &&
                        !words_equal(cand + (size_t)l * W, cb, W)) { c_ties = 1; break; }
                }
            }
            if (a.kmax_shot) atomicMax(&a.kmax_shot[shot], kmax);
        }
        uint64_t *co = a.corr[part] + (size_t)shot * W;
        for (int w = 0; w < W; ++w) co[w] = best >= 0 ? cand[(size_t)best * W + w] : 0ull;
        a.conv[part][shot] = convm;
        a.basis[part][shot] = (int16_t)best;
    }
    if (a.counters) {
        c_sumk = wave_sum_i64(c_sumk);
        c_edges = wave_sum_i64(c_edges);
        c_noconv = wave_sum_i64(c_noconv);
        c_ties = wave_sum_i64(c_ties);
        if ((threadIdx.x & 63) == 0) {
            atomicAdd((unsigned long long *)&a.counters[4], (unsigned long long)c_sumk);
            atomicAdd((unsigned long long *)&a.counters[5], (unsigned long long)c_edges);
            atomicAdd((unsigned long long *)&a.counters[6], (unsigned long long)c_noconv);
            atomicAdd((unsigned long long *)&a.counters[7], (unsigned long long)c_ties);
        }
    }
}

// ----------------------------------------------------------------------------- failures

// One thread per shot.  Part X: residual r = e_X ^ corr_x fails iff H_Z r != 0 or
// L_Z r != 0 (it is then not a product of X stabilizers); part Z symmetric.
// part[0] holds H_Z and L_Z, part[1] holds H_X and L_X.
__global__ __launch_bounds__(256) void fail_kernel(FailArgs a) {
    const int64_t shot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    long long c_fail = 0, c_fx = 0, c_fz = 0, c_kmax = 0;
    if (shot < a.shots) {
        uint32_t flags = 0;
        for (int pt = 0; pt < 2; ++pt) {
            const DevPart &P = a.part[pt];
            const int W = P.W;
            const uint64_t *e = a.err[pt] + (size_t)shot * W;
            const uint64_t *c = a.corr[pt] + (size_t)shot * W;
            bool bad = false;
            for (int j = 0; j < P.m && !bad; ++j) {
                uint32_t par = 0;
                for (int k = P.hrow_ptr[j]; k < P.hrow_ptr[j + 1]; ++k) {
                    const int col = P.hrow_idx[k];
                    par ^= (uint32_t)((e[col >> 6] ^ c[col >> 6]) >> (col & 63)) & 1u;
                }
                bad = par != 0;
            }
            for (int r = 0; r < P.k && !bad; ++r) {
                int cnt = 0;
                for (int w = 0; w < W; ++w) cnt += __popcll((e[w] ^ c[w]) & P.logical[(size_t)r * W + w]);
                bad = (cnt & 1) != 0;
            }
            if (bad) flags |= 1u << pt;
        }
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

hipError_t launch_select(const SelectArgs &a, hipStream_t s) {
    const int64_t total = a.shots * a.nparts;
    hipLaunchKernelGGL(select_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
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

size_t bp_lds_limit() { return 64 * 1024; }  // per workgroup

// Instantiated (PV, PC): variable and check passes of 64 lanes.
struct PassPair {
    int pv, pc;
};
static const PassPair kPairs[] = {{1, 1}, {2, 1}, {2, 2}, {3, 2}, {3, 3}, {5, 5}, {9, 9}, {14, 14}, {16, 16}};

static bool pick_pair(int pv_need, int pc_need, PassPair &out) {
    for (const PassPair &p : kPairs)
        if (p.pv >= pv_need && p.pc >= pc_need) { out = p; return true; }
    return false;
}

static void passes_needed(const BPArgs &a, int &pv, int &pc) {
    pv = 1; pc = 1;
    for (int p = a.part0; p < a.part0 + a.nparts; ++p) {
        pv = max(pv, (a.part[p].n + 63) / 64);
        pc = max(pc, (a.part[p].Mmax + 1 + 63) / 64);  // + the sink row
    }
}

int bp_max_passes(int lpi) { return lpi == 64 ? 16 : 0; }

bool bp_supported(int lpi, int passes, int dc_uniform, int rule, int schedule) {
    (void)dc_uniform;
    if ((schedule != 0 && schedule != 1) || (rule != 0 && rule != 1) || lpi != 64) return false;
    PassPair pp;
    return pick_pair(passes, passes, pp);
}

bool bp_layout(const BPArgs &a, int &mpad) {
    int pv, pc;
    passes_needed(a, pv, pc);
    PassPair pp;
    if (!pick_pair(pv, pc, pp)) return false;
    mpad = 64 * pp.pc;
    return true;
}

template <int PV, int PC, int DC, int RULE, int SCHED>
static hipError_t launch_wave_t(const BPArgs &a, const BPConfig &cfg, hipStream_t s) {
    const int wpb = cfg.waves_per_block;
    const size_t lds = (size_t)wpb * a.inst_bytes;
    const int64_t blocks = a.persistent ? cfg.blocks : (a.n_items + wpb - 1) / wpb;
    hipLaunchKernelGGL((bp_wave_kernel<PV, PC, DC, RULE, SCHED>), dim3((unsigned)blocks), dim3(64 * wpb), lds, s,
                       a);
    return hipGetLastError();
}

template <int PV, int PC, int SCHED>
static hipError_t launch_pair(const BPArgs &a, const BPConfig &cfg, int rule, hipStream_t s) {
    bool u6 = true;
    for (int p = a.part0; p < a.part0 + a.nparts; ++p) u6 = u6 && a.part[p].uniform_dc == 6;
    if (rule == 0)
        return u6 ? launch_wave_t<PV, PC, 6, 0, SCHED>(a, cfg, s) : launch_wave_t<PV, PC, 8, 0, SCHED>(a, cfg, s);
    return u6 ? launch_wave_t<PV, PC, 6, 1, SCHED>(a, cfg, s) : launch_wave_t<PV, PC, 8, 1, SCHED>(a, cfg, s);
}

template <int SCHED>
static hipError_t launch_sched(const BPArgs &a, const BPConfig &cfg, int rule, const PassPair &pp, hipStream_t s) {
#ifndef MBBP_KERNEL_PROBE
    switch (pp.pv * 100 + pp.pc) {
    case 101: return launch_pair<1, 1, SCHED>(a, cfg, rule, s);
    case 201: return launch_pair<2, 1, SCHED>(a, cfg, rule, s);
    case 202: return launch_pair<2, 2, SCHED>(a, cfg, rule, s);
    case 302: return launch_pair<3, 2, SCHED>(a, cfg, rule, s);
    case 303: return launch_pair<3, 3, SCHED>(a, cfg, rule, s);
    case 505: return launch_pair<5, 5, SCHED>(a, cfg, rule, s);
    case 909: return launch_pair<9, 9, SCHED>(a, cfg, rule, s);
    case 1414: return launch_pair<14, 14, SCHED>(a, cfg, rule, s);
    case 1616: return launch_pair<16, 16, SCHED>(a, cfg, rule, s);
    }
#else
    (void)a; (void)cfg; (void)rule; (void)pp; (void)s;
#endif
    return hipErrorInvalidValue;
}

hipError_t launch_bp(const BPArgs &a, const BPConfig &cfg, int schedule, int rule, hipStream_t s) {
    if ((schedule != 0 && schedule != 1) || cfg.lpi != 64) return hipErrorInvalidValue;
    int pv, pc;
    passes_needed(a, pv, pc);
    PassPair pp;
    if (!pick_pair(pv, pc, pp)) return hipErrorInvalidValue;
    return schedule == 0 ? launch_sched<0>(a, cfg, rule, pp, s) : launch_sched<1>(a, cfg, rule, pp, s);
}

}  // namespace mbbp
