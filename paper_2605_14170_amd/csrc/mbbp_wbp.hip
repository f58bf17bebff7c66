// Adjoint (backward) kernel of the weighted min-sum decoder for gfx950 (wave64),
// and the deterministic reduction of its per-instance gradients.
//
// Forward map (flooding, T iterations, no early stop) of one instance:
//   r^(t) = clamp((1 - beta_t) * S * (alpha_t * M(q^(t-1))) + beta_t * r^(t-1)),
//   q^(t) = mu + exclusion sums of r^(t),  P^(T) = mu + sum r^(T),
// with r^(0) = 0 and q^(0) = mu.  Given dL/dP^(T), the adjoint runs t = T .. 1:
//   check rows:  rb^(t) -> (through the clamp) wb; dL/dbeta_t += wb (r^(t-1) - v);
//                dL/dalpha_t += wb (1 - beta_t) S M;  rb^(t-1) = wb beta_t;
//                qb^(t-1) at the minimizing slot += wb (1 - beta_t) S alpha_t sgn(q)
//   variables:   rb^(t-1)_e += sum over the variable's other edges e' of qb^(t-1)_e'.
// The forward stores r^(t) every ckpt_every iterations; the adjoint recomputes each
// segment from its checkpoint with the forward's own arithmetic (the shared rule
// functions), so gradients do not depend on the checkpoint interval.
//
// One instance per wavefront, the decoding kernel's table layout.  LDS per
// instance (A = one [DC][S] float array, S the slot stride): Q (v->c messages) at 0, RB (adjoint
// of c->v messages) at A, QB (adjoint of v->c messages) at 2A, the segment's
// c->v messages R[0..ckpt_every) at 3A, then syndrome words and per-shot priors.
#include <hip/hip_runtime.h>

#include "mbbp_bp_rules.h"
#include "mbbp_device.h"
#include "mbbp_wave.h"

namespace mbbp {

// q = mu + exclusion sums of the c->v messages read at ea + roff, written at ea.
template <int D>
__device__ __forceinline__ void var_q(const uint32_t *ea, int deg, float mu, uint32_t roff) {
    float r[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const float x = *lds_ptr_f32(ea[k] + roff);
        r[k] = k < deg ? x : 0.0f;
    }
    float q[D];
    (void)excl_sums<D>(r, mu, q);
#pragma unroll
    for (int k = 0; k < D; ++k) *lds_ptr_f32(ea[k]) = q[k];
}

// Adjoint of the exclusion sums: rb_e += sum over the variable's other edges of qb.
template <int D>
__device__ __forceinline__ void var_adj(const uint32_t *ea, int deg, uint32_t qboff, uint32_t rboff) {
    float g[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const float x = *lds_ptr_f32(ea[k] + qboff);
        g[k] = k < deg ? x : 0.0f;
    }
    float s[D];
    (void)excl_sums<D>(g, 0.0f, s);
#pragma unroll
    for (int k = 0; k < D; ++k)
        if (k < deg) *lds_ptr_f32(ea[k] + rboff) += s[k];
}

// Variable phase of every pass: q = mu + exclusion sums of the c->v messages at
// byte offset roff from each edge address.
template <int PV>
__device__ __forceinline__ void var_phase(const uint32_t (&ea)[PV][kMaxVarDegree], const uint32_t (&vinfo)[PV],
                                          const int (&dmaxp)[PV], const float (&mu)[PV], int vp, uint32_t roff) {
#pragma unroll
    for (int v = 0; v < PV; ++v) {
        if (v < vp) {
            const int deg = (int)((vinfo[v] >> 16) & 0xffu);
            switch (uniform_i32(dmaxp[v])) {
            case 1: var_q<1>(ea[v], deg, mu[v], roff); break;
            case 2: var_q<2>(ea[v], deg, mu[v], roff); break;
            case 3: var_q<3>(ea[v], deg, mu[v], roff); break;
            case 4: var_q<4>(ea[v], deg, mu[v], roff); break;
            case 5: var_q<5>(ea[v], deg, mu[v], roff); break;
            case 6: var_q<6>(ea[v], deg, mu[v], roff); break;
            case 7: var_q<7>(ea[v], deg, mu[v], roff); break;
            case 8: var_q<8>(ea[v], deg, mu[v], roff); break;
            default: break;
            }
        }
    }
}

template <int PV, int PC, int DC>
__global__ __launch_bounds__(256) void wbp_backward_kernel(WBPBackArgs a) {
    using LY = Layout<PC, kRuleNMS, DC>;
    constexpr int S = LY::S;           // slot stride of the LDS arrays (words)
    constexpr uint32_t A = LY::kMsg;   // bytes of one [DC][S] float array
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int64_t item = (int64_t)blockIdx.x * (blockDim.x >> 6) + wib;
    if (item >= a.n_items) return;  // wave-uniform
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char *ibase = smem + (size_t)wib * a.inst_bytes;
    const uint32_t ibase_addr = (uint32_t)(size_t)(lds_u8 *)ibase;
    const int C = a.ckpt_every;
    uint64_t *synl = reinterpret_cast<uint64_t *>(ibase + (3u + (uint32_t)C) * A);
    float *mul = reinterpret_cast<float *>(synl + a.ws);

    const int l = (int)(item / a.shots);
    const int64_t shot = item - (int64_t)l * a.shots;
    const DevPart *pt = a.dpart;
    const int n = pt->n, Mmax = pt->Mmax, Ws = pt->Ws, L = pt->L;
    const int vp = (n + 63) >> 6;
    const size_t inst = (size_t)shot * L + l;
    const float rmax = a.rmax;

    uint32_t ea[PV][kMaxVarDegree];
    uint32_t vinfo[PV];
    int dmaxp[PV];
    uint32_t cwp[PC];
    float mu[PV];
    {
        const uint4 *vo4 = reinterpret_cast<const uint4 *>(pt->voff) + (size_t)l * n;
        const uint16_t *vid = pt->vid + (size_t)l * n;
        const uint8_t *vdg = pt->vdeg + (size_t)l * n;
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
                ea[v][k] = ibase_addr + 4u * ((e & 7u) * (uint32_t)S + (e >> 3));
            }
            vinfo[v] = id | ((uint32_t)deg << 16) | (valid ? 0x80000000u : 0u);
            dmaxp[v] = uniform_i32(wave_max_i32(deg));
            if (!a.prior_per_shot) mu[v] = valid ? a.prior[id] + 0.0f : 0.0f;
        }
#pragma unroll
        for (int c = 0; c < PC; ++c) {
            const int j = c * 64 + lane;
            cwp[c] = (DC == 8 && j < Mmax) ? (uint32_t)pt->cw[(size_t)l * Mmax + j] : 8u;
        }
    }
    // clear Q, RB, QB and the segment arrays; stage the syndrome and priors
    {
        uint4 *z = reinterpret_cast<uint4 *>(ibase);
        const int nz = (int)((3u + (uint32_t)C) * A / 16u);
        for (int i = lane; i < nz; i += 64) z[i] = make_uint4(0u, 0u, 0u, 0u);
        if (lane < Ws) synl[lane] = a.syn[shot * Ws + lane];
        if (a.prior_per_shot)
            for (int i = lane; i < n; i += 64) mul[i] = a.prior[shot * n + i] + 0.0f;
    }
    wave_sync();
    if (a.prior_per_shot) {
#pragma unroll
        for (int v = 0; v < PV; ++v) mu[v] = (vinfo[v] >> 31) ? mul[vinfo[v] & 0xffffu] + 0.0f : 0.0f;
    }
    uint32_t sbits = 0, rowv = 0;  // syndrome bit and "real check" flag per pass
    {
        const int32_t *csrc = pt->csrc + (size_t)l * Mmax;
#pragma unroll
        for (int c = 0; c < PC; ++c) {
            const int j = c * 64 + lane;
            const int src = j < Mmax ? csrc[j] : kJunkRow;
            if (src != kJunkRow) {
                rowv |= 1u << c;
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
            }
        }
    }
    // adjoint of P^(T) = mu + sum r^(T): every edge of variable i receives dL/dP_i
#pragma unroll
    for (int v = 0; v < PV; ++v) {
        if (vinfo[v] >> 31) {
            const float g = a.grad_llr[inst * n + (vinfo[v] & 0xffffu)];
            const int deg = (int)((vinfo[v] >> 16) & 0xffu);
#pragma unroll
            for (int k = 0; k < kMaxVarDegree; ++k)
                if (k < deg) *lds_ptr_f32(ea[v][k] + A) = g;
        }
    }
    wave_sync();

    const int T = a.T;
    const int nseg = (T + C - 1) / C;
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int t0 = seg * C, t1 = min(T, t0 + C);
        {
            uint4 *r0 = reinterpret_cast<uint4 *>(ibase + 3u * A);
            if (t0 == 0) {
                for (int i = lane; i < (int)(A / 16); i += 64) r0[i] = make_uint4(0u, 0u, 0u, 0u);
            } else {
                const uint4 *src =
                    reinterpret_cast<const uint4 *>(a.ckpt + (inst * a.n_ck + (size_t)(seg - 1)) * (A / 4));
                for (int i = lane; i < (int)(A / 16); i += 64) r0[i] = src[i];
            }
        }
        wave_sync();
        // recompute r^(t0+1) .. r^(t1-1) into R[1 ..]
        for (int t = t0 + 1; t < t1; ++t) {
            const uint32_t rprev = (3u + (uint32_t)(t - 1 - t0)) * A, rnew = rprev + A;
            var_phase<PV>(ea, vinfo, dmaxp, mu, vp, rprev);
            wave_sync();
            const float al = a.walpha[(size_t)(t - 1) * L + l], be = a.wbeta[(size_t)(t - 1) * L + l];
            const float keep = 1.0f - be;
#pragma unroll
            for (int c = 0; c < PC; ++c) {
                const int j = c * 64 + lane;
                const lds_f32 *qrow = lds_ptr_f32(ibase_addr + 4u * (uint32_t)j);
                lds_f32 *rrow = lds_ptr_f32(ibase_addr + rprev + 4u * (uint32_t)j);
                float q[DC], rp[DC];
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    q[k] = qrow[k * S];
                    rp[k] = rrow[k * S];
                    if (DC == 8 && k >= 2 && k >= (int)cwp[c]) q[k] = 3.402823466e38f;
                }
                WeightedRule::apply<DC>(q, rp, (int)((sbits >> c) & 1u), al, keep, be, rmax);
                lds_f32 *orow = lds_ptr_f32(ibase_addr + rnew + 4u * (uint32_t)j);
#pragma unroll
                for (int k = 0; k < DC; ++k) orow[k * S] = q[k];
            }
            wave_sync();
        }
        // adjoint of iterations t1 .. t0+1
        for (int t = t1; t > t0; --t) {
            const uint32_t rprev = (3u + (uint32_t)(t - 1 - t0)) * A;
            var_phase<PV>(ea, vinfo, dmaxp, mu, vp, rprev);  // q^(t-1)
            wave_sync();
            const float al = a.walpha[(size_t)(t - 1) * L + l], be = a.wbeta[(size_t)(t - 1) * L + l];
            const float keep = 1.0f - be;
            float ga = 0.0f, gb = 0.0f;
#pragma unroll
            for (int c = 0; c < PC; ++c) {
                const int j = c * 64 + lane;
                const lds_f32 *qrow = lds_ptr_f32(ibase_addr + 4u * (uint32_t)j);
                const lds_f32 *rrow = lds_ptr_f32(ibase_addr + rprev + 4u * (uint32_t)j);
                lds_f32 *rbrow = lds_ptr_f32(ibase_addr + A + 4u * (uint32_t)j);
                lds_f32 *qbrow = lds_ptr_f32(ibase_addr + 2u * A + 4u * (uint32_t)j);
                float q[DC], rp[DC], rb[DC];
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    q[k] = qrow[k * S];
                    rp[k] = rrow[k * S];
                    rb[k] = rbrow[k * S];
                    if (DC == 8 && k >= 2 && k >= (int)cwp[c]) {
                        q[k] = 3.402823466e38f;
                        rb[k] = 0.0f;
                    }
                }
                float rbp[DC], qb[DC];
                float gal = 0.0f, gbl = 0.0f;
                WeightedRule::adjoint<DC>(q, rp, rb, (int)((sbits >> c) & 1u), al, keep, be, rmax, rbp, qb, gal,
                                          gbl);
                if ((rowv >> c) & 1u) {
                    ga += gal;
                    gb += gbl;
                }
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    rbrow[k * S] = rbp[k];
                    qbrow[k * S] = qb[k];
                }
            }
            wave_sync();
            if (t > 1) {  // q^(0) = mu does not depend on the weights
#pragma unroll
                for (int v = 0; v < PV; ++v) {
                    if (v < vp) {
                        const int deg = (int)((vinfo[v] >> 16) & 0xffu);
                        switch (uniform_i32(dmaxp[v])) {
                        case 1: var_adj<1>(ea[v], deg, 2u * A, A); break;
                        case 2: var_adj<2>(ea[v], deg, 2u * A, A); break;
                        case 3: var_adj<3>(ea[v], deg, 2u * A, A); break;
                        case 4: var_adj<4>(ea[v], deg, 2u * A, A); break;
                        case 5: var_adj<5>(ea[v], deg, 2u * A, A); break;
                        case 6: var_adj<6>(ea[v], deg, 2u * A, A); break;
                        case 7: var_adj<7>(ea[v], deg, 2u * A, A); break;
                        case 8: var_adj<8>(ea[v], deg, 2u * A, A); break;
                        default: break;
                        }
                    }
                }
                wave_sync();
            }
            ga = wave_sum_f32(ga);
            gb = wave_sum_f32(gb);
            if (lane == 0) a.partial[(size_t)(t - 1) * a.n_items + item] = make_float2(ga, gb);
        }
    }
}

// One block per (t, l): FP64 sums over shots in a fixed order.
__global__ __launch_bounds__(256) void wbp_reduce_kernel(const float2 *partial, int64_t shots, int T, int L,
                                                          float *galpha, float *gbeta) {
    __shared__ double sa[256], sb[256];
    const int b = blockIdx.x;
    const int t = b / L, l = b - (b / L) * L;
    const float2 *p = partial + (size_t)t * L * shots + (size_t)l * shots;
    double xa = 0.0, xb = 0.0;
    for (int64_t i = threadIdx.x; i < shots; i += blockDim.x) {
        const float2 v = p[i];
        xa += (double)v.x;
        xb += (double)v.y;
    }
    sa[threadIdx.x] = xa;
    sb[threadIdx.x] = xb;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sa[threadIdx.x] += sa[threadIdx.x + o];
            sb[threadIdx.x] += sb[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        galpha[b] += (float)sa[0];
        gbeta[b] += (float)sb[0];
    }
}

struct WPair {
    int pv, pc;
};
static const WPair kWPairs[] = {{1, 1}, {2, 1}, {2, 2}, {3, 2}, {3, 3}, {5, 5}};

bool wbp_backward_supported(int pv, int pc) {
    for (const WPair &p : kWPairs)
        if (p.pv == pv && p.pc == pc) return true;
    return false;
}

template <int PV, int PC, int DC>
static hipError_t launch_wbp_t(const WBPBackArgs &a, int wpb, hipStream_t s) {
    const int64_t blocks = (a.n_items + wpb - 1) / wpb;
    // one wave per item: the dispatch's thread count must fit 32 bits
    if (blocks * 64 * wpb >= (int64_t)1 << 32) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((wbp_backward_kernel<PV, PC, DC>), dim3((unsigned)blocks), dim3(64 * wpb),
                       (size_t)wpb * a.inst_bytes, s, a);
    return hipGetLastError();
}

template <int PV, int PC>
static hipError_t launch_wbp_dc(const WBPBackArgs &a, int dc, int wpb, hipStream_t s) {
    return dc == 6 ? launch_wbp_t<PV, PC, 6>(a, wpb, s) : launch_wbp_t<PV, PC, 8>(a, wpb, s);
}

hipError_t launch_wbp_backward(const WBPBackArgs &a, int pv, int pc, int dc, int waves_per_block, hipStream_t s) {
    if (a.n_items <= 0) return hipSuccess;
    switch (pv * 100 + pc) {
    case 101: return launch_wbp_dc<1, 1>(a, dc, waves_per_block, s);
    case 201: return launch_wbp_dc<2, 1>(a, dc, waves_per_block, s);
    case 202: return launch_wbp_dc<2, 2>(a, dc, waves_per_block, s);
    case 302: return launch_wbp_dc<3, 2>(a, dc, waves_per_block, s);
    case 303: return launch_wbp_dc<3, 3>(a, dc, waves_per_block, s);
    case 505: return launch_wbp_dc<5, 5>(a, dc, waves_per_block, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_wbp_reduce(const float2 *partial, int64_t shots, int T, int L, float *grad_alpha,
                             float *grad_beta, hipStream_t s) {
    if (T <= 0 || L <= 0) return hipSuccess;
    hipLaunchKernelGGL(wbp_reduce_kernel, dim3((unsigned)(T * L)), dim3(256), 0, s, partial, shots, T, L,
                       grad_alpha, grad_beta);
    return hipGetLastError();
}

}  // namespace mbbp
