// BP kernel of the MBBP-LD library for gfx950 (CDNA4, wave64): BP on the L
// representations [H; H_t] (eqs. (1)-(2), Section II-B), flooding or serial
// schedule, normalized min-sum, weighted (per-iteration, per-representation
// alpha and damping beta) min-sum, or sum-product.  The plain form (one work item
// per wave) and the persistent form (atomic work queue, per-instance refill)
// share this one kernel.
//
// One BP instance (shot, representation, CSS part) per wavefront; the instance
// state is wave-uniform.  Lane i handles variable slots v * 64 + i and checks
// c * 64 + i (v < PV, c < PC, compile-time), so per-lane graph tables and priors
// live in VGPRs.  Per-edge messages live in LDS, one float per edge, slot-major,
// in place: the check phase reads v->c messages of its row and overwrites them
// with c->v messages, the variable phase reads c->v messages and overwrites them
// with v->c messages (the weighted rule keeps c->v messages in a second array,
// since its damping reads the previous iteration's c->v message).  The variable
// phase also writes its hard decision as a byte cell beside every edge, so a
// check reads its row's decisions with its message loads (syndrome test).
// Phases are wave-synchronous, except for large codes under the flooding schedule,
// where WPI wavefronts of a workgroup share one instance (each takes PV variable and
// PC check passes of the instance's WPI * PV and WPI * PC) and workgroup barriers
// separate the phases: half the per-lane tables each, so twice the wavefronts fit.
#include <hip/hip_runtime.h>

#include "mbbp_bp_rules.h"
#include "mbbp_device.h"
#include "mbbp_wave.h"

namespace mbbp {

struct ItemPos {
    int part, l;
    int64_t begin, end;
};

__device__ __forceinline__ ItemPos decode_item(const BPArgs &a, int64_t item) {
    const int64_t rank = item / a.n_chunks;
    const int64_t ch = item - rank * a.n_chunks;
    // (a load through a generic pointer counts as divergent: keep the index uniform)
    const int pl = __builtin_amdgcn_readfirstlane(a.item_order ? a.item_order[rank] : (int)rank);
    ItemPos p;
    p.part = a.part0 + pl / a.L;
    p.l = pl - (pl / a.L) * a.L;
    p.begin = ch * a.chunk;
    p.end = min(p.begin + (int64_t)a.chunk, a.shots);
    return p;
}

template <typename T>
__device__ __forceinline__ T pick(const T (&v)[2], int part) { return part == 0 ? v[0] : v[1]; }



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
// WPI: wavefronts per instance (1, or up to 8 for the flooding schedule with NMS or
// sum-product: then one instance per workgroup of WPI wavefronts, the instance's
// passes split between them).
template <int PV, int PC, int DC, int RULE, int SCHED, int WPI = 1>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(
    WPI > 1 ? 6 : PV <= 3 ? (RULE == kRuleWeighted ? 3 : 4) : (PV <= 5 ? 3 : 1))))
void bp_wave_kernel(BPArgs a) {
    // flooding min-sum and sum-product keep messages in slot pairs (edge (p, k) at word
    // (k >> 1) * 2S + 2p + (k & 1)): a check row moves two slots per 8-byte access
    constexpr bool kPairs = SCHED == 0 && RULE != kRuleWeighted;
    using LY = LayoutM<64 * PC * WPI, RULE, DC, (PC * WPI >= 9), kPairs>;
    static_assert(RULE != kRuleWeighted || SCHED == 0, "the weighted rule is defined for flooding");
    static_assert(WPI == 1 || (SCHED == 0 && RULE != kRuleWeighted && WPI <= 8), "shared instances: flooding NMS / SPA");
    constexpr int S = LY::S;  // slot stride of the LDS arrays (words)
    static_assert(!kPairs || (DC % 2 == 0 && S % 16 == 1), "slot pairs");
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave-uniform
    const int sub = WPI > 1 ? wib : 0;  // this wave's share of the instance's passes
    extern __shared__ __align__(16) unsigned char smem[];
    // 32-bit LDS byte addresses of this wave's instance (wave-uniform: scalar registers)
    const uint32_t ibase_addr = (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)((uint32_t)(size_t)(lds_u8 *)smem + (uint32_t)(WPI > 1 ? 0 : wib * a.inst_bytes)));
    // the DC message slots of check position j (flooding: from slot pairs)
    auto row_load = [&](int j, float (&q)[DC]) {
        if constexpr (kPairs) {
#pragma unroll
            for (int u = 0; u < DC / 2; ++u) {
                const f32x2 w = *lds_ptr_f32x2(ibase_addr + 8u * ((uint32_t)(u * S) + (uint32_t)j));
                q[2 * u] = w.x;
                q[2 * u + 1] = w.y;
            }
        } else {
            const lds_f32 *row = lds_ptr_f32(ibase_addr + 4u * (uint32_t)j);
#pragma unroll
            for (int k = 0; k < DC; ++k) q[k] = row[k * S];
        }
    };
    auto row_store = [&](int j, const float (&q)[DC]) {
        if constexpr (kPairs) {
#pragma unroll
            for (int u = 0; u < DC / 2; ++u) {
                f32x2 w;
                w.x = q[2 * u];
                w.y = q[2 * u + 1];
                *lds_ptr_f32x2(ibase_addr + 8u * ((uint32_t)(u * S) + (uint32_t)j)) = w;
            }
        } else {
            lds_f32 *row = lds_ptr_f32(ibase_addr + 4u * (uint32_t)j);
#pragma unroll
            for (int k = 0; k < DC; ++k) row[k * S] = q[k];
        }
    };
    // shared instances: the work item and two halting flags after the instance's LDS
    lds_u32 *ctl = lds_ptr_u32((uint32_t)(size_t)(lds_u8 *)smem + (uint32_t)a.inst_bytes);
    // the instance's phase boundary: its wavefronts' LDS writes seen by all of them
    auto inst_sync = [&]() {
        if constexpr (WPI > 1) __syncthreads();
        else wave_sync();
    };
    lds_u64 *synl = lds_ptr_u64(ibase_addr + LY::kTail);                           // syndrome words
    lds_u32 *stage = lds_ptr_u32(ibase_addr + LY::kTail + 8u * (uint32_t)a.ws_max);  // output staging
    // flooding min-sum / sum-product: absent edges of pass g (slots beyond a variable's
    // degree) read and write word g here, which the check phase zeroes, so a variable
    // phase reads +0 there; their decision cells are those of position Mmax, which no
    // check of any representation uses (other forms: absent edges use position Mmax)
    constexpr bool kZSink = SCHED == 0 && RULE != kRuleWeighted;
    const uint32_t zsk_addr = ibase_addr + LY::kTail + 8u * (uint32_t)(a.ws_max + a.w_max);
    lds_f32 *zsk = lds_ptr_f32(zsk_addr);  // 16 words
    lds_f32 *mul = lds_ptr_f32(zsk_addr + 64u);  // priors
    lds_u8 *sbl = lds_ptr_u8(zsk_addr + 64u +
                             4u * (uint32_t)a.n_max);  // serial: syndrome byte per check
    constexpr bool kMuLds = SCHED == 1;  // the serial sweep reads priors from LDS

    // next work item: from the queue (persistent), or the grid position and then a
    // grid-sized stride (the grid is capped: its thread count must fit 32 bits); with
    // shared instances wave 0 takes it and the workgroup reads it from LDS
    auto next_item = [&](int64_t cur) -> int64_t {
        if (!a.persistent) {
            const int64_t waves = WPI > 1 ? 1 : (int64_t)(blockDim.x >> 6);
            if (cur >= 0) return cur + (int64_t)gridDim.x * waves;
            return WPI > 1 ? (int64_t)blockIdx.x : (int64_t)blockIdx.x * waves + wib;
        }
        if constexpr (WPI > 1) {
            if (threadIdx.x == 0) {
                const unsigned long long v = atomicAdd(a.queue, 1ull);
                ctl[0] = (uint32_t)v;
                ctl[1] = (uint32_t)(v >> 32);
            }
            __syncthreads();
            const int64_t it = (int64_t)(((uint64_t)ctl[1] << 32) | ctl[0]);
            __syncthreads();
            return uniform_i64(it);
        } else {
            unsigned long long v = 0;
            if (lane == 0) v = atomicAdd(a.queue, 1ull);
            return uniform_i64((long long)v);
        }
    };
    int64_t item = next_item(-1);
    const float alpha = a.alpha, rmax = a.rmax;
    const int T = a.T;
    int cur_key = -1;
    int dmax_rep = 0;  // largest variable degree of the representation (wave-uniform)

    uint32_t ea[PV][kMaxVarDegree];  // LDS byte address of every edge of the lane's variables
    uint32_t vinfo[PV];              // variable id | degree << 16
    int dmaxp[PV];                   // max degree of pass v (wave-uniform)
    uint32_t cwp[PC];                // row weights (DC == 8 only)
    float mu[PV];
    int32_t csrcp[PC];               // syndrome source of each check position (kJunkRow: none)
    uint32_t cpass_live = 0;         // bit c: check pass c holds a check of the representation
    // flooding min-sum / sum-product start every shot from stores only (iteration 0
    // needs no c->v message), so the LDS arrays are cleared only when a wave takes up
    // a representation; the weighted rule (damping reads r^(0) = 0) and the serial
    // schedule (posteriors read c->v messages) clear them for every shot
    constexpr bool kClearPerShot = RULE == kRuleWeighted || SCHED == 1;
    bool clear_now = true;
    // flooding min-sum with one positive prior mu0 on every variable of the part: the
    // first iteration's outcome is known without running it (see the shot set-up)
    constexpr bool kKnownFirst = RULE == kRuleNMS && SCHED == 0;
    bool uni = false;
    float a_first = 0.0f;  // min(alpha * mu0, rmax)

    while (item < a.n_items) {
        const ItemPos ip = decode_item(a, item);
        const DevPart *pt = a.dparts + ip.part;
        const int n = pt->n, Mmax = pt->Mmax, W = pt->W, Ws = pt->Ws, L = pt->L;
        const int l = ip.l;
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
            const uint32_t absent_dec = LY::dec(LY::edge_word(ibase_addr, sink)) << 16;
#pragma unroll
            for (int v = 0; v < PV; ++v) {
                const int s = (sub * PV + v) * 64 + lane;
                const bool valid = sub * PV + v < vp && s < n;
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
                const uint32_t absent = absent_dec | (zsk_addr + 4u * (uint32_t)(sub * PV + v));
#pragma unroll
                for (int k = 0; k < kMaxVarDegree; ++k) {
                    const uint32_t e = (w4[k >> 1] >> (16 * (k & 1))) & 0xffffu;
                    ea[v][k] = kZSink && e == sink ? absent : LY::edge_word(ibase_addr, e);
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
                    const int j = (sub * PC + c) * 64 + lane;
                    cwp[c] = j < Mmax ? (uint32_t)pt->cw[(size_t)l * Mmax + j] : 8u;
                }
            }
            const int32_t *csrc = pt->csrc + (size_t)l * Mmax;
            cpass_live = 0;
#pragma unroll
            for (int c = 0; c < PC; ++c) {
                const int j = (sub * PC + c) * 64 + lane;
                csrcp[c] = j < Mmax ? csrc[j] : kJunkRow;
                if (__ballot(csrcp[c] != kJunkRow) != 0ull) cpass_live |= 1u << c;
            }
            clear_now = true;
            if constexpr (kKnownFirst) {
                // every wave of an instance scans the whole prior vector, so they agree
                const float mu0 = pr0[0] + 0.0f;
                bool same = true;
                for (int i = lane; i < n; i += 64) same = same && pr0[i] + 0.0f == mu0;
                uni = !a.prior_per_shot && !a.fixed_T && mu0 > 0.0f && __ballot(!same) == 0ull;
                a_first = fminf(alpha * mu0, rmax);
            }
        }
        const float *prior = pick(a.prior, ip.part);
        const uint64_t *syn = pick(a.syn, ip.part);
        uint64_t *cand = pick(a.cand, ip.part);
        uint16_t *kstat = pick(a.kstat, ip.part);
        float *llr = pick(a.llr, ip.part);

        for (int64_t shot = ip.begin; shot < ip.end; ++shot) {
            // ---------------- fill: clear messages and decisions, stage syndrome (and priors)
            {
                if (kClearPerShot || clear_now) {
                    constexpr int nz = (int)(LY::kTail / 8);
                    for (int i = sub * 64 + lane; i < nz; i += 64 * WPI) lds_ptr_u64(ibase_addr)[i] = 0ull;
                    if (kZSink && sub == 0 && lane < 16) zsk[lane] = 0.0f;
                    clear_now = false;
                }
                if (sub == 0 && lane < Ws) synl[lane] = syn[shot * Ws + lane];
                if (a.prior_per_shot || kMuLds) {
                    const float *pr = prior + (a.prior_per_shot ? shot * n : 0);
                    for (int i = sub * 64 + lane; i < n; i += 64 * WPI) mul[i] = pr[i] + 0.0f;
                }
                if (WPI > 1 && threadIdx.x == 0) ctl[2] = ctl[3] = 0u;  // halting flags
            }
            inst_sync();
            if (a.prior_per_shot) {
#pragma unroll
                for (int v = 0; v < PV; ++v) {
                    const int s = (sub * PV + v) * 64 + lane;
                    mu[v] = (sub * PV + v < vp && s < n) ? mul[vinfo[v] & 0xffffu] + 0.0f : 0.0f;
                }
            }
            uint32_t sbits = 0, rowv = 0;  // syndrome bit and "real check" flag per pass
#pragma unroll
            for (int c = 0; c < PC; ++c) {
                const int j = (sub * PC + c) * 64 + lane;
                int src = csrcp[c];
                asm volatile("" : "+v"(src));  // derive the syndrome word address per shot (not kept live)
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
                    if (SCHED == 1) sbl[j] = (unsigned char)bit;
                }
            }
            int it = 0, kfix = -1, K = T;
            bool conv = false;
            uint32_t decb = 0;
            float Pl[PV];  // posteriors of the last variable phase (written out at the end)
#pragma unroll
            for (int v = 0; v < PV; ++v) Pl[v] = 0.0f;
            bool run_bp = true;
            if (kKnownFirst && uni) {
                // Iteration 0 with q = mu0 > 0 on every edge: every hard decision is 0,
                // so the shot has converged at K = 0 (zero correction) iff its syndrome
                // is 0, and with T = 0 it stops there in any case.  Otherwise both
                // minima of every check are mu0 and every sign product is +, so the
                // message to each edge of check j is (-1)^{s_j} min(alpha mu0, rmax) (on
                // a row of weight 1 its one edge gets min(alpha * FLT_MAX, rmax), the
                // second minimum being an unused slot's FLT_MAX): written here, with the
                // decision cells 0, and BP resumes at iteration 1.
                const uint64_t sw = lane < Ws ? synl[lane] : 0ull;
                const bool zero = __ballot(sw != 0ull) == 0ull;
                if (zero || T == 0) {
                    conv = zero;
                    K = 0;
                    run_bp = false;
#pragma unroll
                    for (int v = 0; v < PV; ++v) Pl[v] = mu[v];
                } else {
                    const float a_one = fminf(alpha * 3.402823466e38f, rmax);
#pragma unroll
                    for (int c = 0; c < PC; ++c) {
                        const int j = (sub * PC + c) * 64 + lane;
                        const uint32_t sg = ((sbits >> c) & 1u) << 31;
                        const float m = bitsf(fbits(a_first) | sg);
                        float q[DC];
#pragma unroll
                        for (int k = 0; k < DC; ++k) q[k] = m;
                        if (DC == 8 && cwp[c] < 2u) q[0] = bitsf(fbits(a_one) | sg);
                        row_store(j, q);
                        *lds_ptr_u64(ibase_addr + LY::kDecOff + 8u * (uint32_t)j) = 0ull;
                    }
                    it = 1;
                    inst_sync();
                }
            }
            if constexpr (SCHED == 1) {
                const int32_t *lp = pt->lev_ptr + pt->lev_off[l];
                const int nlev = pt->lev_off[l + 1] - pt->lev_off[l] - 1;
                const uint16_t *lc = pt->lev_chk + (size_t)l * Mmax;
                const uint4 *lt = pt->ltab + (size_t)l * Mmax * 8;
                while (true) {
    #pragma unroll
                    for (int v = 0; v < PV; ++v)
    #pragma unroll
                        for (int k = 0; k < kMaxVarDegree; ++k) asm volatile("" : "+v"(ea[v][k]));
                    // ---------------- posterior phase (r = 0 at iteration 0)
#pragma unroll
                    for (int v = 0; v < PV; ++v) {
                        if (v < vp) {
                            const int deg = (int)(vinfo[v] >> 16);
                            float Pv = 0.0f;
                            bool d = false;
                            switch (uniform_i32(dmaxp[v])) {
                            case 1: var_post<1, LY>(ea[v], deg, mu[v], Pv, d); break;
                            case 2: var_post<2, LY>(ea[v], deg, mu[v], Pv, d); break;
                            case 3: var_post<3, LY>(ea[v], deg, mu[v], Pv, d); break;
                            case 4: var_post<4, LY>(ea[v], deg, mu[v], Pv, d); break;
                            case 5: var_post<5, LY>(ea[v], deg, mu[v], Pv, d); break;
                            case 6: var_post<6, LY>(ea[v], deg, mu[v], Pv, d); break;
                            case 7: var_post<7, LY>(ea[v], deg, mu[v], Pv, d); break;
                            case 8: var_post<8, LY>(ea[v], deg, mu[v], Pv, d); break;
                            default: Pv = mu[v]; d = Pv < 0.0f; break;
                            }
                            decb = (decb & ~(1u << v)) | ((uint32_t)d << v);
                            Pl[v] = Pv;
                        }
                    }
                    wave_sync();
                    // ---------------- syndrome test
                    uint32_t unsat = 0;
#pragma unroll
                    for (int c = 0; c < PC; ++c) {
                        const int j = c * 64 + lane;
                        const uint64_t dw = *lds_ptr_u64(ibase_addr + LY::kDecOff + 8u * (uint32_t)j);
                        unsat |= (row_parity(dw) ^ (sbits >> c)) & ((rowv >> c) & 1u);
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
                                                                         4u * ((eo & 7u) * (uint32_t)S + (eo >> 3)));
                                            acc += u < deg - 1 ? x : 0.0f;
                                        }
                                    }
                                    q[k] = deg == 0 ? 3.402823466e38f : acc;
                                }
                                CheckRule<RULE>::template apply<DC>(q, (int)sb, alpha, rmax);
                                lds_f32 *row = lds_ptr_f32(ibase_addr + 4u * (uint32_t)j);
#pragma unroll
                                for (int k = 0; k < DC; ++k) row[k * S] = q[k];
                            }
                            wave_sync();
                        }
                    }
                    ++it;
                }
            } else if (run_bp) {
                while (true) {
                    // ---------------- checkpoint of the c->v messages r^(it) (weighted, training)
                    if constexpr (RULE == kRuleWeighted) {
                        if (a.ckpt && it > 0 && it < T && it % a.ckpt_every == 0) {
                            const lds_u64 *src = lds_ptr_u64(ibase_addr + LY::kROff);
                            uint64_t *dst = reinterpret_cast<uint64_t *>(
                                a.ckpt + (((size_t)shot * L + l) * a.n_ck + (it / a.ckpt_every - 1)) * (LY::kMsg / 4));
                            for (int i = lane; i < (int)(LY::kMsg / 8); i += 64) dst[i] = src[i];
                        }
                    }
                    // ---------------- variable phase
                    // the edge words are unpacked where they are used, not once per shot (which
                    // would keep both halves of every word live in registers)
    #pragma unroll
                    for (int v = 0; v < PV; ++v)
    #pragma unroll
                        for (int k = 0; k < kMaxVarDegree; ++k) asm volatile("" : "+v"(ea[v][k]));
    #pragma unroll
                    for (int v = 0; v < PV; ++v) {
                        if (sub * PV + v < vp && (sub * PV + v) * 64 + lane < n) {
                            const int deg = (int)(vinfo[v] >> 16);
                            float Pv = 0.0f;
                            bool d = false;
                            const bool prevd = (decb >> v) & 1u;
                            if (!kClearPerShot && it == 0) {
                                switch (uniform_i32(dmaxp[v])) {
                                case 1: var_first<1, LY>(ea[v], mu[v], Pv, d); break;
                                case 2: var_first<2, LY>(ea[v], mu[v], Pv, d); break;
                                case 3: var_first<3, LY>(ea[v], mu[v], Pv, d); break;
                                case 4: var_first<4, LY>(ea[v], mu[v], Pv, d); break;
                                case 5: var_first<5, LY>(ea[v], mu[v], Pv, d); break;
                                case 6: var_first<6, LY>(ea[v], mu[v], Pv, d); break;
                                case 7: var_first<7, LY>(ea[v], mu[v], Pv, d); break;
                                case 8: var_first<8, LY>(ea[v], mu[v], Pv, d); break;
                                default: Pv = mu[v]; d = Pv < 0.0f; break;
                                }
                            } else {
                            switch (uniform_i32(dmaxp[v])) {
                            case 1: var_rule<1, LY, kZSink>(ea[v], deg, mu[v], prevd, Pv, d); break;
                            case 2: var_rule<2, LY, kZSink>(ea[v], deg, mu[v], prevd, Pv, d); break;
                            case 3: var_rule<3, LY, kZSink>(ea[v], deg, mu[v], prevd, Pv, d); break;
                            case 4: var_rule<4, LY, kZSink>(ea[v], deg, mu[v], prevd, Pv, d); break;
                            case 5: var_rule<5, LY, kZSink>(ea[v], deg, mu[v], prevd, Pv, d); break;
                            case 6: var_rule<6, LY, kZSink>(ea[v], deg, mu[v], prevd, Pv, d); break;
                            case 7: var_rule<7, LY, kZSink>(ea[v], deg, mu[v], prevd, Pv, d); break;
                            case 8: var_rule<8, LY, kZSink>(ea[v], deg, mu[v], prevd, Pv, d); break;
                            default: Pv = mu[v]; d = Pv < 0.0f; break;
                            }
                            }
                            decb = (decb & ~(1u << v)) | ((uint32_t)d << v);
                            Pl[v] = Pv;
                        }
                    }
                    inst_sync();
                    // ---------------- check phase: syndrome test of the decisions, c->v messages.
                    // Rows beyond the representation's checks are junk rows (unused by it).
                    uint32_t unsat = 0;
                    // every pass's loads are issued before any pass's stores (rows of different
                    // passes are disjoint), so the LDS latency of later passes overlaps
                    float qa[PC][DC];
                    float w_alpha = 0.0f, w_beta = 0.0f, w_keep = 1.0f;
                    if constexpr (RULE == kRuleWeighted) {
                        if (it < T) {
                            w_alpha = a.walpha[(size_t)it * L + l];
                            w_beta = a.wbeta[(size_t)it * L + l];
                            w_keep = 1.0f - w_beta;
                        }
                    }
    #pragma unroll
                    for (int c = 0; c < PC; ++c) {
                        const int j = (sub * PC + c) * 64 + lane;
                        row_load(j, qa[c]);
                        const uint64_t dw = *lds_ptr_u64(ibase_addr + LY::kDecOff + 8u * (uint32_t)j);
                        unsat |= (row_parity(dw) ^ (sbits >> c)) & ((rowv >> c) & 1u);
                    }
    #pragma unroll
                    for (int c = 0; c < PC; ++c) {
                        // a pass without a check of this representation: nothing to compute
                        if (!((cpass_live >> c) & 1u)) continue;
                        const int j = (sub * PC + c) * 64 + lane;
                        float (&q)[DC] = qa[c];
                        if constexpr (DC == 8) {
                            const int w = (int)cwp[c];
    #pragma unroll
                            for (int k = 2; k < DC; ++k)
                                if (k >= w) q[k] = 3.402823466e38f;
                        }
                        if constexpr (RULE == kRuleWeighted) {
                            // c->v messages of iteration it + 1 (none after the last)
                            if (it < T) {
                                lds_f32 *rrow = lds_ptr_f32(ibase_addr + LY::kROff + 4u * (uint32_t)j);
                                float rp[DC];
    #pragma unroll
                                for (int k = 0; k < DC; ++k) rp[k] = rrow[k * S];
                                WeightedRule::apply<DC>(q, rp, (int)((sbits >> c) & 1u), w_alpha, w_keep, w_beta,
                                                        rmax);
    #pragma unroll
                                for (int k = 0; k < DC; ++k) rrow[k * S] = q[k];
                            }
                        } else {
                            CheckRule<RULE>::template apply<DC>(q, (int)((sbits >> c) & 1u), alpha, rmax);
                            row_store(j, q);
                        }
                    }
                    // this wave's absent-edge words back to +0 for the next variable phase
                    if (kZSink && lane < PV) zsk[sub * PV + lane] = 0.0f;
                    bool sat = __ballot(unsat != 0u) == 0ull;
                    if constexpr (WPI > 1) {
                        // the instance's test: flag it & 1 raised by any wave with an unsatisfied
                        // row; the other flag (read last before the previous barrier, written
                        // next after the coming one) cleared for iteration it + 1
                        if (!sat && lane == 0) atomicOr((uint32_t *)(ctl + 2 + (it & 1)), 1u);
                        __syncthreads();
                        sat = ctl[2 + (it & 1)] == 0u;
                        if (threadIdx.x == 0) ctl[2 + ((it + 1) & 1)] = 0u;
                    }
                    // ---------------- halting (Section II-B)
                    if (!a.fixed_T) {
                        if (sat) { conv = true; K = it; break; }
                        if (it == T) { K = T; break; }
                    } else {
                        if (sat && kfix < 0) kfix = it;
                        if (it == T) { conv = kfix >= 0; K = conv ? kfix : T; break; }
                    }
                    ++it;
                    // (shared instances: the flag barrier above already ordered the check
                    // phase's writes before the next variable phase)
                    if constexpr (WPI == 1) wave_sync();
                }
            }
            // the output path recomputes what it derives from the variable ids (hoisting
            // those per-shot values out of the loops would keep them live, spilled, all along)
            uint32_t vidc[PV];
#pragma unroll
            for (int v = 0; v < PV; ++v) {
                vidc[v] = vinfo[v];
                asm volatile("" : "+v"(vidc[v]));
            }
            if (llr) {
#pragma unroll
                for (int v = 0; v < PV; ++v) {
                    const int s = (sub * PV + v) * 64 + lane;
                    if (sub * PV + v < vp && s < n) llr[((size_t)shot * L + l) * n + (vidc[v] & 0xffffu)] = Pl[v];
                }
            }
            // ---------------- output: bit-packed hard decisions via the staging words
            if (sub == 0 && lane < 2 * W) stage[lane] = 0u;
            inst_sync();
#pragma unroll
            for (int v = 0; v < PV; ++v) {
                const int s = (sub * PV + v) * 64 + lane;
                if (sub * PV + v < vp && s < n && ((decb >> v) & 1u)) {
                    const uint32_t id = vidc[v] & 0xffffu;
                    atomicOr((uint32_t *)(stage + (id >> 5)), 1u << (id & 31));
                }
            }
            inst_sync();
            // representation-major: a work item's records are contiguous (whole-line writes)
            const size_t inst = a.cand_rm ? (size_t)l * a.shots + shot : (size_t)shot * L + l;
            if (sub == 0 && lane < W) cand[inst * W + lane] = ((const lds_u64 *)stage)[lane];
            if (sub == 0 && lane == 0) kstat[inst] = (uint16_t)(K | (conv ? 0x8000 : 0));
            inst_sync();
        }

        item = next_item(item);
    }
}

size_t bp_lds_limit() { return 64 * 1024; }  // per workgroup

// The BP kernel function most recently launched by this host thread (graph capture
// records which node is the BP kernel).
static thread_local const void *t_last_bp_kernel = nullptr;
const void *last_bp_kernel() { return t_last_bp_kernel; }
void set_last_bp_kernel(const void *f) { t_last_bp_kernel = f; }

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
    if ((schedule != 0 && schedule != 1) || rule < 0 || rule > 2 || lpi != 64) return false;
    if (rule == kRuleWeighted && schedule != 0) return false;
    PassPair pp;
    return pick_pair(passes, passes, pp);
}

bool bp_passes(const BPArgs &a, int &pv, int &pc) {
    int nv, nc;
    passes_needed(a, nv, nc);
    PassPair pp;
    if (!pick_pair(nv, nc, pp)) return false;
    pv = pp.pv;
    pc = pp.pc;
    return true;
}

bool bp_layout(const BPArgs &a, int &mpad) {
    int pv, pc;
    passes_needed(a, pv, pc);
    PassPair pp;
    if (!pick_pair(pv, pc, pp)) return false;
    mpad = 64 * pp.pc;
    return true;
}

template <int PV, int PC, int DC, int RULE, int SCHED, int WPI = 1>
static hipError_t launch_wave_t(const BPArgs &a, const BPConfig &cfg, hipStream_t s) {
    // shared instances: one per workgroup of WPI waves, 16 bytes of control words after it
    const int wpb = WPI > 1 ? WPI : cfg.waves_per_block;
    const size_t lds = WPI > 1 ? (size_t)a.inst_bytes + 16u : (size_t)wpb * a.inst_bytes;
    const int64_t blocks =
        a.persistent ? cfg.blocks : plain_grid(WPI > 1 ? a.n_items : (a.n_items + wpb - 1) / wpb);
    hipLaunchKernelGGL((bp_wave_kernel<PV, PC, DC, RULE, SCHED, WPI>), dim3((unsigned)blocks), dim3(64 * wpb), lds,
                       s, a);
    set_last_bp_kernel(reinterpret_cast<const void *>(&bp_wave_kernel<PV, PC, DC, RULE, SCHED, WPI>));
    return hipGetLastError();
}

template <int PV, int PC, int SCHED>
static hipError_t launch_pair(const BPArgs &a, const BPConfig &cfg, int rule, hipStream_t s) {
    bool u6 = true;
    for (int p = a.part0; p < a.part0 + a.nparts; ++p) u6 = u6 && a.part[p].uniform_dc == 6;
    // the largest codes under flooding NMS / sum-product: PV / 2 waves per instance,
    // two variable and two check passes each
    if constexpr (SCHED == 0 && PV >= 14 && PV == PC && PV % 2 == 0) {
        constexpr int WPI = PV / 2;
        if (rule == kRuleNMS)
            return u6 ? launch_wave_t<2, 2, 6, 0, 0, WPI>(a, cfg, s) : launch_wave_t<2, 2, 8, 0, 0, WPI>(a, cfg, s);
        if (rule == kRuleSPA)
            return u6 ? launch_wave_t<2, 2, 6, 1, 0, WPI>(a, cfg, s) : launch_wave_t<2, 2, 8, 1, 0, WPI>(a, cfg, s);
    }
    if (rule == kRuleNMS)
        return u6 ? launch_wave_t<PV, PC, 6, 0, SCHED>(a, cfg, s) : launch_wave_t<PV, PC, 8, 0, SCHED>(a, cfg, s);
    if (rule == kRuleSPA)
        return u6 ? launch_wave_t<PV, PC, 6, 1, SCHED>(a, cfg, s) : launch_wave_t<PV, PC, 8, 1, SCHED>(a, cfg, s);
    if constexpr (SCHED == 0) {
        if (rule == kRuleWeighted)
            return u6 ? launch_wave_t<PV, PC, 6, kRuleWeighted, 0>(a, cfg, s)
                      : launch_wave_t<PV, PC, 8, kRuleWeighted, 0>(a, cfg, s);
    }
    return hipErrorInvalidValue;
}

template <int SCHED>
static hipError_t launch_sched(const BPArgs &a, const BPConfig &cfg, int rule, const PassPair &pp, hipStream_t s) {
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
    return hipErrorInvalidValue;
}

hipError_t launch_bp(const BPArgs &a, const BPConfig &cfg, int schedule, int rule, hipStream_t s) {
    if ((schedule != 0 && schedule != 1) || cfg.lpi != 64) return hipErrorInvalidValue;
    if (a.dual) return schedule == 0 && rule == kRuleNMS ? launch_bp_dual(a, cfg, s) : hipErrorInvalidValue;
    int pv, pc;
    passes_needed(a, pv, pc);
    PassPair pp;
    if (!pick_pair(pv, pc, pp)) return hipErrorInvalidValue;
    return schedule == 0 ? launch_sched<0>(a, cfg, rule, pp, s) : launch_sched<1>(a, cfg, rule, pp, s);
}

}  // namespace mbbp
