// Paired form of the flooding min-sum BP kernel (Section II-B, eqs. (1)-(2)): two
// BP instances of one representation (two shots of a work item) per wavefront.
//
// With one instance per wavefront a code of n = 144 variables and up to 96 check
// positions fills 3 variable passes and 2 check passes of 64 lanes, 75% and at most
// 75% of them useful; every pass costs the same LDS instructions however few of its
// lanes are live.  Pairing interleaves the two instances lane by lane: lane i works
// for instance i & 1 on variable rank 32 * v + (i >> 1) and check position
// 32 * c + (i >> 1), so 2n variables take ceil(2n / 64) passes and 2 * Mpad
// positions 2 * Mpad / 64 passes (5 and 3 for the code above, instead of 6 and 4).
//
// Each instance keeps its own LDS region (messages, decisions), its own shot and
// iteration count.  When an instance halts (Section II-B: syndrome satisfied, or T
// iterations) its outputs are written (each 64-bit word of its hard decisions packed
// by one ballot, every lane fetching the decision bits of its variable's lane), its
// c->v messages are reset to 0 and it takes the next shot of the work item at once,
// while the other instance keeps iterating; an iteration with all c->v messages 0
// computes exactly what the first variable phase of a shot computes (q = P = mu), and
// with a uniform positive prior even that iteration is written directly.  Values are
// those of the one-instance kernel bit for bit.  Used for normalized min-sum with
// early stop; with per-shot priors an instance's lanes load their variables' priors
// when it takes a shot.  The other forms use one instance per wavefront.
#include <hip/hip_runtime.h>

#include "mbbp_bp_rules.h"
#include "mbbp_device.h"
#include "mbbp_wave.h"

namespace mbbp {

namespace {

struct DualItem {
    int part, l;
    int64_t begin, end;
};

__device__ __forceinline__ DualItem dual_item(const BPArgs &a, int64_t item) {
    const int64_t rank = item / a.n_chunks;
    const int64_t ch = item - rank * a.n_chunks;
    // (a load through a generic pointer counts as divergent: keep the index uniform)
    const int pl = __builtin_amdgcn_readfirstlane(a.item_order ? a.item_order[rank] : (int)rank);
    DualItem p;
    p.part = a.part0 + pl / a.L;
    p.l = pl - (pl / a.L) * a.L;
    p.begin = ch * a.chunk;
    p.end = min(p.begin + (int64_t)a.chunk, a.shots);
    return p;
}

template <typename T>
__device__ __forceinline__ T pick2(const T (&v)[2], int part) { return part == 0 ? v[0] : v[1]; }

constexpr uint64_t kLanes0 = 0x5555555555555555ull;  // lanes of instance 0

}  // namespace

// PV2 / PC2: variable / check passes of 64 lanes covering both instances; an
// instance has 32 * PC2 check positions.  DC as in bp_wave_kernel; MAXD: largest
// variable degree (edge words kept per variable); RICH: the instantiation that also
// writes posteriors (when a.llr is set) and takes per-shot priors (when
// a.prior_per_shot is set); the other one does neither and keeps fewer registers.
template <int PV2, int PC2, int DC, int MAXD, bool RICH>
// Up to three variable passes the kernel fits five wavefronts per SIMD (96 VGPRs, a few
// spills off the loop); with five passes the spills would land in the loop, so four.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PV2 <= 3 ? 5 : 4)))
void bp_dual_kernel(BPArgs a) {
    using LY = LayoutM<32 * PC2, kRuleNMS, DC, true, true>;  // slot pairs, DC message slots per row
    static_assert(DC % 2 == 0 && LY::S % 16 == 1, "slot pairs");
    constexpr int S = LY::S;
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave-uniform
    const int comp = lane & 1;   // instance of this lane
    const int half = lane >> 1;  // rank within the instance's pass
    extern __shared__ __align__(16) unsigned char smem[];
    const int istride = a.dual_stride;  // bytes per instance region
    // 32-bit LDS byte addresses; the wave's own ones are wave-uniform (scalar registers)
    const uint32_t wbase_addr = (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)((uint32_t)(size_t)(lds_u8 *)smem + (uint32_t)(wib * a.inst_bytes)));
    const uint32_t cbase_addr = wbase_addr + (uint32_t)(comp * istride);
    // after both regions, the syndrome words of every shot of the work item (staged
    // once per item, so no shot waits on memory)
    const uint32_t sbuf_addr = wbase_addr + 2u * (uint32_t)istride;
    // after the syndrome words: where each variable of the representation sits, for
    // the bit-packed outputs (entry 64 w + t: variable 64 w + t as 2 rank | pass << 8;
    // 31 << 8 for ids beyond n, whose pass bit is never set)
    constexpr int kW = (32 * PV2 + 63) / 64;  // output words an instance can need
    const uint32_t map_addr = sbuf_addr + (uint32_t)((a.chunk * a.ws_max * 8 + 15) & ~15);

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

    uint32_t ea[PV2][MAXD];           // packed edge words (message | decision << 16)
    uint32_t vinfo[PV2];              // variable id | degree << 16
    int dmaxp[PV2];
    uint32_t cwp[PC2];
    float mu[PV2];
    int32_t csrcp[PC2];
    uint32_t rowv = 0;   // check pass c holds a real check of this lane's instance
    uint32_t decb = 0;   // decisions of the last variable phase (as stored in the cells)
    // one positive prior mu0 on every variable of the part (checked per representation):
    // a shot's first iteration is then known without running it (see the fresh-shot step)
    bool uni = false;
    float a_first = 0.0f;  // min(alpha * mu0, rmax): magnitude of every first c->v message
    float Pl[RICH ? PV2 : 1];         // posteriors of the last variable phase (RICH only)

    while (item < a.n_items) {
        const DualItem ip = dual_item(a, item);
        const DevPart *pt = a.dparts + ip.part;
        const int n = pt->n, Mmax = pt->Mmax, W = pt->W, Ws = pt->Ws, L = pt->L;
        const int l = ip.l;
        const int key = ip.part * 256 + l;
        if (key != cur_key) {
            cur_key = key;
            const uint4 *vo4 = reinterpret_cast<const uint4 *>(pt->voff) + (size_t)l * n;
            const uint16_t *vid = pt->vid + (size_t)l * n;
            const uint8_t *vdg = pt->vdeg + (size_t)l * n;
            const float *pr0 = pick2(a.prior, ip.part);
            // Absent edges of pass v (slots beyond a variable's degree) read and write a
            // padding word of their own, Z_v: position Mpad of slot pair v / 2, word v % 2,
            // which no check touches; the check phase zeroes it, so each variable phase
            // reads +0 there.  Their decision cells are those of position Mmax, which no
            // check of any representation uses.
            const uint32_t sink = (uint32_t)Mmax * 8u;
            const uint32_t absent_dec = LY::dec(LY::edge_word(cbase_addr, sink)) << 16;
#pragma unroll
            for (int v = 0; v < PV2; ++v) {
                const uint32_t absent = absent_dec | (cbase_addr + 4u * ((uint32_t)(v >> 1) * 2u * (uint32_t)S +
                                                                        2u * (uint32_t)LY::Mpad + (uint32_t)(v & 1)));
                const int s1 = v * 32 + half;
                const bool valid = s1 < n;
                const uint32_t sk2 = sink | (sink << 16);
                uint4 o = make_uint4(sk2, sk2, sk2, sk2);
                int deg = 0;
                uint32_t id = 0;
                if (valid) {
                    o = vo4[s1];
                    deg = vdg[s1];
                    id = vid[s1];
                }
                const uint32_t w4[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
                for (int k = 0; k < MAXD; ++k) {
                    const uint32_t e = (w4[k >> 1] >> (16 * (k & 1))) & 0xffffu;
                    ea[v][k] = e == sink ? absent : LY::edge_word(cbase_addr, e);
                }
                vinfo[v] = id | ((uint32_t)deg << 16);
                dmaxp[v] = uniform_i32(wave_max_i32(deg));
                mu[v] = valid ? pr0[id] + 0.0f : 0.0f;
                if constexpr (RICH) Pl[v] = 0.0f;
            }
            if constexpr (!RICH) {
                const float mu0 = bitsf((uint32_t)uniform_i32((int)fbits(mu[0])));  // lane 0: rank 0
                bool same = true;
#pragma unroll
                for (int v = 0; v < PV2; ++v)
                    if (v * 32 + half < n) same = same && mu[v] == mu0;
                uni = mu0 > 0.0f && __ballot(!same) == 0ull;
                a_first = fminf(alpha * mu0, rmax);
            }
            const int32_t *csrc = pt->csrc + (size_t)l * Mmax;
            rowv = 0;
#pragma unroll
            for (int c = 0; c < PC2; ++c) {
                const int p = c * 32 + half;
                csrcp[c] = p < Mmax ? csrc[p] : kJunkRow;
                if (csrcp[c] != kJunkRow) rowv |= 1u << c;
                if (DC == 8) cwp[c] = p < Mmax ? (uint32_t)pt->cw[(size_t)l * Mmax + p] : 8u;
            }
            // both regions from scratch: messages, decisions (and the decision bits) 0
            const int nz = a.inst_bytes >> 2;
            for (int i = lane; i < nz; i += 64) lds_ptr_u32(wbase_addr)[i] = 0u;
            decb = 0;
#pragma unroll
            for (int w = 0; w < kW; ++w) lds_ptr_u32(map_addr)[64 * w + lane] = 31u << 8;
            wave_sync();
            if (comp == 0) {
#pragma unroll
                for (int v = 0; v < PV2; ++v)
                    if (v * 32 + half < n)
                        lds_ptr_u32(map_addr)[vinfo[v] & 0xffffu] = (uint32_t)(2 * half) | ((uint32_t)v << 8);
            }
        }
        const uint64_t *syn = pick2(a.syn, ip.part);
        const float *prior = pick2(a.prior, ip.part);
        uint64_t *cand = pick2(a.cand, ip.part);
        uint16_t *kstat = pick2(a.kstat, ip.part);
        float *llr = pick2(a.llr, ip.part);
        (void)llr;

        // syndrome words of the item's shots (at most the chunk the host sized sbuf for)
        {
            const int nw = (int)(ip.end - ip.begin) * Ws;
            for (int i = lane; i < nw; i += 64) lds_ptr_u64(sbuf_addr)[i] = syn[ip.begin * Ws + i];
        }
        // per-instance state (wave-uniform): current shot (-1: idle) and iteration
        int64_t next = ip.begin;
        int64_t shot[2] = {-1, -1};
        int it[2] = {0, 0};
        uint32_t fresh = 0;
#pragma unroll
        for (int c = 0; c < 2; ++c)
            if (next < ip.end) { shot[c] = next++; fresh |= 1u << c; }
        uint32_t sbits = 0;  // syndrome bit of this lane's check in each pass
        wave_sync();

        while (shot[0] >= 0 || shot[1] >= 0) {
            // ---------------- a fresh shot (its syndrome words already staged): derive the
            // check bits, then the c->v messages it starts from (an idle instance kept
            // iterating on its last shot)
            if (fresh) {
                if (uni) {
                    // All q = mu0 > 0 at iteration 0, so every hard decision is 0: a shot
                    // whose syndrome is 0 has converged at K = 0 with a zero correction,
                    // and with T = 0 every shot stops there.  Such shots are written here
                    // without running BP.
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        while ((fresh >> c) & 1u) {
                            const lds_u64 *sy = lds_ptr_u64(sbuf_addr) + (shot[c] - ip.begin) * Ws;
                            const uint64_t sw = lane < Ws ? sy[lane] : 0ull;
                            const bool zero = __ballot(sw != 0ull) == 0ull;
                            if (!zero && T > 0) break;
                            const size_t oi = a.cand_rm ? (size_t)l * a.shots + shot[c] : (size_t)shot[c] * L + l;
                            if (lane < W) cand[oi * W + lane] = 0ull;
                            if (lane == 0) kstat[oi] = (uint16_t)(zero ? 0x8000 : 0);
                            if (next < ip.end) {
                                shot[c] = next++;
                            } else {
                                shot[c] = -1;
                                fresh &= ~(1u << c);
                            }
                        }
                    }
                    if (shot[0] < 0 && shot[1] < 0) break;
                }
                if ((fresh >> comp) & 1u) {
                    sbits = 0;
                    const lds_u64 *sy = lds_ptr_u64(sbuf_addr) + (shot[comp] - ip.begin) * Ws;
#pragma unroll
                    for (int c = 0; c < PC2; ++c) {
                        int src = csrcp[c];
                        asm volatile("" : "+v"(src));
                        if (src != kJunkRow) {
                            uint32_t bit = 0;
                            if (src >= 0) {
                                bit = (uint32_t)(sy[src >> 6] >> (src & 63)) & 1u;
                            } else {
                                for (int t = pt->comb_ptr[-src - 1]; t < pt->comb_ptr[-src]; ++t) {
                                    const int r = pt->comb_idx[t];
                                    bit ^= (uint32_t)(sy[r >> 6] >> (r & 63)) & 1u;
                                }
                            }
                            sbits |= bit << c;
                        }
                    }
                }
                if (RICH && a.prior_per_shot && ((fresh >> comp) & 1u)) {
                    const float *pr = prior + shot[comp] * n;
#pragma unroll
                    for (int v = 0; v < PV2; ++v)
                        if (v * 32 + half < n) mu[v] = pr[vinfo[v] & 0xffffu] + 0.0f;
                }
                if ((fresh >> comp) & 1u) {
                    if (uni) {
                        // iteration 0 run on paper: its check phase sees q = mu0 on every
                        // edge, so both minima are mu0, every sign product is +, and the
                        // message to each edge of check j is (-1)^{s_j} min(alpha mu0, rmax)
                        // (on a row of weight 1 its one edge gets min(alpha * FLT_MAX, rmax),
                        // the second minimum being an unused slot's FLT_MAX)
                        const float a_one = fminf(alpha * 3.402823466e38f, rmax);
#pragma unroll
                        for (int c = 0; c < PC2; ++c) {
                            const uint32_t row = cbase_addr + 8u * (uint32_t)(c * 32 + half);
                            const uint32_t sg = ((sbits >> c) & 1u) << 31;
                            f32x2 w;
                            w.x = bitsf(fbits(a_first) | sg);
                            w.y = w.x;
                            if (DC == 8 && cwp[c] < 2u) w.x = bitsf(fbits(a_one) | sg);
#pragma unroll
                            for (int u = 0; u < DC / 2; ++u) {
                                *lds_ptr_f32x2(row + 8u * (uint32_t)(u * S)) = w;
                                if (u == 0) w.x = w.y;
                            }
                        }
                    } else {
                        // c->v messages 0: iteration 0 computes q = P = mu
#pragma unroll
                        for (int c = 0; c < PC2; ++c) {
                            const uint32_t row = cbase_addr + 8u * (uint32_t)(c * 32 + half);
#pragma unroll
                            for (int u = 0; u < DC / 2; ++u) *lds_ptr_u64(row + 8u * (uint32_t)(u * S)) = 0ull;
                        }
                    }
                }
                if (uni) {
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        if ((fresh >> c) & 1u) it[c] = 1;  // iteration 0 is done
                }
                fresh = 0;
                wave_sync();
            }
            // ---------------- variable phase (both instances)
#pragma unroll
            for (int v = 0; v < PV2; ++v)
#pragma unroll
                for (int k = 0; k < MAXD; ++k) asm volatile("" : "+v"(ea[v][k]));
            // Every lane runs every pass: a lane past the last variable has a 0 prior and
            // only absent edges, so it reads +0, writes its pass's absent-edge word (zeroed
            // again before it is read) and keeps decision 0.  The code of each degree is
            // then free of lane-dependent branches; the decision cells (absent edges: those
            // of the unused position) are stored after it, by the lanes whose decision
            // changed.
#pragma unroll
            for (int v = 0; v < PV2; ++v) {
                float Pv;
                // degrees 3 and 4 (most passes of codes with column weight 3) are tested
                // first, each by one compare; the opaque copy keeps the compiler from
                // merging the tests into one balanced search over all degrees
                int dm = uniform_i32(dmaxp[v]);
                if (dm == 3) {
                    Pv = var_msgs<3, LY>(ea[v], mu[v]);
                } else {
                asm volatile("" : "+s"(dm));
                if (dm == 4) {
                    if constexpr (MAXD >= 4) Pv = var_msgs<4, LY>(ea[v], mu[v]); else Pv = mu[v];
                } else {
                asm volatile("" : "+s"(dm));
                switch (dm) {
                case 1: Pv = var_msgs<1, LY>(ea[v], mu[v]); break;
                case 2: Pv = var_msgs<2, LY>(ea[v], mu[v]); break;
                case 5: if constexpr (MAXD >= 5) Pv = var_msgs<5, LY>(ea[v], mu[v]); else Pv = mu[v]; break;
                case 6: if constexpr (MAXD >= 6) Pv = var_msgs<6, LY>(ea[v], mu[v]); else Pv = mu[v]; break;
                case 7: if constexpr (MAXD >= 7) Pv = var_msgs<7, LY>(ea[v], mu[v]); else Pv = mu[v]; break;
                case 8: if constexpr (MAXD >= 8) Pv = var_msgs<8, LY>(ea[v], mu[v]); else Pv = mu[v]; break;
                default: Pv = mu[v]; break;
                }
                }
                }
                const bool d = Pv < 0.0f;
                if (d != (bool)((decb >> v) & 1u)) {
                    // slots below the pass's largest degree (a higher slot is absent in every
                    // lane: stores there would all meet at one byte)
                    // (slots 0..2 first: most passes have degree 3 or more)
                    const unsigned char db = (unsigned char)d;
                    int dd = uniform_i32(dmaxp[v]);
                    if (dd >= 3) {
#pragma unroll
                        for (int k = 0; k < 3; ++k) *lds_ptr_u8(LY::dec(ea[v][k])) = db;
#pragma unroll
                        for (int k = 3; k < MAXD; ++k) {
                            asm volatile("" : "+s"(dd));
                            if (dd <= k) break;
                            *lds_ptr_u8(LY::dec(ea[v][k])) = db;
                        }
                    } else {
                        if (dd >= 1) *lds_ptr_u8(LY::dec(ea[v][0])) = db;
                        if (dd >= 2) *lds_ptr_u8(LY::dec(ea[v][1])) = db;
                    }
                }
                decb = (decb & ~(1u << v)) | ((uint32_t)d << v);
                if constexpr (RICH) Pl[v] = Pv;
            }
            wave_sync();
            // ---------------- check phase: syndrome test and c->v messages
            uint32_t unsat = 0;
            float qa[PC2][DC];
#pragma unroll
            for (int c = 0; c < PC2; ++c) {
                const int p = c * 32 + half;
                const uint32_t row = cbase_addr + 8u * (uint32_t)p;  // slot pair u at + 8 u S
#pragma unroll
                for (int u = 0; u < DC / 2; ++u) {
                    const f32x2 w = *lds_ptr_f32x2(row + 8u * (uint32_t)(u * S));
                    qa[c][2 * u] = w.x;
                    qa[c][2 * u + 1] = w.y;
                }
                const uint64_t dw = *lds_ptr_u64(cbase_addr + LY::kDecOff + 8u * (uint32_t)p);
                unsat |= (row_parity(dw) ^ (sbits >> c)) & ((rowv >> c) & 1u);
            }
#pragma unroll
            for (int c = 0; c < PC2; ++c) {
                const int p = c * 32 + half;
                const uint32_t row = cbase_addr + 8u * (uint32_t)p;
                float (&q)[DC] = qa[c];
                if constexpr (DC == 8) {
                    const int w = (int)cwp[c];
#pragma unroll
                    for (int k = 2; k < DC; ++k)
                        if (k >= w) q[k] = 3.402823466e38f;
                }
                CheckRule<kRuleNMS>::template apply<DC>(q, (int)((sbits >> c) & 1u), alpha, rmax);
#pragma unroll
                for (int u = 0; u < DC / 2; ++u) {
                    f32x2 w;
                    w.x = q[2 * u];
                    w.y = q[2 * u + 1];
                    *lds_ptr_f32x2(row + 8u * (uint32_t)(u * S)) = w;
                }
            }
            // the absent-edge words Z_v back to +0 for the next variable phase (lanes
            // 0..5: slot pair half of instance comp)
            if (half < (PV2 + 1) / 2)
                *lds_ptr_u64(cbase_addr + 8u * ((uint32_t)half * (uint32_t)S + (uint32_t)LY::Mpad)) = 0ull;
            // ---------------- halting of each instance (Section II-B)
            const uint64_t ub = __ballot(unsat != 0u);
            uint32_t done = 0, sat = 0;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const bool s_c = (ub & (kLanes0 << c)) == 0ull;
                sat |= (uint32_t)s_c << c;
                if (shot[c] >= 0 && (s_c || it[c] == T)) done |= 1u << c;
            }
            if (done) {
                wave_sync();
                // the posterior output recomputes what it derives from the variable ids
                // (hoisting those per-shot values out of the loop would keep them live)
                uint32_t vid[PV2];
#pragma unroll
                for (int v = 0; v < PV2; ++v) {
                    vid[v] = vinfo[v];
                    if constexpr (RICH) asm volatile("" : "+v"(vid[v]));
                }
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    if (!((done >> c) & 1u)) continue;
                    const bool conv = (sat >> c) & 1u;
                    const int K = conv ? it[c] : T;
                    const size_t inst = (size_t)shot[c] * L + l;
                    if constexpr (RICH) if (llr) {
                        if (comp == c) {
#pragma unroll
                            for (int v = 0; v < PV2; ++v)
                                if (v * 32 + half < n) llr[inst * n + (vid[v] & 0xffffu)] = Pl[v];
                        }
                    }
                    // bit-packed hard decisions: lane t of word w fetches the decision bits
                    // of the lane holding variable 64 w + t of instance c and keeps the
                    // bit of that variable's pass; a ballot packs the word
                    uint64_t wb[kW];
#pragma unroll
                    for (int w = 0; w < kW; ++w) {
                        const uint32_t m = lds_ptr_u32(map_addr)[64 * w + lane];
                        const uint32_t x = (uint32_t)__builtin_amdgcn_ds_bpermute(
                            (int)(((m & 0xffu) + (uint32_t)c) << 2), (int)decb);
                        wb[w] = __ballot((x >> (m >> 8)) & 1u);
                    }
                    // representation-major: a work item's records are contiguous
                    const size_t oi = a.cand_rm ? (size_t)l * a.shots + shot[c] : inst;
                    if (lane < W) {
                        uint64_t word = wb[0];
#pragma unroll
                        for (int w = 1; w < kW; ++w)
                            if (lane == w) word = wb[w];
                        cand[oi * W + lane] = word;
                    }
                    if (lane == 0) kstat[oi] = (uint16_t)(K | (conv ? 0x8000 : 0));
                    it[c] = 0;
                    if (next < ip.end) {
                        shot[c] = next++;
                        fresh |= 1u << c;
                    } else {
                        shot[c] = -1;
                    }
                }
                wave_sync();
            }
#pragma unroll
            for (int c = 0; c < 2; ++c)
                if (!((done >> c) & 1u)) ++it[c];
            wave_sync();
        }

        if (a.persistent) {
            unsigned long long v = 0;
            if (lane == 0) v = atomicAdd(a.queue, 1ull);
            item = uniform_i64((long long)v);
        } else {
            item += (int64_t)gridDim.x * (blockDim.x >> 6);  // grid-sized stride (capped grid)
        }
    }
}

namespace {

struct DualPair {
    int pv, pc;
};
// (variable passes, check passes) of the paired kernels, both instances together
const DualPair kDualPairs[] = {{1, 1}, {2, 1}, {2, 2}, {3, 2}, {3, 3}, {4, 3}, {5, 3}, {5, 4}};
constexpr int kDualMaxChunk = 128;         // shots of a work item (syndromes staged in LDS)
constexpr int kDualMaxSynBytes = 4096;     // LDS for those syndrome words

bool dual_pick_passes(int pv, int pc, DualPair &out) {
    for (const DualPair &d : kDualPairs)
        if (d.pv >= pv && d.pc >= pc) { out = d; return true; }
    return false;
}

bool dual_pick(const BPArgs &a, DualPair &out) {
    int pv = 1, pc = 1;
    for (int p = a.part0; p < a.part0 + a.nparts; ++p) {
        pv = max(pv, (2 * a.part[p].n + 63) / 64);
        pc = max(pc, (a.part[p].Mmax + 1 + 31) / 32);  // positions of an instance incl. the sink
    }
    return dual_pick_passes(pv, pc, out);
}

template <int PV2, int PC2, int DC, int MAXD, bool RICH>
hipError_t launch_dual_t(const BPArgs &a, const BPConfig &cfg, hipStream_t s) {
    const int wpb = cfg.waves_per_block;
    const size_t lds = (size_t)wpb * a.inst_bytes;
    const int64_t blocks = a.persistent ? cfg.blocks : plain_grid((a.n_items + wpb - 1) / wpb);
    hipLaunchKernelGGL((bp_dual_kernel<PV2, PC2, DC, MAXD, RICH>), dim3((unsigned)blocks), dim3(64 * wpb), lds, s,
                       a);
    set_last_bp_kernel(reinterpret_cast<const void *>(&bp_dual_kernel<PV2, PC2, DC, MAXD, RICH>));
    return hipGetLastError();
}

template <int PV2, int PC2, int DC>
hipError_t launch_dual_dc(const BPArgs &a, const BPConfig &cfg, hipStream_t s) {
    int maxd = 0;
    bool llr = false;
    for (int p = a.part0; p < a.part0 + a.nparts; ++p) {
        maxd = max(maxd, a.part[p].max_deg);
        llr = llr || a.llr[p] != nullptr;
    }
    const bool rich = llr || a.prior_per_shot != 0;  // posteriors or per-shot priors
    llr = rich;
    if (maxd <= 6)
        return llr ? launch_dual_t<PV2, PC2, DC, 6, true>(a, cfg, s) : launch_dual_t<PV2, PC2, DC, 6, false>(a, cfg, s);
    return llr ? launch_dual_t<PV2, PC2, DC, 8, true>(a, cfg, s) : launch_dual_t<PV2, PC2, DC, 8, false>(a, cfg, s);
}

template <int PV2, int PC2>
hipError_t launch_dual_pair(const BPArgs &a, const BPConfig &cfg, hipStream_t s) {
    bool u6 = true;
    for (int p = a.part0; p < a.part0 + a.nparts; ++p) u6 = u6 && a.part[p].uniform_dc == 6;
    return u6 ? launch_dual_dc<PV2, PC2, 6>(a, cfg, s) : launch_dual_dc<PV2, PC2, 8>(a, cfg, s);
}

}  // namespace

bool bp_dual_layout(const BPArgs &a, int schedule, int rule, int &inst_bytes, int &stride) {
    if (schedule != 0 || rule != kRuleNMS || a.fixed_T) return false;
    if (a.chunk > kDualMaxChunk || a.chunk * a.ws_max * 8 > kDualMaxSynBytes) return false;
    DualPair d;
    if (!dual_pick(a, d)) return false;
    const int mpad = 32 * d.pc;
    bool u6 = true;
    for (int p = a.part0; p < a.part0 + a.nparts; ++p) u6 = u6 && a.part[p].uniform_dc == 6;
    const int slots = u6 ? 6 : 8;  // message slots per row: DC of the kernel launched
    const int msg = (4 * slots * (mpad + kSlotPad) + 15) & ~15;  // LayoutM<mpad, NMS, DC, true, true>
    const int dec = (8 * mpad + 15) & ~15;
    const int bytes = msg + dec + a.w_max * 8;
    // instance regions 64 bytes off a multiple of 128: the two instances' copies of
    // one row lie 16 banks apart, so interleaved lanes never share a bank
    stride = ((bytes + 127) & ~127) + 64;
    // + the variable map of the output path: 64 words per output word of an instance
    inst_bytes = 2 * stride + ((a.chunk * a.ws_max * 8 + 15) & ~15) + 4 * 64 * ((32 * d.pv + 63) / 64);
    return true;
}

bool bp_dual_fits(int n, int mmax) {
    DualPair d;
    return dual_pick_passes((2 * n + 63) / 64, (mmax + 1 + 31) / 32, d);
}

hipError_t launch_bp_dual(const BPArgs &a, const BPConfig &cfg, hipStream_t s) {
    DualPair d;
    if (!dual_pick(a, d)) return hipErrorInvalidValue;
    switch (d.pv * 16 + d.pc) {
    case 1 * 16 + 1: return launch_dual_pair<1, 1>(a, cfg, s);
    case 2 * 16 + 1: return launch_dual_pair<2, 1>(a, cfg, s);
    case 2 * 16 + 2: return launch_dual_pair<2, 2>(a, cfg, s);
    case 3 * 16 + 2: return launch_dual_pair<3, 2>(a, cfg, s);
    case 3 * 16 + 3: return launch_dual_pair<3, 3>(a, cfg, s);
    case 4 * 16 + 3: return launch_dual_pair<4, 3>(a, cfg, s);
    case 5 * 16 + 3: return launch_dual_pair<5, 3>(a, cfg, s);
    case 5 * 16 + 4: return launch_dual_pair<5, 4>(a, cfg, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mbbp
