// Serial-schedule BP kernel for normalized min-sum (Section II-B, eq. (1)) with the
// slots of a check spread over lanes: eight lanes per shot, lane k holding row slot
// k, and up to eight shots of one representation per wavefront.
//
// The serial schedule updates the augmented rows 0..M-1 one after another, each from
// the latest messages, so inside one shot a sweep is a chain of M steps.  Here the
// eight lanes of a group do the one step of their shot together: lane k forms the
// variable-to-check message of its slot (the exclusion sum of its variable), the
// group combines the eight values by a three-step butterfly (the two smallest
// magnitudes and the XOR of the signs are the only row quantities normalized
// min-sum needs, and both are independent of the order they are combined in), and
// lane k writes the message back.  A row costs the group a few dozen instructions,
// where a lane holding a whole shot would spend several hundred; the messages of a
// shot take the same LDS either way.
//
// LDS of one wavefront: G shot blocks of SB bytes (SB / 4 = 8 mod 32, so the blocks
// of the groups start eight banks apart), then the shared prior vector and the
// decisions it gives at t = 0:
//   junk      float [8]          what the lanes of absent slots read and write (word 0
//                                 holds +FLT_MAX, the value an absent slot enters)
//   messages  float [Emax]       edges numbered variable by variable, a variable's
//                                 edges in ascending row order
//   decisions u32 [n / 32 + 1]   hard decision of v in bit v % 32 of word v / 32 (bit n
//                                 is never set: the rows of H read it for padding)
//   aug       u32 [NMW]          augmented syndrome bits
//   synw      u32 [2 Ws]         the shot's syndrome words
//   prior     float [n + 1]      per-shot priors (prior_per_shot only), then a 0
// Per row slot a record (two words, one lane's load) holds the byte offsets of the
// slot's variable v (its first edge, the edge of this row (rank t among v's rows), its
// prior and its decision word), the decision's bit, v's degree, whether t is v's last
// rank, and the largest degree in the row (which bounds the exclusion sums of the whole
// row).  An absent slot's lane reads a 0 prior and the junk words, so its value is
// +FLT_MAX exactly, and writes only junk.
// The exclusion sum mu_v + v's other messages in ascending row order is formed with
// the slot's own message set to 0 first (adding +0 changes none of these sums: they
// start at a canonical prior and are never -0).  At v's last row the posterior is
// that sum plus the new message, so the decision is taken in the sweep.
//
// A group whose shot halts (syndrome met, or T sweeps) writes its outputs and takes
// the work item's next shot before the next sweep; its messages are cleared first.
#include <hip/hip_runtime.h>

#include "mbbp_device.h"
#include "mbbp_wave.h"

namespace mbbp {

namespace {

struct SlotItem {
    int part, l;
    int64_t begin, end;
};

__device__ __forceinline__ SlotItem slot_item(const BPArgs &a, int64_t item) {
    const int64_t rank = item / a.n_chunks;
    const int64_t ch = item - rank * a.n_chunks;
    typedef __attribute__((address_space(4))) const int32_t c_i32_;
    const int pl = uniform_i32(a.item_order ? ((const c_i32_ *)a.item_order)[rank] : (int)rank);
    SlotItem p;
    p.part = a.part0 + pl / a.L;
    p.l = pl - (pl / a.L) * a.L;
    p.begin = ch * a.chunk;
    p.end = min(p.begin + (int64_t)a.chunk, a.shots);
    return p;
}

template <typename T>
__device__ __forceinline__ T pick2(const T (&v)[2], int part) { return part == 0 ? v[0] : v[1]; }

// Lane permutations inside each group of eight lanes (DPP controls): swap with lane
// i ^ 1, with lane i ^ 2 (quad permutations), and lane i <-> 7 - i (half-row mirror,
// which pairs each lane of one quad with a lane of the other).
constexpr int kDppX1 = 0xB1;          // quad_perm [1, 0, 3, 2]
constexpr int kDppX2 = 0x4E;          // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141; // row_half_mirror

template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xf, 0xf, true);
}

// Two smallest magnitudes of the group's eight values (m1 <= m2, equal on a tie) and
// the XOR of their sign bits, in every lane of the group.  Merging two sorted pairs
// (m1, m2) and (p1, p2): the smaller is min(m1, p1) and the second smallest is
// med3(m1, p1, min(m2, p2)).
__device__ __forceinline__ void group_min2(float q, float &m1, float &m2, uint32_t &sx) {
    const float a = fabsf(q);
    const float p = dpp_f<kDppX1>(a);
    m1 = fminf(a, p);
    m2 = fmaxf(a, p);
    float p1 = dpp_f<kDppX2>(m1), p2 = dpp_f<kDppX2>(m2);
    m2 = __builtin_amdgcn_fmed3f(m1, p1, fminf(m2, p2));
    m1 = fminf(m1, p1);
    p1 = dpp_f<kDppHalfMirror>(m1);
    p2 = dpp_f<kDppHalfMirror>(m2);
    m2 = __builtin_amdgcn_fmed3f(m1, p1, fminf(m2, p2));
    m1 = fminf(m1, p1);
    uint32_t s = fbits(q);
    s ^= dpp_u<kDppX1>(s);
    s ^= dpp_u<kDppX2>(s);
    s ^= dpp_u<kDppHalfMirror>(s);
    sx = s;
}

}  // namespace

// D: largest variable degree of the launch's representations (6 or 8); LLR: the
// posteriors are stored.
template <int D, bool LLR>
__global__ __launch_bounds__(64) void bp_serial_slots_kernel(BPArgs a) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 3, k = lane & 7;
    // groups beyond G have no shot block: they leave at once, so every ballot below
    // sees only the lanes of real groups (and DPP never crosses a group)
    if (g >= a.serial_groups) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t base = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(size_t)(lds_u8 *)smem);
    const uint32_t SB = (uint32_t)a.s_sb;
    const uint32_t blk_g = base + SB * (uint32_t)g;               // this group's shot block
    const uint32_t msg_g = blk_g + 32u;                           // after the 8 junk words
    const uint32_t dec_g = msg_g + 4u * (uint32_t)a.s_emax;
    const uint32_t aug_g = dec_g + 4u * (uint32_t)a.s_ndw;
    const uint32_t syn_g = aug_g + 4u * (uint32_t)a.s_nmw;
    const uint32_t pri_g = syn_g + 8u * (uint32_t)a.ws_max;
    const uint32_t mu_a = base + SB * (uint32_t)a.serial_groups;  // shared priors [n], then a 0
    const uint32_t dec0_a = mu_a + 4u * (uint32_t)(a.n_max + 1);  // their decisions
    const uint32_t gsh = 8u * (uint32_t)g;                         // the group's bits in a ballot
    const int nlanes = 8 * a.serial_groups;
    // junk word 0: the value absent slots read first (nothing writes it later)
    if (k == 0) *lds_ptr_f32(blk_g) = 3.402823466e38f;

    int64_t item;
    if (a.persistent) {
        unsigned long long v = 0;
        if (lane == 0) v = atomicAdd(a.queue, 1ull);
        item = uniform_i64((long long)v);
    } else {
        item = (int64_t)blockIdx.x;
    }
    const float alpha = a.alpha, rmax = a.rmax;
    const int T = a.T;
    const bool pps = a.prior_per_shot != 0;

    while (item < a.n_items) {
        const SlotItem ip = slot_item(a, item);
        typedef __attribute__((address_space(4))) const DevPart c_part;
        typedef __attribute__((address_space(4))) const int32_t c_i32;
        const c_part *pt = (const c_part *)(a.dparts + ip.part);
        const int n = pt->n, m = pt->m, W = pt->W, Ws = pt->Ws, L = pt->L, l = ip.l;
        const int M = ((const c_i32 *)pt->M)[l];
        const int E = ((const c_i32 *)pt->E)[l];
        const int so = ((const c_i32 *)pt->stab_off)[l];
        const uint2 *srec = pt->srec + (size_t)so * 8 + k;  // this slot's records (vector loads)
        const int32_t *csrc = pt->scsrc + so;
        const uint4 *sht4 = reinterpret_cast<const uint4 *>(pt->sht);
        const int32_t *comb_ptr = pt->comb_ptr;
        const int32_t *comb_idx = pt->comb_idx;
        const float *prior = pick2(a.prior, ip.part);
        const uint64_t *syn = pick2(a.syn, ip.part);
        uint64_t *cand = pick2(a.cand, ip.part);
        uint16_t *kstat = pick2(a.kstat, ip.part);
        float *llr = LLR ? pick2(a.llr, ip.part) : nullptr;
        const int ndw = (n >> 5) + 1;
        if (!pps) {
            // the prior vector (and the 0 after it) and its decisions, staged once per item
            for (int v = lane; v <= n; v += nlanes)
                *lds_ptr_f32(mu_a + 4u * (uint32_t)v) = v < n ? prior[v] + 0.0f : 0.0f;
            wave_sync();
            for (int w = lane; w < ndw; w += nlanes) {
                uint32_t word = 0;
                for (int b = 0; b < 32; ++b) {
                    const int v = 32 * w + b;
                    if (v < n && *lds_ptr_f32(mu_a + 4u * (uint32_t)v) < 0.0f) word |= 1u << b;
                }
                *lds_ptr_u32(dec0_a + 4u * (uint32_t)w) = word;
            }
            wave_sync();
        }
        auto mu_of = [&](uint32_t v) -> float {
            return pps ? *lds_ptr_f32(pri_g + 4u * v) : *lds_ptr_f32(mu_a + 4u * v);
        };
        const uint32_t mu_g = pps ? pri_g : mu_a;  // the priors this group reads
        // any lane of the group holding b (every lane of the wave calls it)
        auto group_any = [&](bool b) -> bool { return ((__ballot(b) >> gsh) & 0xffull) != 0ull; };
        // whether some row of H is unsatisfied by the group's decisions; rows k, k + 8,
        // ... go to lane k.  With `early`, stops once every busy group has one.
        auto group_unsat = [&](bool busy, bool early) -> bool {
            bool un = false;
            for (int r0 = 0; r0 < m; r0 += 8) {
                const int r = r0 + k;
                uint32_t par = 0;
                if (r < m) {
                    const uint4 e0 = sht4[2 * r], e1 = sht4[2 * r + 1];
                    const uint32_t e[8] = {e0.x, e0.y, e0.z, e0.w, e1.x, e1.y, e1.z, e1.w};
                    par = *lds_ptr_u32(syn_g + 4u * (uint32_t)(r >> 5)) >> (r & 31);
#pragma unroll
                    for (int t = 0; t < 8; ++t) par ^= *lds_ptr_u32(dec_g + (e[t] >> 8)) >> (e[t] & 31u);
                }
                un = group_any((par & 1u) != 0u) || un;
                if (early && __ballot(busy && !un) == 0ull) break;
            }
            return un;
        };
        // outputs of a halted group: decisions (two words per candidate word),
        // iterations | converged
        auto write_out = [&](int64_t s, int K, bool conv) {
            const size_t inst = a.cand_rm ? (size_t)l * a.shots + s : (size_t)s * L + l;
            for (int w = k; w < W; w += 8) {
                const uint32_t lo = *lds_ptr_u32(dec_g + 8u * (uint32_t)w);
                const uint32_t hi = 2 * w + 1 < ndw ? *lds_ptr_u32(dec_g + 8u * (uint32_t)w + 4u) : 0u;
                cand[inst * W + w] = (uint64_t)lo | ((uint64_t)hi << 32);
            }
            if (k == 0) kstat[inst] = (uint16_t)(K | (conv ? 0x8000 : 0));
        };

        int64_t next = ip.begin;  // next shot of the item to hand out (wave-uniform)
        int64_t shot = -1;        // the group's shot (-1: idle); equal in the group's lanes
        int it = 0, kfix = -1;
        bool fresh = false;       // the shot has not had its first sweep

        while (true) {
            // ---------------- refill rounds: idle groups take the item's next shots and meet
            // the t = 0 halting test; groups done at t = 0 are refilled again
            while (true) {
                const uint64_t idle = __ballot(shot < 0 && k == 0);  // bit 8 g per idle group
                const int64_t left = ip.end - next;
                const int take = (int)min((int64_t)__popcll(idle), left);
                bool mine = false;
                if (take > 0) {
                    // idle groups below this one: the set bits below the lane, less the
                    // group's own bit for lanes 1..7
                    const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                    const int rank = below - ((k > 0 && ((idle >> gsh) & 1ull)) ? 1 : 0);
                    mine = shot < 0 && rank < take;
                    if (mine) {
                        shot = next + rank;
                        it = 0;
                        kfix = -1;
                        fresh = true;
                        for (int w = k; w < 2 * Ws; w += 8) {
                            const uint64_t sv = syn[shot * Ws + (w >> 1)];
                            *lds_ptr_u32(syn_g + 4u * (uint32_t)w) = (w & 1) ? (uint32_t)(sv >> 32) : (uint32_t)sv;
                        }
                        if (pps)
                            for (int v = k; v <= n; v += 8)
                                *lds_ptr_f32(pri_g + 4u * (uint32_t)v) = v < n ? prior[shot * n + v] + 0.0f : 0.0f;
                    }
                    next += take;
                    wave_sync();
                    // augmented syndrome bits: row j = 8 i + k copies its source row's bit (an
                    // explicit appended row: the sum of its source rows' bits); the group's
                    // eight bits of a ballot are rows 8 i .. 8 i + 7
                    uint32_t word = 0;
                    for (int i = 0; 8 * i < M; ++i) {
                        const int j = 8 * i + k;
                        uint32_t bit = 0;
                        if (j < M) {
                            const int src = csrc[j];
                            if (src >= 0) {
                                bit = *lds_ptr_u32(syn_g + 4u * (uint32_t)(src >> 5)) >> (src & 31);
                            } else {
                                for (int t = comb_ptr[-src - 1]; t < comb_ptr[-src]; ++t) {
                                    const int r = comb_idx[t];
                                    bit ^= *lds_ptr_u32(syn_g + 4u * (uint32_t)(r >> 5)) >> (r & 31);
                                }
                            }
                        }
                        word |= (uint32_t)((__ballot((bit & 1u) != 0u) >> gsh) & 0xffull) << (8 * (i & 3));
                        if ((i & 3) == 3 || 8 * (i + 1) >= M) {
                            if (mine && k == 0) *lds_ptr_u32(aug_g + 4u * (uint32_t)(i >> 2)) = word;
                            word = 0;
                        }
                    }
                    // t = 0: decisions (and posteriors) from the priors
                    if (!pps) {
                        if (mine)
                            for (int w = k; w < ndw; w += 8)
                                *lds_ptr_u32(dec_g + 4u * (uint32_t)w) = *lds_ptr_u32(dec0_a + 4u * (uint32_t)w);
                    } else {
                        uint32_t dw = 0;
                        for (int i = 0; 8 * i < n; ++i) {
                            const int v = 8 * i + k;
                            const bool neg = v < n && *lds_ptr_f32(pri_g + 4u * (uint32_t)v) < 0.0f;
                            dw |= (uint32_t)((__ballot(neg) >> gsh) & 0xffull) << (8 * (i & 3));
                            if ((i & 3) == 3 || 8 * (i + 1) >= n) {
                                if (mine && k == 0) *lds_ptr_u32(dec_g + 4u * (uint32_t)(i >> 2)) = dw;
                                dw = 0;
                            }
                        }
                        // the word holding bit n when n is a multiple of 32
                        if (mine && k == 0 && (n & 31) == 0) *lds_ptr_u32(dec_g + 4u * (uint32_t)(n >> 5)) = 0u;
                    }
                    if (LLR && mine)
                        for (int v = k; v < n; v += 8) llr[((size_t)shot * L + l) * n + v] = mu_of((uint32_t)v);
                }
                // halting test at t = 0 of the groups just handed a shot
                if (__ballot(mine) == 0ull) break;
                wave_sync();
                const bool un = group_unsat(mine, false);
                bool done = false;
                if (mine) {
                    const bool sat = !un;
                    if (sat) kfix = 0;
                    done = a.fixed_T ? T == 0 : (sat || T == 0);
                    if (done) {
                        write_out(shot, sat ? 0 : T, sat);
                        shot = -1;
                    }
                }
                // groups done at t = 0 are idle again: hand out more shots while any are left
                if (__ballot(done) == 0ull || ip.end <= next) break;
            }
            // no busy group after the refill rounds: the item has no shots left
            if (__ballot(shot >= 0) == 0ull) break;
            // a shot's first sweep starts from messages 0 (the rows of later checks are read
            // before this sweep writes them)
            if (fresh && shot >= 0) {
                typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
                typedef __attribute__((address_space(3))) u32x4 lds_u32x4;
                const u32x4 zero4 = {0u, 0u, 0u, 0u};
                for (int e4 = k; 4 * e4 < E; e4 += 8) *(lds_u32x4 *)(size_t)(msg_g + 16u * (uint32_t)e4) = zero4;
                fresh = false;
            }

            // ---------------- one sweep over the augmented rows in order
            const bool busy = shot >= 0;
            auto row_step = [&](uint2 rec, int j, uint32_t augw) {
                const uint32_t A = rec.x, B = rec.y;
                const uint32_t own_a = blk_g + (A >> 16);
                *lds_ptr_f32(own_a) = 0.0f;
                const lds_f32 *row = lds_ptr_f32(blk_g + (A & 0xffffu));
                float x[D];
#pragma unroll
                for (int u = 0; u < D; ++u) x[u] = row[u];
                const float muv = *lds_ptr_f32(mu_g + (B & 0xfffu));
                // every row read issued before the sum (none is moved into its masked add)
                if constexpr (D == 6) asm volatile("" : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]));
                else asm volatile("" : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]), "+v"(x[6]), "+v"(x[7]));
                // mu_v + v's rows in ascending order, the own row reading 0; rows past v's
                // degree add +0 (no change: the sum is never -0); no slot of the row has
                // more than rdm + 1 rows (every lane's record carries rdm)
                const int rdm = (__builtin_amdgcn_readfirstlane((int)B) >> 12) & 7;
                float acc = muv + x[0];
#pragma unroll
                for (int u = 1; u < D; ++u) {
                    if (u > rdm) break;
                    acc += B >= ((uint32_t)u << 29) ? x[u] : 0.0f;
                }
                const float q = acc;
                float m1, m2;
                uint32_t sx;
                group_min2(q, m1, m2, sx);
                // (-1)^{s_j} * product of the other slots' signs * min(alpha * min over the
                // other slots' magnitudes, rmax): min2 for the slot holding the minimum
                const uint32_t sgn = (sx ^ (augw << (31 - (j & 31)))) & 0x80000000u;
                const float mag = (fabsf(q) == m1) ? m2 : m1;
                const uint32_t Am = fbits(fminf(alpha * mag, rmax)) | sgn;
                const float qn = bitsf((fbits(q) & 0x80000000u) ^ Am);
                *lds_ptr_f32(own_a) = qn;
                if ((B & 0x8000u) != 0u) {
                    // posterior of v at its last row: the exclusion sum plus the new message;
                    // its bit cleared, then set if negative (atomics: the group's other lanes
                    // may change other bits of the word)
                    const float P = acc + qn;
                    lds_u32 *dw = lds_ptr_u32(dec_g + ((B >> 16) & 0xffu));
                    const uint32_t bit = 1u << (B >> 24);
                    __hip_atomic_fetch_and(dw, ~bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                    __hip_atomic_fetch_or(dw, P < 0.0f ? bit : 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                    if (LLR && busy) llr[((size_t)shot * L + l) * n + ((B & 0xfffu) >> 2)] = P;
                }
            };
            // two rows per trip, each record register reloaded (two rows ahead; the table is
            // padded past its last row) right after its row is done (every trip issues both
            // loads, so the wait before a row's record leaves the younger load in flight)
            uint2 r_a = srec[0], r_b = srec[8];
            uint32_t augw = 0;
            int j = 0;
            for (; j + 1 < M; j += 2) {
                if ((j & 31) == 0) augw = *lds_ptr_u32(aug_g + 4u * (uint32_t)(j >> 5));
                row_step(r_a, j, augw);
                r_a = srec[(size_t)(j + 2) * 8];
                row_step(r_b, j + 1, augw);
                r_b = srec[(size_t)(j + 3) * 8];
            }
            if (j < M) {
                if ((j & 31) == 0) augw = *lds_ptr_u32(aug_g + 4u * (uint32_t)(j >> 5));
                row_step(r_a, j, augw);
            }
            if (busy) ++it;
            // ---------------- halting test (Section II-B) against the rows of H
            const bool un = group_unsat(busy, true);
            if (busy) {
                const bool sat = !un;
                bool done, conv;
                int K;
                if (!a.fixed_T) {
                    done = sat || it == T;
                    conv = sat;
                    K = sat ? it : T;
                } else {
                    if (sat && kfix < 0) kfix = it;
                    done = it == T;
                    conv = kfix >= 0;
                    K = conv ? kfix : T;
                }
                if (done) {
                    write_out(shot, K, conv);
                    shot = -1;
                }
            }
        }

        if (a.persistent) {
            unsigned long long v = 0;
            if (lane == 0) v = atomicAdd(a.queue, 1ull);
            item = uniform_i64((long long)v);
        } else {
            item += (int64_t)gridDim.x;  // grid-sized stride (capped grid)
        }
    }
}

namespace {

template <int D, bool LLR>
hipError_t launch_slots_t(const BPArgs &a, const BPConfig &cfg, hipStream_t s) {
    const size_t lds = (size_t)a.inst_bytes;
    const auto kern = bp_serial_slots_kernel<D, LLR>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int64_t blocks = a.persistent ? cfg.blocks : plain_grid(a.n_items);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64), lds, s, a);
    set_last_bp_kernel(reinterpret_cast<const void *>(kern));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_bp_serial_slots(const BPArgs &a, const BPConfig &cfg, hipStream_t s) {
    if (a.serial_groups < 1 || a.serial_groups > 8) return hipErrorInvalidValue;
    int dmax = 0;
    for (int p = a.part0; p < a.part0 + a.nparts; ++p) dmax = std::max(dmax, a.part[p].max_deg);
    if (dmax > 8) return hipErrorInvalidValue;
    bool llr = false;
    for (int p = a.part0; p < a.part0 + a.nparts; ++p) llr = llr || a.llr[p] != nullptr;
    if (llr) return dmax <= 6 ? launch_slots_t<6, true>(a, cfg, s) : launch_slots_t<8, true>(a, cfg, s);
    return dmax <= 6 ? launch_slots_t<6, false>(a, cfg, s) : launch_slots_t<8, false>(a, cfg, s);
}

}  // namespace mbbp
