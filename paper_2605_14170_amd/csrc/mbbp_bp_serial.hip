// Serial-schedule BP kernel (Section II-B: check nodes updated one after another,
// each from the latest messages) with one lane per shot.
//
// The serial schedule is a chain: check j reads the check-to-variable messages
// that checks 0..j-1 wrote in this sweep, so one instance has almost no
// parallelism inside a sweep (the exact conflict-free levels of a [[144]]
// representation hold one or two checks each).  Here the lanes of a wavefront are
// SL shots of the same representation, and every lane walks the augmented rows
// 0..M-1 in order: the control flow, the check record and every LDS offset are
// wave-uniform, only the values differ per lane.
//
// LDS of one wavefront (lane-minor, so every access of the wave is SL consecutive
// words, conflict-free):
//   messages  float [E][SL]          c->v message of each edge
//   decisions u32 [ceil(n/4)][SL]    hard decision of variable v in byte v % 4 of row v / 4
//   aug       u32 [NMW][SL]          augmented syndrome bits (row j: bit j % 32 of word j / 32)
//   synw      u32 [2 Ws][SL]         the shot's syndrome words (staged at refill)
//   prior     float [n][SL]          per-shot priors (prior_per_shot only)
//   mu        float [n]              the one prior vector otherwise (broadcast reads)
//
// Edges are numbered variable by variable, a variable's edges in ascending row
// order, so per check j and row slot k one word describes everything: the
// variable v, its first edge, its degree and the rank t of row j among v's rows.
// The variable-to-check message is the exclusion sum mu_v + v's other messages in
// ascending order: the contiguous LDS rows before rank t (written earlier in this
// sweep) and after it (the previous sweep's).  The check's own rows are set to 0
// before they are read, so the sum runs over all of v's rows (adding +0 changes no
// sum here: it starts at a canonical prior and is never -0), with no per-row
// selection.  After the check rule the new messages are written.  At v's last row
// (t = degree - 1) the posterior mu_v + sum over all of v's rows (ascending) is
// exactly that sum plus the new message, so the decision of v is taken there, in
// the sweep itself.  The records of a representation (one word per slot, about
// 2 KB for [[144]]) stay in the scalar cache.
//
// A lane whose shot halts (Section II-B: syndrome met, or T sweeps) writes its
// outputs and takes the next shot of the work item at once; its message column is
// cleared before the new shot's first sweep (the rows of later checks are read
// before that sweep writes them, and start at 0).
#include <hip/hip_runtime.h>

#include "mbbp_bp_rules.h"
#include "mbbp_device.h"
#include "mbbp_wave.h"

namespace mbbp {

namespace {

struct SerialItem {
    int part, l;
    int64_t begin, end;
};

__device__ __forceinline__ SerialItem serial_item(const BPArgs &a, int64_t item) {
    const int64_t rank = item / a.n_chunks;
    const int64_t ch = item - rank * a.n_chunks;
    typedef __attribute__((address_space(4))) const int32_t c_i32_;
    const int pl = uniform_i32(a.item_order ? ((const c_i32_ *)a.item_order)[rank] : (int)rank);
    SerialItem p;
    p.part = a.part0 + pl / a.L;
    p.l = pl - (pl / a.L) * a.L;
    p.begin = ch * a.chunk;
    p.end = min(p.begin + (int64_t)a.chunk, a.shots);
    return p;
}

template <typename T>
__device__ __forceinline__ T pick3(const T (&v)[2], int part) { return part == 0 ? v[0] : v[1]; }

// the record word of a row slot: variable, rank t of the row among the variable's
// rows, degree - 1, first edge of the variable
__device__ __forceinline__ int rec_var(uint32_t w) { return (int)(w & 0x3ffu); }
__device__ __forceinline__ int rec_rank(uint32_t w) { return (int)((w >> 10) & 7u); }
__device__ __forceinline__ int rec_dm1(uint32_t w) { return (int)((w >> 13) & 7u); }
__device__ __forceinline__ uint32_t rec_first(uint32_t w) { return w >> 16; }
__device__ __forceinline__ bool rec_absent(uint32_t w) { return w == 0xffffffffu; }

// Constant-address-space views of the tables: a uniform load from them is a
// scalar load (the kernel never writes them), kept in the scalar cache.
typedef __attribute__((address_space(4))) const uint32_t c_u32;
typedef __attribute__((address_space(4))) const int32_t c_i32;
template <typename T, typename P>
__device__ __forceinline__ const T *as_const(const P *p) { return (const T *)(p); }

// 4 decision bytes (0 or 1) of a word -> 4 bits, byte b to bit b
__device__ __forceinline__ uint32_t pack4(uint32_t w) { return ((w & 0x01010101u) * 0x01020408u) >> 24; }

}  // namespace

// DC: record slots per check (6: every row of weight 6; 8: weights 2..8, absent
// slots read as +FLT_MAX); SL: shots per wavefront (the LDS row stride), a
// compile-time constant so that row offsets are instruction immediates.
template <int DC, int RULE, int SL>
__global__ __launch_bounds__(64) void bp_serial_kernel(BPArgs a) {
    const int lane = threadIdx.x & 63;
    // lanes beyond SL have no LDS column (their addresses would fall in the next
    // row's words): they leave at once, and every wave-wide operation below sees
    // only the shot lanes
    if (lane >= SL) return;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr uint32_t RS = 4u * SL;  // bytes per LDS row
    const uint32_t base = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(size_t)(lds_u8 *)smem);
    const uint32_t lane4 = 4u * (uint32_t)lane;
    const int nq_max = (a.n_max + 3) >> 2;
    const uint32_t msg_addr = base + lane4;                                        // [E][SL]
    const uint32_t dec_addr = msg_addr + RS * (uint32_t)a.s_emax;                 // [ceil(n/4)][SL]
    const uint32_t aug_addr = dec_addr + RS * (uint32_t)nq_max;                   // [NMW][SL]
    const uint32_t syn_addr = aug_addr + RS * (uint32_t)a.s_nmw;                  // [2 Ws][SL]
    const uint32_t pri_addr = syn_addr + RS * (uint32_t)(2 * a.ws_max);           // [n][SL] (per-shot priors)
    const uint32_t mu_addr = base + RS * (uint32_t)(a.s_emax + nq_max + a.s_nmw + 2 * a.ws_max +
                                                    (a.prior_per_shot ? a.n_max : 0));  // [n]
    constexpr uint64_t lanes_mask = SL >= 64 ? ~0ull : ((1ull << SL) - 1ull);

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

    while (item < a.n_items) {
        const SerialItem ip = serial_item(a, item);
        // the part's tables through a constant-address-space pointer: every field below
        // is a scalar load into scalar registers
        typedef __attribute__((address_space(4))) const DevPart c_part;
        const c_part *pt = (const c_part *)(a.dparts + ip.part);
        const int n = pt->n, m = pt->m, W = pt->W, Ws = pt->Ws, L = pt->L, l = ip.l;
        const int M = as_const<c_i32>(pt->M)[l];
        const int E = as_const<c_i32>(pt->E)[l];
        const int dcs = pt->dcs;  // record slots of this part (<= DC)
        const int so = as_const<c_i32>(pt->stab_off)[l];
        const c_u32 *rec0 = as_const<c_u32>(pt->stab) + (size_t)so * dcs;
        const c_i32 *csrc = as_const<c_i32>(pt->scsrc) + so;  // syndrome source of each row
        // rows of H, 8 u16 slots each, read as 4 dwords per row (scalar loads have no
        // 16-bit form)
        const c_u32 *htab = as_const<c_u32>(reinterpret_cast<const uint32_t *>(pt->htab));
        const c_i32 *comb_ptr = as_const<c_i32>(pt->comb_ptr);
        const c_i32 *comb_idx = as_const<c_i32>(pt->comb_idx);
        const float *prior = pick3(a.prior, ip.part);
        const uint64_t *syn = pick3(a.syn, ip.part);
        uint64_t *cand = pick3(a.cand, ip.part);
        uint16_t *kstat = pick3(a.kstat, ip.part);
        float *llr = pick3(a.llr, ip.part);
        const int nmw = (M + 31) >> 5;
        const int nq = (n + 3) >> 2;
        const bool pps = a.prior_per_shot != 0;
        if (!pps) {  // the prior vector, staged once per item
            for (int v = lane; v < n; v += SL) *lds_ptr_f32(mu_addr + 4u * (uint32_t)v) = prior[v] + 0.0f;
            wave_sync();
        }
        auto mu_of = [&](int v) -> float {
            return pps ? *lds_ptr_f32(pri_addr + RS * (uint32_t)v) : *lds_ptr_f32(mu_addr + 4u * (uint32_t)v);
        };
        // byte address of variable v's decision in this lane's column
        auto dec_byte = [&](int v) -> uint32_t { return dec_addr + RS * (uint32_t)(v >> 2) + (uint32_t)(v & 3); };
        // parity of the decisions on row j of H, xor its syndrome bit (1: unsatisfied)
        auto row_unsat = [&](int j) -> uint32_t {
            uint32_t hw[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) hw[h] = htab[j * 4 + h];
            const uint32_t swj = *lds_ptr_u32(aug_addr + RS * (uint32_t)(j >> 5));
            uint32_t par = (swj >> (j & 31)) & 1u;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int v = (int)((hw[k >> 1] >> (16 * (k & 1))) & 0xffffu);
                if (v == 0xffff) break;
                par ^= (uint32_t)*lds_ptr_u8(dec_byte(v));
            }
            return par & 1u;
        };
        // outputs of a halted lane: decisions packed into W words, iterations | converged
        auto write_out = [&](int64_t s, int K, bool conv) {
            const size_t inst = a.cand_rm ? (size_t)l * a.shots + s : (size_t)s * L + l;
            for (int w = 0; w < W; ++w) {
                uint64_t word = 0;
#pragma unroll 4
                for (int g = 0; g < 16; ++g) {
                    const int q = 16 * w + g;
                    if (q >= nq) break;
                    word |= (uint64_t)pack4(*lds_ptr_u32(dec_addr + RS * (uint32_t)q)) << (4 * g);
                }
                cand[inst * W + w] = word;
            }
            kstat[inst] = (uint16_t)(K | (conv ? 0x8000 : 0));
        };

        int64_t next = ip.begin;  // next shot of the item to hand out (wave-uniform)
        int64_t shot = -1;        // this lane's shot (-1: idle)
        int it = 0, kfix = -1;
        bool fresh = false;       // the shot has not had its first sweep

        while (true) {
            // ---------------- refill rounds: idle lanes take the item's next shots and
            // meet the t = 0 halting test; lanes done at t = 0 are refilled again
            while (true) {
                const uint64_t idle = __ballot(shot < 0) & lanes_mask;
                const int64_t left = ip.end - next;
                const int take = (int)min((int64_t)__popcll(idle), left);
                bool mine = false;
                if (take > 0) {
                    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                    mine = ((idle >> lane) & 1ull) && rank < take;
                    if (mine) {
                        shot = next + rank;
                        it = 0;
                        kfix = -1;
                        fresh = true;
                        // stage the shot's syndrome words and (per-shot priors) its priors
                        for (int w = 0; w < Ws; ++w) {
                            const uint64_t sv = syn[shot * Ws + w];
                            *lds_ptr_u32(syn_addr + RS * (uint32_t)(2 * w)) = (uint32_t)sv;
                            *lds_ptr_u32(syn_addr + RS * (uint32_t)(2 * w + 1)) = (uint32_t)(sv >> 32);
                        }
                        if (pps)
                            for (int v = 0; v < n; ++v)
                                *lds_ptr_f32(pri_addr + RS * (uint32_t)v) = prior[shot * n + v] + 0.0f;
                    }
                    next += take;
                    // augmented syndrome bits of the fresh lanes: row j copies its source row's
                    // bit (an explicit appended row: the sum of its source rows' bits)
                    for (int g = 0; g < nmw; ++g) {
                        uint32_t word = 0;
                        const int j1 = min(M, 32 * g + 32);
                        for (int j = 32 * g; j < j1; ++j) {
                            const int src = csrc[j];
                            uint32_t bit = 0;
                            if (src >= 0) {
                                bit = *lds_ptr_u32(syn_addr + RS * (uint32_t)(src >> 5)) >> (src & 31);
                            } else {
                                for (int t = comb_ptr[-src - 1]; t < comb_ptr[-src]; ++t) {
                                    const int r = comb_idx[t];
                                    bit ^= *lds_ptr_u32(syn_addr + RS * (uint32_t)(r >> 5)) >> (r & 31);
                                }
                            }
                            word |= (bit & 1u) << (j & 31);
                        }
                        if (mine) *lds_ptr_u32(aug_addr + RS * (uint32_t)g) = word;
                    }
                    // t = 0: decisions (and posteriors) from the priors
                    if (mine) {
                        for (int q = 0; q < nq; ++q) {
                            uint32_t word = 0;
#pragma unroll
                            for (int b = 0; b < 4; ++b) {
                                const int v = 4 * q + b;
                                if (v < n && mu_of(v) < 0.0f) word |= 1u << (8 * b);
                            }
                            *lds_ptr_u32(dec_addr + RS * (uint32_t)q) = word;
                        }
                        if (llr)
                            for (int v = 0; v < n; ++v) llr[((size_t)shot * L + l) * n + v] = mu_of(v);
                    }
                }
                // halting test at t = 0 of the lanes just handed a shot
                if (__ballot(mine) == 0ull) break;
                uint32_t unsat = 0;
                for (int j = 0; j < m; ++j) unsat |= row_unsat(j);
                bool done = false;
                if (mine) {
                    const bool sat = unsat == 0u;
                    if (sat) kfix = 0;
                    done = a.fixed_T ? T == 0 : (sat || T == 0);
                    if (done) {
                        write_out(shot, sat ? 0 : T, sat);
                        shot = -1;
                    }
                }
                // lanes done at t = 0 are idle again: hand out more shots while any are left
                if (__ballot(done) == 0ull || ip.end <= next) break;
            }
            // no busy lane after the refill rounds: the item has no shots left
            if (__ballot(shot >= 0) == 0ull) break;
            // a shot's first sweep starts from messages 0 (the rows of later checks are read
            // before this sweep writes them): clear the columns of the lanes just filled
            if (fresh && shot >= 0) {
                for (int e = 0; e < E; ++e) *lds_ptr_f32(msg_addr + RS * (uint32_t)e) = 0.0f;
                fresh = false;
            }

            // ---------------- one sweep over the augmented rows in order
            const bool busy = shot >= 0;
            uint32_t sw = 0;
            for (int j = 0; j < M; ++j) {
                if ((j & 31) == 0) sw = *lds_ptr_u32(aug_addr + RS * (uint32_t)(j >> 5));
                // the row's record words in one batch (tables are padded past their end)
                const c_u32 *rec = rec0 + (size_t)j * dcs;
                uint32_t rw[DC];
#pragma unroll
                for (int k = 0; k < DC; ++k) rw[k] = rec[k];
                if (DC == 8) {
#pragma unroll
                    for (int k = 6; k < DC; ++k) rw[k] = k < dcs ? rw[k] : 0xffffffffu;
                }
                // the row's own messages first set to 0, then every read of the row: priors
                // and up to six rows of each slot's variable
                uint32_t own[DC];
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    if (DC == 8 && rec_absent(rw[k])) continue;
                    own[k] = msg_addr + RS * (rec_first(rw[k]) + (uint32_t)rec_rank(rw[k]));
                    *lds_ptr_f32(own[k]) = 0.0f;
                }
                float mu[DC], x[DC][6];
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    if (DC == 8 && rec_absent(rw[k])) continue;
                    mu[k] = mu_of(rec_var(rw[k]));
                    const lds_f32 *row = lds_ptr_f32(msg_addr + RS * rec_first(rw[k]));
#pragma unroll
                    for (int u = 0; u < 6; ++u) x[k][u] = row[u * SL];
                }
                float q[DC], qs[DC];
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    if (DC == 8 && rec_absent(rw[k])) {
                        q[k] = 3.402823466e38f;
                        qs[k] = 0.0f;
                        continue;
                    }
                    const int dm1 = rec_dm1(rw[k]);
                    // mu_v + v's rows in ascending order, the own row reading 0
                    float acc = mu[k] + x[k][0];
#pragma unroll
                    for (int u = 1; u < 6; ++u) {
                        if (u > dm1) break;
                        acc += x[k][u];
                    }
                    if (dm1 >= 6) {  // degree 7 or 8
                        const lds_f32 *row = lds_ptr_f32(msg_addr + RS * rec_first(rw[k]));
                        acc += row[6 * SL];
                        if (dm1 >= 7) acc += row[7 * SL];
                    }
                    q[k] = acc;
                    qs[k] = acc;
                }
                CheckRule<RULE>::template apply<DC>(q, (int)((sw >> (j & 31)) & 1u), alpha, rmax);
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    if (DC == 8 && rec_absent(rw[k])) continue;
                    *lds_ptr_f32(own[k]) = q[k];
                    if (rec_rank(rw[k]) == rec_dm1(rw[k])) {
                        // posterior of v at its last row: the exclusion sum plus the new message
                        const int v = rec_var(rw[k]);
                        const float P = qs[k] + q[k];
                        *lds_ptr_u8(dec_byte(v)) = (unsigned char)(P < 0.0f ? 1 : 0);
                        if (llr && busy) llr[((size_t)shot * L + l) * n + v] = P;
                    }
                }
            }
            if (busy) ++it;
            // ---------------- halting test (Section II-B) against the rows of H
            uint32_t unsat = 0;
            for (int j = 0; j < m; ++j) {
                unsat |= row_unsat(j);
                // every busy lane already fails a row: the rest of the test cannot change that
                if ((j & 7) == 7 && __ballot(busy && unsat == 0u) == 0ull) break;
            }
            if (busy) {
                const bool sat = unsat == 0u;
                bool done;
                bool conv;
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

template <int DC, int RULE, int SL>
hipError_t launch_serial_t(const BPArgs &a, const BPConfig &cfg, hipStream_t s) {
    const size_t lds = (size_t)a.inst_bytes;
    const auto kern = bp_serial_kernel<DC, RULE, SL>;
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

template <int DC, int RULE>
hipError_t launch_serial_sl(const BPArgs &a, const BPConfig &cfg, hipStream_t s) {
    switch (a.serial_lanes) {
    case 64: return launch_serial_t<DC, RULE, 64>(a, cfg, s);
    case 32: return launch_serial_t<DC, RULE, 32>(a, cfg, s);
    case 16: return launch_serial_t<DC, RULE, 16>(a, cfg, s);
    case 8: return launch_serial_t<DC, RULE, 8>(a, cfg, s);
    case 4: return launch_serial_t<DC, RULE, 4>(a, cfg, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool serial_lanes_supported(int n, int S) {
    return n <= 1024 && (S == 64 || S == 32 || S == 16 || S == 8 || S == 4);
}

hipError_t launch_bp_serial(const BPArgs &a, const BPConfig &cfg, int rule, hipStream_t s) {
    bool u6 = true;
    for (int p = a.part0; p < a.part0 + a.nparts; ++p) u6 = u6 && a.part[p].uniform_dc == 6;
    if (rule == kRuleNMS)
        return u6 ? launch_serial_sl<6, kRuleNMS>(a, cfg, s) : launch_serial_sl<8, kRuleNMS>(a, cfg, s);
    if (rule == kRuleSPA)
        return u6 ? launch_serial_sl<6, kRuleSPA>(a, cfg, s) : launch_serial_sl<8, kRuleSPA>(a, cfg, s);
    return hipErrorInvalidValue;
}

}  // namespace mbbp
