// Check and variable rules of the BP kernels (Section II-B, eqs. (1)-(2)) and the
// LDS layout of one BP instance, shared by the decoding kernel and the adjoint
// (backward) kernel of the weighted decoder, so a recomputed iteration is the
// same arithmetic as the forward one.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mbbp_device.h"
#include "mbbp_wave.h"

namespace mbbp {

constexpr int kRuleNMS = 0, kRuleSPA = 1, kRuleWeighted = 2;

template <int RULE>
struct CheckRule;

// XOR of N >= 2 words with three-input XORs (v_bitop3, truth table 0x96).
template <int N>
__device__ __forceinline__ uint32_t xor_all(const uint32_t (&x)[N]) {
    uint32_t acc;
    int k;
    if constexpr (N >= 3) {
        acc = __builtin_amdgcn_bitop3_b32(x[0], x[1], x[2], 0x96);
        k = 3;
    } else {
        acc = x[0] ^ x[1];
        k = 2;
    }
#pragma unroll
    for (; k + 2 <= N; k += 2) acc = __builtin_amdgcn_bitop3_b32(acc, x[k], x[k + 1], 0x96);
    if (k < N) acc ^= x[k];
    return acc;
}

// Two smallest magnitudes of a row (m1 <= m2, equal on a tie) and the XOR of all
// sign bits.  Both are order statistics (exact, no rounding), so any comparison
// order gives the same values: groups of three give their smallest and second
// smallest with one min3 and one med3, and two groups (a1 <= a2, b1 <= b2) merge as
// m1 = min(a1, b1), m2 = med3(a1, b1, min(a2, b2)): the smaller of the larger first
// element and the two seconds.
template <int DC>
__device__ __forceinline__ void row_min2(const float (&q)[DC], float &m1, float &m2, uint32_t &sx) {
    uint32_t b[DC];
#pragma unroll
    for (int k = 0; k < DC; ++k) b[k] = fbits(q[k]);
    sx = xor_all<DC>(b);
    if constexpr (DC == 6 || DC == 8) {
        const float a1 = fminf(fminf(fabsf(q[0]), fabsf(q[1])), fabsf(q[2]));
        const float a2 = __builtin_amdgcn_fmed3f(fabsf(q[0]), fabsf(q[1]), fabsf(q[2]));
        const float b1 = fminf(fminf(fabsf(q[3]), fabsf(q[4])), fabsf(q[5]));
        const float b2 = __builtin_amdgcn_fmed3f(fabsf(q[3]), fabsf(q[4]), fabsf(q[5]));
        m1 = fminf(a1, b1);
        m2 = __builtin_amdgcn_fmed3f(a1, b1, fminf(a2, b2));
        if constexpr (DC == 8) {
            const float c1 = fminf(fabsf(q[6]), fabsf(q[7]));
            const float c2 = fmaxf(fabsf(q[6]), fabsf(q[7]));
            m2 = __builtin_amdgcn_fmed3f(m1, c1, fminf(m2, c2));
            m1 = fminf(m1, c1);
        }
    } else {
        m1 = fminf(fabsf(q[0]), fabsf(q[1]));
        m2 = fmaxf(fabsf(q[0]), fabsf(q[1]));
#pragma unroll
        for (int k = 2; k < DC; ++k) {
            const float a = fabsf(q[k]);
            m2 = __builtin_amdgcn_fmed3f(m1, m2, a);
            m1 = fminf(m1, a);
        }
    }
}

// Normalized min-sum (eq. (1)) with syndrome sign and clamp: the message to slot k
// is (-1)^{s_j} * prod_{k' != k} sgn(q_k') * min(alpha * min_{k' != k} |q_k'|, rmax).
// min over the others is min2 for the (first) minimum and min1 for every other slot.
template <>
struct CheckRule<kRuleNMS> {
    template <int DC>
    __device__ __forceinline__ static void apply(float (&q)[DC], int sbit, float alpha, float rmax) {
        float m1, m2;
        uint32_t sx;
        row_min2<DC>(q, m1, m2, sx);
        const uint32_t sgn = (sx & 0x80000000u) ^ ((uint32_t)sbit << 31);
        // magnitudes with the row's sign product applied; each slot then flips by its
        // own sign: sign(q_k) * row product = product over the other slots
        uint32_t A1s = fbits(fminf(alpha * m1, rmax)) | sgn;
        uint32_t A2s = fbits(fminf(alpha * m2, rmax)) | sgn;
        // keep the signed forms as values (one select plus one three-input bit
        // operation per slot), rather than letting the sign be re-split per slot
        asm volatile("" : "+v"(A1s), "+v"(A2s));
        // all slot tests first (one asm block, so each lands in its own scalar register
        // pair), then the selects: no select waits on the test just before it
        uint64_t at1[DC];
        if constexpr (DC == 6) {
            asm volatile(
                "v_cmp_eq_f32_e64 %0, |%6|, %12\n\t"
                "v_cmp_eq_f32_e64 %1, |%7|, %12\n\t"
                "v_cmp_eq_f32_e64 %2, |%8|, %12\n\t"
                "v_cmp_eq_f32_e64 %3, |%9|, %12\n\t"
                "v_cmp_eq_f32_e64 %4, |%10|, %12\n\t"
                "v_cmp_eq_f32_e64 %5, |%11|, %12"
                : "=s"(at1[0]), "=s"(at1[1]), "=s"(at1[2]), "=s"(at1[3]), "=s"(at1[4]), "=s"(at1[5])
                : "v"(q[0]), "v"(q[1]), "v"(q[2]), "v"(q[3]), "v"(q[4]), "v"(q[5]), "v"(m1));
        } else {
#pragma unroll
            for (int k = 0; k < DC; ++k) at1[k] = __ballot(fabsf(q[k]) == m1);
        }
#pragma unroll
        for (int k = 0; k < DC; ++k) {
            const uint32_t mag = __builtin_amdgcn_inverse_ballot_w64(at1[k]) ? A2s : A1s;
            q[k] = bitsf((fbits(q[k]) & 0x80000000u) ^ mag);
        }
    }
};

// Sum-product: pairwise box-plus x [+] y = sgn(x) sgn(y) min(|x|,|y|)
//   + log(1 + e^{-|x+y|}) - log(1 + e^{-|x-y|}), forward/backward over the row so
// slot k gets the box-plus of all other slots; syndrome sign; clamp.
template <>
struct CheckRule<kRuleSPA> {
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

// Weighted min-sum with damping (the differentiable form of the decoder):
//   r_k = clamp((1 - beta) * v_k + beta * rprev_k),  v_k = S_k * (alpha * M_k),
// M_k the smallest |q| over the row's other slots, S_k the product of their signs
// and of (-1)^{s_j}; keep = 1 - beta is passed in, evaluated once per iteration.
// With beta = 0 and a constant alpha the result equals normalized min-sum.
struct WeightedRule {
    template <int DC>
    __device__ __forceinline__ static void apply(float (&q)[DC], const float (&rp)[DC], int sbit, float alpha,
                                                 float keep, float beta, float rmax) {
        float m1, m2;
        uint32_t sx;
        row_min2<DC>(q, m1, m2, sx);
        const float u1 = alpha * m1, u2 = alpha * m2;
        const uint32_t sgn = (sx & 0x80000000u) ^ ((uint32_t)sbit << 31);
#pragma unroll
        for (int k = 0; k < DC; ++k) {
            const float u = (fabsf(q[k]) == m1) ? u2 : u1;
            const float v = bitsf(fbits(u) ^ ((fbits(q[k]) ^ sgn) & 0x80000000u));  // any sign of alpha
            const float w = keep * v + beta * rp[k];
            q[k] = fminf(fmaxf(w, -rmax), rmax);
        }
    }

    // Adjoint of apply for one row.  In: q, rprev, the adjoint rb of the new
    // messages (0 on unused slots).  Out: rb_prev[k] = the adjoint reaching rprev_k
    // through the damping term, qb = the adjoint of q, and the row's contributions
    // to dL/dalpha and dL/dbeta added to ga, gb.  Subgradients: the minimum passes
    // its adjoint to the first slot (in row order) holding the smallest magnitude
    // among the others, d|x|/dx follows the sign bit of x, sign factors are
    // constant, the clamp passes the adjoint only strictly inside (-rmax, rmax).
    template <int DC>
    __device__ __forceinline__ static void adjoint(const float (&q)[DC], const float (&rp)[DC],
                                                   const float (&rb)[DC], int sbit, float alpha, float keep,
                                                   float beta, float rmax, float (&rb_prev)[DC], float (&qb)[DC],
                                                   float &ga, float &gb) {
        // i1: first slot of the smallest |q|; i2: first other slot of the smallest
        // |q| among the rest.  Their values equal the forward's m1 and m2.
        float m1 = fabsf(q[0]);
        int i1 = 0;
#pragma unroll
        for (int k = 1; k < DC; ++k) {
            const float a = fabsf(q[k]);
            if (a < m1) { m1 = a; i1 = k; }
        }
        float m2 = 3.402823466e38f;
        int i2 = i1 == 0 ? 1 : 0;
        bool have = false;
#pragma unroll
        for (int k = 0; k < DC; ++k) {
            const float a = fabsf(q[k]);
            if (k != i1 && (!have || a < m2)) { m2 = a; i2 = k; have = true; }
        }
        uint32_t sx = 0;
#pragma unroll
        for (int k = 0; k < DC; ++k) sx ^= fbits(q[k]);
        const float u1 = alpha * m1, u2 = alpha * m2;
        const uint32_t sgn = (sx & 0x80000000u) ^ ((uint32_t)sbit << 31);
        float to_i1 = 0.0f, to_i2 = 0.0f;
#pragma unroll
        for (int k = 0; k < DC; ++k) {
            const bool at1 = k == i1;
            const float M = at1 ? m2 : m1;
            const float u = at1 ? u2 : u1;
            const uint32_t sk = (fbits(q[k]) ^ sgn) & 0x80000000u;  // sign of S_k
            const float v = bitsf(fbits(u) ^ sk);
            const float w = keep * v + beta * rp[k];
            const float wb = (w > -rmax && w < rmax) ? rb[k] : 0.0f;
            gb += wb * (rp[k] - v);
            rb_prev[k] = wb * beta;
            const float vb = wb * keep;
            ga += vb * bitsf(fbits(M) ^ sk);
            const float Mb = vb * bitsf(fbits(alpha) ^ sk);
            if (at1) to_i2 += Mb;
            else to_i1 += Mb;
        }
#pragma unroll
        for (int k = 0; k < DC; ++k) {
            const float g = k == i1 ? to_i1 : (k == i2 ? to_i2 : 0.0f);
            qb[k] = bitsf(fbits(g) ^ (fbits(q[k]) & 0x80000000u));
        }
    }
};

// LDS layout of one BP instance, Mpad row positions, slot stride
// S = Mpad + kSlotPad words.  Two forms: the wide one (8 message slots) and, for
// large codes whose instances would otherwise leave most of a CU idle for want of
// LDS, the compact one (DC slots):
//   messages  float [slots][S]  slot-major: edge (p, k) at k * S + p
//   decisions u8 [Mpad][8]      row-major: edge (p, k) at 8 * p + k, so a check lane
//                               reads all of its row's decisions with one 8-byte load
//   weighted rule only: c->v messages float [slots][S] (the message array then holds
//                               the v->c messages only)
//   syndrome words, output staging words, per-shot priors.
// A variable lane keeps one word per edge: the message's byte address in the low
// half and its decision byte's address in the high half (LDS addresses fit 16 bits).
// Junk positions are unused by representation l; position Mmax (of the part) is the
// sink of absent edges.
// PAIRS (the paired kernel): messages in slot pairs, edge (p, k) at word
// (k >> 1) * 2S + 2p + (k & 1), so a check lane moves two slots of its row with one
// 8-byte access; with S = 1 (mod 16) its bank is (2 (p + (k >> 1)) + (k & 1)) mod 32.
template <int MPAD, int RULE, int DC, bool COMPACT, bool PAIRS = false>
struct LayoutM {
    static constexpr bool kCompact = COMPACT;
    static constexpr int kSlots = kCompact ? DC : 8;
    static constexpr int Mpad = MPAD;
    static constexpr int S = Mpad + kSlotPad;                                   // slot stride (words)
    static constexpr uint32_t kMsg = (4u * kSlots * S + 15u) & ~15u;            // bytes of a message array
    static constexpr uint32_t kDec = (8u * Mpad + 15u) & ~15u;                  // bytes of the decisions
    static constexpr uint32_t kDecOff = kMsg;                                   // decisions after the messages
    static constexpr uint32_t kROff = RULE == kRuleWeighted ? kMsg + kDec : 0u;  // where c->v messages live
    static constexpr uint32_t kTail = kMsg + kDec + (RULE == kRuleWeighted ? kMsg : 0u);  // syndrome words
    // the two halves of a packed edge word
    __device__ __forceinline__ static uint32_t msg(uint32_t ea) { return ea & 0xffffu; }
    __device__ __forceinline__ static uint32_t dec(uint32_t ea) { return ea >> 16; }
    // packed edge word of edge id e = position * 8 + slot
    __device__ __forceinline__ static uint32_t edge_word(uint32_t ibase_addr, uint32_t e) {
        const uint32_t k = e & 7u, p = e >> 3;
        const uint32_t m =
            ibase_addr + 4u * (PAIRS ? (k >> 1) * 2u * (uint32_t)S + 2u * p + (k & 1u) : k * (uint32_t)S + p);
        const uint32_t d = ibase_addr + kDecOff + 8u * (e >> 3) + (e & 7u);
        return m | (d << 16);
    }
};
// one instance per wavefront: 64 * PC positions
template <int PC, int RULE = kRuleNMS, int DC = 8>
struct Layout : LayoutM<64 * PC, RULE, DC, (PC >= 9)> {};

// Parity of a row's hard decisions (one byte, 0 or 1, per slot; unused slots 0).
__device__ __forceinline__ uint32_t row_parity(uint64_t dw) { return (uint32_t)__popcll(dw) & 1u; }

// Exclusion sums of a variable of degree <= D with incoming messages r (unused
// slots hold 0): q_k = mu + sum_{k' != k} r_k' and P = mu + sum r, both
// accumulated in ascending check order (never P - r_k).
template <int D>
__device__ __forceinline__ float excl_sums(const float (&r)[D], float mu, float (&q)[D]) {
    float pre = mu;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        float acc = pre;
#pragma unroll
        for (int k2 = k + 1; k2 < D; ++k2) acc += r[k2];
        q[k] = acc;
        pre += r[k];
    }
    return pre;
}

// Variable rule (eq. (2) and the posterior of Section II-B) for a variable of
// degree deg <= D (edges k >= deg point at the sink and read as 0): reads the c->v
// messages at msg(ea) + ROFF, writes every q_k at msg(ea) and the hard decision at
// dec(ea).  prev is the decision already stored in the cells: only lanes whose
// decision changed store it (the fewer lanes a byte store carries, the fewer of them
// share an LDS bank), and the stores are skipped when no lane changed.
// ZSINK: absent edges point at a word that holds +0 whenever this rule reads it (the
// caller zeroes it between the store here and the next read), so no degree test.
template <int D, typename LY, bool ZSINK = false>
__device__ __forceinline__ void var_rule(const uint32_t *ea, int deg, float mu, bool prev, float &P, bool &dec) {
    constexpr uint32_t ROFF = LY::kROff;
    float r[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const float x = *lds_ptr_f32(LY::msg(ea[k]) + ROFF);
        r[k] = (ZSINK || k < deg) ? x : 0.0f;
    }
    float q[D];
    const float pre = excl_sums<D>(r, mu, q);
    dec = pre < 0.0f;
    P = pre;
#pragma unroll
    for (int k = 0; k < D; ++k) *lds_ptr_f32(LY::msg(ea[k])) = q[k];
    if (dec != prev) {
#pragma unroll
        for (int k = 0; k < D; ++k) *lds_ptr_u8(LY::dec(ea[k])) = (unsigned char)dec;
    }
}

// The message part of the variable rule for a degree <= D whose absent edges read +0
// (the ZSINK form above): loads, exclusion sums and the stores of every q_k; returns
// the posterior.  The caller stores the hard decision, so that the code of one degree
// holds no lane-dependent branch.
template <int D, typename LY>
__device__ __forceinline__ float var_msgs(const uint32_t *ea, float mu) {
    constexpr uint32_t ROFF = LY::kROff;
    float r[D];
#pragma unroll
    for (int k = 0; k < D; ++k) r[k] = *lds_ptr_f32(LY::msg(ea[k]) + ROFF);
    float q[D];
    const float pre = excl_sums<D>(r, mu, q);
#pragma unroll
    for (int k = 0; k < D; ++k) *lds_ptr_f32(LY::msg(ea[k])) = q[k];
    return pre;
}

// Variable rule at iteration 0 of the flooding schedule, where every c->v message is
// 0: q_k = P = mu (stored as-is; mu is canonical, never -0), and every decision cell
// is written, so nothing left from an earlier shot is read later.
template <int D, typename LY>
__device__ __forceinline__ void var_first(const uint32_t *ea, float mu, float &P, bool &dec) {
    dec = mu < 0.0f;
    P = mu;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        *lds_ptr_f32(LY::msg(ea[k])) = mu;
        *lds_ptr_u8(LY::dec(ea[k])) = (unsigned char)dec;
    }
}

// Posterior only (serial schedule): P = mu + sum r in ascending check order and the
// hard decision written to every edge's decision cell; messages are left alone.
template <int D, typename LY>
__device__ __forceinline__ void var_post(const uint32_t *ea, int deg, float mu, float &P, bool &dec) {
    float pre = mu;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const float x = *lds_ptr_f32(LY::msg(ea[k]));
        pre += k < deg ? x : 0.0f;
    }
    dec = pre < 0.0f;
    P = pre;
#pragma unroll
    for (int k = 0; k < D; ++k) *lds_ptr_u8(LY::dec(ea[k])) = (unsigned char)dec;
}

}  // namespace mbbp
