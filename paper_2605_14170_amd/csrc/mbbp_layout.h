// Bank-aware LDS layout of one representation (host preprocessing, internal).
//
// In the variable phase of the BP kernel lane i of a pass loads, at instruction k,
// the message of the k-th check of its variable: word k' * S + p, where p is the LDS
// position of that check and k' its slot in the row.  With S = 1 (mod 64) that word
// lies in bank (k' + p) mod B.  Lanes of one access that hit the same bank at
// different words are served one after another; the LDS serves a wave in two
// half-waves of 32 lanes over 32 banks.  This annealer chooses the check positions
// and the variable-to-lane assignment so that, for every half-wave and k, the lanes
// spread over the banks: cost = sum over (group of G consecutive variable slots, k)
// of the largest multiplicity over B banks.  One instance per wavefront: a half-wave
// is 32 slots, G = B = 32.  Two interleaved instances per wavefront: a half-wave
// holds 16 slots of each instance and the two copies of a row lie 16 banks apart,
// so G = B = 16.  It only permutes storage: which check or variable a lane handles
// never changes any value.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace mbbp {
namespace layout {

struct Rng {  // splitmix64
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed) {}
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double unit() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
    uint32_t below(uint32_t n) { return (uint32_t)(next() % n); }
};

struct Result {
    std::vector<int32_t> pos;       // check -> position in [0, npos)
    std::vector<int32_t> slot_var;  // lane slot -> variable (the first n slots are used)
    long cost_before = 0, cost_after = 0, ideal = 0;
};

// rows[j]: variables of check j (in row-slot order).  Variables start sorted by
// degree (descending, stable); moves keep every pass's degree profile: two
// variables swap lanes when they are in the same pass or have the same degree.
// pairs: messages stored in slot pairs (edge (p, k) at word (k >> 1) * 2S + 2p + (k & 1),
// S = 1 mod 16), so the bank is 2 (p + (k >> 1)) + (k & 1) instead of k + p.
inline void optimize(const std::vector<std::vector<int>> &rows, int n, int npos, uint64_t seed, long iters,
                     Result &out, int G = 32, int B = 32, bool pairs = false) {
    const int M = (int)rows.size();
    const int NG = (n + G - 1) / G;  // slot groups
    std::vector<std::vector<std::pair<int, int>>> ve(n);  // (check, row slot), ascending check
    for (int j = 0; j < M; ++j)
        for (int k = 0; k < (int)rows[j].size(); ++k) ve[rows[j][k]].push_back({j, k});
    std::vector<int> deg(n);
    for (int i = 0; i < n; ++i) deg[i] = (int)ve[i].size();
    std::vector<int32_t> sv(n), slot_of(n);
    for (int i = 0; i < n; ++i) sv[i] = i;
    std::stable_sort(sv.begin(), sv.end(), [&](int a, int b) { return deg[a] > deg[b]; });
    for (int s = 0; s < n; ++s) slot_of[sv[s]] = s;
    std::vector<int32_t> pos(M), at(npos, -1);
    for (int j = 0; j < M; ++j) { pos[j] = j; at[j] = j; }
    const int K = 8;
    std::vector<uint8_t> cnt((size_t)NG * K * B, 0);
    auto add_var = [&](int i, int d) {
        const int s = slot_of[i];
        for (int k = 0; k < deg[i]; ++k) {
            const int t = ve[i][k].second, p = pos[ve[i][k].first];
            const int b = (pairs ? 2 * (p + (t >> 1)) + (t & 1) : t + p) % B;
            cnt[((size_t)(s / G) * K + k) * B + b] += (uint8_t)d;
        }
    };
    auto keycost = [&](int key) {
        const uint8_t *c = &cnt[(size_t)key * B];
        int m = 0;
        for (int b = 0; b < B; ++b) m = std::max(m, (int)c[b]);
        return m;
    };
    for (int i = 0; i < n; ++i) add_var(i, 1);
    long cost = 0, ideal = 0;
    for (int g = 0; g < NG * K; ++g) { const int m = keycost(g); cost += m; ideal += m > 0; }
    out.cost_before = cost;
    out.ideal = ideal;
    Rng rng(seed);
    std::vector<int> vars, keys;
    for (long it = 0; it < iters && M > 0 && npos > 1; ++it) {
        const double T = 0.6 * (1.0 - (double)it / (double)iters) + 0.02;
        vars.clear();
        keys.clear();
        const bool rowmove = (rng.next() & 1u) == 0;
        int j1 = -1, j2 = -1, p1 = -1, p2 = -1, s1 = -1, s2 = -1;
        if (rowmove) {
            j1 = (int)rng.below((uint32_t)M);
            p1 = pos[j1];
            p2 = (int)rng.below((uint32_t)npos);
            if (p2 == p1) continue;
            j2 = at[p2];
            for (int v : rows[j1]) vars.push_back(v);
            if (j2 >= 0)
                for (int v : rows[j2]) vars.push_back(v);
        } else {
            s1 = (int)rng.below((uint32_t)n);
            s2 = (int)rng.below((uint32_t)n);
            if (s1 == s2) continue;
            if (s1 / (2 * G) != s2 / (2 * G) && deg[sv[s1]] != deg[sv[s2]]) continue;  // keep pass profiles
            vars.push_back(sv[s1]);
            vars.push_back(sv[s2]);
        }
        std::sort(vars.begin(), vars.end());
        vars.erase(std::unique(vars.begin(), vars.end()), vars.end());
        auto collect = [&]() {
            for (int v : vars) {
                const int s = slot_of[v];
                for (int k = 0; k < deg[v]; ++k) keys.push_back((s / G) * K + k);
            }
        };
        auto apply = [&](bool fwd) {
            for (int v : vars) add_var(v, -1);
            if (rowmove) {
                const int pa = fwd ? p2 : p1, pb = fwd ? p1 : p2;
                pos[j1] = pa;
                at[pa] = j1;
                at[pb] = j2;
                if (j2 >= 0) pos[j2] = pb;
            } else {
                std::swap(sv[s1], sv[s2]);
                slot_of[sv[s1]] = s1;
                slot_of[sv[s2]] = s2;
            }
            for (int v : vars) add_var(v, 1);
        };
        collect();
        apply(true);
        collect();
        std::sort(keys.begin(), keys.end());
        keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
        long nw = 0;
        for (int key : keys) nw += keycost(key);
        apply(false);
        long old = 0;
        for (int key : keys) old += keycost(key);
        const long delta = nw - old;
        if (delta <= 0 || rng.unit() < std::exp(-(double)delta / T)) {
            apply(true);
            cost += delta;
        }
    }
    out.cost_after = cost;
    out.pos = pos;
    out.slot_var = sv;
}

}  // namespace layout
}  // namespace mbbp
