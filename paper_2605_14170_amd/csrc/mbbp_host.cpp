// Host side of the MBBP-LD library: argument validation, GF(2) algebra, maximal
// subtrees (Algorithm 2), representation assembly, packing of the per-representation
// tables consumed by the kernels, device memory, and the C ABI of include/mbbp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mbbp.h"
#include "mbbp_layout.h"
#include "mbbp_device.h"

namespace {

thread_local std::string g_last_error;

// Scratch of the allocation-free entry point mbbp_run_static: every buffer of the
// whole path (noise, syndromes, candidates, decisions, counters, work queue) is
// carved from this array, which each GPU holds from module load to process end.
// Host code never passes its name to a kernel: it is a host-side stand-in, and
// the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

mbbp_status fail(mbbp_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

#define MBBP_HIP(call)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(MBBP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

using Row = std::vector<int32_t>;  // sorted column indices

// ----------------------------------------------------------------------------- GF(2)

struct BitMat {
    int cols = 0, words = 0;
    std::vector<uint64_t> data;  // rows x words
    int rows() const { return words ? (int)(data.size() / words) : 0; }
    uint64_t *row(int r) { return data.data() + (size_t)r * words; }
    const uint64_t *row(int r) const { return data.data() + (size_t)r * words; }
};

inline bool bit(const uint64_t *v, int i) { return (v[i >> 6] >> (i & 63)) & 1u; }

// Reduced row-echelon basis of a row space, with, for each reduced row, the set of
// original rows it is the sum of (so membership also yields the combination).
struct RowSpace {
    int n = 0, m = 0, wn = 0, wm = 0;
    std::vector<std::vector<uint64_t>> red, comb;
    std::vector<int> pivot;

    void build(const std::vector<Row> &rows, int ncols) {
        n = ncols;
        m = (int)rows.size();
        wn = (n + 63) / 64;
        wm = std::max(1, (m + 63) / 64);
        red.clear(); comb.clear(); pivot.clear();
        for (int j = 0; j < m; ++j) {
            std::vector<uint64_t> v(wn, 0), c(wm, 0);
            for (int col : rows[j]) v[col >> 6] ^= 1ull << (col & 63);
            c[j >> 6] |= 1ull << (j & 63);
            insert(v, c);
        }
    }
    // Reduce v (and its combination c) by the basis; returns true iff v becomes 0.
    bool reduce(std::vector<uint64_t> &v, std::vector<uint64_t> *c) const {
        for (size_t r = 0; r < red.size(); ++r) {
            if (bit(v.data(), pivot[r])) {
                for (int w = 0; w < wn; ++w) v[w] ^= red[r][w];
                if (c)
                    for (int w = 0; w < wm; ++w) (*c)[w] ^= comb[r][w];
            }
        }
        for (uint64_t x : v)
            if (x) return false;
        return true;
    }
    // Insert a vector (no-op if dependent).  Keeps every stored row reduced
    // against the pivots of the others.
    bool insert(std::vector<uint64_t> v, std::vector<uint64_t> c) {
        if (reduce(v, &c)) return false;
        int p = -1;
        for (int w = 0; w < wn && p < 0; ++w)
            if (v[w]) p = w * 64 + __builtin_ctzll(v[w]);
        for (size_t r = 0; r < red.size(); ++r) {
            if (bit(red[r].data(), p)) {
                for (int w = 0; w < wn; ++w) red[r][w] ^= v[w];
                for (int w = 0; w < wm; ++w) comb[r][w] ^= c[w];
            }
        }
        red.push_back(std::move(v));
        comb.push_back(std::move(c));
        pivot.push_back(p);
        return true;
    }
    int rank() const { return (int)red.size(); }
};

// Basis of the kernel {x : A x = 0} of A (rows as column lists), as bit vectors.
std::vector<std::vector<uint64_t>> kernel_basis(const std::vector<Row> &A, int n) {
    RowSpace rs;
    rs.build(A, n);
    const int wn = (n + 63) / 64;
    std::vector<char> is_pivot(n, 0);
    for (int p : rs.pivot) is_pivot[p] = 1;
    std::vector<std::vector<uint64_t>> out;
    for (int f = 0; f < n; ++f) {
        if (is_pivot[f]) continue;
        // x_f = 1, other free = 0; pivot variables from the reduced rows
        std::vector<uint64_t> x(wn, 0);
        x[f >> 6] |= 1ull << (f & 63);
        for (size_t r = 0; r < rs.red.size(); ++r)
            if (bit(rs.red[r].data(), f)) x[rs.pivot[r] >> 6] |= 1ull << (rs.pivot[r] & 63);
        out.push_back(std::move(x));
    }
    return out;
}

// Logical operators: a basis of ker(A) modulo the row space of B (A B^T = 0).
std::vector<std::vector<uint64_t>> logicals(const std::vector<Row> &A, const std::vector<Row> &B, int n) {
    RowSpace rs;
    rs.build(B, n);
    std::vector<std::vector<uint64_t>> out;
    const int wm = rs.wm;
    for (auto &v : kernel_basis(A, n)) {
        std::vector<uint64_t> c(wm, 0);
        std::vector<uint64_t> t = v;
        if (!rs.reduce(t, nullptr)) {
            out.push_back(v);
            rs.insert(v, c);
        }
    }
    return out;
}

// ----------------------------------------------------------------------------- validation

mbbp_status read_sparse(const mbbp_sparse *H, const char *name, std::vector<Row> &rows) {
    if (!H || !H->row_ptr || (!H->col_idx && H->rows > 0 && H->row_ptr[H->rows] > 0))
        return fail(MBBP_EINVAL, std::string(name) + ": null matrix pointer");
    if (H->rows <= 0 || H->cols <= 0) return fail(MBBP_EINVAL, std::string(name) + ": empty matrix");
    if (H->row_ptr[0] != 0) return fail(MBBP_EINVAL, std::string(name) + ": row_ptr[0] != 0");
    rows.assign(H->rows, Row());
    for (int r = 0; r < H->rows; ++r) {
        const int a = H->row_ptr[r], b = H->row_ptr[r + 1];
        if (b < a) return fail(MBBP_EINVAL, std::string(name) + ": row_ptr not non-decreasing");
        for (int k = a; k < b; ++k) {
            const int c = H->col_idx[k];
            if (c < 0 || c >= H->cols) return fail(MBBP_EINVAL, std::string(name) + ": column out of range");
            if (k > a && c <= H->col_idx[k - 1])
                return fail(MBBP_EINVAL, std::string(name) + ": columns not strictly ascending");
            rows[r].push_back(c);
        }
    }
    return MBBP_OK;
}

// ----------------------------------------------------------------------------- Algorithm 2

// Maximal cycle-free subtrees.  Roots in the order of perm; a subtree grows
// breadth-first (FIFO, neighbours in ascending index): a dequeued check with at
// most one already-visited variable joins the current subtree, marks its variables
// visited and queues their untested unassigned checks.  Variables and test marks
// are reset for every root.
mbbp_status subtrees(const std::vector<Row> &H, int n, const int32_t *perm, std::vector<int32_t> &cs,
                     std::vector<int32_t> &order, int &nsub) {
    const int m = (int)H.size();
    std::vector<std::vector<int32_t>> vchk(n);
    for (int j = 0; j < m; ++j)
        for (int v : H[j]) vchk[v].push_back(j);
    std::vector<char> seen(m, 0);
    for (int i = 0; i < m; ++i) {
        if (perm[i] < 0 || perm[i] >= m || seen[perm[i]])
            return fail(MBBP_EINVAL, "perm is not a permutation of the checks");
        seen[perm[i]] = 1;
    }
    cs.assign(m, 0);
    order.clear();
    nsub = 0;
    std::vector<char> visited(n), tested(m);
    std::vector<int32_t> queue;
    for (int i = 0; i < m; ++i) {
        const int root = perm[i];
        if (cs[root]) continue;
        ++nsub;
        std::fill(visited.begin(), visited.end(), 0);
        std::fill(tested.begin(), tested.end(), 0);
        queue.assign(1, root);
        for (size_t head = 0; head < queue.size(); ++head) {
            const int u = queue[head];
            tested[u] = 1;
            int eta = 0;
            for (int v : H[u]) eta += visited[v];
            if (eta > 1 || cs[u]) continue;
            cs[u] = nsub;
            order.push_back(u);
            for (int v : H[u]) {
                visited[v] = 1;
                for (int c : vchk[v])
                    if (!tested[c] && !cs[c]) queue.push_back(c);
            }
        }
    }
    return MBBP_OK;
}

// ----------------------------------------------------------------------------- parts

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

struct HostPart {
    int m = 0, n = 0, L = 0, Mmax = 0, uniform_dc = 0;
    std::vector<Row> H;
    std::vector<int32_t> M, E;
    std::vector<uint16_t> voff, vid;
    std::vector<uint8_t> vdeg, cw;
    std::vector<int32_t> csrc, comb_ptr{0}, comb_idx;
    std::vector<uint64_t> logical;
    int k = 0;
    // serial schedule: conflict-free levels of every representation and, per
    // check slot, the variable and its other edges (ascending check order)
    std::vector<int32_t> lev_off{0}, lev_ptr;
    std::vector<uint16_t> lev_chk, ltab;
    // serial schedule, one lane per shot: per-row records, row-order syndrome
    // sources, the rows of H
    std::vector<uint32_t> stab;
    std::vector<int32_t> stab_off{0}, scsrc;
    std::vector<uint16_t> htab;
    int dcs = 8, emax = 0, maug = 0, serial_ok = 1;
    // serial schedule, eight lanes per shot: per-row slot records, and the halting
    // test's entries of the rows of H
    std::vector<uint32_t> srec, sht;
};

// pair_hint: launches will run two instances per wavefront where the code fits the
// paired kernel (its bank-aware layout then targets interleaved lanes).
mbbp_status build_part(const std::vector<Row> &H, int n, const mbbp_basis_list &bl, const char *name,
                       HostPart &P, bool pair_hint) {
    const int m = (int)H.size();
    P.m = m; P.n = n; P.H = H;
    if (bl.L < 1) return fail(MBBP_EINVAL, std::string(name) + ": L < 1");
    if (bl.L > mbbp::kMaxL) return fail(MBBP_EUNSUPPORTED, std::string(name) + ": L > 64");
    if (!bl.basis_ptr) return fail(MBBP_EINVAL, std::string(name) + ": null basis_ptr");
    if (bl.basis_ptr[0] != 0) return fail(MBBP_EINVAL, std::string(name) + ": basis_ptr[0] != 0");
    for (int l = 0; l < bl.L; ++l)
        if (bl.basis_ptr[l + 1] < bl.basis_ptr[l])
            return fail(MBBP_EINVAL, std::string(name) + ": basis_ptr decreasing");
    if (bl.basis_ptr[bl.L] > 0 && !bl.rows) return fail(MBBP_EINVAL, std::string(name) + ": null rows");
    std::vector<Row> extra;
    if (bl.extra) {
        mbbp_status st = read_sparse(bl.extra, name, extra);
        if (st != MBBP_OK) return st;
        if (bl.extra->cols != n) return fail(MBBP_EINVAL, std::string(name) + ": extra rows have wrong width");
    }
    for (int j = 0; j < m; ++j) {
        if ((int)H[j].size() < 2) return fail(MBBP_EINVAL, std::string(name) + ": row weight < 2");
    }
    RowSpace rs;
    bool rs_built = false;
    P.L = bl.L;
    P.M.resize(bl.L);
    P.E.resize(bl.L);
    std::vector<std::vector<Row>> reps(bl.L);
    std::vector<std::vector<int32_t>> srcs(bl.L);
    for (int l = 0; l < bl.L; ++l) {
        reps[l] = H;
        srcs[l].resize(m);
        for (int j = 0; j < m; ++j) srcs[l][j] = j;
        for (int t = bl.basis_ptr[l]; t < bl.basis_ptr[l + 1]; ++t) {
            const int r = bl.rows[t];
            if (r >= 0) {
                if (r >= m) return fail(MBBP_EINVAL, std::string(name) + ": basis row out of range");
                reps[l].push_back(H[r]);
                srcs[l].push_back(r);
            } else {
                const int e = -r - 1;
                if (e >= (int)extra.size()) return fail(MBBP_EINVAL, std::string(name) + ": extra row out of range");
                if ((int)extra[e].size() < 2) return fail(MBBP_EINVAL, std::string(name) + ": row weight < 2");
                if (!rs_built) { rs.build(H, n); rs_built = true; }
                std::vector<uint64_t> v(rs.wn, 0), c(rs.wm, 0);
                for (int col : extra[e]) v[col >> 6] ^= 1ull << (col & 63);
                if (!rs.reduce(v, &c))
                    return fail(MBBP_ENOTINROWSPACE, std::string(name) + ": appended row not in the row space of H");
                const int cix = (int)P.comb_ptr.size() - 1;
                for (int j = 0; j < m; ++j)
                    if (bit(c.data(), j)) P.comb_idx.push_back(j);
                P.comb_ptr.push_back((int32_t)P.comb_idx.size());
                reps[l].push_back(extra[e]);
                srcs[l].push_back(-(cix + 1));
            }
        }
        P.M[l] = (int)reps[l].size();
        P.Mmax = std::max(P.Mmax, P.M[l]);
    }
    // LDS row positions: the largest representation plus the sink, rounded up to a
    // multiple of 32 (half a 64-lane pass, so two instances fill whole passes in the
    // paired kernel); position Mmax is the sink, the others are free for the layout
    P.Mmax = 32 * ((P.Mmax + 1 + 31) / 32) - 1;
    if ((int64_t)(P.Mmax + 1) * 8 > 65535)
        return fail(MBBP_EUNSUPPORTED, std::string(name) + ": too many checks in a representation");
    bool all6 = true;
    for (int l = 0; l < bl.L; ++l)
        for (auto &r : reps[l]) {
            if ((int)r.size() > mbbp::kMaxRowWeight)
                return fail(MBBP_EUNSUPPORTED, std::string(name) + ": row weight > 8");
            all6 = all6 && r.size() == 6;
        }
    P.uniform_dc = all6 ? 6 : 0;
    const int L = bl.L, Mmax = P.Mmax;
    const uint16_t sink = (uint16_t)(Mmax * 8);
    const bool paired = pair_hint && mbbp::bp_dual_fits(n, Mmax);
    const int lay_group = paired ? 16 : 32;  // variable slots per half-wave of one instance
    // both flooding kernels keep messages in slot pairs, so the bank model is the
    // slot-pair one either way (the serial and weighted forms, on plain slots, only
    // see a layout tuned for the other addressing)
    P.voff.assign((size_t)L * n * 8, sink);
    P.vid.assign((size_t)L * n, 0);
    P.vdeg.assign((size_t)L * n, 0);
    P.cw.assign((size_t)L * Mmax, 8);
    P.csrc.assign((size_t)L * Mmax, mbbp::kJunkRow);
    // annealing budget of the bank-aware layout, per representation
    const long iters = std::min<long>(30L * (n + P.Mmax), 400000L / std::max(1, L));
    for (int l = 0; l < L; ++l) {
        const int Ml = P.M[l];
        for (int j = 0; j < Ml; ++j)
            if ((int)reps[l][j].size() > mbbp::kMaxRowWeight)
                return fail(MBBP_EUNSUPPORTED, std::string(name) + ": row weight > 8");
        {
            std::vector<int> degc(n, 0);
            for (int j = 0; j < Ml; ++j)
                for (int v : reps[l][j]) degc[v]++;
            for (int i = 0; i < n; ++i)
                if (degc[i] > mbbp::kMaxVarDegree)
                    return fail(MBBP_EUNSUPPORTED, std::string(name) + ": column weight > 8");
        }
        // positions of the checks and lanes of the variables (storage only)
        mbbp::layout::Result lay;
        {
            std::vector<std::vector<int>> rows(Ml);
            for (int j = 0; j < Ml; ++j) rows[j].assign(reps[l][j].begin(), reps[l][j].end());
            // a representation's checks take the positions [0, Ml rounded up to a 64-lane
            // check pass), so the flooding kernels skip the passes it leaves empty
            const int npos = std::min(Mmax, (Ml + 63) / 64 * 64);
            mbbp::layout::optimize(rows, n, npos, 0x5eed0000ull + (uint64_t)l * 7919u + (uint64_t)Mmax, iters,
                                   lay, lay_group, lay_group, true);
        }
        const std::vector<int32_t> &pos = lay.pos;
        // edges of every variable in ascending check order, as LDS edge ids pos * 8 + slot
        std::vector<std::vector<uint16_t>> vedges(n);
        int E = 0;
        for (int j = 0; j < Ml; ++j) {
            const Row &r = reps[l][j];
            P.cw[(size_t)l * Mmax + pos[j]] = (uint8_t)r.size();
            P.csrc[(size_t)l * Mmax + pos[j]] = srcs[l][j];
            for (size_t k = 0; k < r.size(); ++k) vedges[r[k]].push_back((uint16_t)(pos[j] * 8 + k));
            E += (int)r.size();
        }
        P.E[l] = E;
        for (int s = 0; s < n; ++s) {
            const int i = lay.slot_var[s];
            P.vid[(size_t)l * n + s] = (uint16_t)i;
            P.vdeg[(size_t)l * n + s] = (uint8_t)vedges[i].size();
            for (int k = 0; k < (int)vedges[i].size(); ++k)  // absent edges point at the sink
                P.voff[((size_t)l * n + s) * 8 + k] = vedges[i][k];
        }
        // Serial schedule (Section II-B): checks are visited in row order, each seeing
        // the latest check messages.  Level of check j = 1 + the highest level of an
        // earlier check sharing a variable with it; checks of one level share no
        // variable, so running levels in order equals the row-order sweep exactly.
        std::vector<int> lastlev(n, -1), level(Ml, 0);
        int nlev = 0;
        for (int j = 0; j < Ml; ++j) {
            int lv = 0;
            for (int v : reps[l][j]) lv = std::max(lv, lastlev[v] + 1);
            level[j] = lv;
            for (int v : reps[l][j]) lastlev[v] = std::max(lastlev[v], lv);
            nlev = std::max(nlev, lv + 1);
        }
        std::vector<int> cnt(nlev + 1, 0);
        for (int j = 0; j < Ml; ++j) cnt[level[j] + 1]++;
        for (int t = 0; t < nlev; ++t) cnt[t + 1] += cnt[t];
        for (int t = 0; t <= nlev; ++t) P.lev_ptr.push_back(cnt[t]);
        P.lev_off.push_back((int32_t)P.lev_ptr.size());
        std::vector<uint16_t> order(Mmax, 0);
        {
            std::vector<int> fill(cnt.begin(), cnt.end() - 1);
            for (int j = 0; j < Ml; ++j) order[fill[level[j]]++] = (uint16_t)pos[j];
        }
        P.lev_chk.insert(P.lev_chk.end(), order.begin(), order.end());
        // per check slot (position p, k): word 0 = variable id | degree << 12, words
        // 1..7 = the variable's other edges in ascending check order (sink beyond its
        // degree)
        std::vector<uint16_t> tab((size_t)Mmax * 8 * 8, sink);
        for (int p = 0; p < Mmax; ++p)
            for (int k = 0; k < 8; ++k) tab[((size_t)p * 8 + k) * 8] = 0;
        for (int j = 0; j < Ml; ++j) {
            const Row &r = reps[l][j];
            for (size_t k = 0; k < r.size(); ++k) {
                const int v = r[k];
                const uint16_t self = (uint16_t)(pos[j] * 8 + k);
                uint16_t *e = &tab[(size_t)self * 8];
                e[0] = (uint16_t)(v | ((int)vedges[v].size() << 12));
                int t = 1;
                for (uint16_t other : vedges[v])
                    if (other != self) e[t++] = other;
            }
        }
        P.ltab.insert(P.ltab.end(), tab.begin(), tab.end());
        // records of the one-lane-per-shot serial kernel, rows in order 0..Ml-1; edges
        // numbered variable by variable, a variable's edges in ascending row order
        {
            const int dcs = P.uniform_dc == 6 ? 6 : 8;
            P.dcs = dcs;
            std::vector<std::vector<int>> vck(n);  // rows of each variable, ascending
            for (int j = 0; j < Ml; ++j)
                for (int v : reps[l][j]) vck[v].push_back(j);
            std::vector<int> vstart(n + 1, 0);
            for (int v = 0; v < n; ++v) vstart[v + 1] = vstart[v] + (int)vck[v].size();
            if (vstart[n] > 65535) P.serial_ok = 0;
            P.emax = std::max(P.emax, vstart[n]);
            P.maug = std::max(P.maug, Ml);
            // eight-lanes-per-shot records: per row 8 slots of 2 words, byte offsets
            // within a shot's LDS block (8 junk words, then the messages):
            //   A = 32 + 4 first | (32 + 4 (first + t)) << 16
            //   B = 4 v | rdm << 12 | (t = deg - 1) << 15 | 4 (v >> 5) << 16 |
            //       (v & 31) << 24 | (deg - 1) << 29
            // rdm: the largest deg - 1 in the row.  An absent slot reads and writes the
            // junk words (A = 4 << 16) and reads the prior of v = n (a 0 kept there): its
            // sum is 0 + junk word 0 (+FLT_MAX).
            if (32 + 4 * (vstart[n] + 8) > 65535) P.serial_ok = 0;
            for (int j = 0; j < Ml; ++j) {
                uint32_t rdm = 0;
                for (int v : reps[l][j]) rdm = std::max(rdm, (uint32_t)vck[v].size() - 1u);
                for (int k = 0; k < 8; ++k) {
                    uint32_t A = 4u << 16, B = (uint32_t)(4 * n) | (rdm << 12);
                    if (k < (int)reps[l][j].size()) {
                        const int v = reps[l][j][k];
                        const int deg = (int)vck[v].size();
                        const int t = (int)(std::find(vck[v].begin(), vck[v].end(), j) - vck[v].begin());
                        A = (uint32_t)(32 + 4 * vstart[v]) | ((uint32_t)(32 + 4 * (vstart[v] + t)) << 16);
                        B = (uint32_t)(4 * v) | (rdm << 12) | ((uint32_t)(t == deg - 1) << 15) |
                            ((uint32_t)(4 * (v >> 5)) << 16) | ((uint32_t)(v & 31) << 24) |
                            ((uint32_t)(deg - 1) << 29);
                    }
                    P.srec.push_back(A);
                    P.srec.push_back(B);
                }
            }
            for (int j = 0; j < Ml; ++j) {
                P.scsrc.push_back(srcs[l][j]);
                for (int k = 0; k < dcs; ++k) {
                    uint32_t w = 0xffffffffu;  // absent slot
                    if (k < (int)reps[l][j].size()) {
                        const int v = reps[l][j][k];
                        const int deg = (int)vck[v].size();
                        const int t = (int)(std::find(vck[v].begin(), vck[v].end(), j) - vck[v].begin());
                        w = (uint32_t)v | ((uint32_t)t << 10) | ((uint32_t)(deg - 1) << 13) |
                            ((uint32_t)vstart[v] << 16);
                    }
                    P.stab.push_back(w);
                }
            }
            P.stab_off.push_back(P.stab_off.back() + Ml);
        }
    }
    // padding: a row's record is read as 8 words, and the kernel with eight lanes per
    // shot loads the records of two rows ahead
    P.stab.insert(P.stab.end(), 16, 0xffffffffu);
    // padding: the eight-lanes-per-shot kernel loads slot records two rows ahead
    P.srec.insert(P.srec.end(), 2 * 16, 0u);
    P.htab.assign((size_t)m * 8, 0xffff);
    for (int j = 0; j < m; ++j)
        for (size_t k = 0; k < H[j].size() && k < 8; ++k) P.htab[(size_t)j * 8 + k] = (uint16_t)H[j][k];
    // halting-test entries of the eight-lanes-per-shot kernel: per row of H 8 words
    // (v & 31) | 4 (v >> 5) << 8 (bit and byte offset of v's decision word); padding
    // takes v = n, whose bit is never set
    P.sht.assign((size_t)m * 8, 0u);
    for (int j = 0; j < m; ++j)
        for (int k = 0; k < 8; ++k) {
            const int v = k < (int)H[j].size() ? H[j][k] : n;
            P.sht[(size_t)j * 8 + k] = (uint32_t)(v & 31) | ((uint32_t)(4 * (v >> 5)) << 8);
        }
    return MBBP_OK;
}

template <typename T>
mbbp_status upload(DevBuf &b, const std::vector<T> &v) {
    const size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
    MBBP_HIP(hipMalloc(&b.p, bytes));
    if (!v.empty()) MBBP_HIP(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return MBBP_OK;
}

}  // namespace

// ----------------------------------------------------------------------------- context

// Buffers of the whole path of mbbp_run: allocated per context on first use, or
// carved from the static scratch array by mbbp_run_static.
struct RunWs {
    uint64_t *err[2], *syn[2], *corr[2], *conv[2];
    int16_t *basis[2];
    float *prior[2];
    int *kmax;
    int64_t *counters;
    mbbp::RunDesc *desc;
    unsigned long long *queue;
    uint64_t *cand[2];
    uint16_t *kstat[2];
};

// A captured mbbp_run: its BP kernel node was launched with `cfg`; the two event
// record nodes around it take fresh events at every timed replay.
struct RunGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t prep = nullptr;
    hipKernelNodeParams prep_params{};
    hipGraphNode_t ev_node[2] = {nullptr, nullptr};
    const void *bp_func = nullptr;
    mbbp::BPConfig cfg{};
};

struct mbbp_ctx {
    int device = 0;
    int n = 0, T = 0, schedule = 0;
    int noise = MBBP_NOISE_DEPOLARIZING;  // noise model of mbbp_sample / mbbp_run / mbbp_autotune
    mbbp_params params{};
    HostPart hp[2];  // [0] = part X (H_Z), [1] = part Z (H_X)
    std::vector<Row> HX, HZ;
    std::vector<std::vector<uint64_t>> LX, LZ;
    std::vector<std::unique_ptr<DevBuf>> bufs;
    mbbp::DevPart dp[2]{};
    const mbbp::DevPart *dparts = nullptr;  // dp[] copied to device memory
    // workspace
    uint64_t *cand[2]{};
    uint16_t *kstat[2]{};
    uint64_t *w_err[2]{}, *w_syn[2]{}, *w_corr[2]{}, *w_conv[2]{};
    int16_t *w_basis[2]{};
    float *w_prior[2]{};
    int *w_kmax = nullptr;
    int64_t *w_counters = nullptr;
    mbbp::RunDesc *w_desc = nullptr;
    unsigned long long *w_queue = nullptr;
    int32_t *item_order = nullptr;
    // weighted rule: user weights for decoding ([T][L] device floats, not owned)
    const float *walpha = nullptr, *wbeta = nullptr;
    // adjoint of the weighted decoder: per-instance gradient partials (grown on demand)
    std::unique_ptr<DevBuf> gpart;
    size_t gpart_bytes = 0;
    int cu_count = 256;
    int lds_block = 65536;  // largest LDS of one workgroup on this device
    mbbp::BPConfig plain_cfg{16, 4, 0, 0};
    mbbp::BPConfig batched_cfg{16, 4, 8, 0};
    hipStream_t capture_stream = nullptr;
    std::map<int64_t, RunGraph> graphs;
    bool use_graph = true;  // mbbp_run replays a captured graph
    hipEvent_t graph_ev[2] = {nullptr, nullptr};  // events of the captured record nodes (untimed replays)
    bool per_basis = false;  // mbbp_decode: one BP launch per (part, representation)
    int serial_lanes = 0;    // serial schedule: shots per wavefront (0 = chosen from the LDS size)
    int serial_kernel = 0;   // serial schedule: MBBP_SERIAL_* (0 = automatic)
    int64_t *stats = nullptr;  // device counters mbbp_decode / mbbp_decode_batched add to (or null)
    unsigned char *scratch_dev = nullptr;  // this device's copy of the static scratch array
    const int32_t *rep_ids = nullptr;  // device [2L]: p * L + l in order (single-pair launches)
    // BP kernel event timing
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    double timed_ms = 0.0;
    int64_t timed_launches = 0;

    template <typename T>
    mbbp_status alloc(T *&p, size_t count) {
        auto b = std::make_unique<DevBuf>();
        hipError_t e = hipMalloc(&b->p, std::max<size_t>(count * sizeof(T), 16));
        if (e != hipSuccess) return fail(MBBP_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        p = static_cast<T *>(b->p);
        bufs.push_back(std::move(b));
        return MBBP_OK;
    }
    template <typename T>
    mbbp_status put(const T *&p, const std::vector<T> &v) {
        auto b = std::make_unique<DevBuf>();
        mbbp_status st = upload(*b, v);
        if (st != MBBP_OK) return st;
        p = static_cast<const T *>(b->p);
        bufs.push_back(std::move(b));
        return MBBP_OK;
    }
};

namespace {

mbbp_status upload_part(mbbp_ctx *c, int pi, const std::vector<std::vector<uint64_t>> &logi) {
    HostPart &P = c->hp[pi];
    mbbp::DevPart &D = c->dp[pi];
    D.m = P.m; D.n = P.n; D.L = P.L;
    D.W = (P.n + 63) / 64;
    D.Ws = (P.m + 63) / 64;
    D.Mmax = P.Mmax;
    D.uniform_dc = P.uniform_dc;
    D.max_deg = 0;
    for (uint8_t d : P.vdeg) D.max_deg = std::max(D.max_deg, (int)d);
    mbbp_status st;
    if ((st = c->put(D.M, P.M)) != MBBP_OK) return st;
    if ((st = c->put(D.E, P.E)) != MBBP_OK) return st;
    if ((st = c->put(D.voff, P.voff)) != MBBP_OK) return st;
    if ((st = c->put(D.vid, P.vid)) != MBBP_OK) return st;
    if ((st = c->put(D.vdeg, P.vdeg)) != MBBP_OK) return st;
    if ((st = c->put(D.cw, P.cw)) != MBBP_OK) return st;
    if ((st = c->put(D.csrc, P.csrc)) != MBBP_OK) return st;
    if ((st = c->put(D.lev_off, P.lev_off)) != MBBP_OK) return st;
    if ((st = c->put(D.lev_ptr, P.lev_ptr)) != MBBP_OK) return st;
    if ((st = c->put(D.lev_chk, P.lev_chk)) != MBBP_OK) return st;
    {
        const uint16_t *lt = nullptr;
        if ((st = c->put(lt, P.ltab)) != MBBP_OK) return st;
        D.ltab = reinterpret_cast<const uint4 *>(lt);
    }
    if ((st = c->put(D.stab, P.stab)) != MBBP_OK) return st;
    if ((st = c->put(D.stab_off, P.stab_off)) != MBBP_OK) return st;
    if ((st = c->put(D.scsrc, P.scsrc)) != MBBP_OK) return st;
    if ((st = c->put(D.htab, P.htab)) != MBBP_OK) return st;
    {
        const uint32_t *sr = nullptr;
        if ((st = c->put(sr, P.srec)) != MBBP_OK) return st;
        D.srec = reinterpret_cast<const uint2 *>(sr);
    }
    if ((st = c->put(D.sht, P.sht)) != MBBP_OK) return st;
    D.dcs = P.dcs;
    D.emax = P.emax;
    D.maug = P.maug;
    D.serial_ok = P.serial_ok;
    if ((st = c->put(D.comb_ptr, P.comb_ptr)) != MBBP_OK) return st;
    std::vector<int32_t> ci = P.comb_idx;
    if ((st = c->put(D.comb_idx, ci)) != MBBP_OK) return st;
    std::vector<int32_t> hp{0}, hi;
    for (auto &r : P.H) {
        hi.insert(hi.end(), r.begin(), r.end());
        hp.push_back((int32_t)hi.size());
    }
    if ((st = c->put(D.hrow_ptr, hp)) != MBBP_OK) return st;
    if ((st = c->put(D.hrow_idx, hi)) != MBBP_OK) return st;
    std::vector<uint64_t> lg;
    for (auto &v : logi) lg.insert(lg.end(), v.begin(), v.end());
    P.logical = lg;
    P.k = (int)logi.size();
    D.k = P.k;
    if ((st = c->put(D.logical, lg)) != MBBP_OK) return st;
    return MBBP_OK;
}

// Row slots the BP kernel is instantiated with for these parts: 6 when every row of
// every representation has weight 6, else 8 (must match the kernel launcher).
int launch_dc(const mbbp_ctx *c, int part0, int nparts) {
    bool u6 = true;
    for (int p = part0; p < part0 + nparts; ++p) u6 = u6 && c->dp[p].uniform_dc == 6;
    return u6 ? 6 : 8;
}

// Slots per LDS row (must match Layout in mbbp_bp_rules.h): the compact layout of
// large codes (64 * kCompactPC positions or more) keeps the row weight, the wide one 8.
constexpr int kCompactPC = 9;
int lds_slots(const mbbp_ctx *c, int part0, int nparts, int mpad) {
    return mpad >= 64 * kCompactPC ? launch_dc(c, part0, nparts) : 8;
}

// LDS bytes of one BP instance (must match Layout in mbbp_bp_rules.h): messages
// (slots of stride Mpad + kSlotPad words, 16-byte rounded), 8 decision bytes per row, for
// the weighted rule the c->v messages, the syndrome words, the output staging words,
// 16 words for absent edges and, for per-shot priors or the serial schedule, the
// shot's n priors.
bool inst_layout(const mbbp_ctx *c, int part0, int nparts, bool per_shot_prior, int schedule, int rule,
                 mbbp::BPArgs &a) {
    int W = 0, Ws = 0, n = 0;
    for (int p = part0; p < part0 + nparts; ++p) {
        W = std::max(W, c->dp[p].W);
        Ws = std::max(Ws, c->dp[p].Ws);
        n = std::max(n, c->dp[p].n);
    }
    int mpad = 0;
    if (!mbbp::bp_layout(a, mpad)) return false;
    a.ws_max = Ws;
    a.w_max = W;
    a.n_max = n;
    const int stride = mpad + mbbp::kSlotPad;  // slot stride of the LDS arrays (words)
    const int slots = lds_slots(c, part0, nparts, mpad);
    const int msg = (4 * slots * stride + 15) & ~15, dec = (8 * mpad + 15) & ~15;  // decisions: 8 bytes per row
    a.msg_bytes = msg;
    a.zero_bytes = msg + dec;
    // serial schedule: priors always staged (n floats) plus one syndrome byte per row
    const bool serial = schedule == MBBP_LAYERED;
    // the weighted rule keeps the c->v messages in a second message array
    // + 16 words for the absent edges of the flooding passes
    const int bytes = msg + dec + (rule == MBBP_WEIGHTED ? msg : 0) + Ws * 8 + W * 8 + 64 +
                      ((per_shot_prior || serial) ? n * 4 : 0) + (serial ? mpad : 0);
    a.inst_bytes = (bytes + 15) & ~15;
    return true;
}

mbbp_status ensure_run_workspace(mbbp_ctx *c) {
    if (c->w_kmax) return MBBP_OK;
    const int64_t B = c->params.max_batch;
    mbbp_status st;
    for (int p = 0; p < 2; ++p) {
        const int W = c->dp[p].W, Ws = c->dp[p].Ws;
        if ((st = c->alloc(c->w_err[p], (size_t)B * W)) != MBBP_OK) return st;
        if ((st = c->alloc(c->w_syn[p], (size_t)B * Ws)) != MBBP_OK) return st;
        if ((st = c->alloc(c->w_corr[p], (size_t)B * W)) != MBBP_OK) return st;
        if ((st = c->alloc(c->w_conv[p], (size_t)B)) != MBBP_OK) return st;
        if ((st = c->alloc(c->w_basis[p], (size_t)B)) != MBBP_OK) return st;
        if ((st = c->alloc(c->w_prior[p], (size_t)c->n)) != MBBP_OK) return st;
    }
    if ((st = c->alloc(c->w_counters, (size_t)MBBP_NUM_COUNTERS)) != MBBP_OK) return st;
    if ((st = c->alloc(c->w_desc, 1)) != MBBP_OK) return st;
    return c->alloc(c->w_kmax, (size_t)B);
}

mbbp_status check_stream_ptrs(const void *p, const char *what) {
    if (!p) return fail(MBBP_EINVAL, std::string("null pointer: ") + what);
    return MBBP_OK;
}

// Serial schedule with one lane per shot: shots per wavefront S and LDS bytes of its
// wavefront (messages [E][S], augmented syndrome words, the shot's syndrome words,
// per-shot priors).  The largest S in {64, 32, 16, 8, 4} that leaves room for two
// wavefronts per compute unit, else the largest that fits one; false if none does
// (the level-parallel kernel then runs the schedule).
bool serial_lane_layout(const mbbp_ctx *c, int part0, int nparts, bool pps, mbbp::BPArgs &a) {
    int emax = 0, maug = 0, ws = 0, n = 0;
    for (int p = part0; p < part0 + nparts; ++p) {
        if (!c->dp[p].serial_ok) return false;
        emax = std::max(emax, c->dp[p].emax);
        maug = std::max(maug, c->dp[p].maug);
        ws = std::max(ws, c->dp[p].Ws);
        n = std::max(n, c->dp[p].n);
    }
    const int nmw = (maug + 31) / 32;
    // per shot lane: messages, decision bytes (4 a word), augmented syndrome bits,
    // syndrome words and (per-shot priors) the priors, one word each
    const size_t per_lane = 4u * (size_t)(emax + (n + 3) / 4 + nmw + 2 * ws + (pps ? n : 0));
    const size_t cu_lds = 160u * 1024u;  // LDS of one gfx950 compute unit
    int pick = 0;
    if (c->serial_lanes > 0 && mbbp::serial_lanes_supported(n, c->serial_lanes) &&
        (size_t)c->serial_lanes * per_lane <= (size_t)c->lds_block)
        pick = c->serial_lanes;
    for (int S : {64, 32, 16, 8, 4})
        if (!pick && mbbp::serial_lanes_supported(n, S) && (size_t)S * per_lane <= (size_t)c->lds_block &&
            2 * (size_t)S * per_lane <= cu_lds) { pick = S; break; }
    if (!pick)
        for (int S : {64, 32, 16, 8, 4})
            if (mbbp::serial_lanes_supported(n, S) && (size_t)S * per_lane <= (size_t)c->lds_block) { pick = S; break; }
    if (!pick) return false;
    a.serial_lanes = pick;
    a.s_emax = emax;
    a.s_nmw = nmw;
    a.ws_max = ws;
    a.n_max = n;
    a.inst_bytes = (int)((size_t)pick * per_lane + 4u * (size_t)n);  // + the shared prior vector
    return true;
}

// LDS layout of the serial kernel with eight lanes per shot (normalized min-sum):
// G shot blocks of sb bytes (8 junk words, messages, decision words, augmented
// syndrome words, syndrome words, per-shot priors and a 0), sb / 4 = 8 mod 32 so that the groups' blocks
// start eight banks apart, then the shared prior vector and its decision words.  G
// is the count (8, 4, 2, 1) that keeps the most shots resident per compute unit,
// counting at most eight wavefronts (two per SIMD); ties go to the larger G.  Sets
// the persistent grid to the wavefronts that fit.  False if one shot does not fit.
bool serial_slot_layout(const mbbp_ctx *c, int part0, int nparts, bool pps, mbbp::BPArgs &a, int &waves_per_cu) {
    int emax = 0, maug = 0, ws = 0, n = 0;
    for (int p = part0; p < part0 + nparts; ++p) {
        if (!c->dp[p].serial_ok || c->dp[p].max_deg > 8) return false;
        emax = std::max(emax, c->dp[p].emax);
        maug = std::max(maug, c->dp[p].maug);
        ws = std::max(ws, c->dp[p].Ws);
        n = std::max(n, c->dp[p].n);
    }
    if (emax > 65000) return false;  // the junk words' index must fit a record's edge field
    const int nmw = (maug + 31) / 32, ndw = n / 32 + 1;
    size_t sb = 4u * (size_t)(emax + 8 + ndw + nmw + 2 * ws + (pps ? n + 1 : 0));
    sb = (sb + 15u) & ~(size_t)15u;
    while ((sb / 4u) % 32u != 8u) sb += 16u;
    // shared priors and their decisions; 32 bytes of slack past the last block (the
    // exclusion sums read up to seven words past a variable's first edge)
    const size_t tail = (pps ? 0u : 4u * (size_t)(n + 1) + 4u * (size_t)ndw) + 32u;
    const size_t cu_lds = 160u * 1024u;
    int best = 0, best_score = 0, best_fit = 0;
    for (int G : {8, 4, 2, 1}) {
        const size_t bytes = (size_t)G * sb + tail;
        if (bytes > (size_t)c->lds_block) continue;
        const int fit = (int)std::min<size_t>(16, cu_lds / bytes);
        const int score = G * std::min(fit, 8);
        if (score > best_score) { best = G; best_score = score; best_fit = fit; }
    }
    if (!best) return false;
    a.serial_groups = best;
    a.s_sb = (int)sb;
    a.s_ndw = ndw;
    a.s_emax = emax;
    a.s_nmw = nmw;
    a.ws_max = ws;
    a.n_max = n;
    a.inst_bytes = (int)((size_t)best * sb + tail);
    waves_per_cu = best_fit;
    return true;
}

// Weighted-decoder training call: explicit weights, no early stop, checkpoints.
struct WeightedCall {
    const float *alpha, *beta;
    float *ckpt;
    int ckpt_every, n_ck;
};

mbbp_status run_bp(mbbp_ctx *c, int part0, int nparts, int64_t shots, const uint64_t *const syn[2],
                   const float *const prior[2], int pps, uint64_t *const cand[2], uint16_t *const kstat[2],
                   float *const llr[2], bool persistent, hipStream_t s, const WeightedCall *wc = nullptr,
                   bool rep_major = true, bool capturing = false, unsigned long long *queue = nullptr) {
    if (!queue) queue = c->w_queue;
    const int rule = wc ? (int)MBBP_WEIGHTED : c->params.rule;
    if (rule == MBBP_WEIGHTED && !wc && (!c->walpha || !c->wbeta))
        return fail(MBBP_EINVAL, "weighted rule: no weights set (mbbp_set_weights)");
    mbbp::BPArgs a{};
    a.part[0] = c->dp[0];
    a.part[1] = c->dp[1];
    a.dparts = c->dparts;
    a.part0 = part0;
    a.nparts = nparts;
    a.L = c->dp[0].L;
    a.T = c->T;
    a.alpha = c->params.alpha;
    a.rmax = c->params.r_max;
    a.fixed_T = (wc || (c->params.flags & MBBP_FLAG_FIXED_T)) ? 1 : 0;
    if (rule == MBBP_WEIGHTED) {
        a.walpha = wc ? wc->alpha : c->walpha;
        a.wbeta = wc ? wc->beta : c->wbeta;
        a.ckpt = wc ? wc->ckpt : nullptr;
        a.ckpt_every = wc ? wc->ckpt_every : 1;
        a.n_ck = wc ? wc->n_ck : 0;
    }
    a.shots = shots;
    a.cand_rm = rep_major ? 1 : 0;
    a.prior_per_shot = pps;
    for (int p = 0; p < 2; ++p) {
        a.syn[p] = syn[p];
        a.prior[p] = prior[p];
        a.cand[p] = cand[p];
        a.kstat[p] = kstat[p];
        a.llr[p] = llr[p];
    }
    const mbbp::BPConfig cfg = persistent ? c->batched_cfg : c->plain_cfg;
    const int G = 1;  // one instance per wavefront
    a.persistent = persistent ? 1 : 0;
    a.chunk = cfg.chunk;  // shots of a work item, decoded one after another by a wave
    a.n_chunks = (shots + a.chunk - 1) / a.chunk;
    a.n_pl = nparts * c->dp[part0].L;
    a.n_items = a.n_chunks * a.n_pl;
    a.item_order = persistent ? c->item_order + (part0 == 1 ? 0 : 0) : nullptr;
    if (persistent && nparts != 2) a.item_order = nullptr;
    a.queue = queue;
    if (!inst_layout(c, part0, nparts, pps != 0, c->schedule, rule, a))
        return fail(MBBP_EUNSUPPORTED, "code too large for the BP kernel's register tables");
    // two instances per wavefront where the paired kernel serves the launch
    int dual_bytes = 0, dual_stride = 0;
    if (!(c->params.flags & MBBP_FLAG_ONE_PER_WAVE) &&
        mbbp::bp_dual_layout(a, c->schedule, rule, dual_bytes, dual_stride)) {
        a.dual = 1;
        a.inst_bytes = dual_bytes;
        a.dual_stride = dual_stride;
    }
    // serial schedule: normalized min-sum on eight lanes per shot, else one lane per
    // shot (both rules), where their layouts fit; else the level-synchronous kernel
    const bool layered = c->schedule == MBBP_LAYERED && !wc;
    const int sk = c->serial_kernel;
    int slot_waves = 0;
    const bool serial_slots = layered && rule == MBBP_NMS && (sk == MBBP_SERIAL_AUTO || sk == MBBP_SERIAL_SLOTS) &&
                              serial_slot_layout(c, part0, nparts, pps != 0, a, slot_waves);
    const bool serial_lane = !serial_slots && layered && (rule == MBBP_NMS || rule == MBBP_SPA) &&
                             sk != MBBP_SERIAL_LEVELS && serial_lane_layout(c, part0, nparts, pps != 0, a);
    if (serial_lane || serial_slots) {
        a.dual = 0;
        // a work item gives every lane (every group) `chunk` shots
        a.chunk = cfg.chunk * (serial_lane ? a.serial_lanes : a.serial_groups);
        a.n_chunks = (shots + a.chunk - 1) / a.chunk;
        a.n_items = a.n_chunks * a.n_pl;
    }
    mbbp::BPConfig run = cfg;
    if (persistent) {
        run.blocks = cfg.blocks > 0 ? cfg.blocks : c->cu_count * 5;
        // the eight-lanes-per-shot kernel: as many wavefronts as the LDS holds
        if (serial_slots) run.blocks = c->cu_count * slot_waves;
        hipError_t e = mbbp::launch_reset(queue, nullptr, 0, s);
        if (e != hipSuccess) return fail(MBBP_EDEVICE, std::string("reset launch: ") + hipGetErrorString(e));
    }
    if (!serial_lane && !serial_slots) {
        while (run.waves_per_block > 1 && (size_t)run.waves_per_block * G * a.inst_bytes > mbbp::bp_lds_limit())
            run.waves_per_block /= 2;
        if ((size_t)run.waves_per_block * G * a.inst_bytes > mbbp::bp_lds_limit())
            return fail(MBBP_EUNSUPPORTED, "representation too large for LDS with this configuration");
    }
    auto launch = [&](const mbbp::BPArgs &x) {
        if (serial_slots) return mbbp::launch_bp_serial_slots(x, run, s);
        return serial_lane ? mbbp::launch_bp_serial(x, run, rule, s) : mbbp::launch_bp(x, run, c->schedule, rule, s);
    };
    // timing: events around the launch(es); a captured launch (mbbp_run's graph) gets
    // event record nodes of its own after capture, given fresh events per replay
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (c->timing && !capturing) {
        MBBP_HIP(hipEventCreate(&ev0));
        MBBP_HIP(hipEventCreate(&ev1));
        MBBP_HIP(hipEventRecord(ev0, s));
    }
    hipError_t e = hipSuccess;
    if (!persistent && c->per_basis && !wc && nparts == 2) {
        // the naive form: one launch per (part, representation) over all shots
        for (int k = 0; k < a.n_pl && e == hipSuccess; ++k) {
            mbbp::BPArgs one = a;
            one.item_order = c->rep_ids + k;
            one.n_pl = 1;
            one.n_items = a.n_chunks;
            e = launch(one);
        }
    } else {
        e = launch(a);
    }
    if (e != hipSuccess) return fail(MBBP_EDEVICE, std::string("bp launch: ") + hipGetErrorString(e));
    if (c->timing && !capturing) {
        MBBP_HIP(hipEventRecord(ev1, s));
        c->events.push_back({ev0, ev1});
    }
    return MBBP_OK;
}

mbbp_status run_select(mbbp_ctx *c, int part0, int nparts, int64_t shots, uint64_t *const corr[2],
                       uint64_t *const conv[2], int16_t *const basis[2], int64_t *counters, int *kmax,
                       hipStream_t s, uint64_t *const *cand = nullptr, uint16_t *const *kstat = nullptr) {
    if (!cand) cand = c->cand;
    if (!kstat) kstat = c->kstat;
    mbbp::SelectArgs a{};
    a.part[0] = c->dp[0];
    a.part[1] = c->dp[1];
    a.part0 = part0;
    a.nparts = nparts;
    a.rule = c->params.select;
    a.shots = shots;
    for (int p = 0; p < 2; ++p) {
        a.cand[p] = cand[p];
        a.kstat[p] = kstat[p];
        a.corr[p] = corr[p];
        a.conv[p] = conv[p];
        a.basis[p] = basis[p];
    }
    a.counters = counters;
    a.kmax_shot = kmax;
    hipError_t e = mbbp::launch_select(a, s);
    if (e != hipSuccess) return fail(MBBP_EDEVICE, std::string("select launch: ") + hipGetErrorString(e));
    return MBBP_OK;
}

}  // namespace

// ----------------------------------------------------------------------------- C ABI

extern "C" {

const char *mbbp_last_error(void) { return g_last_error.c_str(); }

mbbp_status mbbp_params_default(mbbp_params *p) {
    if (!p) return fail(MBBP_EINVAL, "null params");
    p->rule = MBBP_NMS;
    p->alpha = 0.875f;
    p->r_max = 65536.0f;
    p->select = MBBP_MIN_WEIGHT;
    p->max_batch = 1 << 20;
    p->flags = 0;
    return MBBP_OK;
}

mbbp_status mbbp_subtrees(const mbbp_sparse *H, const int32_t *perm, int32_t *check_sets, int32_t *order,
                          int32_t *n_subtrees) {
    std::vector<Row> rows;
    mbbp_status st = read_sparse(H, "H", rows);
    if (st != MBBP_OK) return st;
    if (!perm || !check_sets || !order || !n_subtrees) return fail(MBBP_EINVAL, "null output pointer");
    std::vector<int32_t> cs, ord;
    int ns = 0;
    try {
        st = subtrees(rows, H->cols, perm, cs, ord, ns);
    } catch (const std::bad_alloc &) {
        return fail(MBBP_ENOMEM, "out of host memory");
    }
    if (st != MBBP_OK) return st;
    std::copy(cs.begin(), cs.end(), check_sets);
    std::copy(ord.begin(), ord.end(), order);
    *n_subtrees = ns;
    return MBBP_OK;
}

mbbp_status mbbp_build_bases(const mbbp_sparse *H, int32_t mode, int32_t L, int32_t n_perms, const int32_t *perms,
                             int32_t *basis_ptr, int32_t *rows_out, int32_t rows_cap) {
    std::vector<Row> rows;
    mbbp_status st = read_sparse(H, "H", rows);
    if (st != MBBP_OK) return st;
    if (L < 1 || n_perms < 1 || !perms || !basis_ptr || (!rows_out && rows_cap > 0) || rows_cap < 0)
        return fail(MBBP_EINVAL, "bad arguments to mbbp_build_bases");
    const int m = H->rows;
    std::vector<std::vector<int32_t>> reps;
    try {
        if (mode == 0) {
            std::vector<std::vector<int32_t>> seen_sets;
            for (int k = 0; k < n_perms && (int)reps.size() < L; ++k) {
                std::vector<int32_t> cs, ord;
                int ns = 0;
                st = subtrees(rows, H->cols, perms + (size_t)k * m, cs, ord, ns);
                if (st != MBBP_OK) return st;
                size_t pos = 0;
                for (int s = 1; s <= ns && (int)reps.size() < L; ++s) {
                    std::vector<int32_t> t;
                    while (pos < ord.size() && cs[ord[pos]] == s) t.push_back(ord[pos++]);
                    std::vector<int32_t> key = t;
                    std::sort(key.begin(), key.end());
                    if (std::find(seen_sets.begin(), seen_sets.end(), key) != seen_sets.end()) continue;
                    seen_sets.push_back(key);
                    reps.push_back(t);
                }
            }
            if ((int)reps.size() < L) return fail(MBBP_EINVAL, "not enough distinct subtrees for L");
        } else if (mode == 1) {
            if (n_perms < L) return fail(MBBP_EINVAL, "ramp mode needs n_perms >= L");
            for (int l = 0; l < L; ++l) {
                std::vector<int32_t> cs, ord;
                int ns = 0;
                st = subtrees(rows, H->cols, perms + (size_t)l * m, cs, ord, ns);
                if (st != MBBP_OK) return st;
                const int r = L == 1 ? 0 : (int)((2LL * l * m + (L - 1)) / (2LL * (L - 1)));
                reps.emplace_back(ord.begin(), ord.begin() + r);
            }
        } else {
            return fail(MBBP_EINVAL, "unknown basis mode");
        }
    } catch (const std::bad_alloc &) {
        return fail(MBBP_ENOMEM, "out of host memory");
    }
    int64_t total = 0;
    for (auto &r : reps) total += (int64_t)r.size();
    if (total > rows_cap) return fail(MBBP_EINVAL, "rows_cap too small");
    basis_ptr[0] = 0;
    int64_t used = 0;
    for (int l = 0; l < L; ++l) {
        for (int32_t r : reps[l]) rows_out[used++] = r;
        basis_ptr[l + 1] = (int32_t)used;
    }
    return MBBP_OK;
}

mbbp_status mbbp_create(const mbbp_sparse *H_X, const mbbp_sparse *H_Z, const mbbp_bases *bases, int32_t T,
                        int32_t schedule, const mbbp_params *params, mbbp_ctx **out) {
    if (!out) return fail(MBBP_EINVAL, "null out");
    *out = nullptr;
    if (!bases) return fail(MBBP_EINVAL, "null bases");
    if (T < 0) return fail(MBBP_EINVAL, "T < 0");
    if (T > 32767) return fail(MBBP_EUNSUPPORTED, "T > 32767");
    if (schedule != MBBP_FLOODING && schedule != MBBP_LAYERED) return fail(MBBP_EINVAL, "unknown schedule");
    mbbp_params prm;
    mbbp_params_default(&prm);
    if (params) prm = *params;
    if (prm.rule != MBBP_NMS && prm.rule != MBBP_SPA && prm.rule != MBBP_WEIGHTED)
        return fail(MBBP_EINVAL, "unknown rule");
    if (prm.rule == MBBP_WEIGHTED && schedule != MBBP_FLOODING)
        return fail(MBBP_EUNSUPPORTED, "the weighted rule is built for the flooding schedule");
    if (prm.select != MBBP_MIN_WEIGHT && prm.select != MBBP_FWS) return fail(MBBP_EINVAL, "unknown select rule");
    if (!(prm.alpha > 0.0f) || !(prm.r_max > 0.0f) || !std::isfinite(prm.alpha) || !std::isfinite(prm.r_max))
        return fail(MBBP_EINVAL, "alpha and r_max must be positive and finite");
    if (prm.max_batch < 1) return fail(MBBP_EINVAL, "max_batch < 1");
    std::unique_ptr<mbbp_ctx> c;
    try {
        c.reset(new mbbp_ctx());
        std::vector<Row> hx, hz;
        mbbp_status st;
        if ((st = read_sparse(H_X, "H_X", hx)) != MBBP_OK) return st;
        if ((st = read_sparse(H_Z, "H_Z", hz)) != MBBP_OK) return st;
        if (H_X->cols != H_Z->cols) return fail(MBBP_EINVAL, "H_X and H_Z have different n");
        const int n = H_X->cols;
        if (n > mbbp::kMaxN) return fail(MBBP_EUNSUPPORTED, "n > 1024");
        // H_X H_Z^T = 0 (Section II-A)
        {
            std::vector<std::vector<uint64_t>> zb(hz.size(), std::vector<uint64_t>((n + 63) / 64, 0));
            for (size_t j = 0; j < hz.size(); ++j)
                for (int col : hz[j]) zb[j][col >> 6] |= 1ull << (col & 63);
            for (auto &rx : hx)
                for (auto &z : zb) {
                    int par = 0;
                    for (int col : rx) par ^= (int)((z[col >> 6] >> (col & 63)) & 1u);
                    if (par) return fail(MBBP_EINVAL, "H_X H_Z^T != 0");
                }
        }
        c->n = n;
        c->T = T;
        c->schedule = schedule;
        c->params = prm;
        c->HX = hx;
        c->HZ = hz;
        const bool pair_hint = prm.rule == MBBP_NMS && schedule == MBBP_FLOODING &&
                               !(prm.flags & (MBBP_FLAG_FIXED_T | MBBP_FLAG_ONE_PER_WAVE));
        if ((st = build_part(hz, n, bases->hz, "bases.hz", c->hp[0], pair_hint)) != MBBP_OK) return st;
        if ((st = build_part(hx, n, bases->hx, "bases.hx", c->hp[1], pair_hint)) != MBBP_OK) return st;
        if (c->hp[0].L != c->hp[1].L) return fail(MBBP_EINVAL, "bases.hx and bases.hz have different L");
        c->LZ = logicals(hx, hz, n);  // ker H_X mod rowspace H_Z
        c->LX = logicals(hz, hx, n);  // ker H_Z mod rowspace H_X
        MBBP_HIP(hipGetDevice(&c->device));
        hipDeviceProp_t prop;
        MBBP_HIP(hipGetDeviceProperties(&prop, c->device));
        c->cu_count = prop.multiProcessorCount;
        {
            int lb = 0;
            if (hipDeviceGetAttribute(&lb, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) == hipSuccess &&
                lb > 0)
                c->lds_block = lb;
        }
        // device address of the static scratch array on this device (taken once per
        // device, with the device current)
        {
            if (c->device < 0 || c->device >= kMaxDevices) return fail(MBBP_EUNSUPPORTED, "device index too large");
            std::lock_guard<std::mutex> lk(g_scratch_mu);
            if (!g_scratch_ptr[c->device]) {
                void *ptr = nullptr;
                hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
                if (e != hipSuccess || !ptr)
                    return fail(MBBP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
                g_scratch_ptr[c->device] = ptr;
            }
            c->scratch_dev = static_cast<unsigned char *>(g_scratch_ptr[c->device]);
        }
        // part X (H_Z) tests residuals with H_Z and L_Z; part Z with H_X and L_X
        if ((st = upload_part(c.get(), 0, c->LZ)) != MBBP_OK) return st;
        if ((st = upload_part(c.get(), 1, c->LX)) != MBBP_OK) return st;
        {
            std::vector<mbbp::DevPart> both{c->dp[0], c->dp[1]};
            if ((st = c->put(c->dparts, both)) != MBBP_OK) return st;
        }
        // schedule support
        for (int lpi : {16, 32, 64}) {
            (void)lpi;
        }
        // default launch shape: one instance per wavefront (measured fastest on MI355X;
        // the autotuner may pick another)
        const int lpi = 64;
        int need = 0;
        for (int p = 0; p < 2; ++p)
            need = std::max({need, (c->dp[p].n + lpi - 1) / lpi, (c->dp[p].Mmax + lpi - 1) / lpi});
        if (!mbbp::bp_supported(lpi, need, c->dp[0].uniform_dc, prm.rule, schedule))
            return fail(MBBP_EUNSUPPORTED, "code too large for the register tables");
        c->plain_cfg = mbbp::BPConfig{lpi, 4, 8, 0};
        c->batched_cfg = mbbp::BPConfig{lpi, 4, 64, c->cu_count * 5};
        // workspace
        const int64_t B = prm.max_batch;
        for (int p = 0; p < 2; ++p) {
            const int L = c->dp[p].L, W = c->dp[p].W, Ws = c->dp[p].Ws;
            if ((st = c->alloc(c->cand[p], (size_t)B * L * W)) != MBBP_OK) return st;
            if ((st = c->alloc(c->kstat[p], (size_t)B * L)) != MBBP_OK) return st;
            (void)Ws;
        }
        if ((st = c->alloc(c->w_queue, 1)) != MBBP_OK) return st;
        {
            std::vector<int32_t> ids(2 * c->dp[0].L);
            for (size_t i = 0; i < ids.size(); ++i) ids[i] = (int32_t)i;
            if ((st = c->put(c->rep_ids, ids)) != MBBP_OK) return st;
        }
        // heavy-first order of (part, representation) work for the persistent form
        {
            std::vector<std::pair<int64_t, int32_t>> w;
            const int L = c->dp[0].L;
            for (int p = 0; p < 2; ++p)
                for (int l = 0; l < L; ++l) w.push_back({-(int64_t)c->hp[p].E[l], p * L + l});
            std::stable_sort(w.begin(), w.end());
            std::vector<int32_t> order;
            for (auto &x : w) order.push_back(x.second);
            const int32_t *d = nullptr;
            if ((st = c->put(d, order)) != MBBP_OK) return st;
            c->item_order = const_cast<int32_t *>(d);
        }
    } catch (const std::bad_alloc &) {
        return fail(MBBP_ENOMEM, "out of host memory");
    }
    *out = c.release();
    return MBBP_OK;
}

void mbbp_destroy(mbbp_ctx *ctx) {
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    for (auto &ev : ctx->events) {
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    for (auto &kv : ctx->graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    for (hipEvent_t ev : ctx->graph_ev)
        if (ev) (void)hipEventDestroy(ev);
    delete ctx;
}

mbbp_status mbbp_decode_detail(mbbp_ctx *ctx, int32_t part, int64_t shots, const uint64_t *syn, const float *prior,
                               int32_t prior_per_shot, uint64_t *cand, uint16_t *kstat, float *llr,
                               void *hip_stream) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    if (part != 0 && part != 1) return fail(MBBP_EINVAL, "part must be 0 (X) or 1 (Z)");
    if (shots < 1 || shots > ctx->params.max_batch) return fail(MBBP_EINVAL, "shots out of range");
    mbbp_status st;
    if ((st = check_stream_ptrs(syn, "syn")) != MBBP_OK) return st;
    if ((st = check_stream_ptrs(prior, "prior")) != MBBP_OK) return st;
    if ((st = check_stream_ptrs(cand, "cand")) != MBBP_OK) return st;
    if ((st = check_stream_ptrs(kstat, "kstat")) != MBBP_OK) return st;
    const uint64_t *sy[2] = {syn, syn};
    const float *pr[2] = {prior, prior};
    uint64_t *cd[2] = {cand, cand};
    uint16_t *ks[2] = {kstat, kstat};
    float *ll[2] = {llr, llr};
    return run_bp(ctx, part, 1, shots, sy, pr, prior_per_shot ? 1 : 0, cd, ks, ll, false,
                  static_cast<hipStream_t>(hip_stream), nullptr, false);
}

static mbbp_status decode_common(mbbp_ctx *ctx, int64_t shots, const uint64_t *syn_x, const uint64_t *syn_z,
                                 const float *prior_x, const float *prior_z, int32_t pps, uint64_t *corr_x,
                                 uint64_t *corr_z, uint64_t *conv_x, uint64_t *conv_z, int16_t *basis_x,
                                 int16_t *basis_z, void *hip_stream, bool persistent) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    if (shots < 1 || shots > ctx->params.max_batch) return fail(MBBP_EINVAL, "shots out of range");
    const void *ptrs[] = {syn_x, syn_z, prior_x, prior_z, corr_x, corr_z, conv_x, conv_z, basis_x, basis_z};
    for (const void *p : ptrs)
        if (!p) return fail(MBBP_EINVAL, "null device pointer");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const uint64_t *sy[2] = {syn_x, syn_z};
    const float *pr[2] = {prior_x, prior_z};
    float *ll[2] = {nullptr, nullptr};
    mbbp_status st = run_bp(ctx, 0, 2, shots, sy, pr, pps ? 1 : 0, ctx->cand, ctx->kstat, ll, persistent, s);
    if (st != MBBP_OK) return st;
    uint64_t *co[2] = {corr_x, corr_z};
    uint64_t *cv[2] = {conv_x, conv_z};
    int16_t *bs[2] = {basis_x, basis_z};
    return run_select(ctx, 0, 2, shots, co, cv, bs, ctx->stats, nullptr, s);
}

mbbp_status mbbp_decode(mbbp_ctx *ctx, int64_t shots, const uint64_t *syn_x, const uint64_t *syn_z,
                        const float *prior_x, const float *prior_z, int32_t prior_per_shot, uint64_t *corr_x,
                        uint64_t *corr_z, uint64_t *conv_x, uint64_t *conv_z, int16_t *basis_x, int16_t *basis_z,
                        void *hip_stream) {
    return decode_common(ctx, shots, syn_x, syn_z, prior_x, prior_z, prior_per_shot, corr_x, corr_z, conv_x,
                         conv_z, basis_x, basis_z, hip_stream, false);
}

mbbp_status mbbp_decode_batched(mbbp_ctx *ctx, int64_t shots, const uint64_t *syn_x, const uint64_t *syn_z,
                                const float *prior_x, const float *prior_z, int32_t prior_per_shot,
                                uint64_t *corr_x, uint64_t *corr_z, uint64_t *conv_x, uint64_t *conv_z,
                                int16_t *basis_x, int16_t *basis_z, void *hip_stream) {
    return decode_common(ctx, shots, syn_x, syn_z, prior_x, prior_z, prior_per_shot, corr_x, corr_z, conv_x,
                         conv_z, basis_x, basis_z, hip_stream, true);
}

// Sampler thresholds: u < t1 -> X, u < t2 -> Y, u < t3 -> Z.  Depolarizing:
// t_k = floor(k (p/3) 2^32).  X errors only: t1 = t2 = t3 = floor(p 2^32), so a
// qubit takes X iff u < floor(p 2^32) and never Y or Z.
static void thresholds(double p, int noise, uint64_t t[3]) {
    if (noise == MBBP_NOISE_X_ONLY) {
        t[0] = t[1] = t[2] = (uint64_t)std::floor(p * 4294967296.0);
        return;
    }
    for (int k = 1; k <= 3; ++k) t[k - 1] = (uint64_t)std::floor((double)k * (p / 3.0) * 4294967296.0);
}

mbbp_status mbbp_set_noise(mbbp_ctx *ctx, int32_t model) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    if (model != MBBP_NOISE_DEPOLARIZING && model != MBBP_NOISE_X_ONLY) return fail(MBBP_EINVAL, "unknown noise model");
    ctx->noise = model;
    return MBBP_OK;
}

mbbp_status mbbp_sample(mbbp_ctx *ctx, uint64_t seed, double p, int64_t shot0, int64_t shots, uint64_t *err_x,
                        uint64_t *err_z, uint64_t *syn_x, uint64_t *syn_z, void *hip_stream) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    if (!(p >= 0.0 && p <= 1.0)) return fail(MBBP_EINVAL, "p outside [0, 1]");
    if (shots < 1 || shots > ctx->params.max_batch || shot0 < 0) return fail(MBBP_EINVAL, "shots out of range");
    if (!err_x || !err_z || !syn_x || !syn_z) return fail(MBBP_EINVAL, "null device pointer");
    mbbp::SampleArgs a{};
    a.part[0] = ctx->dp[0];
    a.part[1] = ctx->dp[1];
    a.n = ctx->n;
    a.seed = seed;
    uint64_t t[3];
    thresholds(p, ctx->noise, t);
    a.t1 = t[0]; a.t2 = t[1]; a.t3 = t[2];
    a.shot0 = shot0;
    a.shots = shots;
    a.err[0] = err_x; a.err[1] = err_z;
    a.syn[0] = syn_x; a.syn[1] = syn_z;
    a.desc = nullptr;
    hipError_t e = mbbp::launch_sample(a, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(MBBP_EDEVICE, std::string("sample launch: ") + hipGetErrorString(e));
    return MBBP_OK;
}

mbbp_status mbbp_failures(mbbp_ctx *ctx, int64_t shots, const uint64_t *err_x, const uint64_t *err_z,
                          const uint64_t *corr_x, const uint64_t *corr_z, uint8_t *fail_out, void *hip_stream) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    if (shots < 1 || shots > ctx->params.max_batch) return fail(MBBP_EINVAL, "shots out of range");
    if (!err_x || !err_z || !corr_x || !corr_z || !fail_out) return fail(MBBP_EINVAL, "null device pointer");
    mbbp::FailArgs a{};
    a.part[0] = ctx->dp[0];
    a.part[1] = ctx->dp[1];
    a.shots = shots;
    a.err[0] = err_x; a.err[1] = err_z;
    a.corr[0] = corr_x; a.corr[1] = corr_z;
    a.fail = fail_out;
    hipError_t e = mbbp::launch_fail(a, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(MBBP_EDEVICE, std::string("failure launch: ") + hipGetErrorString(e));
    return MBBP_OK;
}

// The whole path of one call, enqueued on s: descriptor and clearing (prep), noise
// and syndromes, persistent BP, decision with counters, failure test, counters
// added into the caller's.  Every node reads its per-call values from the device
// descriptor, so a captured copy is replayed by changing only the prep node.
static mbbp_status run_enqueue(mbbp_ctx *ctx, const mbbp::RunPrepArgs &prep, int64_t shots, hipStream_t s,
                               const RunWs &ws, bool capturing = false) {
    hipError_t e = mbbp::launch_run_prep(prep, s);
    if (e != hipSuccess) return fail(MBBP_EDEVICE, std::string("prep launch: ") + hipGetErrorString(e));
    mbbp::SampleArgs sa{};
    sa.part[0] = ctx->dp[0];
    sa.part[1] = ctx->dp[1];
    sa.n = ctx->n;
    sa.shots = shots;
    sa.err[0] = ws.err[0]; sa.err[1] = ws.err[1];
    sa.syn[0] = ws.syn[0]; sa.syn[1] = ws.syn[1];
    sa.desc = ws.desc;
    e = mbbp::launch_sample(sa, s);
    if (e != hipSuccess) return fail(MBBP_EDEVICE, std::string("sample launch: ") + hipGetErrorString(e));
    const uint64_t *sy[2] = {ws.syn[0], ws.syn[1]};
    const float *pr[2] = {ws.prior[0], ws.prior[1]};
    float *ll[2] = {nullptr, nullptr};
    mbbp_status st;
    if ((st = run_bp(ctx, 0, 2, shots, sy, pr, 0, ws.cand, ws.kstat, ll, true, s, nullptr, true, capturing,
                     ws.queue)) != MBBP_OK)
        return st;
    if ((st = run_select(ctx, 0, 2, shots, ws.corr, ws.conv, ws.basis, ws.counters, ws.kmax, s, ws.cand,
                         ws.kstat)) != MBBP_OK)
        return st;
    mbbp::FailArgs a{};
    a.part[0] = ctx->dp[0];
    a.part[1] = ctx->dp[1];
    a.shots = shots;
    a.err[0] = ws.err[0]; a.err[1] = ws.err[1];
    a.corr[0] = ws.corr[0]; a.corr[1] = ws.corr[1];
    a.fail = nullptr;
    a.counters = ws.counters;
    a.kmax_shot = ws.kmax;
    e = mbbp::launch_fail(a, s);
    if (e != hipSuccess) return fail(MBBP_EDEVICE, std::string("failure launch: ") + hipGetErrorString(e));
    e = mbbp::launch_accumulate(ws.counters, ws.desc, MBBP_NUM_COUNTERS, s);
    if (e != hipSuccess) return fail(MBBP_EDEVICE, std::string("accumulate launch: ") + hipGetErrorString(e));
    return MBBP_OK;
}

// The context's own run workspace (allocated by ensure_run_workspace).
static RunWs ctx_ws(mbbp_ctx *ctx) {
    RunWs w{};
    for (int p = 0; p < 2; ++p) {
        w.err[p] = ctx->w_err[p];
        w.syn[p] = ctx->w_syn[p];
        w.corr[p] = ctx->w_corr[p];
        w.conv[p] = ctx->w_conv[p];
        w.basis[p] = ctx->w_basis[p];
        w.prior[p] = ctx->w_prior[p];
        w.cand[p] = ctx->cand[p];
        w.kstat[p] = ctx->kstat[p];
    }
    w.kmax = ctx->w_kmax;
    w.counters = ctx->w_counters;
    w.desc = ctx->w_desc;
    w.queue = ctx->w_queue;
    return w;
}

// Validation and the per-call descriptor of mbbp_run / mbbp_run_static.
static mbbp_status run_prep_args(mbbp_ctx *ctx, uint64_t seed, double p, int64_t shot0, int64_t shots,
                                 int64_t *counters, const RunWs &ws, mbbp::RunPrepArgs &prep) {
    prep = mbbp::RunPrepArgs{};
    prep.d.seed = seed;
    prep.d.shot0 = shot0;
    uint64_t t[3];
    thresholds(p, ctx->noise, t);
    prep.d.t1 = t[0]; prep.d.t2 = t[1]; prep.d.t3 = t[2];
    prep.d.counters = counters;
    prep.desc = ws.desc;
    prep.prior0 = ws.prior[0];
    prep.prior1 = ws.prior[1];
    prep.n = ctx->n;
    mbbp_status st = mbbp_prior_llr(ctx->noise, p, &prep.mu);
    if (st != MBBP_OK) return st;
    prep.kmax = ws.kmax;
    prep.shots = shots;
    prep.queue = ws.queue;
    prep.counters = ws.counters;
    return MBBP_OK;
}

static bool same_config(const mbbp::BPConfig &a, const mbbp::BPConfig &b) {
    return a.lpi == b.lpi && a.waves_per_block == b.waves_per_block && a.chunk == b.chunk && a.blocks == b.blocks;
}

static void drop_graphs(mbbp_ctx *ctx) {
    (void)hipDeviceSynchronize();
    for (auto &kv : ctx->graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    ctx->graphs.clear();
}

static mbbp_status capture_run_graph(mbbp_ctx *ctx, const mbbp::RunPrepArgs &prep, int64_t shots, RunGraph &g) {
    if (!ctx->capture_stream) MBBP_HIP(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
    for (hipEvent_t &ev : ctx->graph_ev)
        if (!ev) MBBP_HIP(hipEventCreate(&ev));
    MBBP_HIP(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
    mbbp::set_last_bp_kernel(nullptr);
    mbbp_status st = run_enqueue(ctx, prep, shots, ctx->capture_stream, ctx_ws(ctx), true);
    g.bp_func = mbbp::last_bp_kernel();
    g.cfg = ctx->batched_cfg;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->capture_stream, &graph);
    if (st != MBBP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(MBBP_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    g.graph = graph;
    size_t count = 0;
    MBBP_HIP(hipGraphGetNodes(graph, nullptr, &count));
    std::vector<hipGraphNode_t> nodes(count);
    MBBP_HIP(hipGraphGetNodes(graph, nodes.data(), &count));
    hipGraphNode_t bp = nullptr;
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType ty;
        MBBP_HIP(hipGraphNodeGetType(nd, &ty));
        if (ty != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp;
        MBBP_HIP(hipGraphKernelNodeGetParams(nd, &kp));
        if (kp.func == mbbp::run_prep_kernel_ptr()) {
            g.prep = nd;
            g.prep_params = kp;
        }
        if (kp.func == g.bp_func) bp = nd;
    }
    if (!g.prep) return fail(MBBP_EDEVICE, "captured graph has no preparation node");
    if (!bp) return fail(MBBP_EDEVICE, "captured graph has no BP kernel node");
    // event record nodes around the BP kernel node: pred -> ev0 -> bp -> ev1 -> succ
    {
        size_t nd = 0, ns = 0;
        MBBP_HIP(hipGraphNodeGetDependencies(bp, nullptr, &nd));
        std::vector<hipGraphNode_t> pred(nd);
        if (nd) MBBP_HIP(hipGraphNodeGetDependencies(bp, pred.data(), &nd));
        MBBP_HIP(hipGraphNodeGetDependentNodes(bp, nullptr, &ns));
        std::vector<hipGraphNode_t> succ(ns);
        if (ns) MBBP_HIP(hipGraphNodeGetDependentNodes(bp, succ.data(), &ns));
        for (hipGraphNode_t p : pred) MBBP_HIP(hipGraphRemoveDependencies(graph, &p, &bp, 1));
        for (hipGraphNode_t q : succ) MBBP_HIP(hipGraphRemoveDependencies(graph, &bp, &q, 1));
        MBBP_HIP(hipGraphAddEventRecordNode(&g.ev_node[0], graph, pred.data(), pred.size(), ctx->graph_ev[0]));
        MBBP_HIP(hipGraphAddDependencies(graph, &g.ev_node[0], &bp, 1));
        MBBP_HIP(hipGraphAddEventRecordNode(&g.ev_node[1], graph, &bp, 1, ctx->graph_ev[1]));
        for (hipGraphNode_t q : succ) MBBP_HIP(hipGraphAddDependencies(graph, &g.ev_node[1], &q, 1));
    }
    MBBP_HIP(hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
    return MBBP_OK;
}

mbbp_status mbbp_run(mbbp_ctx *ctx, uint64_t seed, double p, int64_t shot0, int64_t shots, int64_t *counters,
                     void *hip_stream) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    if (!(p > 0.0 && p <= 1.0)) return fail(MBBP_EINVAL, "p must be in (0, 1]");
    if (shots < 1 || shots > ctx->params.max_batch || shot0 < 0) return fail(MBBP_EINVAL, "shots out of range");
    if (!counters) return fail(MBBP_EINVAL, "null counters");
    mbbp_status st = ensure_run_workspace(ctx);
    if (st != MBBP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    mbbp::RunPrepArgs prep{};
    if ((st = run_prep_args(ctx, seed, p, shot0, shots, counters, ctx_ws(ctx), prep)) != MBBP_OK) return st;
    if (!ctx->use_graph) return run_enqueue(ctx, prep, shots, s, ctx_ws(ctx));
    auto it = ctx->graphs.find(shots);
    if (it != ctx->graphs.end() && !same_config(it->second.cfg, ctx->batched_cfg)) {
        // captured with another launch shape: capture again
        (void)hipStreamSynchronize(s);
        if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
        if (it->second.graph) (void)hipGraphDestroy(it->second.graph);
        ctx->graphs.erase(it);
        it = ctx->graphs.end();
    }
    if (it == ctx->graphs.end()) {
        RunGraph g;
        st = capture_run_graph(ctx, prep, shots, g);
        if (st != MBBP_OK) {
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            if (g.graph) (void)hipGraphDestroy(g.graph);
            return st;
        }
        it = ctx->graphs.emplace(shots, g).first;
    }
    RunGraph &g = it->second;
    hipKernelNodeParams kp = g.prep_params;
    void *args[] = {&prep};
    kp.kernelParams = args;
    kp.extra = nullptr;
    MBBP_HIP(hipGraphExecKernelNodeSetParams(g.exec, g.prep, &kp));
    hipEvent_t ev[2] = {ctx->graph_ev[0], ctx->graph_ev[1]};
    if (ctx->timing) {
        MBBP_HIP(hipEventCreate(&ev[0]));
        MBBP_HIP(hipEventCreate(&ev[1]));
    }
    for (int k = 0; k < 2; ++k) MBBP_HIP(hipGraphExecEventRecordNodeSetEvent(g.exec, g.ev_node[k], ev[k]));
    MBBP_HIP(hipGraphLaunch(g.exec, s));
    if (ctx->timing) ctx->events.push_back({ev[0], ev[1]});
    return MBBP_OK;
}

// Carves the run buffers for `shots` out of the scratch array at `base`; returns
// the bytes used (256-byte aligned pieces).  With base == nullptr only sizes.
static size_t carve_ws(const mbbp_ctx *ctx, int64_t shots, unsigned char *base, RunWs &w) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> unsigned char * {
        unsigned char *p = base ? base + off : nullptr;
        off += (bytes + 255) & ~size_t(255);
        return p;
    };
    const size_t S = (size_t)shots;
    w.desc = reinterpret_cast<mbbp::RunDesc *>(take(sizeof(mbbp::RunDesc)));
    w.counters = reinterpret_cast<int64_t *>(take(8 * MBBP_NUM_COUNTERS));
    w.queue = reinterpret_cast<unsigned long long *>(take(8));
    w.kmax = reinterpret_cast<int *>(take(4 * S));
    for (int p = 0; p < 2; ++p) {
        const size_t W = ctx->dp[p].W, Ws = ctx->dp[p].Ws, L = ctx->dp[p].L;
        w.prior[p] = reinterpret_cast<float *>(take(4 * (size_t)ctx->n));
        w.err[p] = reinterpret_cast<uint64_t *>(take(8 * S * W));
        w.syn[p] = reinterpret_cast<uint64_t *>(take(8 * S * Ws));
        w.corr[p] = reinterpret_cast<uint64_t *>(take(8 * S * W));
        w.conv[p] = reinterpret_cast<uint64_t *>(take(8 * S));
        w.basis[p] = reinterpret_cast<int16_t *>(take(2 * S));
        w.cand[p] = reinterpret_cast<uint64_t *>(take(8 * S * L * W));
        w.kstat[p] = reinterpret_cast<uint16_t *>(take(2 * S * L));
    }
    return off;
}

mbbp_status mbbp_run_static(mbbp_ctx *ctx, uint64_t seed, double p, int64_t shot0, int64_t shots, int64_t *counters,
                            void *hip_stream) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    if (!(p > 0.0 && p <= 1.0)) return fail(MBBP_EINVAL, "p must be in (0, 1]");
    if (shots < 1 || shot0 < 0) return fail(MBBP_EINVAL, "shots out of range");
    if (!counters) return fail(MBBP_EINVAL, "null counters");
    if (!ctx->scratch_dev) return fail(MBBP_EDEVICE, "no scratch address for this device");
    RunWs ws{};
    if (carve_ws(ctx, shots, nullptr, ws) > kScratchBytes) {
        int64_t lo = 0, hi = shots;  // largest batch that fits, for the message
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (carve_ws(ctx, mid, nullptr, ws) <= kScratchBytes) lo = mid;
            else hi = mid - 1;
        }
        return fail(MBBP_EINVAL, "shots = " + std::to_string(shots) + " exceed the static scratch of " +
                                     std::to_string(kScratchBytes >> 20) + " MiB (at most " + std::to_string(lo) +
                                     " shots for this decoder)");
    }
    int dev = -1;
    MBBP_HIP(hipGetDevice(&dev));
    if (dev != ctx->device) return fail(MBBP_EINVAL, "the decoder's device is not the current device");
    carve_ws(ctx, shots, ctx->scratch_dev, ws);
    mbbp::RunPrepArgs prep{};
    mbbp_status st = run_prep_args(ctx, seed, p, shot0, shots, counters, ws, prep);
    if (st != MBBP_OK) return st;
    const bool timing = ctx->timing;  // no event objects are made here
    ctx->timing = false;
    st = run_enqueue(ctx, prep, shots, static_cast<hipStream_t>(hip_stream), ws);
    ctx->timing = timing;
    return st;
}

mbbp_status mbbp_run_graph_config(mbbp_ctx *ctx, int64_t shots, mbbp_launch_config *cfg) {
    if (!ctx || !cfg) return fail(MBBP_EINVAL, "null argument");
    auto it = ctx->graphs.find(shots);
    if (it == ctx->graphs.end()) return fail(MBBP_EINVAL, "no graph captured for this number of shots");
    const RunGraph &g = it->second;
    size_t count = 0;
    MBBP_HIP(hipGraphGetNodes(g.graph, nullptr, &count));
    std::vector<hipGraphNode_t> nodes(count);
    MBBP_HIP(hipGraphGetNodes(g.graph, nodes.data(), &count));
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType ty;
        MBBP_HIP(hipGraphNodeGetType(nd, &ty));
        if (ty != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp;
        MBBP_HIP(hipGraphKernelNodeGetParams(nd, &kp));
        if (kp.func != g.bp_func) continue;
        cfg->lanes_per_instance = 64;
        cfg->waves_per_block = (int32_t)(kp.blockDim.x / 64);
        cfg->chunk = g.cfg.chunk;
        cfg->blocks = (int32_t)kp.gridDim.x;
        return MBBP_OK;
    }
    return fail(MBBP_EDEVICE, "captured graph has no BP kernel node");
}

static bool config_fits(const mbbp_ctx *c, int lpi) {
    int need = 0;
    for (int p = 0; p < 2; ++p)
        need = std::max({need, (c->dp[p].n + lpi - 1) / lpi, (c->dp[p].Mmax + lpi - 1) / lpi});
    return mbbp::bp_supported(lpi, need, c->dp[0].uniform_dc, c->params.rule, c->schedule);
}

mbbp_status mbbp_set_config(mbbp_ctx *ctx, int32_t form, const mbbp_launch_config *cfg) {
    if (!ctx || !cfg) return fail(MBBP_EINVAL, "null argument");
    if (form != 0 && form != 1) return fail(MBBP_EINVAL, "form must be 0 (plain) or 1 (batched)");
    const int lpi = cfg->lanes_per_instance;
    if (lpi != 64) return fail(MBBP_EUNSUPPORTED, "lanes_per_instance: only 64 (one instance per wavefront) is built");
    if (cfg->waves_per_block < 1 || cfg->waves_per_block > 4)  // kernels are built for 256 threads
        return fail(MBBP_EINVAL, "waves_per_block in [1, 4]");
    if (cfg->chunk < 1 || cfg->chunk > (1 << 20)) return fail(MBBP_EINVAL, "chunk in [1, 2^20]");
    if (cfg->blocks < 0) return fail(MBBP_EINVAL, "blocks < 0");
    if (!config_fits(ctx, lpi)) return fail(MBBP_EUNSUPPORTED, "code too large for this lane count");
    mbbp::BPConfig b{lpi, cfg->waves_per_block, cfg->chunk, cfg->blocks > 0 ? cfg->blocks : ctx->cu_count * 5};
    if (form == 0) {
        ctx->plain_cfg = b;
    } else {
        if (!same_config(ctx->batched_cfg, b)) drop_graphs(ctx);  // captured launches hold the old shape
        ctx->batched_cfg = b;
    }
    return MBBP_OK;
}

mbbp_status mbbp_get_config(mbbp_ctx *ctx, int32_t form, mbbp_launch_config *cfg) {
    if (!ctx || !cfg) return fail(MBBP_EINVAL, "null argument");
    if (form != 0 && form != 1) return fail(MBBP_EINVAL, "form must be 0 (plain) or 1 (batched)");
    const mbbp::BPConfig &b = form == 0 ? ctx->plain_cfg : ctx->batched_cfg;
    cfg->lanes_per_instance = b.lpi;
    cfg->waves_per_block = b.waves_per_block;
    cfg->chunk = b.chunk;
    cfg->blocks = b.blocks;
    return MBBP_OK;
}

mbbp_status mbbp_prior_llr(int32_t noise, double p, float *mu) {
    if (!mu) return fail(MBBP_EINVAL, "null mu");
    if (noise != MBBP_NOISE_DEPOLARIZING && noise != MBBP_NOISE_X_ONLY) return fail(MBBP_EINVAL, "unknown noise model");
    const double q = noise == MBBP_NOISE_X_ONLY ? p : 2.0 * p / 3.0;
    if (!(q > 0.0 && q < 1.0)) return fail(MBBP_EINVAL, "flip probability outside (0, 1)");
    *mu = (float)std::log((1.0 - q) / q);
    return MBBP_OK;
}

mbbp_status mbbp_set_per_basis(mbbp_ctx *ctx, int32_t enable) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    ctx->per_basis = enable != 0;
    return MBBP_OK;
}

mbbp_status mbbp_set_serial_lanes(mbbp_ctx *ctx, int32_t lanes) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    if (lanes != 0 && lanes != 4 && lanes != 8 && lanes != 16 && lanes != 32 && lanes != 64)
        return fail(MBBP_EINVAL, "lanes must be 0, 4, 8, 16, 32 or 64");
    if (ctx->serial_lanes != lanes) drop_graphs(ctx);
    ctx->serial_lanes = lanes;
    return MBBP_OK;
}

mbbp_status mbbp_set_stats(mbbp_ctx *ctx, int64_t *counters) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    ctx->stats = counters;
    return MBBP_OK;
}

mbbp_status mbbp_set_serial_kernel(mbbp_ctx *ctx, int32_t kernel) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    if (kernel < MBBP_SERIAL_AUTO || kernel > MBBP_SERIAL_LEVELS)
        return fail(MBBP_EINVAL, "serial kernel must be MBBP_SERIAL_AUTO, _SLOTS, _LANES or _LEVELS");
    if (ctx->serial_kernel != kernel) drop_graphs(ctx);
    ctx->serial_kernel = kernel;
    return MBBP_OK;
}

mbbp_status mbbp_set_graph(mbbp_ctx *ctx, int32_t enable) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    ctx->use_graph = enable != 0;
    return MBBP_OK;
}

mbbp_status mbbp_autotune(mbbp_ctx *ctx, int32_t form, uint64_t seed, double p, int64_t shots,
                          mbbp_launch_config *chosen) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    if (form != 0 && form != 1) return fail(MBBP_EINVAL, "form must be 0 (plain) or 1 (batched)");
    if (!(p > 0.0 && p <= 1.0)) return fail(MBBP_EINVAL, "p must be in (0, 1]");
    if (shots < 1 || shots > ctx->params.max_batch) return fail(MBBP_EINVAL, "shots out of range");
    mbbp_status st = ensure_run_workspace(ctx);
    if (st != MBBP_OK) return st;
    if (!ctx->capture_stream) MBBP_HIP(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
    hipStream_t s = ctx->capture_stream;
    if ((st = mbbp_sample(ctx, seed, p, 0, shots, ctx->w_err[0], ctx->w_err[1], ctx->w_syn[0], ctx->w_syn[1], s)) !=
        MBBP_OK)
        return st;
    float mu0 = 0.0f;
    if ((st = mbbp_prior_llr(ctx->noise, p, &mu0)) != MBBP_OK) return st;
    std::vector<float> mu(ctx->n, mu0);
    for (int pt = 0; pt < 2; ++pt)
        MBBP_HIP(hipMemcpyAsync(ctx->w_prior[pt], mu.data(), mu.size() * 4, hipMemcpyHostToDevice, s));
    std::vector<mbbp::BPConfig> cands;
    const int cu = ctx->cu_count;
    if (form == 1) {
        for (int wpb : {2, 4})
            for (int chunk : {4, 16, 64, 128})
                for (int bpc : {2, 4, 8}) cands.push_back({64, wpb, chunk, cu * bpc});
    } else {
        for (int wpb : {1, 2, 4})
            for (int chunk : {1, 4, 16, 64}) cands.push_back({64, wpb, chunk, 0});
    }
    mbbp::BPConfig &slot = form == 0 ? ctx->plain_cfg : ctx->batched_cfg;
    const mbbp::BPConfig keep = slot;
    const bool timing = ctx->timing;
    ctx->timing = false;
    hipEvent_t e0, e1;
    MBBP_HIP(hipEventCreate(&e0));
    MBBP_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    mbbp::BPConfig best = keep;
    for (const mbbp::BPConfig &cfg : cands) {
        slot = cfg;
        float total = 0.0f;
        for (int rep = 0; rep < 3 && st == MBBP_OK; ++rep) {
            if (rep == 1) (void)hipEventRecord(e0, s);
            st = decode_common(ctx, shots, ctx->w_syn[0], ctx->w_syn[1], ctx->w_prior[0], ctx->w_prior[1], 0,
                               ctx->w_corr[0], ctx->w_corr[1], ctx->w_conv[0], ctx->w_conv[1], ctx->w_basis[0],
                               ctx->w_basis[1], s, form == 1);
        }
        if (st != MBBP_OK) break;
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&total, e0, e1) != hipSuccess) {
            st = fail(MBBP_EDEVICE, "autotune timing failed");
            break;
        }
        if (total < best_ms) {
            best_ms = total;
            best = cfg;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->timing = timing;
    slot = st == MBBP_OK ? best : keep;
    if (form == 1 && !same_config(slot, keep)) drop_graphs(ctx);  // captured launches hold the old shape
    if (st != MBBP_OK) return st;
    if (chosen) {
        chosen->lanes_per_instance = best.lpi;
        chosen->waves_per_block = best.waves_per_block;
        chosen->chunk = best.chunk;
        chosen->blocks = best.blocks;
    }
    return MBBP_OK;
}

mbbp_status mbbp_set_timing(mbbp_ctx *ctx, int32_t enable) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    ctx->timing = enable != 0;
    return MBBP_OK;
}

mbbp_status mbbp_bp_time(mbbp_ctx *ctx, double *ms, int64_t *launches, int32_t reset) {
    if (!ctx || !ms || !launches) return fail(MBBP_EINVAL, "null argument");
    for (auto &ev : ctx->events) {
        MBBP_HIP(hipEventSynchronize(ev.second));
        float t = 0.0f;
        MBBP_HIP(hipEventElapsedTime(&t, ev.first, ev.second));
        ctx->timed_ms += t;
        ctx->timed_launches += 1;
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    ctx->events.clear();
    *ms = ctx->timed_ms;
    *launches = ctx->timed_launches;
    if (reset) {
        ctx->timed_ms = 0.0;
        ctx->timed_launches = 0;
    }
    return MBBP_OK;
}

mbbp_status mbbp_logicals(mbbp_ctx *ctx, uint64_t *LX, uint64_t *LZ, int32_t *k) {
    if (!ctx || !k) return fail(MBBP_EINVAL, "null argument");
    *k = (int32_t)ctx->LX.size();
    const int W = (ctx->n + 63) / 64;
    if (LX)
        for (size_t r = 0; r < ctx->LX.size(); ++r) std::memcpy(LX + r * W, ctx->LX[r].data(), W * 8);
    if (LZ)
        for (size_t r = 0; r < ctx->LZ.size(); ++r) std::memcpy(LZ + r * W, ctx->LZ[r].data(), W * 8);
    return MBBP_OK;
}

mbbp_status mbbp_edge_counts(mbbp_ctx *ctx, int32_t part, int64_t *edges) {
    if (!ctx || !edges) return fail(MBBP_EINVAL, "null argument");
    if (part != 0 && part != 1) return fail(MBBP_EINVAL, "part must be 0 or 1");
    for (int l = 0; l < ctx->hp[part].L; ++l) edges[l] = ctx->hp[part].E[l];
    return MBBP_OK;
}

mbbp_status mbbp_set_weights(mbbp_ctx *ctx, const float *alpha, const float *beta) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    if ((alpha == nullptr) != (beta == nullptr)) return fail(MBBP_EINVAL, "alpha and beta: both or neither");
    if (ctx->walpha != alpha || ctx->wbeta != beta) drop_graphs(ctx);  // captured launches hold the pointers
    ctx->walpha = alpha;
    ctx->wbeta = beta;
    return MBBP_OK;
}

static mbbp_status wbp_common(mbbp_ctx *ctx, int32_t part, int64_t shots, const void *syn, const void *prior,
                              const float *alpha, const float *beta, int32_t ckpt_every, int &n_ck, int &mpad) {
    if (!ctx) return fail(MBBP_EINVAL, "null ctx");
    if (part != 0 && part != 1) return fail(MBBP_EINVAL, "part must be 0 (X) or 1 (Z)");
    if (shots < 1 || shots > ctx->params.max_batch) return fail(MBBP_EINVAL, "shots out of range");
    if (!syn || !prior || !alpha || !beta) return fail(MBBP_EINVAL, "null device pointer");
    if (ckpt_every < 1) return fail(MBBP_EINVAL, "ckpt_every < 1");
    if (ctx->schedule != MBBP_FLOODING) return fail(MBBP_EUNSUPPORTED, "the weighted rule is built for flooding");
    const int T = ctx->T;
    n_ck = T >= 1 ? (T + ckpt_every - 1) / ckpt_every - 1 : 0;
    mbbp::BPArgs a{};
    a.part[0] = ctx->dp[0];
    a.part[1] = ctx->dp[1];
    a.part0 = part;
    a.nparts = 1;
    if (!mbbp::bp_layout(a, mpad)) return fail(MBBP_EUNSUPPORTED, "code too large for the BP kernel");
    return MBBP_OK;
}

mbbp_status mbbp_wbp_ckpt_floats(mbbp_ctx *ctx, int32_t part, int64_t shots, int32_t ckpt_every, int64_t *floats) {
    if (!floats) return fail(MBBP_EINVAL, "null floats");
    int n_ck = 0, mpad = 0;
    const float one = 0.0f;
    mbbp_status st = wbp_common(ctx, part, shots, &one, &one, &one, &one, ckpt_every, n_ck, mpad);
    if (st != MBBP_OK) return st;
    const int msg = (4 * lds_slots(ctx, part, 1, mpad) * (mpad + mbbp::kSlotPad) + 15) & ~15;
    *floats = shots * (int64_t)ctx->dp[part].L * n_ck * (msg / 4);
    return MBBP_OK;
}

mbbp_status mbbp_wbp_forward(mbbp_ctx *ctx, int32_t part, int64_t shots, const uint64_t *syn, const float *prior,
                             int32_t prior_per_shot, const float *alpha, const float *beta, int32_t ckpt_every,
                             float *ckpt, float *llr, void *hip_stream) {
    int n_ck = 0, mpad = 0;
    mbbp_status st = wbp_common(ctx, part, shots, syn, prior, alpha, beta, ckpt_every, n_ck, mpad);
    if (st != MBBP_OK) return st;
    if (!llr) return fail(MBBP_EINVAL, "null llr");
    if (n_ck > 0 && !ckpt) return fail(MBBP_EINVAL, "null ckpt (checkpoints are needed for this T and interval)");
    WeightedCall wc{alpha, beta, ckpt, ckpt_every, n_ck};
    const uint64_t *sy[2] = {syn, syn};
    const float *pr[2] = {prior, prior};
    float *ll[2] = {llr, llr};
    return run_bp(ctx, part, 1, shots, sy, pr, prior_per_shot ? 1 : 0, ctx->cand, ctx->kstat, ll, false,
                  static_cast<hipStream_t>(hip_stream), &wc);
}

mbbp_status mbbp_wbp_backward(mbbp_ctx *ctx, int32_t part, int64_t shots, const uint64_t *syn, const float *prior,
                              int32_t prior_per_shot, const float *alpha, const float *beta, int32_t ckpt_every,
                              const float *ckpt, const float *grad_llr, float *grad_alpha, float *grad_beta,
                              void *hip_stream) {
    int n_ck = 0, mpad = 0;
    mbbp_status st = wbp_common(ctx, part, shots, syn, prior, alpha, beta, ckpt_every, n_ck, mpad);
    if (st != MBBP_OK) return st;
    if (!grad_llr || !grad_alpha || !grad_beta) return fail(MBBP_EINVAL, "null gradient pointer");
    if (n_ck > 0 && !ckpt) return fail(MBBP_EINVAL, "null ckpt");
    const int T = ctx->T, L = ctx->dp[part].L;
    if (T == 0) return MBBP_OK;
    mbbp::BPArgs ba{};
    ba.part[0] = ctx->dp[0];
    ba.part[1] = ctx->dp[1];
    ba.part0 = part;
    ba.nparts = 1;
    int pv = 0, pc = 0;
    if (!mbbp::bp_passes(ba, pv, pc) || !mbbp::wbp_backward_supported(pv, pc))
        return fail(MBBP_EUNSUPPORTED, "weighted adjoint: code too large (built for n <= 320, <= 320 checks)");
    const mbbp::DevPart &D = ctx->dp[part];
    mbbp::WBPBackArgs a{};
    a.dpart = ctx->dparts + part;
    a.L = L;
    a.T = T;
    a.shots = shots;
    a.n_items = shots * L;
    a.rmax = ctx->params.r_max;
    a.syn = syn;
    a.prior = prior;
    a.prior_per_shot = prior_per_shot ? 1 : 0;
    a.walpha = alpha;
    a.wbeta = beta;
    a.ckpt = ckpt;
    a.ckpt_every = ckpt_every;
    a.n_ck = n_ck;
    a.grad_llr = grad_llr;
    a.ws = D.Ws;
    a.n = D.n;
    const int msg = (4 * lds_slots(ctx, part, 1, mpad) * (mpad + mbbp::kSlotPad) + 15) & ~15;
    const int bytes = (3 + ckpt_every) * msg + D.Ws * 8 + (prior_per_shot ? D.n * 4 : 0);
    a.inst_bytes = (bytes + 15) & ~15;
    int wpb = 4;
    while (wpb > 1 && (size_t)wpb * a.inst_bytes > mbbp::bp_lds_limit()) wpb /= 2;
    if ((size_t)a.inst_bytes > mbbp::bp_lds_limit())
        return fail(MBBP_EUNSUPPORTED, "weighted adjoint: checkpoint interval too long for LDS");
    const size_t need = (size_t)a.n_items * T * sizeof(float2);
    if (need > ctx->gpart_bytes) {
        auto b = std::make_unique<DevBuf>();
        hipError_t e = hipMalloc(&b->p, need);
        if (e != hipSuccess) return fail(MBBP_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        ctx->gpart = std::move(b);
        ctx->gpart_bytes = need;
    }
    a.partial = static_cast<float2 *>(ctx->gpart->p);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipError_t e = mbbp::launch_wbp_backward(a, pv, pc, D.uniform_dc == 6 ? 6 : 8, wpb, s);
    if (e != hipSuccess) return fail(MBBP_EDEVICE, std::string("adjoint launch: ") + hipGetErrorString(e));
    e = mbbp::launch_wbp_reduce(a.partial, shots, T, L, grad_alpha, grad_beta, s);
    if (e != hipSuccess) return fail(MBBP_EDEVICE, std::string("reduce launch: ") + hipGetErrorString(e));
    return MBBP_OK;
}

}  // extern "C"
