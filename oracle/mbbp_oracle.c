/*
 * Plain single-threaded CPU oracle for MBBP-LD (multiple-bases BP list decoding).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call this
 * file; only the tests, the smoke check and the CPU-baseline leg of the bench do.
 * It shares no code with the HIP library.
 *
 * The arithmetic type is REAL: the default build uses double (the FP64 oracle);
 * a second build with -DREAL=float takes every floating-point decision in single
 * precision so that integer outcomes decided by floating point (hard decisions,
 * convergence, list choice) can be compared bit for bit with a single-precision
 * decoder that evaluates the same definitions in the same order.
 *
 * Contents, each following the paper's text:
 *   - orc_subtrees      : maximal cycle-free subtrees (Algorithm 2, Section III-A)
 *   - orc_build_bases   : the L redundant representations [H; H_t] (eq. (3))
 *   - orc_decode        : BP on each [H; H_t] (Section II-B, eqs. (1)-(2), normalized
 *                         min-sum, flooding or serial schedule; sum-product as the
 *                         textbook tanh rule) and the list decision (Algorithm 1,
 *                         Section III-B: least weight, or FWS)
 *   - weighted min-sum  : the differentiable form of the decoder (not in the paper):
 *                         per-iteration, per-representation scaling alpha_{t,l} and
 *                         damping beta_{t,l} of the min-sum check message,
 *                         r^(t) = clamp((1 - beta) * S * alpha * M + beta * r^(t-1)),
 *                         r^(0) = 0 (rule 2 of orc_decode, flooding only)
 *   - orc_failures      : logical failure = residual not a stabilizer (Section II-A)
 *   - orc_philox4x64_10 / orc_sample : counter-based noise (Philox, Salmon et al.,
 *                         SC'11), syndromes s = H e: depolarizing, or X errors only
 *                         (binary symmetric channel, the noise of Section IV)
 *
 * Conventions (readings where the paper is silent):
 *   - Syndrome BP: the check message carries the factor (-1)^{s_j}.
 *   - sgn(x) = -1 if x < 0 else +1; hard decision e_i = 1 iff posterior < 0.
 *   - Check messages are clamped to [-rmax, rmax].
 *   - Variable-to-check messages are exclusion sums mu_i + sum_{j' != j} r_{j'->i}
 *     accumulated in ascending augmented-check order (never P_i - r_{j->i}).
 *   - Serial schedule: augmented checks 0..M-1 in row order, each using the most
 *     recent check messages.
 *   - Halting: tested at t = 0 and after every iteration against the original
 *     checks (the appended rows are implied by them).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef REAL
#define REAL double
#endif
typedef REAL real;

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOTINROWSPACE (-2)
#define ORC_ENOMEM (-3)

/* ------------------------------------------------------------------------- */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the 4x64
 * Philox S-box with multipliers M0, M1 and Weyl key increments W0, W1.        */

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, x0, &hi0, &lo0);
        mulhilo64(M1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Depolarizing thresholds: u < t1 -> X, u < t2 -> Y, u < t3 -> Z, else I,
 * with t_k = floor(k * (p/3) * 2^32) and u a uniform 32-bit word.            */
static void thresholds(double p, uint64_t t[3]) {
    for (int k = 1; k <= 3; ++k) t[k - 1] = (uint64_t)floor((double)k * (p / 3.0) * 4294967296.0);
}

static int words64(int bits) { return (bits + 63) / 64; }

static int getbit(const uint64_t *w, int i) { return (int)((w[i >> 6] >> (i & 63)) & 1u); }
static void setbit(uint64_t *w, int i) { w[i >> 6] |= (uint64_t)1 << (i & 63); }

static int parity_row(const int *cols, int len, const uint64_t *e) {
    int par = 0;
    for (int k = 0; k < len; ++k) par ^= getbit(e, cols[k]);
    return par;
}

/* Qubit q of shot s takes the 32-bit half (q % 2) of output word (q % 8) / 2 of
 * philox(counter = (s, q / 8, 0, 0), key = (seed, 0)).                         */
/* noise 0: depolarizing (thresholds above); noise 1: X errors only, qubit q
 * flipped iff u < floor(p * 2^32), e_Z = 0.                                     */
int orc_sample(int n, int mx, const int *hx_ptr, const int *hx_idx,
               int mz, const int *hz_ptr, const int *hz_idx,
               uint64_t seed, double p, int noise, int64_t shot0, int64_t shots,
               uint64_t *ex, uint64_t *ez, uint64_t *sx, uint64_t *sz) {
    if (n <= 0 || p < 0.0 || p > 1.0 || shots < 0 || (noise != 0 && noise != 1)) return ORC_EINVAL;
    uint64_t t[3];
    thresholds(p, t);
    const uint64_t tb = (uint64_t)floor(p * 4294967296.0);
    int wn = words64(n), wx = words64(mx), wz = words64(mz);
    for (int64_t s = 0; s < shots; ++s) {
        uint64_t *exs = ex + s * wn, *ezs = ez + s * wn;
        memset(exs, 0, sizeof(uint64_t) * (size_t)wn);
        memset(ezs, 0, sizeof(uint64_t) * (size_t)wn);
        uint64_t block[4];
        int last_block = -1;
        for (int q = 0; q < n; ++q) {
            int b = q / 8;
            if (b != last_block) {
                uint64_t ctr[4] = {(uint64_t)(shot0 + s), (uint64_t)b, 0, 0};
                uint64_t key[2] = {seed, 0};
                orc_philox4x64_10(ctr, key, block);
                last_block = b;
            }
            int sub = q % 8;
            uint64_t u = (block[sub / 2] >> (32 * (sub % 2))) & 0xFFFFFFFFULL;
            if (noise == 1) {
                if (u < tb) setbit(exs, q);
            } else if (u < t[0]) {     /* X */
                setbit(exs, q);
            } else if (u < t[1]) {     /* Y = X and Z */
                setbit(exs, q);
                setbit(ezs, q);
            } else if (u < t[2]) {     /* Z */
                setbit(ezs, q);
            }
        }
        /* named by error type: s_X = H_Z e_X (m_Z bits), s_Z = H_X e_Z (m_X bits) */
        uint64_t *sxs = sx + s * wz, *szs = sz + s * wx;
        memset(sxs, 0, sizeof(uint64_t) * (size_t)wz);
        memset(szs, 0, sizeof(uint64_t) * (size_t)wx);
        for (int j = 0; j < mz; ++j)
            if (parity_row(hz_idx + hz_ptr[j], hz_ptr[j + 1] - hz_ptr[j], exs)) setbit(sxs, j);
        for (int j = 0; j < mx; ++j)
            if (parity_row(hx_idx + hx_ptr[j], hx_ptr[j + 1] - hx_ptr[j], ezs)) setbit(szs, j);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* GF(2) row reduction with the combination of original rows tracked, used for
 * row-space membership (bases, failures) and for the syndrome bit of a general
 * appended row h = c^T H, which is c . s.                                      */

typedef struct {
    int m, n, wn, wm;  /* rows, cols, words per row (cols), words per combination */
    int rank;
    uint64_t *row;   /* [rank][wn] reduced rows */
    uint64_t *comb;  /* [rank][wm] which original rows were summed */
    int *pivot;      /* [rank] pivot column of each reduced row */
} gf2_basis;

static void gf2_free(gf2_basis *b) {
    free(b->row); free(b->comb); free(b->pivot);
    memset(b, 0, sizeof(*b));
}

static int gf2_build(gf2_basis *b, int m, int n, const int *ptr, const int *idx) {
    memset(b, 0, sizeof(*b));
    b->m = m; b->n = n; b->wn = words64(n); b->wm = words64(m > 0 ? m : 1);
    uint64_t *R = (uint64_t *)calloc((size_t)(m > 0 ? m : 1) * (size_t)b->wn, sizeof(uint64_t));
    uint64_t *C = (uint64_t *)calloc((size_t)(m > 0 ? m : 1) * (size_t)b->wm, sizeof(uint64_t));
    b->pivot = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    if (!R || !C || !b->pivot) { free(R); free(C); free(b->pivot); return ORC_ENOMEM; }
    for (int j = 0; j < m; ++j) {
        for (int k = ptr[j]; k < ptr[j + 1]; ++k) R[(size_t)j * b->wn + (idx[k] >> 6)] ^= (uint64_t)1 << (idx[k] & 63);
        C[(size_t)j * b->wm + (j >> 6)] |= (uint64_t)1 << (j & 63);
    }
    int r = 0;
    for (int col = 0; col < n && r < m; ++col) {
        int p = -1;
        for (int i = r; i < m; ++i)
            if (getbit(R + (size_t)i * b->wn, col)) { p = i; break; }
        if (p < 0) continue;
        if (p != r) {
            for (int w = 0; w < b->wn; ++w) { uint64_t t = R[(size_t)p * b->wn + w]; R[(size_t)p * b->wn + w] = R[(size_t)r * b->wn + w]; R[(size_t)r * b->wn + w] = t; }
            for (int w = 0; w < b->wm; ++w) { uint64_t t = C[(size_t)p * b->wm + w]; C[(size_t)p * b->wm + w] = C[(size_t)r * b->wm + w]; C[(size_t)r * b->wm + w] = t; }
        }
        for (int i = 0; i < m; ++i) {
            if (i != r && getbit(R + (size_t)i * b->wn, col)) {
                for (int w = 0; w < b->wn; ++w) R[(size_t)i * b->wn + w] ^= R[(size_t)r * b->wn + w];
                for (int w = 0; w < b->wm; ++w) C[(size_t)i * b->wm + w] ^= C[(size_t)r * b->wm + w];
            }
        }
        b->pivot[r] = col;
        ++r;
    }
    b->rank = r;
    b->row = R;
    b->comb = C;
    return ORC_OK;
}

/* Reduce v (wn words, modified in place) by the basis; if comb != NULL it
 * receives the combination of original rows used.  Returns 1 iff v is in the
 * row space.                                                                  */
static int gf2_reduce(const gf2_basis *b, uint64_t *v, uint64_t *comb) {
    if (comb) memset(comb, 0, sizeof(uint64_t) * (size_t)b->wm);
    for (int r = 0; r < b->rank; ++r) {
        if (getbit(v, b->pivot[r])) {
            for (int w = 0; w < b->wn; ++w) v[w] ^= b->row[(size_t)r * b->wn + w];
            if (comb)
                for (int w = 0; w < b->wm; ++w) comb[w] ^= b->comb[(size_t)r * b->wm + w];
        }
    }
    for (int w = 0; w < b->wn; ++w)
        if (v[w]) return 0;
    return 1;
}

int orc_rank(int m, int n, const int *ptr, const int *idx) {
    gf2_basis b;
    if (gf2_build(&b, m, n, ptr, idx) != ORC_OK) return ORC_ENOMEM;
    int r = b.rank;
    gf2_free(&b);
    return r;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 2: maximal subtrees.  check_sets[c] receives the 1-based subtree
 * index of check c; order[] lists the checks in acceptance order (all subtrees
 * concatenated, subtree 1 first); *n_subtrees the number of subtrees.
 * Readings: FIFO queue; neighbours visited in ascending index; eta is counted
 * when a check is dequeued; a check may be queued more than once and is only
 * accepted while unassigned.                                                  */

int orc_subtrees(int m, int n, const int *row_ptr, const int *col_idx,
                 const int *perm, int *check_sets, int *order, int *n_subtrees) {
    if (m <= 0 || n <= 0) return ORC_EINVAL;
    /* column adjacency: checks of each variable, ascending */
    int *vdeg = (int *)calloc((size_t)n + 1, sizeof(int));
    int nnz = row_ptr[m];
    int *vptr = (int *)calloc((size_t)n + 1, sizeof(int));
    int *vchk = (int *)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    int *visited = (int *)malloc(sizeof(int) * (size_t)n);
    int *tested = (int *)malloc(sizeof(int) * (size_t)m);
    /* a check is queued once per (accepted check, shared variable) visit, so
       nnz * (max column degree) + 1 bounds the queue of one subtree */
    int maxcol = 0;
    {
        int *cnt = (int *)calloc((size_t)n, sizeof(int));
        if (cnt) {
            for (int k = 0; k < nnz; ++k) cnt[col_idx[k]]++;
            for (int v = 0; v < n; ++v) if (cnt[v] > maxcol) maxcol = cnt[v];
            free(cnt);
        }
    }
    size_t qcap = (size_t)nnz * (size_t)(maxcol + 1) + 1;
    int *queue = (int *)malloc(sizeof(int) * qcap);
    int *seen = (int *)calloc((size_t)m, sizeof(int));
    if (!vdeg || !vptr || !vchk || !visited || !tested || !queue || !seen) {
        free(vdeg); free(vptr); free(vchk); free(visited); free(tested); free(queue); free(seen);
        return ORC_ENOMEM;
    }
    for (int j = 0; j < m; ++j)
        for (int k = row_ptr[j]; k < row_ptr[j + 1]; ++k) vdeg[col_idx[k]]++;
    for (int v = 0; v < n; ++v) vptr[v + 1] = vptr[v] + vdeg[v];
    memset(vdeg, 0, sizeof(int) * (size_t)n);
    for (int j = 0; j < m; ++j)
        for (int k = row_ptr[j]; k < row_ptr[j + 1]; ++k) {
            int v = col_idx[k];
            vchk[vptr[v] + vdeg[v]++] = j;
        }
    int status = ORC_OK;
    for (int i = 0; i < m; ++i) {
        if (perm[i] < 0 || perm[i] >= m || seen[perm[i]]) { status = ORC_EINVAL; break; }
        seen[perm[i]] = 1;
    }
    int s = 0, n_order = 0;
    if (status == ORC_OK) {
        for (int j = 0; j < m; ++j) check_sets[j] = 0;
        for (int i = 0; i < m; ++i) {
            int c = perm[i];
            if (check_sets[c] != 0) continue;
            s += 1;
            for (int v = 0; v < n; ++v) visited[v] = 0;
            for (int j = 0; j < m; ++j) tested[j] = 0;
            int head = 0, tail = 0;
            queue[tail++] = c;
            while (head < tail) {
                int u = queue[head++];
                tested[u] = 1;
                int eta = 0;
                for (int k = row_ptr[u]; k < row_ptr[u + 1]; ++k) eta += visited[col_idx[k]] ? 1 : 0;
                if (eta <= 1 && check_sets[u] == 0) {
                    check_sets[u] = s;
                    order[n_order++] = u;
                    for (int k = row_ptr[u]; k < row_ptr[u + 1]; ++k) {
                        int v = col_idx[k];
                        visited[v] = 1;
                        for (int t = vptr[v]; t < vptr[v + 1]; ++t) {
                            int c2 = vchk[t];
                            if (!tested[c2] && check_sets[c2] == 0) {
                                if ((size_t)tail >= qcap) {
                                    status = ORC_ENOMEM;
                                    break;
                                }
                                queue[tail++] = c2;
                            }
                        }
                        if (status != ORC_OK) break;
                    }
                }
                if (status != ORC_OK) break;
            }
            if (status != ORC_OK) break;
        }
    }
    *n_subtrees = s;
    free(vdeg); free(vptr); free(vchk); free(visited); free(tested); free(queue); free(seen);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Bases.  mode 0 ("subtrees"): walk pi_0, pi_1, ... (perms[k*m ..]); for each,
 * the subtrees of Algorithm 2 in discovery order, rows in acceptance order;
 * take each subtree whose row set differs from every one already taken, until
 * L are taken.  mode 1 ("ramp"): basis l appends the first
 * r_l = round(l * m / (L - 1)) rows (half rounds up) of pi_l's concatenated
 * acceptance order, so l = 0 is H itself and l = L - 1 is [H; H].
 * Output: basis_ptr[L + 1], rows[] (H row indices).                           */

static int same_set(const int *a, int na, const int *b, int nb, int m, int *mark) {
    if (na != nb) return 0;
    for (int i = 0; i < m; ++i) mark[i] = 0;
    for (int i = 0; i < na; ++i) mark[a[i]] = 1;
    for (int i = 0; i < nb; ++i)
        if (!mark[b[i]]) return 0;
    return 1;
}

int orc_build_bases(int m, int n, const int *row_ptr, const int *col_idx, int mode, int L,
                    int n_perms, const int *perms, int *basis_ptr, int *rows, int rows_cap) {
    if (L <= 0 || n_perms <= 0) return ORC_EINVAL;
    int *cs = (int *)malloc(sizeof(int) * (size_t)m);
    int *ord = (int *)malloc(sizeof(int) * (size_t)m);
    int *mark = (int *)malloc(sizeof(int) * (size_t)m);
    if (!cs || !ord || !mark) { free(cs); free(ord); free(mark); return ORC_ENOMEM; }
    int status = ORC_OK, taken = 0, used = 0;
    basis_ptr[0] = 0;
    if (mode == 0) {
        for (int k = 0; k < n_perms && taken < L && status == ORC_OK; ++k) {
            int ns = 0;
            status = orc_subtrees(m, n, row_ptr, col_idx, perms + (size_t)k * m, cs, ord, &ns);
            if (status != ORC_OK) break;
            int pos = 0;
            for (int s = 1; s <= ns && taken < L; ++s) {
                int start = pos;
                while (pos < m && cs[ord[pos]] == s) ++pos;
                int len = pos - start;
                int dup = 0;
                for (int t = 0; t < taken && !dup; ++t)
                    dup = same_set(rows + basis_ptr[t], basis_ptr[t + 1] - basis_ptr[t], ord + start, len, m, mark);
                if (dup) continue;
                if (used + len > rows_cap) { status = ORC_ENOMEM; break; }
                for (int i = 0; i < len; ++i) rows[used++] = ord[start + i];
                basis_ptr[++taken] = used;
            }
        }
        if (status == ORC_OK && taken < L) status = ORC_EINVAL; /* not enough distinct subtrees */
    } else if (mode == 1) {
        if (n_perms < L) status = ORC_EINVAL;
        for (int l = 0; l < L && status == ORC_OK; ++l) {
            int ns = 0;
            status = orc_subtrees(m, n, row_ptr, col_idx, perms + (size_t)l * m, cs, ord, &ns);
            if (status != ORC_OK) break;
            int r = (L == 1) ? 0 : (int)((2LL * l * m + (L - 1)) / (2LL * (L - 1)));
            if (used + r > rows_cap) { status = ORC_ENOMEM; break; }
            for (int i = 0; i < r; ++i) rows[used++] = ord[i];
            basis_ptr[++taken] = used;
        }
    } else {
        status = ORC_EINVAL;
    }
    free(cs); free(ord); free(mark);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Augmented graph of one representation [H; H_t]. */

typedef struct {
    int m, n, M, E;
    int *cptr, *cvar;   /* check j: variables cvar[cptr[j]..cptr[j+1]) ascending; edge id = position */
    int *vptr, *vedge;  /* var i: edge ids of its checks in ascending check order */
    int *ecol;          /* edge -> variable (same as cvar) */
    uint64_t *comb;     /* [M - m][wm]: original rows summing to each appended row */
    int wm;
} aug_graph;

static void aug_free(aug_graph *g) {
    free(g->cptr); free(g->cvar); free(g->vptr); free(g->vedge); free(g->comb);
    memset(g, 0, sizeof(*g));
}

static int aug_build(aug_graph *g, const gf2_basis *hb, int m, int n, const int *row_ptr, const int *col_idx,
                     int r, const int *app_ptr, const int *app_idx) {
    memset(g, 0, sizeof(*g));
    g->m = m; g->n = n; g->M = m + r; g->wm = hb->wm;
    int E = row_ptr[m] + (r > 0 ? app_ptr[r] - app_ptr[0] : 0);
    g->E = E;
    g->cptr = (int *)malloc(sizeof(int) * (size_t)(g->M + 1));
    g->cvar = (int *)malloc(sizeof(int) * (size_t)(E > 0 ? E : 1));
    g->vptr = (int *)calloc((size_t)n + 1, sizeof(int));
    g->vedge = (int *)malloc(sizeof(int) * (size_t)(E > 0 ? E : 1));
    g->comb = (uint64_t *)calloc((size_t)(r > 0 ? r : 1) * (size_t)g->wm, sizeof(uint64_t));
    if (!g->cptr || !g->cvar || !g->vptr || !g->vedge || !g->comb) { aug_free(g); return ORC_ENOMEM; }
    int e = 0;
    for (int j = 0; j < m; ++j) {
        g->cptr[j] = e;
        for (int k = row_ptr[j]; k < row_ptr[j + 1]; ++k) g->cvar[e++] = col_idx[k];
    }
    uint64_t *v = (uint64_t *)calloc((size_t)hb->wn, sizeof(uint64_t));
    if (!v) { aug_free(g); return ORC_ENOMEM; }
    for (int a = 0; a < r; ++a) {
        g->cptr[m + a] = e;
        memset(v, 0, sizeof(uint64_t) * (size_t)hb->wn);
        for (int k = app_ptr[a]; k < app_ptr[a + 1]; ++k) {
            g->cvar[e++] = app_idx[k];
            setbit(v, app_idx[k]);
        }
        if (!gf2_reduce(hb, v, g->comb + (size_t)a * g->wm)) { free(v); aug_free(g); return ORC_ENOTINROWSPACE; }
    }
    free(v);
    g->cptr[g->M] = e;
    g->ecol = g->cvar;
    for (int k = 0; k < E; ++k) g->vptr[g->cvar[k] + 1]++;
    for (int i = 0; i < n; ++i) g->vptr[i + 1] += g->vptr[i];
    int *fill = (int *)calloc((size_t)n, sizeof(int));
    if (!fill) { aug_free(g); return ORC_ENOMEM; }
    for (int j = 0; j < g->M; ++j)           /* ascending check order */
        for (int k = g->cptr[j]; k < g->cptr[j + 1]; ++k) {
            int i = g->cvar[k];
            g->vedge[g->vptr[i] + fill[i]++] = k;
        }
    free(fill);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Check rules.  Both return the clamped message to variable slot `skip` of a
 * check whose incoming messages are qin[0..d).                                 */

static real clampr(real x, real rmax, int *hit) {
    if (x > rmax) { *hit = 1; return rmax; }
    if (x < -rmax) { *hit = 1; return -rmax; }
    return x;
}

/* normalized min-sum, eq. (1), with syndrome sign */
static real nms_msg(const real *qin, int d, int skip, int sbit, real alpha, real rmax, int *hit, double *msign) {
    real mn = (real)INFINITY;
    int neg = sbit;
    for (int k = 0; k < d; ++k) {
        if (k == skip) continue;
        real a = qin[k] < 0 ? -qin[k] : qin[k];
        if ((double)a < *msign) *msign = (double)a;
        if (a < mn) mn = a;
        if (qin[k] < 0) neg ^= 1;
    }
    real mag = alpha * mn;
    real r = neg ? -mag : mag;
    return clampr(r, rmax, hit);
}

/* Weighted normalized min-sum with damping: the message is
 * clamp((1 - beta) * v + beta * rprev) with v = S * (alpha * M), S the
 * syndrome-signed product of the other slots' signs and M the smallest magnitude
 * among them; rprev is the same edge's message of the previous iteration.
 * *kink receives the smallest distance seen from a point where this map is not
 * smooth: a sign change (|q| = 0), a change of the minimizing slot (the gap
 * between the two smallest magnitudes among the other slots) or the clamp bound.
 * The first two count only when the incoming messages depend on the weights
 * (qvar != 0, i.e. from iteration 2 on; at iteration 1 they are the priors).  */
static real wnms_msg(const real *qin, int d, int skip, int sbit, real alpha, real beta, real rprev, real rmax,
                     int qvar, int *hit, double *kink) {
    real mn = (real)INFINITY, mn2 = (real)INFINITY;
    int neg = sbit;
    for (int k = 0; k < d; ++k) {
        if (k == skip) continue;
        real a = qin[k] < 0 ? -qin[k] : qin[k];
        if (qvar && (double)a < *kink) *kink = (double)a;
        if (a < mn) { mn2 = mn; mn = a; }
        else if (a < mn2) mn2 = a;
        if (qin[k] < 0) neg ^= 1;
    }
    if (qvar && d > 2 && (double)mn2 - (double)mn < *kink) *kink = (double)mn2 - (double)mn;
    real u = alpha * mn;
    real v = neg ? -u : u;
    real keep = (real)1 - beta;
    real wsum = keep * v + beta * rprev;
    double dist = fabs(fabs((double)wsum) - (double)rmax);
    if (dist < *kink) *kink = dist;
    return clampr(wsum, rmax, hit);
}

/* Sum-product (tanh rule, Section II-B): the magnitude of the message to slot
 * `skip` is phi(S) with S = sum over the other slots of phi(|q|), where
 * phi(x) = ln((e^x + 1) / (e^x - 1)) = ln coth(x / 2), its own inverse, phi(0) = inf,
 * phi(inf) = 0; equivalently 2 atanh(prod tanh(|q| / 2)).
 *
 * The magnitudes reach r_max (2^16), far beyond where e^-x is representable, and
 * the message there is about the smallest |q| (exactly min |q| - ln(1 + ...)), not
 * r_max.  So the sum is taken in the log domain: ln phi(x) per slot, S through a
 * log-sum-exp, and phi(S) from ln S.  Every branch below is the same function;
 * the cut-offs only choose the form whose terms stay representable, and the
 * neglected terms are below 1e-26 relative.                                      */
#if defined(ORACLE_SINGLE) /* set together with -DREAL=float */
#define RLOG logf
#define REXP expf
#define RLOG1P log1pf
#define REXPM1 expm1f
#define RLN2 0.69314718f
#else
#define RLOG log
#define REXP exp
#define RLOG1P log1p
#define REXPM1 expm1
#define RLN2 0.69314718055994531
#endif

/* ln phi(x), x > 0: phi(x) = log1p(v) with v = 2 / expm1(x), and
 * ln v = ln 2 - x - log1p(-e^-x); for v < e^-30, ln log1p(v) = ln v - v/2 + O(v^2). */
static real ln_phi(real x) {
    if (x <= 0) return (real)INFINITY;
    real lnv = RLN2 - x - RLOG1P(-REXP(-x));
    if (lnv > (real)-30) return RLOG(RLOG1P(REXP(lnv)));
    return lnv - (real)0.5 * REXP(lnv);
}

/* phi(S) given ln S: direct for moderate S (underflowing to 0 once phi(S) < 1e-300
 * is below every representable magnitude of interest); for S < e^-30,
 * phi(S) = ln(2 / S) + S^2 / 12 + O(S^4).                                        */
static real phi_from_ln(real lnS) {
    if (lnS == (real)INFINITY) return 0;
    if (lnS > (real)-30) return RLOG1P((real)2 / REXPM1(REXP(lnS)));
    return RLN2 - lnS + REXP((real)2 * lnS) / (real)12;
}

/* sum-product (tanh rule): sign product times phi(sum phi(|q|)), with syndrome sign */
static real spa_msg(const real *qin, int d, int skip, int sbit, real rmax, int *hit, double *msign) {
    real lp[64];
    real lmax = -(real)INFINITY;
    int neg = sbit, cnt = 0;
    for (int k = 0; k < d; ++k) {
        if (k == skip) continue;
        real a = qin[k] < 0 ? -qin[k] : qin[k];
        if ((double)a < *msign) *msign = (double)a;
        lp[cnt] = ln_phi(a);
        if (lp[cnt] > lmax) lmax = lp[cnt];
        ++cnt;
        if (qin[k] < 0) neg ^= 1;
    }
    real lnS;
    if (cnt == 0 || lmax == (real)INFINITY) {
        lnS = lmax;  /* no other slot: phi(-inf) handled below; a zero |q|: S = inf */
    } else {
        real acc = 0;
        for (int k = 0; k < cnt; ++k) acc += REXP(lp[k] - lmax);
        lnS = lmax + RLOG(acc);
    }
    real mag = cnt == 0 ? (real)INFINITY : phi_from_ln(lnS);
    real r = neg ? -mag : mag;
    return clampr(r, rmax, hit);
}

/* ------------------------------------------------------------------------- */
/* BP on one representation for one syndrome.
 * schedule: 0 flooding, 1 serial (layered).  rule: 0 normalized min-sum, 1 sum-product,
 * 2 weighted min-sum with damping (flooding only; wa[t-1], wb[t-1] are the weights
 * of iteration t).
 * fixed_T: run exactly T iterations (diagnostic); *K then holds the first
 * iteration at which the syndrome was met (T if never) and dec/P the state after T. */

typedef struct {
    real *q, *r, *P, *qin, *rout;
    uint8_t *dec;
} bp_work;

static int syndrome_met(const aug_graph *g, const uint8_t *dec, const uint8_t *sb) {
    for (int j = 0; j < g->m; ++j) {
        int par = sb[j];
        for (int k = g->cptr[j]; k < g->cptr[j + 1]; ++k) par ^= dec[g->cvar[k]];
        if (par) return 0;
    }
    return 1;
}

static void bp_one(const aug_graph *g, const uint8_t *sb, const real *mu, int T, int schedule, int rule,
                   real alpha, real rmax, int fixed_T, const real *wa, const real *wb, bp_work *w,
                   int *K_out, int *conv_out, double *m_sign, double *m_dec, int *clamp_hit) {
    const int n = g->n, M = g->M;
    double msign = INFINITY, mdec = INFINITY;
    int hit = 0, conv = 0, K = T;
    for (int i = 0; i < n; ++i) {
        w->P[i] = mu[i];
        w->dec[i] = mu[i] < 0;
        double a = fabs((double)mu[i]);
        if (a < mdec) mdec = a;
    }
    if (syndrome_met(g, w->dec, sb)) { conv = 1; K = 0; }
    if (!conv || fixed_T) {
        for (int e = 0; e < g->E; ++e) { w->q[e] = mu[g->ecol[e]]; w->r[e] = 0; }
        for (int t = 1; t <= T; ++t) {
            if (schedule == 0) {
                /* flooding: all check messages from the previous v->c messages */
                for (int j = 0; j < M; ++j) {
                    int d = g->cptr[j + 1] - g->cptr[j];
                    for (int k = 0; k < d; ++k) w->qin[k] = w->q[g->cptr[j] + k];
                    for (int k = 0; k < d; ++k) {
                        real *re = &w->r[g->cptr[j] + k];
                        *re = rule == 0 ? nms_msg(w->qin, d, k, sb[j], alpha, rmax, &hit, &msign)
                            : rule == 1 ? spa_msg(w->qin, d, k, sb[j], rmax, &hit, &msign)
                                        : wnms_msg(w->qin, d, k, sb[j], wa[t - 1], wb[t - 1], *re, rmax, t > 1,
                                                   &hit, &msign);
                    }
                }
                /* variables: posterior and exclusion sums, ascending check order */
                for (int i = 0; i < n; ++i) {
                    int a0 = g->vptr[i], a1 = g->vptr[i + 1];
                    real P = mu[i];
                    for (int a = a0; a < a1; ++a) P += w->r[g->vedge[a]];
                    w->P[i] = P;
                    w->dec[i] = P < 0;
                    for (int a = a0; a < a1; ++a) {
                        real qq = mu[i];
                        for (int b = a0; b < a1; ++b)
                            if (b != a) qq += w->r[g->vedge[b]];
                        w->q[g->vedge[a]] = qq;
                    }
                }
            } else {
                /* serial: checks in augmented row order, each seeing the latest r */
                for (int j = 0; j < M; ++j) {
                    int d = g->cptr[j + 1] - g->cptr[j];
                    for (int k = 0; k < d; ++k) {
                        int e = g->cptr[j] + k, i = g->cvar[e];
                        real qq = mu[i];
                        for (int b = g->vptr[i]; b < g->vptr[i + 1]; ++b)
                            if (g->vedge[b] != e) qq += w->r[g->vedge[b]];
                        w->qin[k] = qq;
                    }
                    for (int k = 0; k < d; ++k)
                        w->rout[k] = rule == 0 ? nms_msg(w->qin, d, k, sb[j], alpha, rmax, &hit, &msign)
                                               : spa_msg(w->qin, d, k, sb[j], rmax, &hit, &msign);
                    for (int k = 0; k < d; ++k) w->r[g->cptr[j] + k] = w->rout[k];
                }
                for (int i = 0; i < n; ++i) {
                    real P = mu[i];
                    for (int a = g->vptr[i]; a < g->vptr[i + 1]; ++a) P += w->r[g->vedge[a]];
                    w->P[i] = P;
                    w->dec[i] = P < 0;
                }
            }
            for (int i = 0; i < n; ++i) {
                double a = fabs((double)w->P[i]);
                if (a < mdec) mdec = a;
            }
            if (!conv && syndrome_met(g, w->dec, sb)) {
                conv = 1;
                K = t;
                if (!fixed_T) break;
            }
        }
    }
    *K_out = K;
    *conv_out = conv;
    if (m_sign) *m_sign = msign;
    if (m_dec) *m_dec = mdec;
    if (clamp_hit) *clamp_hit = hit;
}

/* ------------------------------------------------------------------------- */
/* Decision rules over the list of converged candidates (Section III-B).
 * select_rule 0: least Hamming weight, ties to the smaller basis index.
 * select_rule 1: FWS, argmax count(e) / (w(e) + 1) compared exactly as
 *   cnt_a * (w_b + 1) vs cnt_b * (w_a + 1); ties to the smaller index of first
 *   occurrence.  No converged candidate: failure, all-zero output, index -1.    */

static int popcount_words(const uint64_t *v, int w) {
    int c = 0;
    for (int i = 0; i < w; ++i) c += __builtin_popcountll(v[i]);
    return c;
}

static int select_one(int L, int wn, const uint64_t *cand, const uint8_t *conv, int rule) {
    int best = -1;
    if (rule == 0) {
        int bw = 0;
        for (int l = 0; l < L; ++l) {
            if (!conv[l]) continue;
            int wt = popcount_words(cand + (size_t)l * wn, wn);
            if (best < 0 || wt < bw) { best = l; bw = wt; }
        }
    } else {
        long bc = 0, bw1 = 1;
        for (int l = 0; l < L; ++l) {
            if (!conv[l]) continue;
            int first = 1;  /* is l the first occurrence of its candidate? */
            for (int k = 0; k < l && first; ++k)
                if (conv[k] && memcmp(cand + (size_t)k * wn, cand + (size_t)l * wn, sizeof(uint64_t) * (size_t)wn) == 0) first = 0;
            if (!first) continue;
            long cnt = 0;
            for (int k = 0; k < L; ++k)
                if (conv[k] && memcmp(cand + (size_t)k * wn, cand + (size_t)l * wn, sizeof(uint64_t) * (size_t)wn) == 0) ++cnt;
            long w1 = popcount_words(cand + (size_t)l * wn, wn) + 1;
            if (best < 0 || cnt * bw1 > bc * w1) { best = l; bc = cnt; bw1 = w1; }
        }
    }
    return best;
}

/* ------------------------------------------------------------------------- */
/* Decode `shots` syndromes of one parity-check matrix H (m x n, CSR) with L
 * representations [H; H_l].  Appended rows are given explicitly: basis l owns
 * appended rows basis_ptr[l]..basis_ptr[l+1] of the CSR (app_ptr, app_idx).
 *
 * prior: [n] (prior_per_shot == 0) or [shots][n] LLRs.
 * syn:   [shots][ceil(m/64)] bit-packed, LSB first.
 * Outputs (any may be NULL except chosen/corr):
 *   cand   [shots][L][ceil(n/64)]  candidate of every basis
 *   K      [shots][L]              iterations used
 *   conv   [shots][L]              converged flags
 *   llr    [shots][L][n]           posteriors at stop (or after T if fixed_T)
 *   margin [shots][L][2]           min |q| at sign evaluations, min |P| at decisions
 *   clamp  [shots][L]              1 if the clamp bound
 *   chosen [shots]                 selected basis or -1
 *   corr   [shots][ceil(n/64)]     selected correction
 * Rule 2 (weighted min-sum) takes walpha, wbeta [T][L] (iteration t = 1..T at row
 * t - 1) and reports in margin[0] the distance to the nearest non-smooth point of
 * the forward map instead of the smallest |q|.                                  */

int orc_decode(int m, int n, const int *row_ptr, const int *col_idx,
               int L, const int *basis_ptr, const int *app_ptr, const int *app_idx,
               int T, int schedule, int rule, double alpha, double rmax, int fixed_T,
               int64_t shots, const double *prior, int prior_per_shot, const uint64_t *syn,
               uint64_t *cand, int32_t *K, uint8_t *conv, double *llr, double *margin, uint8_t *clamp,
               int select_rule, int32_t *chosen, uint64_t *corr, const double *walpha, const double *wbeta) {
    if (m <= 0 || n <= 0 || L <= 0 || T < 0 || shots < 0) return ORC_EINVAL;
    if (schedule < 0 || schedule > 1 || rule < 0 || rule > 2) return ORC_EINVAL;
    if (rule == 2 && (schedule != 0 || !walpha || !wbeta)) return ORC_EINVAL;
    for (int j = 0; j < m; ++j)
        if (row_ptr[j + 1] - row_ptr[j] < 2) return ORC_EINVAL;
    gf2_basis hb;
    int status = gf2_build(&hb, m, n, row_ptr, col_idx);
    if (status != ORC_OK) return status;
    aug_graph *g = (aug_graph *)calloc((size_t)L, sizeof(aug_graph));
    if (!g) { gf2_free(&hb); return ORC_ENOMEM; }
    int maxE = 0, maxM = 0, maxd = 0;
    for (int l = 0; l < L && status == ORC_OK; ++l) {
        int r = basis_ptr[l + 1] - basis_ptr[l];
        status = aug_build(&g[l], &hb, m, n, row_ptr, col_idx, r, app_ptr + basis_ptr[l], app_idx);
        if (status == ORC_OK) {
            if (g[l].E > maxE) maxE = g[l].E;
            if (g[l].M > maxM) maxM = g[l].M;
            for (int j = 0; j < g[l].M; ++j) {
                int d = g[l].cptr[j + 1] - g[l].cptr[j];
                if (d < 2) status = ORC_EINVAL;
                if (d > maxd) maxd = d;
            }
        }
    }
    if (status == ORC_OK && maxd > 64) status = ORC_EINVAL; /* spa_msg keeps one slot buffer of 64 */
    int wn = words64(n), ws = words64(m);
    bp_work w;
    w.q = (real *)malloc(sizeof(real) * (size_t)(maxE + 1));
    w.r = (real *)malloc(sizeof(real) * (size_t)(maxE + 1));
    w.P = (real *)malloc(sizeof(real) * (size_t)n);
    w.qin = (real *)malloc(sizeof(real) * (size_t)(maxd + 1));
    w.rout = (real *)malloc(sizeof(real) * (size_t)(maxd + 1));
    w.dec = (uint8_t *)malloc((size_t)n);
    real *mu = (real *)malloc(sizeof(real) * (size_t)n);
    uint8_t *sb = (uint8_t *)malloc((size_t)(maxM + 1));
    uint64_t *cl = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)L * (size_t)wn);
    uint8_t *cv = (uint8_t *)malloc((size_t)L);
    real *wa = (real *)malloc(sizeof(real) * (size_t)(T + 1));
    real *wb = (real *)malloc(sizeof(real) * (size_t)(T + 1));
    if (!w.q || !w.r || !w.P || !w.qin || !w.rout || !w.dec || !mu || !sb || !cl || !cv || !wa || !wb)
        status = ORC_ENOMEM;
    const real ralpha = (real)alpha, rrmax = (real)rmax;
    for (int64_t s = 0; s < shots && status == ORC_OK; ++s) {
        const double *pr = prior + (prior_per_shot ? (size_t)s * n : 0);
        for (int i = 0; i < n; ++i) mu[i] = (real)pr[i];
        const uint64_t *ss = syn + (size_t)s * ws;
        for (int l = 0; l < L; ++l) {
            const aug_graph *gl = &g[l];
            for (int j = 0; j < m; ++j) sb[j] = (uint8_t)getbit(ss, j);
            for (int a = 0; a < gl->M - m; ++a) {
                int par = 0;
                const uint64_t *cb = gl->comb + (size_t)a * gl->wm;
                for (int j = 0; j < m; ++j)
                    if (getbit(cb, j)) par ^= sb[j];
                sb[m + a] = (uint8_t)par;
            }
            if (rule == 2)
                for (int t = 0; t < T; ++t) {
                    wa[t] = (real)walpha[(size_t)t * L + l];
                    wb[t] = (real)wbeta[(size_t)t * L + l];
                }
            int k = 0, c = 0, hit = 0;
            double ms = 0, md = 0;
            bp_one(gl, sb, mu, T, schedule, rule, ralpha, rrmax, fixed_T, wa, wb, &w, &k, &c, &ms, &md, &hit);
            uint64_t *cw = cl + (size_t)l * wn;
            memset(cw, 0, sizeof(uint64_t) * (size_t)wn);
            for (int i = 0; i < n; ++i)
                if (w.dec[i]) setbit(cw, i);
            cv[l] = (uint8_t)c;
            size_t sl = (size_t)s * L + l;
            if (cand) memcpy(cand + sl * wn, cw, sizeof(uint64_t) * (size_t)wn);
            if (K) K[sl] = k;
            if (conv) conv[sl] = (uint8_t)c;
            if (llr)
                for (int i = 0; i < n; ++i) llr[sl * n + i] = (double)w.P[i];
            if (margin) { margin[sl * 2] = ms; margin[sl * 2 + 1] = md; }
            if (clamp) clamp[sl] = (uint8_t)hit;
        }
        int best = select_one(L, wn, cl, cv, select_rule);
        chosen[s] = best;
        uint64_t *co = corr + (size_t)s * wn;
        if (best >= 0) memcpy(co, cl + (size_t)best * wn, sizeof(uint64_t) * (size_t)wn);
        else memset(co, 0, sizeof(uint64_t) * (size_t)wn);
    }
    free(w.q); free(w.r); free(w.P); free(w.qin); free(w.rout); free(w.dec);
    free(mu); free(sb); free(cl); free(cv); free(wa); free(wb);
    for (int l = 0; l < L; ++l) aug_free(&g[l]);
    free(g);
    gf2_free(&hb);
    return status;
}

/* Number of edges of each representation [H; H_l]: nnz(H) + nnz(appended rows). */
int orc_edge_counts(int m, const int *row_ptr, int L, const int *basis_ptr, const int *app_ptr, int *E) {
    for (int l = 0; l < L; ++l) E[l] = row_ptr[m] + (app_ptr[basis_ptr[l + 1]] - app_ptr[basis_ptr[l]]);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Logical failure of one error type: the residual rho = err ^ corr must be a
 * product of stabilizers of the same type, i.e. lie in the row space of S
 * (S = H_X for X errors, H_Z for Z errors).  fail[s] = 1 otherwise.          */

int orc_failures(int ms, int n, const int *s_ptr, const int *s_idx, int64_t shots,
                 const uint64_t *err, const uint64_t *corr, uint8_t *fail) {
    gf2_basis b;
    int status = gf2_build(&b, ms, n, s_ptr, s_idx);
    if (status != ORC_OK) return status;
    int wn = words64(n);
    uint64_t *v = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)wn);
    if (!v) { gf2_free(&b); return ORC_ENOMEM; }
    for (int64_t s = 0; s < shots; ++s) {
        for (int w = 0; w < wn; ++w) v[w] = err[(size_t)s * wn + w] ^ corr[(size_t)s * wn + w];
        fail[s] = (uint8_t)(gf2_reduce(&b, v, NULL) ? 0 : 1);
    }
    free(v);
    gf2_free(&b);
    return ORC_OK;
}

/* Membership of explicit rows in the row space of H (1 = member).  */
int orc_in_rowspace(int m, int n, const int *ptr, const int *idx, int nrows, const int *q_ptr,
                    const int *q_idx, uint8_t *member) {
    gf2_basis b;
    int status = gf2_build(&b, m, n, ptr, idx);
    if (status != ORC_OK) return status;
    uint64_t *v = (uint64_t *)calloc((size_t)b.wn, sizeof(uint64_t));
    if (!v) { gf2_free(&b); return ORC_ENOMEM; }
    for (int a = 0; a < nrows; ++a) {
        memset(v, 0, sizeof(uint64_t) * (size_t)b.wn);
        for (int k = q_ptr[a]; k < q_ptr[a + 1]; ++k) v[q_idx[k] >> 6] ^= (uint64_t)1 << (q_idx[k] & 63);
        member[a] = (uint8_t)gf2_reduce(&b, v, NULL);
    }
    free(v);
    gf2_free(&b);
    return ORC_OK;
}

int orc_real_bytes(void) { return (int)sizeof(real); }

/* The decision rule alone, on given lists: cand [shots][L][wn], conv [shots][L]. */
int orc_select(int L, int wn, int64_t shots, const uint64_t *cand, const uint8_t *conv, int rule,
               int32_t *chosen) {
    if (L <= 0 || wn <= 0 || rule < 0 || rule > 1) return ORC_EINVAL;
    for (int64_t s = 0; s < shots; ++s)
        chosen[s] = select_one(L, wn, cand + (size_t)s * L * wn, conv + (size_t)s * L, rule);
    return ORC_OK;
}
