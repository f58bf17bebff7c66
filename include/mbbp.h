/*
 * mbbp.h -- C ABI of the MI355X (gfx950) multiple-bases BP list decoder (MBBP-LD)
 * for CSS quantum LDPC codes.
 *
 * Method (Sections II-III of the MBBP-LD paper):
 *   - A CSS code has parity-check matrices H_X, H_Z with H_X H_Z^T = 0
 *     (Section II-A).  X errors e_X are seen by H_Z, Z errors e_Z by H_X.
 *   - L redundant representations [H; H_t] of each matrix are built from maximal
 *     cycle-free subtrees of the Tanner graph (Algorithm 2, eq. (3)).
 *   - BP (normalized min-sum, eqs. (1)-(2), or sum-product) runs on every
 *     representation; converged estimates form a list (Algorithm 1) from which a
 *     decision rule picks one (Section III-B: least weight, or FWS); if nothing
 *     converges the estimate is all-zero and the shot is a failure.
 *
 * Naming: everything is named by the ERROR TYPE it concerns.
 *   part X : e_X, syndrome s_X = H_Z e_X (m_Z bits), decoded on representations
 *            of H_Z, correction corr_x; logical failure iff e_X ^ corr_x is not in
 *            the row space of H_X.
 *   part Z : e_Z, s_Z = H_X e_Z (m_X bits), representations of H_X, corr_z;
 *            failure iff e_Z ^ corr_z is not in the row space of H_Z.
 *
 * Layouts: bit vectors are uint64 words, bit i in word i/64 at position i%64
 * (LSB first); per-shot arrays are [shots][words] row-major.  Device pointers
 * are HIP device memory owned by the caller; host pointers are plain memory
 * owned by the caller.  All device work is enqueued on the given hipStream_t
 * (passed as void*, NULL = default stream) and is asynchronous; outputs are
 * valid once the stream has been synchronised.
 *
 * Errors: every call returns mbbp_status; no C++ exception crosses the ABI.
 * Arguments are validated on the host before anything is enqueued, and on
 * error no output is written.  mbbp_last_error() gives a thread-local message
 * for the most recent non-OK status.  A device fault surfaces as MBBP_EDEVICE.
 */
#ifndef MBBP_H
#define MBBP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mbbp_ctx mbbp_ctx;

typedef enum {
    MBBP_OK = 0,
    MBBP_EINVAL = -1,          /* bad argument (shape, pointer, range, H_X H_Z^T != 0, ...) */
    MBBP_ENOTINROWSPACE = -2,  /* an explicit appended row is not in the row space of H */
    MBBP_ENOMEM = -3,          /* host or device allocation failed */
    MBBP_EDEVICE = -4,         /* a HIP call failed (message names it) */
    MBBP_EUNSUPPORTED = -5,    /* beyond the implementation's limits (listed below) */
    MBBP_EABORTED = -6         /* a persistent launch saw the abort flag */
} mbbp_status;

typedef enum { MBBP_FLOODING = 0, MBBP_LAYERED = 1 } mbbp_schedule;  /* Section II-B */
/* eq. (1) / tanh rule / weighted min-sum with damping (see mbbp_set_weights) */
typedef enum { MBBP_NMS = 0, MBBP_SPA = 1, MBBP_WEIGHTED = 2 } mbbp_rule;
typedef enum { MBBP_MIN_WEIGHT = 0, MBBP_FWS = 1 } mbbp_select_rule; /* Section III-B */
typedef enum { MBBP_PART_X = 0, MBBP_PART_Z = 1 } mbbp_part;

/* Host CSR of a 0/1 matrix: row r has columns col_idx[row_ptr[r] .. row_ptr[r+1]),
 * 0-based, strictly ascending. */
typedef struct {
    int32_t rows, cols;
    const int32_t *row_ptr;
    const int32_t *col_idx;
} mbbp_sparse;

/* The L representations of one matrix H (eq. (3)): representation l is H with
 * the rows rows[basis_ptr[l] .. basis_ptr[l+1]) appended in that order.  An
 * entry r >= 0 duplicates row r of H; an entry r < 0 appends row (-r - 1) of
 * `extra`, which must lie in the row space of H (checked by GF(2) elimination;
 * its syndrome bit is then the matching sum of syndrome bits). */
typedef struct {
    int32_t L;
    const int32_t *basis_ptr;  /* [L + 1], basis_ptr[0] = 0, non-decreasing */
    const int32_t *rows;       /* [basis_ptr[L]] */
    const mbbp_sparse *extra;  /* may be NULL when no entry is negative */
} mbbp_basis_list;

typedef struct {
    mbbp_basis_list hx;  /* representations of H_X (used by part Z) */
    mbbp_basis_list hz;  /* representations of H_Z (used by part X) */
} mbbp_bases;

#define MBBP_FLAG_FIXED_T 1u  /* diagnostic: run exactly T iterations, no early stop */
/* One BP instance per wavefront everywhere.  By default flooding min-sum with early
 * stop and one prior vector runs two instances (two shots of a representation) per
 * wavefront; results are identical either way (for comparison and testing). */
#define MBBP_FLAG_ONE_PER_WAVE 2u

typedef struct {
    int32_t rule;        /* mbbp_rule, default MBBP_NMS; MBBP_WEIGHTED needs MBBP_FLOODING */
    float alpha;         /* normalisation of eq. (1), default 0.875 (Section IV); unused by SPA */
    float r_max;         /* check messages are clamped to [-r_max, r_max], default 65536 */
    int32_t select;      /* mbbp_select_rule, default MBBP_MIN_WEIGHT */
    int64_t max_batch;   /* largest `shots` of any later call (sizes the workspace), default 1<<20 */
    uint32_t flags;      /* MBBP_FLAG_* */
} mbbp_params;

/* Fill *p with the defaults above. */
mbbp_status mbbp_params_default(mbbp_params *p);

/* Build a decoder (host preprocessing + device upload, synchronous).
 * H_X (m_X x n) and H_Z (m_Z x n) must satisfy H_X H_Z^T = 0 (Section II-A).
 * T >= 0 is the iteration cap (I_max of Section IV), schedule an mbbp_schedule.
 * Everything is deep-copied; the caller may free its arrays on return.
 * Limits (MBBP_EUNSUPPORTED): row weight of every representation in [2, 8]
 * (weight < 2 is MBBP_EINVAL), column weight <= 8, 1 <= L <= 64, n <= 1024,
 * T <= 32767.  Uses the current HIP device. */
mbbp_status mbbp_create(const mbbp_sparse *H_X, const mbbp_sparse *H_Z, const mbbp_bases *bases,
                        int32_t T, int32_t schedule, const mbbp_params *params, mbbp_ctx **out);

/* Release the decoder and its device memory (synchronises its work first). */
void mbbp_destroy(mbbp_ctx *ctx);

/* Decode `shots` syndrome pairs (Algorithm 1 for both parts).
 * syn_x   device [shots][ceil(m_Z/64)]   s_X = H_Z e_X
 * syn_z   device [shots][ceil(m_X/64)]   s_Z = H_X e_Z
 * prior_x device float [n] (prior_per_shot = 0) or [shots][n]: LLR log((1-q)/q)
 * prior_z likewise (Section II-B initialisation)
 * corr_x, corr_z device [shots][ceil(n/64)]   chosen estimate (all-zero if none converged)
 * conv_x, conv_z device uint64 [shots]  bit l set iff representation l converged
 * basis_x, basis_z device int16 [shots] chosen representation, -1 if none converged
 * 0 < shots <= max_batch.  Deterministic: identical inputs give identical bits. */
mbbp_status mbbp_decode(mbbp_ctx *ctx, int64_t shots,
                        const uint64_t *syn_x, const uint64_t *syn_z,
                        const float *prior_x, const float *prior_z, int32_t prior_per_shot,
                        uint64_t *corr_x, uint64_t *corr_z,
                        uint64_t *conv_x, uint64_t *conv_z,
                        int16_t *basis_x, int16_t *basis_z, void *hip_stream);

/* One part, every representation's own result (for inspection and parity):
 * cand  device [shots][L][ceil(n/64)]  hard decision of each representation at its stop
 * kstat device uint16 [shots][L]       iterations used (low 15 bits), bit 15 = converged
 * llr   device float [shots][L][n] or NULL: posteriors at the stop (after T with FIXED_T)
 * Same syndrome/prior conventions as mbbp_decode. */
mbbp_status mbbp_decode_detail(mbbp_ctx *ctx, int32_t part, int64_t shots, const uint64_t *syn,
                               const float *prior, int32_t prior_per_shot,
                               uint64_t *cand, uint16_t *kstat, float *llr, void *hip_stream);

/* Noise models of mbbp_sample, mbbp_run and mbbp_autotune (per context, set with
 * mbbp_set_noise; default MBBP_NOISE_DEPOLARIZING).  MBBP_NOISE_X_ONLY is the
 * binary symmetric channel on X errors of the paper's experiments (Section IV):
 * each qubit suffers an X error with probability p, never Z.
 * MBBP_EINVAL for any other value; a null ctx is MBBP_EINVAL. */
enum { MBBP_NOISE_DEPOLARIZING = 0, MBBP_NOISE_X_ONLY = 1 };
mbbp_status mbbp_set_noise(mbbp_ctx *ctx, int32_t model);

/* Counter-based code-capacity noise: qubit q of shot s uses the 32-bit half (q%2)
 * of word (q%8)/2 of Philox4x64-10(counter = (s, q/8, 0, 0), key = (seed, 0))
 * [Salmon et al. SC'11].  Depolarizing (X, Y, Z each with probability p/3):
 * u < t1 -> X, u < t2 -> Y, u < t3 -> Z with t_k = floor(k * (p/3) * 2^32) in
 * double precision.  X only: X iff u < floor(p * 2^32), e_Z = 0.  Shots are
 * indexed shot0 .. shot0 + shots - 1.
 * err_x, err_z device [shots][ceil(n/64)]; syn_x = H_Z e_X, syn_z = H_X e_Z as above.
 * 0 <= p <= 1, 0 < shots <= max_batch. */
mbbp_status mbbp_sample(mbbp_ctx *ctx, uint64_t seed, double p, int64_t shot0, int64_t shots,
                        uint64_t *err_x, uint64_t *err_z, uint64_t *syn_x, uint64_t *syn_z,
                        void *hip_stream);

/* Logical-failure test (Section II-A): fail[s] bit 0 = part X failed
 * (residual e_X ^ corr_x not a stabilizer: H_Z r != 0 or L_Z r != 0), bit 1 = part Z.
 * All pointers device memory, [shots][ceil(n/64)] and uint8 [shots]. */
mbbp_status mbbp_failures(mbbp_ctx *ctx, int64_t shots, const uint64_t *err_x, const uint64_t *err_z,
                          const uint64_t *corr_x, const uint64_t *corr_z, uint8_t *fail,
                          void *hip_stream);

/* The batched form of mbbp_decode: one persistent launch over a work queue of
 * (part, representation, shot chunk) items of uneven size, with per-instance
 * early exit and refill.  Outputs are bit-identical to mbbp_decode. */
mbbp_status mbbp_decode_batched(mbbp_ctx *ctx, int64_t shots,
                                const uint64_t *syn_x, const uint64_t *syn_z,
                                const float *prior_x, const float *prior_z, int32_t prior_per_shot,
                                uint64_t *corr_x, uint64_t *corr_z,
                                uint64_t *conv_x, uint64_t *conv_z,
                                int16_t *basis_x, int16_t *basis_z, void *hip_stream);

/* Counter indices of mbbp_run. */
enum {
    MBBP_CNT_FAIL = 0,        /* shots with a logical failure in either part */
    MBBP_CNT_FAIL_X = 1,
    MBBP_CNT_FAIL_Z = 2,
    MBBP_CNT_SUM_KMAX = 3,    /* sum over shots of max iterations over all 2L instances */
    MBBP_CNT_SUM_K = 4,       /* sum over (shot, part, representation) of iterations */
    MBBP_CNT_EDGE_UPDATES = 5,/* sum of iterations x edges of that representation */
    MBBP_CNT_NOCONV = 6,      /* (shot, part) pairs where no representation converged */
    MBBP_CNT_TIES = 7,        /* (shot, part) pairs whose best value under the decision rule is shared
                                 by distinct converged candidates (least weight: the same weight; FWS:
                                 the same score); the smaller index decides those */
    MBBP_NUM_COUNTERS = 8
};

/* The whole path for shots [shot0, shot0 + shots): noise (mbbp_sample), the
 * batched decoder, the decision and the failure test, replayed from a HIP graph
 * captured on first use for this `shots` and launch configuration (also while BP
 * timing is enabled: the graph's own event nodes time its BP kernel, see
 * mbbp_set_timing; direct launches with mbbp_set_graph(ctx, 0)).  counters: device int64
 * [MBBP_NUM_COUNTERS], ACCUMULATED into (the caller zeroes it).  Uniform
 * priors log((1 - q) / q) for both parts, q = 2p/3 under depolarizing noise and
 * q = p under X-only noise (mbbp_set_noise). */
mbbp_status mbbp_run(mbbp_ctx *ctx, uint64_t seed, double p, int64_t shot0, int64_t shots,
                     int64_t *counters, void *hip_stream);

/* mbbp_run for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same path
 * and results as mbbp_run, launched directly on hip_stream (no graph, no event,
 * no hipMalloc / hipFree), with every intermediate buffer in one static device
 * array of 64 MiB that each GPU holds until the process ends.  `shots` is bounded
 * by that array, not by max_batch: per shot 8 (W + Ws) + 8 W + 10 + 8 L W + 2 L
 * bytes for each part (W = ceil(n/64), Ws = ceil(m/64) of the part's matrix, L
 * representations), plus 4, in 256-byte aligned pieces; a larger batch is
 * MBBP_EINVAL and the message names the largest that fits.  The decoder's device
 * must be current.  All calls on one GPU share the array: calls that overlap in
 * time on one GPU (two streams, two threads, two decoders) race and give wrong
 * counters; serialise them.  counters as in mbbp_run (accumulated into). */
mbbp_status mbbp_run_static(mbbp_ctx *ctx, uint64_t seed, double p, int64_t shot0, int64_t shots,
                            int64_t *counters, void *hip_stream);

/* Kernel of the serial schedule (MBBP_LAYERED, Section II-B: rows updated one after
 * another from the latest messages).  Every choice gives the same results.
 *   MBBP_SERIAL_AUTO   (default) SLOTS for normalized min-sum, LANES for
 *                      sum-product, where their LDS layouts fit, else LEVELS;
 *   MBBP_SERIAL_SLOTS  eight lanes per shot, lane k holding slot k of the current
 *                      row, up to eight shots of one representation per wavefront
 *                      (normalized min-sum; sum-product runs LANES);
 *   MBBP_SERIAL_LANES  one shot per lane (mbbp_set_serial_lanes);
 *   MBBP_SERIAL_LEVELS one instance per wavefront, the rows of a representation
 *                      grouped into levels of rows sharing no variable.
 * The weighted rule always runs the flooding schedule.  MBBP_EINVAL: another value. */
typedef enum {
    MBBP_SERIAL_AUTO = 0,
    MBBP_SERIAL_SLOTS = 1,
    MBBP_SERIAL_LANES = 2,
    MBBP_SERIAL_LEVELS = 3
} mbbp_serial_kernel;
mbbp_status mbbp_set_serial_kernel(mbbp_ctx *ctx, int32_t kernel);

/* Statistics of the decode calls: with counters a device int64 [MBBP_NUM_COUNTERS]
 * array, every later mbbp_decode / mbbp_decode_batched on this decoder ADDS its
 * MBBP_CNT_SUM_K, MBBP_CNT_EDGE_UPDATES, MBBP_CNT_NOCONV and MBBP_CNT_TIES to it, on
 * the call's stream (the others are left alone: those calls take no failure test).
 * The caller owns the array and keeps it alive while set; NULL (the default) stops
 * the accounting. */
mbbp_status mbbp_set_stats(mbbp_ctx *ctx, int64_t *counters);

/* Serial schedule with the one-shot-per-lane kernel (MBBP_SERIAL_LANES, or AUTO
 * with sum-product): `lanes` shots of one representation per wavefront, its
 * messages in LDS.  lanes = 0 (default) picks the largest count
 * that leaves room for two wavefronts per compute unit; 4, 8, 16, 32 or 64 asks
 * for that count, used where it fits the LDS of one workgroup (else the default).
 * Codes up to n = 1024 with at most 65535 edges per representation; others run
 * the level-synchronous kernel.  Results do not depend on it.
 * MBBP_EINVAL: lanes not 0, 4, 8, 16, 32 or 64. */
mbbp_status mbbp_set_serial_lanes(mbbp_ctx *ctx, int32_t lanes);

/* Launch configuration of the BP kernel (the autotuner's search space).
 * form: 0 = mbbp_decode / mbbp_decode_detail, 1 = mbbp_decode_batched / mbbp_run.
 * lanes_per_instance: 64 (one instance per wavefront; other values: MBBP_EUNSUPPORTED);
 * waves_per_block >= 1 (reduced automatically to fit 64 KiB of LDS);
 * chunk: shots per work item, decoded one after another by a wave (default 8 for
 *   form 0, 64 for form 1; the paired kernel, two instances per wavefront, serves
 *   items of at most 128 shots, larger ones run one instance per wavefront);
 * blocks: persistent grid size (form 1; 0 = 5 per compute unit).
 * Every configuration gives bit-identical outputs.  MBBP_EUNSUPPORTED if the code
 * does not fit the register tables of that lane count. */
typedef struct {
    int32_t lanes_per_instance, waves_per_block, chunk, blocks;
} mbbp_launch_config;
mbbp_status mbbp_set_config(mbbp_ctx *ctx, int32_t form, const mbbp_launch_config *cfg);
mbbp_status mbbp_get_config(mbbp_ctx *ctx, int32_t form, mbbp_launch_config *cfg);

/* Autotuner: times the candidate launch configurations of `form` (0 plain,
 * 1 batched) on `shots` synthetic shots drawn with (seed, p) and keeps the
 * fastest; *chosen (may be NULL) receives it.  Synchronous.  Outputs of every
 * later call are unchanged bit for bit (only the launch shape differs). */
mbbp_status mbbp_autotune(mbbp_ctx *ctx, int32_t form, uint64_t seed, double p, int64_t shots,
                          mbbp_launch_config *chosen);

/* mbbp_run replays a HIP graph captured per `shots` (enable = 1, default) or
 * launches its kernels directly (enable = 0); results are identical.  A graph
 * captured before the batched launch configuration changed (mbbp_set_config,
 * mbbp_autotune) is captured again. */
mbbp_status mbbp_set_graph(mbbp_ctx *ctx, int32_t enable);

/* The launch configuration held by the BP kernel node of the graph mbbp_run has
 * captured for `shots` (waves_per_block and blocks read from the node itself).
 * MBBP_EINVAL if no graph is captured for that size. */
mbbp_status mbbp_run_graph_config(mbbp_ctx *ctx, int64_t shots, mbbp_launch_config *cfg);

/* Uniform prior LLR of one part (the BP initialisation of Section II-B),
 * log((1 - q) / q) rounded to float, with q the part's flip probability: 2p/3
 * under depolarizing noise (X and Y, or Y and Z, flip it), p under X-only noise.
 * This is the prior mbbp_run and mbbp_autotune use.  MBBP_EINVAL unless
 * 0 < q < 1 or for an unknown model. */
mbbp_status mbbp_prior_llr(int32_t noise, double p, float *mu);

/* mbbp_decode as the naive per-basis form (enable = 1): one BP launch per (part,
 * representation), each over all shots, instead of one launch over every
 * representation of both parts.  Results are identical (for comparison with the
 * batched form).  Default 0. */
mbbp_status mbbp_set_per_basis(mbbp_ctx *ctx, int32_t enable);

/* Event timing of the BP kernel.  While enabled, every BP kernel launch of this
 * context is bracketed by HIP events recorded on the launch's stream (under
 * mbbp_run's graph replay by the graph's own event record nodes around its BP
 * kernel node, given fresh events at every replay).
 * mbbp_bp_time waits for those events and returns the summed elapsed time (ms)
 * and the number of launches since the last reset (reset != 0 clears them). */
mbbp_status mbbp_set_timing(mbbp_ctx *ctx, int32_t enable);
mbbp_status mbbp_bp_time(mbbp_ctx *ctx, double *ms, int64_t *launches, int32_t reset);

/* Algorithm 2 on host memory: perm is a permutation of the m checks (root
 * order); check_sets[m] receives the 1-based subtree of each check, order[m]
 * the checks in acceptance order (subtree 1 first), *n_subtrees their number. */
mbbp_status mbbp_subtrees(const mbbp_sparse *H, const int32_t *perm, int32_t *check_sets,
                          int32_t *order, int32_t *n_subtrees);

/* Representations from subtrees (host).  perms: [n_perms][m] root orders.
 * mode 0: distinct maximal subtrees of perms[0], perms[1], ... in discovery
 *         order, rows in acceptance order, until L are found (fewer: MBBP_EINVAL).
 * mode 1: representation l appends the first round(l m / (L-1)) rows (halves
 *         up) of perms[l]'s acceptance order (needs n_perms >= L): sizes ramp
 *         from 0 to m.
 * Output basis_ptr[L + 1] and rows[rows_cap] (H row indices). */
mbbp_status mbbp_build_bases(const mbbp_sparse *H, int32_t mode, int32_t L, int32_t n_perms,
                             const int32_t *perms, int32_t *basis_ptr, int32_t *rows,
                             int32_t rows_cap);

/* Logical operators (host copies): LX [k][ceil(n/64)] spans ker H_Z modulo the
 * row space of H_X, LZ spans ker H_X modulo the row space of H_Z; *k = n -
 * rank H_X - rank H_Z.  Either array may be NULL to query k. */
mbbp_status mbbp_logicals(mbbp_ctx *ctx, uint64_t *LX, uint64_t *LZ, int32_t *k);

/* Edges of each representation of a part (host int64 [L]). */
mbbp_status mbbp_edge_counts(mbbp_ctx *ctx, int32_t part, int64_t *edges);

/* Message for the last non-OK status returned on this thread. */
const char *mbbp_last_error(void);

/* ---- Weighted (differentiable) form of the decoder ------------------------------
 * Not part of the paper's method: a learned variant of its normalized min-sum
 * (eq. (1)) with a scaling alpha_{t,l} and a damping beta_{t,l} per iteration t and
 * representation l, flooding schedule:
 *   r^(t) = clamp((1 - beta_{t,l}) * S * (alpha_{t,l} * M) + beta_{t,l} * r^(t-1)),
 *   r^(0) = 0, M the smallest |q| over the row's other edges, S the product of
 *   their signs and of (-1)^{s_j}; variables as eq. (2).  beta = 0 and a constant
 *   alpha give plain normalized min-sum bit for bit.
 * Weights are device float arrays [T][L] (iteration t at row t - 1), shared by
 * both parts (representation l of H_Z and of H_X use column l); both parts must
 * have the same L. */

/* Weights used by decode / decode_batched / decode_detail / run when the context
 * was created with rule MBBP_WEIGHTED.  Device pointers, read at every launch
 * (their contents may change between calls; the pointers must stay valid).
 * Pass NULL, NULL to clear.  Decoding with MBBP_WEIGHTED and no weights is
 * MBBP_EINVAL.  Changing the pointers drops captured mbbp_run graphs. */
mbbp_status mbbp_set_weights(mbbp_ctx *ctx, const float *alpha, const float *beta);

/* Floats of the checkpoint buffer of mbbp_wbp_forward for `shots` shots of one part
 * with a checkpoint every ckpt_every >= 1 iterations:
 * shots * L * (ceil(T / ckpt_every) - 1) * 8 * S, S the kernel's slot stride for that
 * part. */
mbbp_status mbbp_wbp_ckpt_floats(mbbp_ctx *ctx, int32_t part, int64_t shots, int32_t ckpt_every, int64_t *floats);

/* Training forward of one part: weighted min-sum for exactly T iterations (no early
 * stop) on every representation, any rule the context was created with.
 * syn, prior as in mbbp_decode_detail; alpha, beta device [T][L].
 * llr  device float [shots][L][n]: the posterior P^(T) of every representation.
 * ckpt device float [mbbp_wbp_ckpt_floats]: c->v messages r^(t) for t = ckpt_every,
 *      2 ckpt_every, ... < T (may be NULL when that list is empty); opaque layout,
 *      read by mbbp_wbp_backward with the same arguments.
 * Candidates and iteration counts go to the context's workspace (overwritten). */
mbbp_status mbbp_wbp_forward(mbbp_ctx *ctx, int32_t part, int64_t shots, const uint64_t *syn, const float *prior,
                             int32_t prior_per_shot, const float *alpha, const float *beta, int32_t ckpt_every,
                             float *ckpt, float *llr, void *hip_stream);

/* Adjoint of mbbp_wbp_forward: given grad_llr = dL/dP^(T) (device float
 * [shots][L][n]), ADDS dL/dalpha and dL/dbeta (device float [T][L]) into grad_alpha,
 * grad_beta.  Same syn, prior, alpha, beta, ckpt_every and ckpt as the forward.
 * Each segment of ckpt_every iterations is recomputed from its checkpoint, so the
 * result does not depend on ckpt_every.  Subgradients: the minimum passes its
 * adjoint to the first edge (in row order) of smallest magnitude among the others,
 * d|x|/dx = sign of x, sign factors are constant, the clamp passes the adjoint only
 * strictly inside (-r_max, r_max).  Per-instance partial sums are added over shots
 * in FP64 in a fixed order: results are deterministic.
 * Limits (MBBP_EUNSUPPORTED): n <= 320 and at most 319 checks per representation;
 * (3 + ckpt_every) * 32 * S bytes of LDS per instance (S the slot stride) must fit
 * 64 KiB. */
mbbp_status mbbp_wbp_backward(mbbp_ctx *ctx, int32_t part, int64_t shots, const uint64_t *syn, const float *prior,
                              int32_t prior_per_shot, const float *alpha, const float *beta, int32_t ckpt_every,
                              const float *ckpt, const float *grad_llr, float *grad_alpha, float *grad_beta,
                              void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MBBP_H */
