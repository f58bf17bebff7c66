// Device-side data shared by the host preprocessing and the HIP kernels of the
// MBBP-LD library (internal; not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>

namespace mbbp {

constexpr int kMaxRowWeight = 8;   // row slots per check in LDS (stride 8)
constexpr int kMaxVarDegree = 8;   // edge slots per variable
constexpr int kMaxL = 64;
constexpr int kMaxN = 1024;

// LDS rows of a representation are "positions": check j of representation l sits at
// position pos_l(j) and owns LDS edge ids pos*8 .. pos*8 + w_j - 1.  Positions run
// over [0, Mmax); Mmax itself is the sink of absent edges (shared by all
// representations); positions no check uses are junk (csrc = kJunkRow).
constexpr int32_t kJunkRow = INT32_MIN;
// Slot stride of the slot-major LDS arrays: Mpad + kSlotPad words, so the slots of one
// row fall in different banks.
constexpr int kSlotPad = 1;

// Tables of one part (one parity-check matrix and its L representations).
struct DevPart {
    int m, n, L;
    int W, Ws;          // 64-bit words of n bits / of m bits
    int Mmax;           // positions per representation (the sink is position Mmax)
    int uniform_dc;     // 6 if every row of every representation has weight 6, else 0
    int max_deg;        // largest variable degree over the representations
    const int32_t *M;   // [L] checks of each representation
    const int32_t *E;   // [L] edges of each representation
    const uint16_t *voff;   // [L][n][8] edge ids of the variable in slot s, ascending check order
    const uint16_t *vid;    // [L][n] variable id of slot s (slots sorted by degree, descending)
    const uint8_t *vdeg;    // [L][n] degree of the variable in slot s
    const uint8_t *cw;      // [L][Mmax] row weight at each position (8 at junk positions)
    const int32_t *csrc;    // [L][Mmax] syndrome source at each position: H row j -> j; duplicate
                            // of H row r -> r; explicit row -> -(c + 1), combination c in
                            // comb_ptr/comb_idx; junk position -> kJunkRow
    const int32_t *comb_ptr;
    const int32_t *comb_idx;
    const int32_t *hrow_ptr;   // H in CSR (sampler / failure test)
    const int32_t *hrow_idx;
    const uint64_t *logical;   // [k][W] logical operators of the other type (failure test)
    int k;
    // serial schedule: levels of representation l are lev_ptr[lev_off[l] ..
    // lev_off[l + 1]) (offsets into lev_chk + l * Mmax, the positions of the checks
    // ordered by level); ltab[(l * Mmax + p) * 8 + k] = 8 x u16: variable id | degree
    // << 12, then the variable's other edge ids in ascending check order (sink beyond
    // its degree)
    const int32_t *lev_off;
    const int32_t *lev_ptr;
    const uint16_t *lev_chk;
    const uint4 *ltab;
    // serial schedule, one lane per shot (bp_serial_kernel): per representation l
    // and augmented row j (row order), rows stab_off[l] + j of
    //   stab  [rows][dcs] u32: per row slot, variable v | t << 10 | (deg - 1) << 13 |
    //         first edge of v << 16 (0xffffffff: absent slot), where edges are numbered
    //         variable by variable (v's deg edges contiguous, ascending row order) and
    //         t is the rank of row j among v's rows
    //   scsrc [rows] syndrome source of the row (as csrc)
    // htab [m][8] u16: the rows of H (0xffff beyond the row weight), for the halting test
    const uint32_t *stab;
    const int32_t *stab_off;   // [L + 1]
    const int32_t *scsrc;
    const uint16_t *htab;
    int dcs;                   // slots per record row: 6 (every row of weight 6) or 8
    int emax, maug;            // largest edge count / augmented row count of a representation
    int serial_ok;             // the records fit their bit fields (edge ids < 65536)
    // serial schedule, eight lanes per shot (bp_serial_slots_kernel): per augmented
    // row (rows stab_off[l] + j), byte offsets within a shot's LDS block (8 junk
    // words, then the messages)
    //   srec  [rows][8] (A, B): A = 32 + 4 first | (32 + 4 (first + t)) << 16,
    //         B = 4 v | rdm << 12 | (t = deg - 1) << 15 | 4 (v >> 5) << 16 |
    //         (v & 31) << 24 | (deg - 1) << 29, rdm the row's largest deg - 1; an absent
    //         slot has A = 4 << 16 and B's v = n
    //   sht   [m][8] u32: rows of H, (v & 31) | 4 (v >> 5) << 8 (v = n pads)
    const uint2 *srec;
    const uint32_t *sht;
};

// One BP launch (plain or persistent).
struct BPArgs {
    DevPart part[2];
    const DevPart *dparts;   // the same two parts in device memory (read by bp_kernel)
    int part0, nparts;       // parts handled: part0 .. part0 + nparts - 1
    int L;                   // representations per part (equal for both parts)
    int T;
    float alpha, rmax;
    int fixed_T;
    int64_t shots;
    const uint64_t *syn[2];  // [shots][Ws]
    const float *prior[2];   // [n] or [shots][n]
    int prior_per_shot;
    uint64_t *cand[2];       // [shots][L][W], or [L][shots][W] with cand_rm
    uint16_t *kstat[2];      // [shots][L], or [L][shots] with cand_rm
    int cand_rm;             // candidates and iteration words representation-major
    float *llr[2];           // [shots][L][n] or null
    // work items
    int persistent;          // 0: item = global wave id, 1: atomic queue
    int chunk;               // shots per item
    int64_t n_items;
    const int32_t *item_order;  // persistent: [n_items_per_shotrange] (part, l) pairs ordered heavy first
    int n_pl;                // number of (part, l) pairs
    int64_t n_chunks;        // chunks per (part, l)
    unsigned long long *queue;
    int dual;                // two instances per wavefront (bp_dual_kernel)
    int dual_stride;         // bytes of one instance's LDS region in the paired kernel
    int inst_bytes;          // LDS bytes per instance (per wavefront with dual: both instances)
    int msg_bytes;           // message rows of an instance: (Mmax + 1) * 8 floats
    int zero_bytes;          // message rows + decision rows (cleared at every fill), multiple of 16
    int ws_max, w_max;       // syndrome words / candidate words of the launch's parts
    int n_max;               // priors staged in LDS (per-shot priors, serial schedule)
    // weighted rule: alpha_{t,l}, beta_{t,l} as [T][L] (iteration t at row t - 1); with
    // ckpt non-null the c->v messages r^(t) of t = ckpt_every, 2 ckpt_every, ... < T
    // are stored per instance (shot * L + l) as n_ck arrays of 8 * Mpad floats
    const float *walpha, *wbeta;
    float *ckpt;
    int ckpt_every, n_ck;
    // serial kernel with one lane per shot: shots per wavefront, and the LDS rows of
    // the messages [s_emax][S] and augmented syndrome words [s_nmw][S]
    int serial_lanes, s_emax, s_nmw;
    // serial kernel with eight lanes per shot: shots (lane groups) per wavefront, the
    // bytes of one shot's LDS block and its decision words
    int serial_groups, s_sb, s_ndw;
};

// Per-call parameters of the captured whole-path graph, written on device by the
// graph's first node (the only node whose parameters change between replays).
struct RunDesc {
    uint64_t seed;
    int64_t shot0;
    uint64_t t1, t2, t3;
    int64_t *counters;       // caller's counters, accumulated at the end of the graph
};

struct RunPrepArgs {
    RunDesc d;
    RunDesc *desc;           // where the descriptor is stored
    float *prior0, *prior1;
    int n;
    float mu;
    int *kmax;
    int64_t shots;
    unsigned long long *queue;
    int64_t *counters;       // internal counters cleared here
};

struct SampleArgs {
    DevPart part[2];         // part[0] uses H_Z (syn_x), part[1] uses H_X (syn_z)
    int n;
    uint64_t seed;
    uint64_t t1, t2, t3;
    int64_t shot0, shots;
    uint64_t *err[2];        // [shots][W]  e_X, e_Z
    uint64_t *syn[2];        // [shots][Ws] s_X = H_Z e_X, s_Z = H_X e_Z
    const RunDesc *desc;     // graph replay: seed, shot0 and thresholds read from here (or null)
};

struct SelectArgs {
    DevPart part[2];
    int part0, nparts;
    int rule;                // 0 least weight, 1 FWS
    int group;               // lanes per (part, shot); set by launch_select
    int64_t shots;
    const uint64_t *cand[2];     // [L][shots][W] (representation-major, as the BP kernels write them)
    const uint16_t *kstat[2];    // [L][shots]
    uint64_t *corr[2];
    uint64_t *conv[2];
    int16_t *basis[2];
    int64_t *counters;       // optional: SUM_KMAX, SUM_K, EDGE_UPDATES, NOCONV, TIES
    int *kmax_shot;          // optional [shots] scratch for the per-shot max over both parts
};

struct FailArgs {
    DevPart part[2];
    int64_t shots;
    const uint64_t *err[2];
    const uint64_t *corr[2];
    uint8_t *fail;           // optional [shots]
    int64_t *counters;       // optional FAIL, FAIL_X, FAIL_Z, SUM_KMAX
    const int *kmax_shot;    // optional
};

// Launchers (mbbp_kernels*.hip).  Return hipError_t of the launch.
struct BPConfig {
    int lpi;        // lanes per instance: 16, 32 or 64
    int waves_per_block;
    int chunk;      // persistent: shots per work item
    int blocks;     // persistent: grid size
};

hipError_t launch_bp(const BPArgs &a, const BPConfig &cfg, int schedule, int rule, hipStream_t s);

// Grid of a non-persistent BP launch that wants `blocks` workgroups: capped (the
// kernels then stride over work items by the grid size), so the dispatch's thread
// count stays far below 2^32.
inline int64_t plain_grid(int64_t blocks) { return blocks < 1 ? 1 : (blocks > 65536 ? 65536 : blocks); }

// Adjoint of the weighted decoder's fixed-T forward map for one part: per instance
// (l, shot), segments of ckpt_every iterations are recomputed from the stored
// checkpoints and run backwards; per-instance dL/dalpha_t, dL/dbeta_t go to partial.
struct WBPBackArgs {
    const DevPart *dpart;    // the part, in device memory
    int L, T;
    int64_t shots, n_items;  // n_items = L * shots, item = l * shots + shot
    float rmax;
    const uint64_t *syn;     // [shots][Ws]
    const float *prior;      // [n] or [shots][n]
    int prior_per_shot;
    const float *walpha, *wbeta;  // [T][L]
    const float *ckpt;       // [shots * L][n_ck][8 * Mpad]
    int ckpt_every, n_ck;
    const float *grad_llr;   // [shots][L][n]: dL/dP^(T)
    float2 *partial;         // [T][n_items]: per-instance (dL/dalpha_t, dL/dbeta_t)
    int inst_bytes, ws, n;
};
hipError_t launch_wbp_backward(const WBPBackArgs &a, int pv, int pc, int dc, int waves_per_block, hipStream_t s);
// grad_alpha[t][l] += sum over shots of partial, likewise grad_beta (FP64 sums in a
// fixed order, so results do not depend on scheduling).
hipError_t launch_wbp_reduce(const float2 *partial, int64_t shots, int T, int L, float *grad_alpha,
                             float *grad_beta, hipStream_t s);
bool wbp_backward_supported(int pv, int pc);
// (pv, pc) instantiation the BP kernel uses for the parts of a
bool bp_passes(const BPArgs &a, int &pv, int &pc);
hipError_t launch_sample(const SampleArgs &a, hipStream_t s);
hipError_t launch_select(SelectArgs a, hipStream_t s);
hipError_t launch_fail(const FailArgs &a, hipStream_t s);
hipError_t launch_reset(unsigned long long *queue, int64_t *counters, int ncounters, hipStream_t s);
// Per-run preparation: descriptor stored, uniform priors mu for both parts, per-shot
// max-iteration scratch, work-queue counter and internal counters cleared.
hipError_t launch_run_prep(const RunPrepArgs &a, hipStream_t s);
// Adds the internal counters into the caller's (desc->counters).
hipError_t launch_accumulate(const int64_t *src, const RunDesc *desc, int nc, hipStream_t s);
const void *run_prep_kernel_ptr();
int bp_max_passes(int lpi);  // register slots available per lane for this lpi
// Rows per instance (Mpad = 64 * check passes) of the kernel a launch would use; false if none fits.
bool bp_layout(const BPArgs &a, int &mpad);
// Paired form (two instances per wavefront): whether it serves this launch and, if
// so, the LDS bytes per wavefront.
bool bp_dual_layout(const BPArgs &a, int schedule, int rule, int &inst_bytes, int &stride);
bool bp_dual_fits(int n, int mmax);  // a part of n variables and mmax + 1 positions fits it
hipError_t launch_bp_dual(const BPArgs &a, const BPConfig &cfg, hipStream_t s);
// Serial schedule with one lane per shot (rule NMS or SPA); a.serial_lanes,
// a.s_emax, a.s_nmw and a.inst_bytes (LDS of the one wavefront of a block) set.
hipError_t launch_bp_serial(const BPArgs &a, const BPConfig &cfg, int rule, hipStream_t s);
// Shots per wavefront the serial kernel is built for at n variables.
bool serial_lanes_supported(int n, int S);
// Serial schedule, normalized min-sum, eight lanes per shot (row slot k in lane k);
// a.serial_groups, a.s_sb, a.s_ndw, a.s_emax, a.s_nmw, a.ws_max, a.n_max and
// a.inst_bytes set.
hipError_t launch_bp_serial_slots(const BPArgs &a, const BPConfig &cfg, hipStream_t s);
bool bp_supported(int lpi, int passes, int dc_uniform, int rule, int schedule);
size_t bp_lds_limit();
// BP kernel function most recently launched by the calling host thread.
const void *last_bp_kernel();
void set_last_bp_kernel(const void *f);

}  // namespace mbbp
