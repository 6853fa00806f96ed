// Internal declarations shared by the HIP sources of libhawkes (not installed).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "hawkes.h"

// Geometry of the pair passes.  A wavefront is 64 lanes on gfx950; a block of
// four wavefronts owns a tile of 256 rows (row pass) or 256 columns (column
// pass); the other index is swept in chunks of 64 staged through LDS.
#define HK_WAVE 64
#define HK_TILE 256
#define HK_WAVES (HK_TILE / HK_WAVE)
#define HK_CHUNKS_PER_TILE (HK_TILE / HK_WAVE)

// Number of row accumulators (row pass) and symmetric column accumulators.
// Row slots: 0 B0, 1 B1, 2 B2, 3 B11, 4 B22, 5 X0, 6 X1, 7 X2, 8 X11, 9 X22.
// Column slots: the five background moments B0, B1, B2, B11, B22.
#define HK_NROW 10
#define HK_NCOL 5
// Per-event sums reduced by the finalize kernels (see hawkes_eval.hip).
#define HK_NSUM 20

// The excitation's time factor is split per 64-event chunk (exp(-omega (t_i -
// t_j)) = exp(-omega (t_i - T_c)) exp(omega (t_j - T_c))) when omega times the
// chunk's time span is at most this: both factors then stay far inside the
// FP32 range.
#define HK_FACT_SPAN 40.0

// The row pass takes its fast form (split time factor, FP32 times relative to
// the chunk's first event) on a chunk that spans at most HK_COMPACT_TAU tau_t
// (and HK_FACT_SPAN / omega) in time; on a wider chunk, the precise form (FP64
// time differences, whole exponents formed in FP64 with an exact power of two).
#define HK_COMPACT_TAU 0.5

// The column passes form the whole exponent of a term c_e E_ij / lambda_i in
// FP64 (log2 units): log2(c_e / lambda_i), the time term and the spatial term.
// Exponents are clamped below at this value (every term with an exponent below
// about -150 is zero in FP32 anyway), which keeps their integer parts inside
// int32 for padding rows, zero weights and very distant pairs.
#define HK_EXP_FLOOR (-1.0e5)

// The column passes' spatial exponent -|s (x_i - x_j)|^2 is expanded as
// 2 s x_i . s x_j - |s x_i|^2 - |s x_j|^2 (one FP64 operation fewer per pair
// than the differences) when the pre-scaled coordinates are small enough for
// the cancellation to cost at most ~2^-30 absolute: |s x|^2 <= HK_DOT_MAX2 for
// every event.  Wider sets (relative to the bandwidth h) take the differences.
#define HK_DOT_MAX2 524288.0

// Floor of Eq. 5's entries under the log in the learned preconditioner's
// training target log max(H_k, HK_LOGH_FLOOR).  An entry without later events
// is exactly 0, and an entry below the floor changes its event's mass
// theta^2 H + P by at most 1e-6 theta^2: the floor spends none of the network's
// capacity on the long tail of such entries (log H reaches -70 on the
// clustered workloads) that the mass does not feel.
#define HK_LOGH_FLOOR 1.0e-6
// Floor of the learned preconditioner's kernel-sum feature, log2 S_m (a sum
// below 2^-32 of a unit term says only that no later event is near).
#define HK_KSUM_LOG2_FLOOR (-32.0)

// Eq. 4 alone: the column passes take the integer part of a row's weight
// lw_i = log2(c_e / lambda_i) out of each exponent exactly and round the rest,
// the pair's own decay, once to FP32.  For a row of large weight (a low
// intensity) that rest can be large on terms that still carry a column's sum,
// so a chunk holding a row with lw_i above HK_LW_SPLIT_MAX splits every
// exponent exactly instead (integer part and FP32 fraction).
#define HK_LW_SPLIT_MAX 8.0

// Time offset given to padding events: their pair terms underflow to exactly
// zero while every square stays finite in FP32.
#define HK_PAD_DT 1.0e15

// Mean relative error of the hardware exp2 (v_exp_f32) over uniformly
// distributed fractional arguments, measured on gfx950 over 2.7e8 arguments
// spanning [-126, 0): -3.4e-9 (the function rounds slightly low on average).
// The FP64 constants that multiply the FP32 pair sums are divided by
// (1 + HK_EXP2_BIAS) so that the sums of many terms are unbiased.
#define HK_EXP2_BIAS (-3.4e-9)

enum { HK_MODE_LOGLIK = 0, HK_MODE_GRAD = 1, HK_MODE_HESS = 2 };

// Largest batch of the allocation-free network training step (its workspace
// is a fixed device array of about 4.3 MB per GPU).
#define HK_NOALLOC_MLP_MAX_B 4096

struct hk_item {  // one piece of a pair-pass block: a chunk range of one tile
    int tile;     // row tile (row pass) or column tile (column pass)
    int c_begin;  // first chunk of the swept index
    int c_end;    // one past the last chunk
    int seg;      // piece number within the tile
};

struct hawkes_plan_s {
    int64_t n;       // events
    int64_t npad;    // padded to a multiple of HK_TILE
    int ntiles;      // npad / HK_TILE
    int nchunks;     // npad / HK_WAVE
    double t0;       // window start
    double t1;       // max t
    double cx, cy;   // centre of the bounding box
    double xmin, xmax, ymin, ymax;  // bounding box of the locations
    int device;

    // sorted, padded structure-of-arrays (device)
    double *ts;      // [npad] sorted times; padding = t1 + HK_PAD_DT
    double *xs, *ys; // [npad] coordinates relative to the centre (x - cx, y - cy)
    int *perm;       // [n] sorted position -> caller index
    int *g;          // [npad] first sorted index with the same time (ties)

    // row pass schedule
    int n_row_items;
    hk_item *row_items;       // [n_row_items] (device)
    int n_row_blocks;         // blocks of the row pass
    int *row_block0;          // [n_row_blocks + 1] first item of each block (device)
    int *row_item0;           // [ntiles] first item of each row tile (device)
    int *row_nseg;            // [ntiles] items per row tile (device)
    int64_t *colpart_off;     // [ntiles] offset of tile I's column partials (device)
    int64_t colpart_len;
    // column pass schedule
    int n_col_items;
    hk_item *col_items;
    int n_col_blocks;
    int *col_block0;
    int *col_item0;
    int *col_nseg;

    // per-evaluation scratch (device)
    float *theta_s;           // [npad] rates in sorted order (FP32), 0 on padding
    float *theta_v;           // [npad] staged rates of the row pass (split time factor applied)
    int *chunk_precise;       // [nchunks] 1 where the row pass takes its precise form on the chunk
    double *tstep;            // [nchunks] exp(-omega (T_{c+1} - T_c)) of the last k_tfac
    double *lw;               // [npad] log2(c_e / lambda_i) of the last evaluation (HK_EXP_FLOOR on padding)
    float *rowpart;           // [n_row_items][HK_NROW][HK_TILE] row partial sums of each piece
    float *colpart;           // triangular [tile][HK_NCOL][(tile+1)*HK_TILE]: background column partials
    double *lam;              // [npad] lambda_i, sorted
    double *a;                // [npad] theta0 (1 - exp(-omega (T1 - t_i)))
    double *colG;             // [n_col_items][2][HK_TILE]: G and H of each column piece
    int nfin_blocks;          // npad / 256 (subset-path reductions)
    double *blockpart;        // [nchunks][HK_NSUM] per-block partial sums
    int *status;              // sticky device status bits
    hipStream_t last_stream;
    int64_t epoch;            // intensity evaluations so far (host counter)
    int cutoff;               // skip chunk pairs whose terms all underflow (off by default)
    int64_t eval_epoch;       // epoch of the last hawkes_eval (its lam, w, a are current)
    hawkes_hyper eval_hyper;  // hyperparameters of that evaluation
    struct hk_profile *prof;  // HIP-event timing of the passes (NULL when off)
    struct hk_subset *sub;    // free-rate subset for the HMC path (NULL until set)
    struct hk_tree *tree;     // phylogenetic prior on the subset log-rates (NULL until set)
};

hipError_t hk_sort_pairs(double *key, int *idx, int64_t n2, hipStream_t stream);
// Phylogenetic prior (hawkes_tree.hip): d_vz [m] = V^{-1} z and d_quad [1] =
// z^T V^{-1} z for z [m] in subset slot order (either output may be NULL).
hawkes_status hk_tree_launch(hawkes_plan p, const double *d_z, double *d_vz, double *d_quad, hipStream_t stream);
int64_t hk_tree_tips(hawkes_plan p);
// diagonal of V^{-1} of the plan's tree [m], slot order (device), or NULL
const double *hk_tree_precision_diag(hawkes_plan p);
void hk_tree_free(hawkes_plan p);
// Blocks of a pair pass (0 = row, 1 = column) resident at once on `device`:
// compute units times the pass kernels' occupancy.
int64_t hk_pass_slots(int device, int pass, int64_t npad);
void hk_subset_free(hawkes_plan p);
// views of the free-rate subset for the preconditioner code
void hk_subset_view(hawkes_plan p, int64_t *m, const int64_t **cidx, const int **pos, const int **slot);
hawkes_status hk_subset_grid(hawkes_plan p, int64_t cells, hipStream_t stream);
int *hk_subset_grid_ptr(hawkes_plan p);

// Exponent constants of the pair kernels (log2 units) and the FP64 constants of
// the finalisation; built per call from the hyperparameters.
struct PairConst {
    // kbx = -1 / (2 tau_x^2 ln 2) and kex = -1 / (2 h^2 ln 2) map a squared
    // distance to the log2 exponents a_b and a_e.
    // The row pass takes times scaled by st = 1 / (tau_t sqrt(2 ln 2)), so the
    // background's time exponent is exactly -dt'^2 (no rounded constant).
    double st;
    float rex;     // kex / kbx: a_e = a_b rex in the row pass
    // low part of rex (rex - (double)rex_f): the log-likelihood-only row pass,
    // which carries no first moments to correct its rounding with, applies it
    // inside the pair loop instead (in an FMA whose exact product is rounded
    // once, so the low part is not lost)
    float rex_lo;
    double omega;  // excitation decay rate (time factors formed in FP64)
    double kw_d;   // -omega / ln 2 in FP64 (exponents formed in FP64)
    double kw_s;   // kw_d / st: the same per scaled time unit (the row pass's precise form)
    double rex_x;  // kex / kbx exact in FP64 (the row pass's precise form, log-likelihood-only mode)
    double span_max;   // row pass: the fast form's largest chunk time span
    double sx;     // sqrt(-kex): coordinate -> scaled coordinate whose squared distance is -a_e
    double sbx;    // sqrt(-kbx): the same for the background exponent a_b
    double dt_cut;     // row pass: time gap past which both terms are below 2^-160 (INFINITY: no cutoff)
    double dt_cut_ex;  // column pass: the same for the excitation term alone
    int dot;           // column passes: expand the spatial exponent (HK_DOT_MAX2 holds for the plan)
};

struct FinConst {
    double mu0, tau_x, tau_t, theta0, omega, h;
    double c_b, c_e;       // normalisers of Sec. 2.1
    double cb1, ce1;       // c_b / mu0 and c_e / theta0
    double Kx, Kh;         // log2-unit moment -> r^2 moment: -2 tau_x^2 ln 2, -2 h^2 ln 2
    double corr;           // 1 / (1 + exp2 bias)
    double log2_ce;        // log2(c_e) (-inf when theta0 = 0)
    double t0, t1;
    // The row pass's time moments are in scaled time (t' = st t): dt^2 moments
    // are dt'^2 moments times Kt = 1/st^2 = 2 tau_t^2 ln 2, dt moments dt'
    // moments times 1/st.
    double Kt, inv_st;
    // First-order correction for the rounding of the FP32 ratio rex: a term
    // computed as exp2(a + d) equals exp2(a) (1 + d ln 2 + O(d^2)), and d is
    // linear in the excitation's spatial exponent, whose weighted sum X2 the
    // row pass accumulates.  (The background's exponent carries no rounded
    // constant; the excitation's time term is exact or formed in FP64.)
    double rho_ex;         // (rex_f - rex) / rex_f: the row pass forms a_e = a_b rex_f
    // The pair passes' FP32 terms lose what falls below FP32's normal range
    // (2^-126 per term): at most (c_b + c_e) n 2^-126 of lambda_i.  A row whose
    // lambda_i comes out below lam_exact = (c_b + c_e) n 2^-96, where that loss
    // could exceed 2^-30 of it, is recomputed exactly in FP64 by k_fin.
    double lam_exact;
};

bool hk_hyper_ok(const hawkes_hyper *h);
// Eq. 4 and Eq. 5 on the subset at the rates d_theta (O(N M) path); device
// pointers to the results in time order
hawkes_status hk_subset_exact(hawkes_plan p, const hawkes_hyper *hy, const double *d_theta, hipStream_t stream,
                              const double **gsub, const double **hsub);
void hk_make_consts(const hawkes_plan p, const hawkes_hyper *hy, PairConst *kc, FinConst *fc);
// Log-likelihood-only row pass (no moments) with the sorted FP32 rates already
// in p->theta_s; leaves the partial sums B0 (row slot 0, column slot 0) and X0
// (row slot 5) in p->rowpart / p->colpart.
void hk_launch_row_loglik(hawkes_plan p, const PairConst &kc, hipStream_t stream);

// Optional timing of the passes with HIP events recorded on the launch stream.
enum { HK_PROF_ROW = 0, HK_PROF_COL = 1, HK_PROF_EVAL = 2, HK_PROF_KINDS = 3 };
void hk_prof_mark(hawkes_plan p, int kind, bool start, hipStream_t stream);
void hk_prof_free(hawkes_plan p);

// status bits on the device
#define HK_ST_ZERO 1
#define HK_ST_NONFINITE 2
#define HK_ST_BADTHETA 4

#define HK_CHECK(call)                                  \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return HAWKES_E_DEVICE;   \
    } while (0)
