// Free-rate subset and Hamiltonian Monte Carlo on its log-rates (Sec. 2.2,
// Sec. 2.3.2).
//
// Only the M rates in the subset change along an HMC trajectory; every other
// rate is fixed (1 in the paper).  lambda_i therefore splits exactly into a
// static part -- the background over all pairs plus the excitation from fixed-
// rate events -- and the excitation from the subset:
//   lambda_i = lambda_static_i + c_e sum_{k in M, t_k < t_i} theta_k E_ik .
// The static part costs one O(N^2) row pass per hyperparameter setting and is
// cached; each gradient inside a trajectory then costs one row pass over
// N x M pairs (subset excitation) and one column pass over M x N pairs
// (Eq. 4 and Eq. 5 restricted to the subset), i.e. O(N M) as the paper notes.
//
// Kernels:
//   k_sub_static   partial sums of the static row pass -> lambda_static_i
//   k_sub_offset   temporal-trend offsets beta t_k (Sec. 2.2)
//   k_sub_theta    theta_k = exp(z_k + beta t_k) into the caller's theta, and the
//                  subset entries staged in time order for the subset passes
//   k_sub_row      X_i = sum_{k in M, t_k < t_i} theta_k E_ik (rows = all events),
//                  one-wavefront items with partial sums
//   k_sub_fin      lambda_i, block sums of log lambda_i, and the column
//                  pass's row weights log2(c_e / lambda_i)
//   k_sub_col      G_k = sum_{t_i > t_k} E_ik w_i, H_k = sum (E_ik w_i)^2, items
//   k_sub_colfin   Eq. 4 / Eq. 5 on the subset; inside hmc_step also the
//                  leapfrog's gradient in z, kick and drift
//   k_hmc_*        momenta (Philox-4x32-10 + Box-Muller), energy, accept
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "hawkes_internal.h"

struct hk_subset {
    int64_t m;           // subset size
    int64_t mpad;        // padded to a multiple of HK_TILE
    int *pos;            // [mpad] sorted position of subset entry r (time order); pad = INT_MAX
    int *slot;           // [mpad] caller's subset slot k of entry r
    int64_t *cidx;       // [m] caller index of slot k (copy of the caller's idx)
    // row pass schedule: (row chunk, range of subset entries before its end)
    int n_ritems;
    hk_item *ritems;     // (row chunk, entry begin, entry end, seg)
    int *ritem0, *rnseg; // per row chunk
    double *xpart;       // [n_ritems][HK_WAVE] excitation partial sums of each item
    // column pass schedule: (64-entry subset chunk, row chunk begin, end)
    int n_items;
    hk_item *items;      // (subset chunk, row chunk begin, end, seg)
    int *item0, *nseg;   // per subset chunk
    int nq;              // subset chunks: mpad / HK_WAVE
    // cached static part
    bool static_valid;
    hawkes_hyper static_hyper;
    double *lam_static;  // [npad]
    double *Lam_static;  // [1] integral term of the fixed-rate events + background
    double *a;           // [mpad] theta0 (1 - exp(-omega (T1 - t_k))) per subset entry r
    // per-evaluation buffers
    // staged subset entries (time order), written once per evaluation
    float *tv;           // [mpad] theta_r exp(omega (t_r - T_q)) (theta_r on wide chunks), 0 on padding
    double2 *sxy;        // [mpad] coordinates pre-scaled by sqrt(-kex)
    double *sts;         // [mpad] times
    int *qwide;          // [nq] 1 where the 64-entry chunk q spans more than HK_SUB_FACT_SPAN / omega
    double *qstep;       // [nq] exp(-omega (T_{q+1} - T_q)), T_q the time of chunk q's first entry
    // the subset column pass's row weights, written by k_sub_fin
    double *lw;          // [npad] log2(c_e / lambda_i) (HK_EXP_FLOOR on padding)
    double *colG;        // [n_items][2][HK_WAVE]
    double *gsub;        // [mpad] Eq. 4 on the subset, time order
    double *hsub;        // [mpad] Eq. 5 on the subset, time order
    double *sums;        // [8] loglik pieces of the last evaluation
    // HMC state
    double *z0, *p;      // [m] slot order
    double *off;         // [m] temporal-trend offsets beta t_k, slot order
    double *vz;          // [m] V^{-1} z of the phylogenetic prior, slot order
    double *scal;        // [16] energies and flags
    // feature grids of the learned preconditioner
    int *grid;
    int64_t grid_cap;
};

namespace {

// The subset passes are split into many one-wavefront items (about this many
// each, and at most SUB_ITEM_BATCHES 64-wide batches per item, so that the
// few items that still have work under the underflow cutoff stay short) so
// that the whole chip takes part; partial sums per item are combined in a
// fixed order afterwards.  Measured on the N = 23,422 HMC iteration (M = 1,610):
// column items 4096 -> 8192 (one row chunk per item there) 0.616 -> 0.607 ms,
// 2048 0.623 ms; row items 4096 0.639 ms, 16384 no change (one batch per item
// already).
#ifndef HK_SUB_ROW_ITEMS
#define HK_SUB_ROW_ITEMS 8192
#endif
#ifndef HK_SUB_COL_ITEMS
#define HK_SUB_COL_ITEMS 8192
#endif
constexpr int64_t SUB_ROW_ITEMS = HK_SUB_ROW_ITEMS;
constexpr int64_t SUB_COL_ITEMS = HK_SUB_COL_ITEMS;
#ifndef HK_SUB_FIN_WAVES
#define HK_SUB_FIN_WAVES 16
#endif
constexpr int SUB_FIN_WAVES = HK_SUB_FIN_WAVES;
// partial-sum loads a finalisation wavefront keeps in flight (16 in the
// column finalisation measured slower: 4.95 -> 5.7 us at N = 23,422)
constexpr int SUB_FIN_BATCH = 8;
// wavefronts per row chunk in the subset row finalisation
#ifndef HK_SUB_ROWFIN_WAVES
#define HK_SUB_ROWFIN_WAVES 4
#endif
constexpr int SUB_ROWFIN_WAVES = HK_SUB_ROWFIN_WAVES;
constexpr int64_t SUB_ITEM_BATCHES = 16;
// unroll of the subset sweeps: 8 measured fastest (114 VGPRs, 4 wavefronts per
// SIMD); shorter loops fit more wavefronts but lose more instruction-level
// parallelism than that hides (N = 23,422 HMC iteration, 0.603 ms at 8: 4 ->
// +1.5%, 6 -> +5%, 16 -> +8%, 1 -> +20%)
#ifndef HK_SUB_UNROLL
#define HK_SUB_UNROLL 8
#endif
constexpr int kSubUnroll = HK_SUB_UNROLL;
// a 64-entry (or 64-event) chunk whose times span more than this over omega
// takes the direct exponent instead of the split time factor
#define HK_SUB_FACT_SPAN 40.0

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }

__device__ __forceinline__ void two_sum_acc(float &hi, float &lo, float v) {
    float s = hi + v;
    float bp = s - hi;
    float err = (hi - (s - bp)) + (v - bp);
    hi = s;
    lo += err;
}

__global__ void k_invperm(const int *__restrict__ perm, int64_t n, int *__restrict__ inv) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) inv[perm[i]] = (int)i;
}

__global__ void k_sub_keys(const int64_t *__restrict__ idx, int64_t m, int64_t m2, const int *__restrict__ inv,
                           int64_t n, double *__restrict__ key, int *__restrict__ slot, int *__restrict__ bad) {
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= m2) return;
    if (k < m) {
        int64_t c = idx[k];
        if (c < 0 || c >= n) {
            atomicOr(bad, 1);
            key[k] = 0.0;
        } else {
            key[k] = (double)inv[c];
        }
    } else {
        key[k] = INFINITY;
    }
    slot[k] = (int)k;
}

__global__ void k_sub_layout(const double *__restrict__ key, const int *__restrict__ slot2, int64_t m, int64_t mpad,
                             int *__restrict__ pos, int *__restrict__ slot, int *__restrict__ bad) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= mpad) return;
    if (r < m) {
        pos[r] = (int)key[r];
        slot[r] = slot2[r];
        if (r > 0 && key[r] == key[r - 1]) atomicOr(bad, 1);  // repeated index
    } else {
        pos[r] = 0x7fffffff;
        slot[r] = 0;
    }
}

// ---- static part ---------------------------------------------------------------------
// theta with the subset entries zeroed, sorted, FP32
__global__ void k_sub_static_theta(const double *__restrict__ theta, const int *__restrict__ perm,
                                   const int *__restrict__ pos, int64_t m, int64_t n, int64_t npad,
                                   float *__restrict__ theta_s, int *__restrict__ status) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < npad) {
        float v = 0.0f;
        if (i < n) {
            double th = theta[perm[i]];
            if (!(th >= 0.0) || !isfinite(th)) atomicOr(status, HK_ST_BADTHETA);
            v = (float)th;
        }
        theta_s[i] = v;
    }
}

__global__ void k_sub_zero_subset(const int *__restrict__ pos, int64_t m, float *__restrict__ theta_s) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r < m) theta_s[pos[r]] = 0.0f;
}

// lambda_static_i from the row pass partials (log-likelihood mode: B0, X0) and
// the integral term of everything that does not depend on the subset rates.
__global__ __launch_bounds__(256) void k_sub_static(const double *__restrict__ ts, const double *__restrict__ xs,
                                                    const double *__restrict__ ys, const int *__restrict__ g,
                                                    const double *__restrict__ theta,
                                                    const int *__restrict__ perm, const float *__restrict__ theta_s,
                                                    int64_t n, int ntiles, const int *__restrict__ row_item0,
                                                    const int *__restrict__ row_nseg,
                                                    const float *__restrict__ rowpart,
                                                    const float *__restrict__ colpart,
                                                    const int64_t *__restrict__ colpart_off, const FinConst fc,
                                                    double *__restrict__ lam_static, double *__restrict__ blockpart) {
    __shared__ double sh[HK_WAVES];
    __shared__ double red[HK_WAVES][2];
    __shared__ uint64_t low_mask[HK_WAVES];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (HK_WAVE - 1), wq = threadIdx.x / HK_WAVE;
    double lam_part = 0.0;
    double ls = 1.0;
    if (i < n) {
        const int I = (int)(i / HK_TILE), r = (int)(i % HK_TILE);
        // the log-likelihood-only row pass: B0 (row and column partials) and X0
        double b0 = 0.0, x0 = 0.0;
        for (int sg = 0; sg < row_nseg[I]; ++sg) {
            const float *rp = rowpart + (int64_t)(row_item0[I] + sg) * HK_NROW * HK_TILE + r;
            b0 += rp[0];
            x0 += rp[5 * HK_TILE];
        }
        for (int J = I; J < ntiles; ++J) b0 += (double)colpart[colpart_off[J] + i];
        ls = fc.c_b * b0 * fc.corr + fc.c_e * x0 * fc.corr;
    }
    // rows whose static intensity is below fc.lam_exact (the FP32 pair terms may
    // have lost more than 2^-30 of it) are recomputed from the definitions in
    // FP64 by the whole block, one row at a time: background over every j != i,
    // excitation from the earlier fixed-rate events (theta_s is zero on the subset)
    const uint64_t mine = __ballot(i < n && ls < fc.lam_exact);
    if (lane == 0) low_mask[wq] = mine;
    __syncthreads();
    for (int w = 0; w < HK_WAVES; ++w) {
        for (uint64_t mk = low_mask[w]; mk != 0; mk &= mk - 1) {
            const int rr = __ffsll((unsigned long long)mk) - 1;
            const int64_t ir = blockIdx.x * (int64_t)blockDim.x + w * HK_WAVE + rr;
            const double xi = xs[ir], yi = ys[ir], tsi = ts[ir];
            const int gi = g[ir];
            const double kb = 0.5 / (fc.tau_x * fc.tau_x), kt = 0.5 / (fc.tau_t * fc.tau_t);
            const double kh = 0.5 / (fc.h * fc.h);
            double B0 = 0.0, X0 = 0.0;
            for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
                if (j == ir) continue;
                const double dx = xi - xs[j], dy = yi - ys[j];
                const double r2 = dx * dx + dy * dy;
                const double dt = tsi - ts[j];
                B0 += exp(-(r2 * kb) - dt * dt * kt);
                if (j < gi && theta_s[j] != 0.0f) X0 += theta[perm[j]] * exp(-fc.omega * dt - r2 * kh);
            }
            for (int off = 32; off > 0; off >>= 1) {
                B0 += __shfl_xor(B0, off);
                X0 += __shfl_xor(X0, off);
            }
            if (lane == 0) {
                red[wq][0] = B0;
                red[wq][1] = X0;
            }
            __syncthreads();
            if (threadIdx.x == w * HK_WAVE + rr) {
                double b = red[0][0], x = red[0][1];
                for (int q = 1; q < HK_WAVES; ++q) {
                    b += red[q][0];
                    x += red[q][1];
                }
                ls = fc.c_b * b + fc.c_e * x;
            }
            __syncthreads();
        }
    }
    if (i < n) {
        lam_static[i] = ls;
        // integral term: background (all events) + excitation of the fixed-rate events
        const double ti = ts[i];
        const double u1 = (fc.t1 - ti) / fc.tau_t, u0 = (fc.t0 - ti) / fc.tau_t;
        const double Cn = 0.5 * erfc(-u1 * 0.7071067811865476) - 0.5 * erfc(-u0 * 0.7071067811865476);
        const double one_m = -expm1(-fc.omega * (fc.t1 - ti));
        const double th_fixed = theta_s[i] == 0.0f ? 0.0 : theta[perm[i]];  // subset entries are zeroed
        lam_part = fc.mu0 * Cn + fc.theta0 * th_fixed * one_m;
    } else if (i < (int64_t)ntiles * HK_TILE) {
        lam_static[i] = 1.0;
    }
    // fixed-order block sum
    for (int off = 32; off > 0; off >>= 1) lam_part += __shfl_xor(lam_part, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = lam_part;
    __syncthreads();
    if (threadIdx.x == 0) blockpart[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__global__ void k_sum_blocks(const double *__restrict__ part, int nb, double *__restrict__ out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0, c = 0.0;
        for (int b = 0; b < nb; ++b) {
            const double v = part[b];
            const double t = s + v;
            c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
            s = t;
        }
        out[0] = s + c;
    }
}

__global__ void k_sub_a(const double *__restrict__ ts, const int *__restrict__ pos, int64_t m, int64_t mpad,
                        const FinConst fc, double *__restrict__ a) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= mpad) return;
    a[r] = r < m ? fc.theta0 * -expm1(-fc.omega * (fc.t1 - ts[pos[r]])) : 0.0;
}

// ---- per-evaluation kernels ---------------------------------------------------------------
// log theta_k = z_k + off_k: off is the temporal-trend term beta f(t_k) of Sec.
// 2.2 (slot order), or NULL for none.
__device__ __forceinline__ double zeff(const double *__restrict__ z, const double *__restrict__ off, int64_t k) {
    return off ? z[k] + off[k] : z[k];
}

// off_k = beta t_k for the subset events (their times, slot order)
__global__ void k_sub_offset(const double *__restrict__ ts, const int *__restrict__ pos,
                             const int *__restrict__ slot, int64_t m, double beta, double *__restrict__ off) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r < m) off[slot[r]] = beta * ts[pos[r]];
}

// theta_k = exp(z_k) into the caller's full rate vector, and the staged subset
// entries of this evaluation in time order: pre-scaled coordinates, times, the
// rate with the split time factor of its 64-entry chunk, the chunk's split flag
// and step factor.  One wavefront per chunk (the grid covers mpad exactly).
__global__ __launch_bounds__(256) void k_sub_theta(
    const double *__restrict__ z, const double *__restrict__ off, const int *__restrict__ slot,
    const int64_t *__restrict__ cidx, int64_t m, const int *__restrict__ pos, const double *__restrict__ ts,
    const double *__restrict__ xs, const double *__restrict__ ys, const PairConst kc, float *__restrict__ tv,
    double2 *__restrict__ sxy, double *__restrict__ sts, int *__restrict__ qwide, double *__restrict__ qstep,
    double *__restrict__ theta_full) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (HK_WAVE - 1);
    const int64_t r0 = r - lane;  // the chunk's first entry
    const bool valid = r < m;
    const int pj = valid ? pos[r] : 0;
    const double t = ts[pj];
    const double Tq = r0 < m ? ts[pos[r0]] : 0.0;  // chunks past m hold padding only
    const double dt = valid ? t - Tq : 0.0;
    const bool wide = __any(valid && kc.omega * dt > HK_SUB_FACT_SPAN);
    if (valid) {
        const int k = slot[r];
        const double ze = zeff(z, off, k);
        if (theta_full) theta_full[cidx[k]] = exp(ze);
        tv[r] = (float)exp(wide ? ze : ze + kc.omega * dt);
        sxy[r] = make_double2(xs[pj] * kc.sx, ys[pj] * kc.sx);
        sts[r] = t;
    } else {
        tv[r] = 0.0f;
        sxy[r] = make_double2(0.0, 0.0);
        sts[r] = 0.0;
    }
    if (lane == 0) {
        const int64_t q = r0 / HK_WAVE;
        qwide[q] = wide;
        qstep[q] = r0 + HK_WAVE < m ? exp(-kc.omega * (ts[pos[r0 + HK_WAVE]] - Tq)) : 0.0;
    }
}

// Subset excitation per event: a wavefront owns the 64 rows of a chunk and
// sweeps subset entries that precede the chunk's end, staged 64 at a time (one
// 64-entry subset chunk) through LDS.  The time factor of E is split at the
// chunk's first entry time as in the full row pass (FP64 factors, spatial
// exponent in the loop) unless the chunk spans more than HK_SUB_FACT_SPAN /
// omega in time.  The exponent is formed in FP64 from coordinates pre-scaled by
// sqrt(-kex), so it carries no rounded FP32 constant; the split form rounds the
// spatial exponent once to FP32, the unsplit one adds the FP64 time term and
// splits the whole exponent into an exact power of two and an FP32 fraction
// (rounding it whole would give a term an error that grows with its decay).

// 2^e for an FP64 exponent: exact integer part, FP32 fraction (a term's
// relative error then does not grow with |e|)
__device__ __forceinline__ float sub_exp2_split(double e) {
    const double n = rint(e);
    return __builtin_amdgcn_ldexpf(fexp2((float)(e - n)), (int)n);
}

template <bool MASKED, bool FACT>
__device__ __forceinline__ void sub_row_sweep(const double2 *__restrict__ rxy, const float *__restrict__ rv,
                                              const double *__restrict__ rtd, const int *__restrict__ rpos,
                                              double tsi, double xr, double yr, int gr, const PairConst kc,
                                              double &acc) {
#pragma unroll kSubUnroll
    for (int s = 0; s < HK_WAVE; ++s) {
        const double2 pk = rxy[s];
        const double dx = xr - pk.x, dy = yr - pk.y;
        const double aed = -fma(dx, dx, dy * dy);
        // unsplit (a wide batch): the whole exponent, time term included, is
        // split into an exact power of two and an FP32 fraction
        float E = FACT ? fexp2((float)aed) : sub_exp2_split(fmax(fma(tsi - rtd[s], kc.kw_d, aed), HK_EXP_FLOOR));
        if (MASKED && !(rpos[s] < gr)) E = 0.0f;
        acc += (double)(E * rv[s]);
    }
}

// One item: the 64 rows of a chunk against a range of the subset entries that
// precede the chunk's end (64 at a time through LDS); the rows' partial sums go
// to the item's slot.
__global__ __launch_bounds__(HK_WAVE) void k_sub_row(
    const double *__restrict__ ts, const double *__restrict__ xs, const double *__restrict__ ys, const int *__restrict__ g,
    const int *__restrict__ pos, const float *__restrict__ tv, const double2 *__restrict__ sxy,
    const double *__restrict__ sts, const int *__restrict__ qwide, const double *__restrict__ qstep,
    const hk_item *__restrict__ ritems, const PairConst kc, double *__restrict__ xpart) {
    __shared__ double2 rxy[HK_WAVE];
    __shared__ float rv[HK_WAVE];
    __shared__ double rtd[HK_WAVE];
    __shared__ int rpos[HK_WAVE];
    const hk_item it = ritems[blockIdx.x];
    const int b = it.tile;
    const int lane = threadIdx.x;
    const int64_t i = (int64_t)b * HK_WAVE + lane;
    const double tsi = ts[i];
    const double xr = xs[i] * kc.sx, yr = ys[i] * kc.sx;
    const int gr = g[i];
    double acc = 0.0;  // every term in FP64 (see the row pass: FP32 sums drop small terms)
    // under the cutoff, batches whose last entry precedes the chunk's first row
    // by more than dt_cut_ex are skipped (entries are in time order)
    const double chunk_tmin = ts[(int64_t)b * HK_WAVE];
    const int g_first = g[(int64_t)b * HK_WAVE];  // g is non-decreasing
    // batches are the 64-entry subset chunks (items start on chunk boundaries),
    // walked from late to early: the row's split factor exp(-omega (t_i - T_q)) is
    // evaluated at the first batch that has a causal pair (where it is at most 1)
    // and carried down by the chunks' step factors
    double ui = 0.0;
    bool have_ui = false;
    const int c_last = it.c_begin + (it.c_end - 1 - it.c_begin) / HK_WAVE * HK_WAVE;
    // a batch's entries are loaded into registers one batch ahead, so that the
    // loads of the next batch are in flight during this one's sweep (the subset
    // arrays are padded to whole 256-entry tiles: every lane's load is in bounds)
    double2 nxy = sxy[c_last + lane];
    float nv = tv[c_last + lane];
    double nt = sts[c_last + lane];
    int np = pos[c_last + lane];
    for (int c0 = c_last; c0 >= it.c_begin; c0 -= HK_WAVE) {
        const int q = c0 / HK_WAVE;
        if (have_ui) ui *= qstep[q];
        const int cend = min(c0 + HK_WAVE, it.c_end);
        const double2 pxy = nxy;
        const float pv = nv;
        const double pt = nt;
        const int pp = np;
        if (c0 - HK_WAVE >= it.c_begin) {
            const int rn = c0 - HK_WAVE + lane;
            nxy = sxy[rn];
            nv = tv[rn];
            nt = sts[rn];
            np = pos[rn];
        }
        if (chunk_tmin - sts[cend - 1] > kc.dt_cut_ex) continue;
        const bool fact = qwide[q] == 0;
        {
            // entries past the item's range carry rate 0 and a time of -inf: the
            // unsplit exponent is then -inf and the term exactly 0 (a later
            // entry's own time could make it +inf, and inf * 0 a NaN)
            const bool valid = c0 + lane < cend;
            rxy[lane] = pxy;
            rv[lane] = valid ? pv : 0.0f;
            rtd[lane] = valid ? pt : -INFINITY;
            rpos[lane] = valid ? pp : 0x7fffffff;
        }
        __syncthreads();
        double accb = 0.0;
        // a batch whose entries all precede the chunk's first tie group needs no
        // causality mask (padding entries carry rate 0)
        if (rpos[cend - 1 - c0] < g_first) {
            if (fact) sub_row_sweep<false, true>(rxy, rv, rtd, rpos, tsi, xr, yr, gr, kc, accb);
            else sub_row_sweep<false, false>(rxy, rv, rtd, rpos, tsi, xr, yr, gr, kc, accb);
        } else {
            if (fact) sub_row_sweep<true, true>(rxy, rv, rtd, rpos, tsi, xr, yr, gr, kc, accb);
            else sub_row_sweep<true, false>(rxy, rv, rtd, rpos, tsi, xr, yr, gr, kc, accb);
        }
        if (accb != 0.0) {
            if (fact) {
                if (!have_ui) {
                    ui = exp(-kc.omega * (tsi - rtd[0]));
                    have_ui = true;
                }
                acc += ui * accb;
            } else {
                acc += accb;
            }
        }
        __syncthreads();
    }
    xpart[(int64_t)blockIdx.x * HK_WAVE + lane] = acc;
}

// One block per 64-row chunk.  Its SUB_ROWFIN_WAVES wavefronts split the
// chunk's row items (late chunks have the most, one per run of subset sources
// before them) and combine their partial sums in a fixed order, so that the
// partial-sum reads are in flight together; wavefront 0 then finalises the
// rows.  The chunk's sum of log lambda goes to blockpart[chunk], and the
// subset column pass's weight w_i = c_e / lambda_i to lw as its log2 (FP64).
__global__ __launch_bounds__(SUB_ROWFIN_WAVES * HK_WAVE) void k_sub_fin(const double *__restrict__ lam_static,
                                                 const int *__restrict__ ritem0, const int *__restrict__ rnseg,
                                                 const double *__restrict__ xpart, const double *__restrict__ ts,
                                                 const double *__restrict__ xs, const double *__restrict__ ys,
                                                 const int *__restrict__ g, const int *__restrict__ pos,
                                                 const float *__restrict__ tv, const double *__restrict__ sts,
                                                 const int *__restrict__ qwide, int64_t m,
                                                 int64_t n, int64_t npad, const FinConst fc,
                                                 double *__restrict__ lam, double *__restrict__ lw,
                                                 double *__restrict__ blockpart, int *__restrict__ status) {
    __shared__ double part[SUB_ROWFIN_WAVES][HK_WAVE];
    const int b = blockIdx.x, lane = threadIdx.x & (HK_WAVE - 1);
    const int wq = __builtin_amdgcn_readfirstlane(threadIdx.x / HK_WAVE);
    const int64_t i0 = (int64_t)b * HK_WAVE;  // the chunk's first event
    const int64_t i = i0 + lane;
    // the static part is fetched before the reduction, so that its latency
    // overlaps the partial-sum reads
    double lst = 0.0;
    if (i < n) lst = lam_static[i];
    {
        double x = 0.0;
        if (i < n) {
            const double *xp = xpart + (int64_t)ritem0[b] * HK_WAVE + lane;
            const int ns = rnseg[b];
            // batches of SUB_FIN_BATCH loads issue together (absent ones read as
            // zero, which adds exactly); the adds keep the items' order
            for (int base = wq; base < ns; base += SUB_FIN_BATCH * SUB_ROWFIN_WAVES) {
                double v[SUB_FIN_BATCH];
#pragma unroll
                for (int k = 0; k < SUB_FIN_BATCH; ++k) {
                    const int sg = base + k * SUB_ROWFIN_WAVES;
                    v[k] = sg < ns ? xp[(int64_t)sg * HK_WAVE] : 0.0;
                }
#pragma unroll
                for (int k = 0; k < SUB_FIN_BATCH; ++k) x += v[k];
            }
        }
        part[wq][lane] = x;
    }
    __syncthreads();
    double x = part[0][lane];
#pragma unroll
    for (int k = 1; k < SUB_ROWFIN_WAVES; ++k) x += part[k][lane];
    // rows whose intensity is below fc.lam_exact (the FP32 terms may have lost
    // more than 2^-30 of it) take the subset excitation from the definitions
    // in FP64, the whole block on one row at a time; every wavefront derives
    // the same mask
    __shared__ double xred[SUB_ROWFIN_WAVES];
    __shared__ double xexact[HK_WAVE];
    const bool low = i < n && lst + fc.c_e * fc.corr * x < fc.lam_exact;
    for (uint64_t mk = __ballot(low); mk != 0; mk &= mk - 1) {
        const int rr = __ffsll((unsigned long long)mk) - 1;
        const int64_t ir = i0 + rr;
        const double xi = xs[ir], yi = ys[ir], ti = ts[ir];
        const int gi = g[ir];
        const double kh = 0.5 / (fc.h * fc.h);
        double xs_sum = 0.0;
        for (int64_t r = threadIdx.x; r < m; r += SUB_ROWFIN_WAVES * HK_WAVE) {
            const int pk = pos[r];
            if (pk >= gi) continue;  // entries are in time order; only earlier events excite
            const double dx = xi - xs[pk], dy = yi - ys[pk];
            const double r2 = dx * dx + dy * dy;
            // tv carries theta_r exp(omega (t_r - T_q)) on a split chunk q
            const int64_t q = r / HK_WAVE;
            const double tq = qwide[q] ? sts[r] : sts[q * HK_WAVE];
            xs_sum += (double)tv[r] * exp(-fc.omega * (ti - tq) - r2 * kh);
        }
        for (int off = 32; off > 0; off >>= 1) xs_sum += __shfl_xor(xs_sum, off);
        if (lane == 0) xred[wq] = xs_sum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double v = xred[0];
            for (int k = 1; k < SUB_ROWFIN_WAVES; ++k) v += xred[k];
            xexact[rr] = v;
        }
        __syncthreads();
    }
    if (wq != 0) return;
    double v = 0.0;
    if (i < n) {
        const double l = low ? lst + fc.c_e * xexact[lane] : lst + fc.c_e * fc.corr * x;
        lam[i] = l;
        if (!(l > 0.0)) atomicOr(status, isnan(l) ? HK_ST_NONFINITE : HK_ST_ZERO);
        v = log(l);
        lw[i] = l > 0.0 ? fmax(fc.log2_ce - v * 1.4426950408889634, HK_EXP_FLOOR) : HK_EXP_FLOOR;
    } else {
        lam[i] = 1.0;
        lw[i] = HK_EXP_FLOOR;
    }
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) blockpart[b] = v;
}

// Column pass on the subset: lanes own subset entries (time order), rows are
// all events after them, broadcast from LDS.  Each term c_e E_ik / lambda_i is
// the exponential of its whole exponent,
//   e_ik = log2(c_e / lambda_i) - omega (t_i - t_k) / ln2 - |s (x_i - x_k)|^2,
// formed in FP64.  With Eq. 5 (WITH_H) the exponent is split into an exact
// power of two and an FP32 fraction, as in the full column pass: Eq. 5 squares
// the terms and its small entries are sums of terms with large |e|.  For
// Eq. 4 alone the row's weight is split instead: n_i = rint(log2(c_e /
// lambda_i)) is applied exactly (ldexp) and the rest of the exponent, which is
// small for the terms that make up G_k, is rounded once to FP32 (relative
// error about 2^-24 ln2 |e_ik - n_i| per term: far below Eq. 4's bound for the
// terms that carry the sum, larger only for terms that are negligible in it).
struct SubColRow {  // one staged row
    double2 u;      // DOT: 2 u_i; else u_i (u = s x)
    double c;       // lw_i + kw (t_i - T_ref) (DOT: minus |u_i|^2), at least HK_EXP_FLOOR; Eq. 4 alone: minus n
    int n;          // Eq. 4 alone: rint(lw_i) (0 for a row at the floor), applied exactly
};

template <bool WITH_H, bool SPLIT, bool MASKED, bool DOT>
__device__ __forceinline__ void sub_col_sweep(const SubColRow *__restrict__ rows, const int *__restrict__ rg, int pj,
                                              double xk, double yk, double dk, float &G, float &H) {
#pragma unroll kSubUnroll
    for (int s = 0; s < HK_WAVE; ++s) {
        const SubColRow r = rows[s];
        double e;
        if (DOT) {
            e = fma(r.u.x, xk, fma(r.u.y, yk, r.c + dk));
        } else {
            const double dx = r.u.x - xk, dy = r.u.y - yk;
            e = fma(-dx, dx, fma(-dy, dy, r.c + dk));
        }
        float T = SPLIT ? sub_exp2_split(e) : __builtin_amdgcn_ldexpf(fexp2((float)e), r.n);
        if (MASKED && !(pj < rg[s])) T = 0.0f;
        G += T;
        if (WITH_H) H = fmaf(T, T, H);
    }
}

// One item: a chunk of 64 subset entries (the lanes) against a range of row
// chunks after them; the entries' partial sums go to the item's slot.  Times
// enter relative to the subset chunk's first entry.
template <bool WITH_H, bool DOT>
__global__ __launch_bounds__(HK_WAVE) void k_sub_col(const double *__restrict__ ts, const double *__restrict__ xs,
                                                      const double *__restrict__ ys, const double *__restrict__ lw,
                                                      const int *__restrict__ g, const int *__restrict__ pos,
                                                      const double2 *__restrict__ sxy, const double *__restrict__ sts,
                                                      int64_t m, const hk_item *__restrict__ items,
                                                      const PairConst kc, double *__restrict__ colG) {
    __shared__ SubColRow rows[HK_WAVE];
    __shared__ int rg[HK_WAVE];
    const hk_item it = items[blockIdx.x];
    const int lane = threadIdx.x;
    const int64_t q0 = (int64_t)it.tile * HK_WAVE;
    const int64_t r = q0 + lane;
    const bool live = r < m;
    const int pj = live ? pos[r] : 0;
    const double t_ref = sts[q0];
    const double2 pxy = sxy[r];
    double dk = -kc.kw_d * (sts[r] - t_ref);
    if (DOT) dk -= fma(pxy.x, pxy.x, pxy.y * pxy.y);
    if (!live) dk = HK_EXP_FLOOR;
    // the chunk's latest entry (entries are in time order)
    const int64_t r_last = min(q0 + HK_WAVE, m) - 1;
    const double q_tmax = sts[r_last];
    const int pos_last = pos[r_last];
    double Gd = 0.0, Hd = 0.0;
    // a row chunk is loaded into registers one chunk ahead, so that the loads of
    // the next chunk are in flight during this one's sweep (items are never empty)
    int ng;
    double nx, ny, nl, nt;
    {
        const int64_t i = (int64_t)it.c_begin * HK_WAVE + lane;
        nx = xs[i];
        ny = ys[i];
        nl = lw[i];
        nt = ts[i];
        ng = g[i];
    }
    for (int c = it.c_begin; c < it.c_end; ++c) {
        const int pg = ng;
        const double px = nx, py = ny, pl = nl, pt = nt;
        if (c + 1 < it.c_end) {
            const int64_t i = (int64_t)(c + 1) * HK_WAVE + lane;
            nx = xs[i];
            ny = ys[i];
            nl = lw[i];
            nt = ts[i];
            ng = g[i];
        }
        const double Tc = ts[(int64_t)c * HK_WAVE];
        if (Tc - q_tmax > kc.dt_cut_ex) break;  // cutoff: all later rows too far
        bool split = WITH_H;
        {
            const double ux = px * kc.sx, uy = py * kc.sx;
            double cr = pl + kc.kw_d * (pt - t_ref);
            SubColRow w;
            if (DOT) {
                cr -= fma(ux, ux, uy * uy);
                w.u = make_double2(2.0 * ux, 2.0 * uy);
            } else {
                w.u = make_double2(ux, uy);
            }
            w.c = fmax(cr, HK_EXP_FLOOR);
            w.n = 0;
            // a row whose weight is at the floor (zero weight, padding) keeps its
            // whole exponent in c, which then stays at the floor; a chunk with a
            // row of large weight splits every exponent exactly
            split = !WITH_H && __ballot(pl > HK_LW_SPLIT_MAX) != 0;
            if (!WITH_H && !split && pl > HK_EXP_FLOOR) {
                const double nw = rint(pl);
                w.n = (int)nw;
                w.c -= nw;
            }
            rows[lane] = w;
            rg[lane] = pg;
        }
        __syncthreads();
        float G = 0.0f, H = 0.0f;
        // rows whose tie groups all start after the chunk's last entry need no mask
        if (pos_last < rg[0]) {
            if (WITH_H || split)
                sub_col_sweep<WITH_H, true, false, DOT>(rows, rg, pj, pxy.x, pxy.y, dk, G, H);
            else
                sub_col_sweep<WITH_H, false, false, DOT>(rows, rg, pj, pxy.x, pxy.y, dk, G, H);
        } else {
            if (WITH_H || split)
                sub_col_sweep<WITH_H, true, true, DOT>(rows, rg, pj, pxy.x, pxy.y, dk, G, H);
            else
                sub_col_sweep<WITH_H, false, true, DOT>(rows, rg, pj, pxy.x, pxy.y, dk, G, H);
        }
        Gd += (double)G;
        if (WITH_H) Hd += (double)H;
        __syncthreads();
    }
    double *cg = colG + (int64_t)blockIdx.x * 2 * HK_WAVE;
    cg[lane] = live ? Gd : 0.0;
    if (WITH_H) cg[HK_WAVE + lane] = live ? Hd : 0.0;
}

// A leapfrog update fused into the column finalisation: with g = Eq. 4 at the
// current z, the log-posterior gradient in z is theta g - P z / sigma^2 (P the
// prior precision direction, pv = z or V^{-1} z), then p += a_p grad and, when
// a_z != 0, z += a_z p / M and the subset rates for the next evaluation.
struct SubUpd {
    const int *slot;
    double *z;
    const double *off;
    const double *pv;
    double inv_s2;
    double *p;
    const double *mass;
    double a_p, a_z;
    float *tv;            // staged subset rates (k_sub_theta's layout)
    const double *sts;
    const int *qwide;
    double omega;
};

// Per 64-entry subset chunk: the SUB_FIN_WAVES wavefronts split the chunk's
// items round robin, then the first combines them in a fixed order (and, with
// UPD, applies the leapfrog update to its entries).
template <bool UPD>
__global__ __launch_bounds__(SUB_FIN_WAVES * HK_WAVE) void k_sub_colfin(
    const int *__restrict__ item0, const int *__restrict__ nseg, const double *__restrict__ colG,
    const double *__restrict__ a, int64_t m, const FinConst fc, bool with_h, double *__restrict__ gsub,
    double *__restrict__ hsub, const SubUpd u) {
    __shared__ double part[SUB_FIN_WAVES][2][HK_WAVE];
    const int q = blockIdx.x, lane = threadIdx.x & (HK_WAVE - 1);
    const int wq = __builtin_amdgcn_readfirstlane(threadIdx.x / HK_WAVE);
    const int64_t r = (int64_t)q * HK_WAVE + lane;
    const bool fin = wq == 0 && r < m;
    // the operands of the finalisation and of the update are fetched before the
    // reduction, so that their latency (a gather through the slot) overlaps the
    // partial-sum reads; each slot belongs to one entry, so no other thread
    // writes them in between
    double ar = 0.0, zk = 0.0, offk = 0.0, pvk = 0.0, pk0 = 0.0, massk = 1.0, dts = 0.0;
    int k = 0, wide = 1;
    if (fin) {
        ar = a[r];
        if (UPD) {
            k = u.slot[r];
            zk = u.z[k];
            if (u.off) offk = u.off[k];
            pvk = u.pv[k];
            pk0 = u.p[k];
            if (u.a_z != 0.0) {
                massk = u.mass[k];
                wide = u.qwide[q];
                dts = u.sts[r] - u.sts[(int64_t)q * HK_WAVE];
            }
        }
    }
    double G = 0.0, H = 0.0;
    const int ns = nseg[q], i0 = item0[q];
    // batches of SUB_FIN_BATCH loads issue together (absent ones read as zero,
    // which adds exactly); the adds keep the items' order
    for (int base = wq; base < ns; base += SUB_FIN_BATCH * SUB_FIN_WAVES) {
        double vg[SUB_FIN_BATCH], vh[SUB_FIN_BATCH];
#pragma unroll
        for (int e = 0; e < SUB_FIN_BATCH; ++e) {
            const int sg = base + e * SUB_FIN_WAVES;
            const double *cg = colG + (int64_t)(i0 + sg) * 2 * HK_WAVE + lane;
            vg[e] = sg < ns ? cg[0] : 0.0;
            vh[e] = with_h && sg < ns ? cg[HK_WAVE] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < SUB_FIN_BATCH; ++e) {
            G += vg[e];
            H += vh[e];
        }
    }
    part[wq][0][lane] = G;
    part[wq][1][lane] = H;
    __syncthreads();
    if (!fin) return;
    double Gs = part[0][0][lane], Hs = part[0][1][lane];
    for (int w = 1; w < SUB_FIN_WAVES; ++w) {
        Gs += part[w][0][lane];
        Hs += part[w][1][lane];
    }
    const double g = Gs * fc.corr - ar;
    gsub[r] = g;
    if (with_h) hsub[r] = Hs * fc.corr * fc.corr;
    if (UPD) {
        const double gz = exp(u.off ? zk + offk : zk) * g - pvk * u.inv_s2;
        const double pk = pk0 + u.a_p * gz;
        u.p[k] = pk;
        if (u.a_z != 0.0) {
            const double zn = zk + u.a_z * pk / massk;
            u.z[k] = zn;
            const double ze = u.off ? zn + offk : zn;
            u.tv[r] = (float)exp(wide ? ze : ze + u.omega * dts);
        }
    }
}

// Scatter the subset results to the caller's slot order.
__global__ void k_sub_scatter(const int *__restrict__ slot, int64_t m, const double *__restrict__ gsub,
                              const double *__restrict__ hsub, double *__restrict__ g_out,
                              double *__restrict__ h_out) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= m) return;
    const int k = slot[r];
    if (g_out) g_out[k] = gsub[r];
    if (h_out) h_out[k] = hsub[r];
}

// Deterministic single-block sums over the subset (m is at most a few 1e4).
// out[0] = sum log lambda (from block partials), out[1] = sum theta_k a_k,
// out[2] = sum z_k^2, out[3] = sum p_k^2 / M_k
constexpr int ENERGY_THREADS = 1024;
constexpr int ENERGY_BATCH = 4;
__global__ __launch_bounds__(ENERGY_THREADS) void k_sub_energy(const double *__restrict__ loglam_part, int nb,
                                                    const double *__restrict__ z, const double *__restrict__ off,
                                                    const double *__restrict__ p,
                                                    const double *__restrict__ mass, const int *__restrict__ slot,
                                                    const double *__restrict__ a, int64_t m,
                                                    double *__restrict__ out) {
    __shared__ double sh[4][ENERGY_THREADS];
    const int t = threadIdx.x;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = t; b < nb; b += ENERGY_THREADS) s[0] += loglam_part[b];
    // a thread's entries are gathered ENERGY_BATCH at a time (the loads through
    // the slot issue together), then summed in entry order
    for (int64_t base = t; base < m; base += (int64_t)ENERGY_BATCH * ENERGY_THREADS) {
        int k[ENERGY_BATCH];
        double zk[ENERGY_BATCH], ok[ENERGY_BATCH], pk[ENERGY_BATCH], mk[ENERGY_BATCH], ak[ENERGY_BATCH];
#pragma unroll
        for (int e = 0; e < ENERGY_BATCH; ++e) {
            const int64_t r = base + (int64_t)e * ENERGY_THREADS;
            k[e] = r < m ? slot[r] : 0;
            ak[e] = r < m ? a[r] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < ENERGY_BATCH; ++e) {
            const bool in = base + (int64_t)e * ENERGY_THREADS < m;
            zk[e] = in ? z[k[e]] : 0.0;
            ok[e] = in && off ? off[k[e]] : 0.0;
            pk[e] = in && p ? p[k[e]] : 0.0;
            mk[e] = in && p ? mass[k[e]] : 1.0;
        }
#pragma unroll
        for (int e = 0; e < ENERGY_BATCH; ++e) {
            if (base + (int64_t)e * ENERGY_THREADS >= m) break;
            s[1] += exp(off ? zk[e] + ok[e] : zk[e]) * ak[e];
            s[2] += zk[e] * zk[e];
            if (p) s[3] += pk[e] * pk[e] / mk[e];
        }
    }
    for (int q = 0; q < 4; ++q) sh[q][t] = s[q];
    __syncthreads();
    for (int h = ENERGY_THREADS / 2; h > 0; h >>= 1) {
        if (t < h)
            for (int q = 0; q < 4; ++q) sh[q][t] += sh[q][t + h];
        __syncthreads();
    }
    if (t < 4) out[t] = sh[t][0];
}

// ---- Philox-4x32-10 (Salmon et al. 2011) ------------------------------------------------
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

// p_k = sqrt(M_k) N(0,1): element k uses counter (k, 0, counter_lo, counter_hi);
// z0 <- z (start of the trajectory)
__global__ void k_hmc_init(int64_t m, uint64_t seed, uint64_t counter, const double *__restrict__ mass,
                           const double *__restrict__ z, double *__restrict__ p, double *__restrict__ z0) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= m) return;
    uint32_t c[4] = {(uint32_t)k, 0u, (uint32_t)counter, (uint32_t)(counter >> 32)};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = u53(c[0], c[1]), u2 = u53(c[2], c[3]);
    const double nrm = sqrt(-2.0 * log1p(-u1)) * cos(6.283185307179586 * u2);
    p[k] = sqrt(mass[k]) * nrm;
    z0[k] = z[k];
}

// Energies: scal[0..3] start sums, scal[4..7] end sums (k_sub_energy layout).
// H = -(sum log lambda - Lam_static - theta0-part) + sum z^2/(2 s^2) + sum p^2/(2M)
__global__ void k_hmc_accept(const double *__restrict__ scal, const double *__restrict__ Lam_static,
                             double inv_s2, uint64_t seed, uint64_t counter, int64_t m,
                             const double *__restrict__ z0, double *__restrict__ z, double *__restrict__ z_prop,
                             double *__restrict__ out, int *__restrict__ flag) {
    __shared__ int acc;
    if (threadIdx.x == 0) {
        const double ll0 = scal[0] - Lam_static[0] - scal[1];
        const double ll1 = scal[4] - Lam_static[0] - scal[5];
        const double lp0 = ll0 - 0.5 * scal[2] * inv_s2;
        const double lp1 = ll1 - 0.5 * scal[6] * inv_s2;
        const double H0 = -lp0 + 0.5 * scal[3];
        const double H1 = -lp1 + 0.5 * scal[7];
        const double dH = H1 - H0;
        uint32_t c[4] = {0u, 1u, (uint32_t)counter, (uint32_t)(counter >> 32)};
        philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        const double u = u53(c[0], c[1]);
        const int a = (isfinite(dH) && log(u) < -dH) ? 1 : 0;
        acc = a;
        flag[0] = a;
        out[0] = (double)a;
        out[1] = dH;
        out[2] = a ? ll1 : ll0;
        out[3] = a ? lp1 : lp0;
        out[4] = isfinite(dH) ? fmin(1.0, exp(-dH)) : 0.0;
        out[5] = ll1;
        out[6] = H0;
        out[7] = H1;
    }
    __syncthreads();
    for (int64_t k = threadIdx.x; k < m; k += blockDim.x) {
        if (z_prop) z_prop[k] = z[k];
        if (!acc) z[k] = z0[k];
    }
}

// theta_full[idx_k] = exp(z_k) (after a rejection restores z)
__global__ void k_sub_theta_full(const double *__restrict__ z, const double *__restrict__ off,
                                 const int64_t *__restrict__ cidx, int64_t m, double *__restrict__ theta_full) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < m) theta_full[cidx[k]] = exp(zeff(z, off, k));
}

template <class T>
hipError_t dalloc(T **p, size_t count) {
    return hipMalloc((void **)p, count * sizeof(T) + 16);
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void hk_subset_free(hawkes_plan p) {
    hk_subset *s = p->sub;
    if (!s) return;
    void *ptrs[] = {s->pos, s->slot, s->cidx, s->ritems, s->ritem0, s->rnseg, s->xpart, s->items, s->item0, s->nseg,
                    s->lam_static, s->Lam_static, s->a, s->tv, s->sxy, s->sts, s->qwide, s->qstep, s->lw, s->colG, s->gsub, s->hsub, s->sums, s->z0, s->p, s->off, s->vz, s->scal,
                    s->grid};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    delete s;
    p->sub = nullptr;
}

extern "C" hawkes_status hawkes_plan_set_subset(hawkes_plan p, int64_t m, const int64_t *d_idx,
                                                hipStream_t stream) {
    if (!p || !d_idx || m < 1 || m > p->n) return HAWKES_E_INVALID;
    hk_subset_free(p);
    hk_subset *s = new hk_subset();
    memset(s, 0, sizeof(*s));
    p->sub = s;
    p->last_stream = stream;
    s->m = m;
    s->mpad = (m + HK_TILE - 1) / HK_TILE * HK_TILE;
#define SC(call)                                                              \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) {                                               \
            hk_subset_free(p);                                                \
            return e_ == hipErrorOutOfMemory ? HAWKES_E_NOMEM : HAWKES_E_DEVICE; \
        }                                                                     \
    } while (0)
    int64_t m2 = 1;
    while (m2 < m) m2 <<= 1;
    int *inv = nullptr, *slot2 = nullptr, *bad = nullptr;
    double *key = nullptr;
    SC(dalloc(&inv, p->n));
    SC(dalloc(&key, m2));
    SC(dalloc(&slot2, m2));
    SC(dalloc(&bad, 1));
    SC(hipMemsetAsync(bad, 0, sizeof(int), stream));
    hipLaunchKernelGGL(k_invperm, dim3(nblk(p->n, 256)), dim3(256), 0, stream, p->perm, p->n, inv);
    hipLaunchKernelGGL(k_sub_keys, dim3(nblk(m2, 256)), dim3(256), 0, stream, d_idx, m, m2, inv, p->n, key, slot2,
                       bad);
    SC(hk_sort_pairs(key, slot2, m2, stream));
    SC(dalloc(&s->pos, s->mpad));
    SC(dalloc(&s->slot, s->mpad));
    SC(dalloc(&s->cidx, m));
    hipLaunchKernelGGL(k_sub_layout, dim3(nblk(s->mpad, 256)), dim3(256), 0, stream, key, slot2, m, s->mpad, s->pos,
                       s->slot, bad);
    SC(hipMemcpyAsync(s->cidx, d_idx, sizeof(int64_t) * m, hipMemcpyDeviceToDevice, stream));
    SC(hipGetLastError());
    std::vector<int> hpos(m);
    int hbad = 0;
    SC(hipMemcpyAsync(hpos.data(), s->pos, sizeof(int) * m, hipMemcpyDeviceToHost, stream));
    SC(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, stream));
    SC(hipStreamSynchronize(stream));
    (void)hipFree(inv);
    (void)hipFree(key);
    (void)hipFree(slot2);
    (void)hipFree(bad);
    if (hbad) {
        hk_subset_free(p);
        return HAWKES_E_INVALID;
    }
    // row pass schedule: row chunk b pairs with the subset entries before its end
    // (cnt_b of them, a prefix in time order), in items of at most BR entries
    const int nch = p->nchunks;
    std::vector<int> cnt(nch);
    {
        int64_t r = 0;
        for (int b = 0; b < nch; ++b) {
            while (r < m && hpos[(size_t)r] < HK_WAVE * (b + 1)) ++r;
            cnt[b] = (int)r;
        }
    }
    int64_t wrow = 0;
    for (int b = 0; b < nch; ++b) wrow += cnt[b];
    const int64_t br = std::min<int64_t>(SUB_ITEM_BATCHES, std::max<int64_t>(1, (wrow + SUB_ROW_ITEMS * HK_WAVE - 1) /
                                                                                   (SUB_ROW_ITEMS * HK_WAVE))) *
                       HK_WAVE;
    std::vector<hk_item> ritems;
    std::vector<int> ritem0(nch), rnseg(nch);
    for (int b = 0; b < nch; ++b) {
        ritem0[b] = (int)ritems.size();
        int seg = 0;
        for (int64_t e = 0; e < cnt[b]; e += br)
            ritems.push_back({b, (int)e, (int)std::min<int64_t>(e + br, cnt[b]), seg++});
        rnseg[b] = seg;
    }
    // column pass schedule: subset chunk q sweeps the row chunks from the chunk of
    // its earliest entry to the end, in items of sc chunks
    s->nq = (int)(s->mpad / HK_WAVE);
    const int nq_live = (int)((m + HK_WAVE - 1) / HK_WAVE);
    int64_t wcol = 0;
    for (int q = 0; q < nq_live; ++q) wcol += nch - hpos[(size_t)q * HK_WAVE] / HK_WAVE;
    const int sc = (int)std::min<int64_t>(SUB_ITEM_BATCHES,
                                          std::max<int64_t>(1, (wcol + SUB_COL_ITEMS - 1) / SUB_COL_ITEMS));
    std::vector<hk_item> items;
    std::vector<int> item0(s->nq, 0), nseg(s->nq, 0);
    for (int q = 0; q < nq_live; ++q) {
        const int first = hpos[(size_t)q * HK_WAVE] / HK_WAVE;
        item0[q] = (int)items.size();
        int seg = 0;
        for (int c = first; c < nch; c += sc) items.push_back({q, c, std::min(c + sc, nch), seg++});
        nseg[q] = seg;
    }
    for (int q = nq_live; q < s->nq; ++q) item0[q] = (int)items.size();
    s->n_ritems = (int)ritems.size();
    s->n_items = (int)items.size();
    SC(dalloc(&s->ritems, std::max<size_t>(1, ritems.size())));
    SC(dalloc(&s->ritem0, nch));
    SC(dalloc(&s->rnseg, nch));
    SC(dalloc(&s->xpart, (size_t)std::max(1, s->n_ritems) * HK_WAVE));
    if (!ritems.empty())
        SC(hipMemcpy(s->ritems, ritems.data(), sizeof(hk_item) * ritems.size(), hipMemcpyHostToDevice));
    SC(hipMemcpy(s->ritem0, ritem0.data(), sizeof(int) * nch, hipMemcpyHostToDevice));
    SC(hipMemcpy(s->rnseg, rnseg.data(), sizeof(int) * nch, hipMemcpyHostToDevice));
    SC(dalloc(&s->items, items.size()));
    SC(dalloc(&s->item0, s->nq));
    SC(dalloc(&s->nseg, s->nq));
    SC(hipMemcpy(s->items, items.data(), sizeof(hk_item) * items.size(), hipMemcpyHostToDevice));
    SC(hipMemcpy(s->item0, item0.data(), sizeof(int) * s->nq, hipMemcpyHostToDevice));
    SC(hipMemcpy(s->nseg, nseg.data(), sizeof(int) * s->nq, hipMemcpyHostToDevice));
    SC(dalloc(&s->lam_static, p->npad));
    SC(dalloc(&s->Lam_static, 1));
    SC(dalloc(&s->a, s->mpad));
    SC(dalloc(&s->tv, s->mpad));
    SC(dalloc(&s->sxy, s->mpad));
    SC(dalloc(&s->sts, s->mpad));
    SC(dalloc(&s->qwide, s->nq));
    SC(dalloc(&s->qstep, s->nq));
    SC(dalloc(&s->lw, p->npad));
    SC(dalloc(&s->colG, (size_t)s->n_items * 2 * HK_WAVE));
    SC(dalloc(&s->gsub, s->mpad));
    SC(dalloc(&s->hsub, s->mpad));
    SC(dalloc(&s->sums, 8));
    SC(dalloc(&s->z0, m));
    SC(dalloc(&s->p, m));
    SC(dalloc(&s->off, m));
    SC(dalloc(&s->vz, m));
    SC(dalloc(&s->scal, 16));
#undef SC
    s->static_valid = false;
    return HAWKES_OK;
}

namespace {

bool same_hyper(const hawkes_hyper &a, const hawkes_hyper &b) {
    return a.mu0 == b.mu0 && a.tau_x == b.tau_x && a.tau_t == b.tau_t && a.theta0 == b.theta0 &&
           a.omega == b.omega && a.h == b.h;
}

// Static part for (hyper, fixed rates) -- recomputed when the hyperparameters
// change or the caller asks.
hawkes_status ensure_static(hawkes_plan p, const hawkes_hyper *hy, const double *d_theta, bool force,
                            const PairConst &kc, const FinConst &fc, hipStream_t stream) {
    hk_subset *s = p->sub;
    if (s->static_valid && !force && same_hyper(s->static_hyper, *hy)) return HAWKES_OK;
    hipLaunchKernelGGL(k_sub_static_theta, dim3(nblk(p->npad, 256)), dim3(256), 0, stream, d_theta, p->perm, s->pos,
                       s->m, p->n, p->npad, p->theta_s, p->status);
    hipLaunchKernelGGL(k_sub_zero_subset, dim3(nblk(s->m, 256)), dim3(256), 0, stream, s->pos, s->m, p->theta_s);
    hk_launch_row_loglik(p, kc, stream);
    hipLaunchKernelGGL(k_sub_static, dim3(p->nfin_blocks), dim3(256), 0, stream, p->ts, p->xs, p->ys, p->g, d_theta,
                       p->perm, p->theta_s,
                       p->n, p->ntiles, p->row_item0, p->row_nseg, p->rowpart, p->colpart,
                       p->colpart_off, fc,
                       s->lam_static, p->blockpart);
    hipLaunchKernelGGL(k_sum_blocks, dim3(1), dim3(64), 0, stream, p->blockpart, p->nfin_blocks, s->Lam_static);
    hipLaunchKernelGGL(k_sub_a, dim3(nblk(s->mpad, 256)), dim3(256), 0, stream, p->ts, s->pos, s->m, s->mpad, fc,
                       s->a);
    HK_CHECK(hipGetLastError());
    s->static_hyper = *hy;
    s->static_valid = true;
    return HAWKES_OK;
}

// The row half of a subset evaluation at z (slot order): (theta,) lambda, w and
// the block partial sums of log lambda in p->blockpart.
static void sub_rows(hawkes_plan p, const double *z, const double *off, double *theta_full, bool with_theta,
                     const PairConst &kc, const FinConst &fc, hipStream_t stream) {
    hk_subset *s = p->sub;
    p->epoch += 1;  // p->lam is overwritten below
    if (with_theta)
        hipLaunchKernelGGL(k_sub_theta, dim3((unsigned)(s->mpad / 256)), dim3(256), 0, stream, z, off, s->slot,
                           s->cidx, s->m, s->pos, p->ts, p->xs, p->ys, kc, s->tv, s->sxy, s->sts, s->qwide, s->qstep,
                           theta_full);
    hipLaunchKernelGGL(k_sub_row, dim3(s->n_ritems), dim3(HK_WAVE), 0, stream, p->ts, p->xs, p->ys, p->g, s->pos,
                       s->tv, s->sxy, s->sts, s->qwide, s->qstep, s->ritems, kc, s->xpart);
    hipLaunchKernelGGL(k_sub_fin, dim3(p->nchunks), dim3(SUB_ROWFIN_WAVES * HK_WAVE), 0, stream, s->lam_static,
                       s->ritem0, s->rnseg, s->xpart, p->ts, p->xs, p->ys, p->g, s->pos, s->tv, s->sts, s->qwide,
                       s->m, p->n, p->npad, fc, p->lam, s->lw, p->blockpart, p->status);
}

// The column half: Eq. 4 (and Eq. 5) on the subset, optionally with the fused
// leapfrog update.
static void sub_cols(hawkes_plan p, bool with_h, const PairConst &kc, const FinConst &fc, const SubUpd *upd,
                     hipStream_t stream) {
    hk_subset *s = p->sub;
#define HK_SUBCOL(H, D)                                                                                        \
    hipLaunchKernelGGL((k_sub_col<H, D>), dim3(s->n_items), dim3(HK_WAVE), 0, stream, p->ts, p->xs, p->ys, s->lw, \
                       p->g, s->pos, s->sxy, s->sts, s->m, s->items, kc, s->colG)
    if (with_h) {
        if (kc.dot) HK_SUBCOL(true, true);
        else HK_SUBCOL(true, false);
    } else {
        if (kc.dot) HK_SUBCOL(false, true);
        else HK_SUBCOL(false, false);
    }
#undef HK_SUBCOL
    if (upd)
        hipLaunchKernelGGL(k_sub_colfin<true>, dim3(s->nq), dim3(SUB_FIN_WAVES * HK_WAVE), 0, stream, s->item0,
                           s->nseg, s->colG, s->a, s->m, fc, with_h, s->gsub, s->hsub, *upd);
    else
        hipLaunchKernelGGL(k_sub_colfin<false>, dim3(s->nq), dim3(SUB_FIN_WAVES * HK_WAVE), 0, stream, s->item0,
                           s->nseg, s->colG, s->a, s->m, fc, with_h, s->gsub, s->hsub, SubUpd{});
}

// One subset evaluation at z (slot order): theta, lambda, w, Eq. 4 (and Eq. 5)
// on the subset, block partial sums of log lambda in p->blockpart.
void sub_eval(hawkes_plan p, const double *z, const double *off, double *theta_full, bool with_h,
              const PairConst &kc, const FinConst &fc, hipStream_t stream) {
    sub_rows(p, z, off, theta_full, true, kc, fc, stream);
    sub_cols(p, with_h, kc, fc, nullptr, stream);
}

__global__ void k_z_from_theta(const double *__restrict__ theta, const int64_t *__restrict__ cidx, int64_t m,
                               double *__restrict__ z) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < m) z[k] = log(theta[cidx[k]]);
}

// z_k = log theta_{idx_k} - beta t_{idx_k} (slot order)
__global__ void k_z_of_rates(const double *__restrict__ theta, const int *__restrict__ pos,
                             const int *__restrict__ slot, const int64_t *__restrict__ cidx,
                             const double *__restrict__ ts, int64_t m, double beta, double *__restrict__ z) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= m) return;
    const int k = slot[r];
    z[k] = log(theta[cidx[k]]) - beta * ts[pos[r]];
}

// d loglik / d z_k = theta_k g_k and d loglik / d beta = sum_k t_k theta_k g_k
// for log theta_k = z_k + beta t_k; one block, fixed-order tree reduction.
__global__ __launch_bounds__(256) void k_sub_trend_out(const int *__restrict__ slot, const int *__restrict__ pos,
                                                       const double *__restrict__ ts, int64_t m,
                                                       const double *__restrict__ gsub, const double *__restrict__ z,
                                                       const double *__restrict__ off, double *__restrict__ grad_z,
                                                       double *__restrict__ grad_beta) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < m; r += 256) {
        const int k = slot[r];
        const double gz = exp(zeff(z, off, k)) * gsub[r];
        if (grad_z) grad_z[k] = gz;
        acc += ts[pos[r]] * gz;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && grad_beta) grad_beta[0] = sh[0];
}

__global__ void k_sub_loglik_out(const double *__restrict__ e, const double *__restrict__ Lam_static,
                                 double *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = e[0] - Lam_static[0] - e[1];
}

}  // namespace

extern "C" hawkes_status hawkes_subset_grad(hawkes_plan p, const hawkes_hyper *hyper, const double *d_theta,
                                            int refresh_static, double *d_loglik, double *d_grad_sub,
                                            double *d_negH_sub, hipStream_t stream) {
    if (!p || !hk_hyper_ok(hyper) || !d_theta) return HAWKES_E_INVALID;
    if (!p->sub) return HAWKES_E_UNSUPPORTED;
    hk_subset *s = p->sub;
    p->last_stream = stream;
    PairConst kc;
    FinConst fc;
    hk_make_consts(p, hyper, &kc, &fc);
    hawkes_status st = ensure_static(p, hyper, d_theta, refresh_static != 0, kc, fc, stream);
    if (st != HAWKES_OK) return st;
    // z = log theta on the subset (the rates are taken from d_theta as given)
    hipLaunchKernelGGL(k_z_from_theta, dim3(nblk(s->m, 256)), dim3(256), 0, stream, d_theta, s->cidx, s->m, s->z0);
    sub_eval(p, s->z0, nullptr, nullptr, d_negH_sub != nullptr, kc, fc, stream);
    hipLaunchKernelGGL(k_sub_scatter, dim3(nblk(s->m, 256)), dim3(256), 0, stream, s->slot, s->m, s->gsub, s->hsub,
                       d_grad_sub, d_negH_sub);
    if (d_loglik) {
        hipLaunchKernelGGL(k_sub_energy, dim3(1), dim3(ENERGY_THREADS), 0, stream, p->blockpart, p->nchunks, s->z0,
                           (const double *)nullptr, (const double *)nullptr, (const double *)nullptr, s->slot, s->a,
                           s->m, s->scal);
        hipLaunchKernelGGL(k_sub_loglik_out, dim3(1), dim3(64), 0, stream, s->scal, s->Lam_static, d_loglik);
    }
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}

extern "C" hawkes_status hmc_step(hawkes_plan p, const hawkes_hyper *hyper, hawkes_hmc_args *a,
                                  hipStream_t stream) {
    if (!p || !a || !hk_hyper_ok(hyper) || !a->d_z || !a->d_theta || !a->d_mass || !a->d_out || a->L < 1 ||
        !(a->eps > 0.0) || !(a->sigma_z > 0.0))
        return HAWKES_E_INVALID;
    if (!p->sub) return HAWKES_E_UNSUPPORTED;
    if (a->prior != 0 && a->prior != 1) return HAWKES_E_INVALID;
    if (a->prior == 1 && hk_tree_tips(p) != p->sub->m) return HAWKES_E_UNSUPPORTED;
    hk_subset *s = p->sub;
    p->last_stream = stream;
    PairConst kc;
    FinConst fc;
    hk_make_consts(p, hyper, &kc, &fc);
    hawkes_status st = ensure_static(p, hyper, a->d_theta, a->refresh_static != 0, kc, fc, stream);
    if (st != HAWKES_OK) return st;
    const int64_t m = s->m;
    const bool tree = a->prior == 1;
    const double *pv = tree ? s->vz : a->d_z;  // prior gradient direction (times 1/sigma^2)
    const double inv_s2 = 1.0 / (a->sigma_z * a->sigma_z);
    const unsigned gb = nblk(m, 256);
    // temporal trend: log theta_k = z_k + beta t_k
    const double *off = nullptr;
    if (a->beta != 0.0) {
        hipLaunchKernelGGL(k_sub_offset, dim3(gb), dim3(256), 0, stream, p->ts, s->pos, s->slot, m, a->beta, s->off);
        off = s->off;
    }
    hipLaunchKernelGGL(k_hmc_init, dim3(gb), dim3(256), 0, stream, m, a->seed, a->counter, a->d_mass, a->d_z, s->p,
                       s->z0);
    // start of the trajectory: the energy at z0, then the gradient there and the
    // first half kick and drift (fused into the column finalisation)
    sub_rows(p, a->d_z, off, a->d_theta, true, kc, fc, stream);
    hipLaunchKernelGGL(k_sub_energy, dim3(1), dim3(ENERGY_THREADS), 0, stream, p->blockpart, p->nchunks, a->d_z, off, s->p,
                       a->d_mass, s->slot, s->a, m, s->scal);
    // phylogenetic prior: the quadratic form z^T V^{-1} z replaces sum z^2
    if (tree && (st = hk_tree_launch(p, a->d_z, s->vz, s->scal + 2, stream)) != HAWKES_OK) return st;
    SubUpd upd{s->slot, a->d_z, off, pv, inv_s2, s->p, a->d_mass, 0.5 * a->eps, a->eps, s->tv, s->sts, s->qwide,
               kc.omega};
    sub_cols(p, false, kc, fc, &upd, stream);
    for (int l = 0; l < a->L; ++l) {
        // evaluation at the drifted position, then a full kick and drift, or the
        // closing half kick after the last one
        sub_rows(p, a->d_z, off, a->d_theta, false, kc, fc, stream);
        if (tree && (st = hk_tree_launch(p, a->d_z, s->vz, nullptr, stream)) != HAWKES_OK) return st;
        const bool last = l == a->L - 1;
        upd.a_p = last ? 0.5 * a->eps : a->eps;
        upd.a_z = last ? 0.0 : a->eps;
        sub_cols(p, false, kc, fc, &upd, stream);
    }
    hipLaunchKernelGGL(k_sub_energy, dim3(1), dim3(ENERGY_THREADS), 0, stream, p->blockpart, p->nchunks, a->d_z, off, s->p,
                       a->d_mass, s->slot, s->a, m, s->scal + 4);
    if (tree && (st = hk_tree_launch(p, a->d_z, nullptr, s->scal + 6, stream)) != HAWKES_OK) return st;
    hipLaunchKernelGGL(k_hmc_accept, dim3(1), dim3(256), 0, stream, s->scal, s->Lam_static, inv_s2, a->seed,
                       a->counter, m, s->z0, a->d_z, a->d_z_proposal, a->d_out, (int *)(s->scal + 8));
    hipLaunchKernelGGL(k_sub_theta_full, dim3(gb), dim3(256), 0, stream, a->d_z, off, s->cidx, m, a->d_theta);
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}

extern "C" hawkes_status hawkes_subset_trend_grad(hawkes_plan p, const hawkes_hyper *hyper, const double *d_z,
                                                  double beta, double *d_theta, double *d_loglik, double *d_grad_z,
                                                  double *d_grad_beta, hipStream_t stream) {
    if (!p || !hk_hyper_ok(hyper) || !d_z || !d_theta || !isfinite(beta)) return HAWKES_E_INVALID;
    if (!p->sub) return HAWKES_E_UNSUPPORTED;
    hk_subset *s = p->sub;
    p->last_stream = stream;
    PairConst kc;
    FinConst fc;
    hk_make_consts(p, hyper, &kc, &fc);
    hawkes_status st = ensure_static(p, hyper, d_theta, false, kc, fc, stream);
    if (st != HAWKES_OK) return st;
    const unsigned gb = nblk(s->m, 256);
    const double *off = nullptr;
    if (beta != 0.0) {
        hipLaunchKernelGGL(k_sub_offset, dim3(gb), dim3(256), 0, stream, p->ts, s->pos, s->slot, s->m, beta, s->off);
        off = s->off;
    }
    sub_eval(p, d_z, off, d_theta, false, kc, fc, stream);
    if (d_grad_z || d_grad_beta)
        hipLaunchKernelGGL(k_sub_trend_out, dim3(1), dim3(256), 0, stream, s->slot, s->pos, p->ts, s->m, s->gsub, d_z,
                           off, d_grad_z, d_grad_beta);
    if (d_loglik) {
        hipLaunchKernelGGL(k_sub_energy, dim3(1), dim3(ENERGY_THREADS), 0, stream, p->blockpart, p->nchunks, d_z, off,
                           (const double *)nullptr, (const double *)nullptr, s->slot, s->a, s->m, s->scal);
        hipLaunchKernelGGL(k_sub_loglik_out, dim3(1), dim3(64), 0, stream, s->scal, s->Lam_static, d_loglik);
    }
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}

void hk_subset_view(hawkes_plan p, int64_t *m, const int64_t **cidx, const int **pos, const int **slot) {
    *m = p->sub->m;
    *cidx = p->sub->cidx;
    *pos = p->sub->pos;
    *slot = p->sub->slot;
}

hawkes_status hk_subset_grid(hawkes_plan p, int64_t cells, hipStream_t stream) {
    hk_subset *s = p->sub;
    if (s->grid_cap >= cells) return HAWKES_OK;
    if (s->grid) {
        HK_CHECK(hipStreamSynchronize(stream));
        (void)hipFree(s->grid);
        s->grid = nullptr;
        s->grid_cap = 0;
    }
    if (hipMalloc((void **)&s->grid, sizeof(int) * cells + 16) != hipSuccess) return HAWKES_E_NOMEM;
    s->grid_cap = cells;
    return HAWKES_OK;
}

int *hk_subset_grid_ptr(hawkes_plan p) { return p->sub->grid; }

hawkes_status hk_subset_exact(hawkes_plan p, const hawkes_hyper *hy, const double *d_theta, hipStream_t stream,
                              const double **gsub, const double **hsub) {
    hk_subset *s = p->sub;
    p->last_stream = stream;
    PairConst kc;
    FinConst fc;
    hk_make_consts(p, hy, &kc, &fc);
    hawkes_status st = ensure_static(p, hy, d_theta, false, kc, fc, stream);
    if (st != HAWKES_OK) return st;
    hipLaunchKernelGGL(k_z_from_theta, dim3(nblk(s->m, 256)), dim3(256), 0, stream, d_theta, s->cidx, s->m, s->z0);
    sub_eval(p, s->z0, nullptr, nullptr, true, kc, fc, stream);
    HK_CHECK(hipGetLastError());
    *gsub = s->gsub;
    *hsub = s->hsub;
    return HAWKES_OK;
}

extern "C" hawkes_status hawkes_subset_z(hawkes_plan p, const double *d_theta, double beta, double *d_z,
                                         hipStream_t stream) {
    if (!p || !d_theta || !d_z || !isfinite(beta)) return HAWKES_E_INVALID;
    if (!p->sub) return HAWKES_E_UNSUPPORTED;
    hk_subset *s = p->sub;
    p->last_stream = stream;
    hipLaunchKernelGGL(k_z_of_rates, dim3(nblk(s->m, 256)), dim3(256), 0, stream, d_theta, s->pos, s->slot, s->cidx,
                       p->ts, s->m, beta, d_z);
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}
