// Evaluation of Eq. 1 (log-likelihood), Eq. 4 (rate gradient), Eq. 5 (rate
// Hessian diagonal) and the hyperparameter derivatives on gfx950.
//
// Kernels, in launch order:
//   k_tfac     theta to sorted order (FP32), validity check, staged rates of
//              the split excitation time factor, the per-chunk split flags and
//              step factors
//   k_row      row pass over causal tile pairs: for each row i the background
//              moments over j < i and the excitation moments over t_j < t_i;
//              the background is symmetric, so each pair also adds its
//              background terms to column j: the FP32 moments through
//              accumulators that rotate one lane per step around the wavefront
//              (DPP wave_rol), the FP64 sum through an LDS add per pair
//   k_fin      per event: partial sums -> lambda_i (FP64), log lambda_i,
//              w_i = c_e / lambda_i staged for the column pass, integral term
//              (App. A), hyperparameter terms; fixed-order block reduction
//   k_fin2     one block: block partials -> loglik, grad/negH of hyperparameters
//   k_col      column pass: G_j = sum_{t_i > t_j} E_ij w_i, H_j = sum (E_ij w_i)^2
//   k_colfin   G_j, H_j -> Eq. 4 / Eq. 5 in the caller's order
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <vector>

#include "hawkes_internal.h"

struct hk_profile {
    std::vector<hipEvent_t> ev[HK_PROF_KINDS];  // start/stop pairs, in order
    int every = 1;                              // record around every `every`-th evaluation
    int64_t count = 0;                          // evaluations seen since enabled
    bool active = false;                        // the current evaluation is recorded
};

// An event recorded between two dependent kernels keeps the command processor
// from starting the second as the first drains (about 6 us per event on this
// part, against no gap without them), so the timing records only a sample of
// the evaluations when asked to.
void hk_prof_mark(hawkes_plan p, int kind, bool start, hipStream_t stream) {
    if (!p->prof) return;
    if (kind == HK_PROF_EVAL && start) p->prof->active = (p->prof->count++ % p->prof->every) == 0;
    if (!p->prof->active) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)start;
    (void)hipEventRecord(e, stream);
    p->prof->ev[kind].push_back(e);
}

void hk_prof_free(hawkes_plan p) {
    if (!p->prof) return;
    for (auto &v : p->prof->ev)
        for (hipEvent_t e : v) (void)hipEventDestroy(e);
    delete p->prof;
    p->prof = nullptr;
}

extern "C" hawkes_status hawkes_profile_enable(hawkes_plan p, int on) {
    if (!p || on < 0) return HAWKES_E_INVALID;
    if (on && !p->prof) p->prof = new hk_profile();
    if (!on) hk_prof_free(p);
    if (on) {
        p->prof->every = on;
        p->prof->count = 0;
    }
    return HAWKES_OK;
}

extern "C" hawkes_status hawkes_profile_read(hawkes_plan p, double *out) {
    if (!p || !out) return HAWKES_E_INVALID;
    for (int k = 0; k < 2 * HK_PROF_KINDS; ++k) out[k] = 0.0;
    if (!p->prof) return HAWKES_OK;
    for (int k = 0; k < HK_PROF_KINDS; ++k) {
        auto &v = p->prof->ev[k];
        for (size_t q = 0; q + 1 < v.size(); q += 2) {
            HK_CHECK(hipEventSynchronize(v[q + 1]));
            float ms = 0.0f;
            HK_CHECK(hipEventElapsedTime(&ms, v[q], v[q + 1]));
            out[2 * k] += ms;
            out[2 * k + 1] += 1.0;
        }
        for (hipEvent_t e : v) (void)hipEventDestroy(e);
        v.clear();
    }
    return HAWKES_OK;
}

namespace {

__device__ __forceinline__ float rot_next(float v) {
    // lane l receives lane l+1 (wave_rol:1); the rotation closes over 64 lanes
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x134, 0xf, 0xf, true));
}

__device__ __forceinline__ double rot_next_d(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x134, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x134, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Knuth's TwoSum: (hi, lo) += v with the rounding error of the high add kept.
__device__ __forceinline__ void two_sum_acc(float &hi, float &lo, float v) {
    float s = hi + v;
    float bp = s - hi;
    float err = (hi - (s - bp)) + (v - bp);
    hi = s;
    lo += err;
}

// ------------------------------------------------------------------------------------
// Per evaluation, before the row pass: the sorted FP32 rates (gathered from the
// caller's order when FROM_CALLER, else already in theta_s), and for the split
// excitation time factor the staged rate of each event,
// theta_v_j = theta_j exp(omega (t_j - T_c)) with T_c its chunk's first time,
// plus a flag per chunk that spans more than `span_max` in time (those chunks
// take the row pass's precise form and stage theta_j itself), and the chunk's step factor
// tstep_c = exp(-omega (T_{c+1} - T_c)) (0 for the last chunk), with which the
// pair passes carry a row's or column's own split factor from one chunk to the
// next instead of evaluating it anew.  One wavefront per chunk.
template <bool FROM_CALLER>
__global__ __launch_bounds__(256) void k_tfac(const double *__restrict__ theta, const int *__restrict__ perm,
                                              const double *__restrict__ ts, int64_t n, double omega,
                                              double span_max, float *__restrict__ theta_s,
                                              float *__restrict__ theta_v, int *__restrict__ chunk_precise,
                                              double *__restrict__ tstep, int *__restrict__ status) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;  // grid covers npad exactly
    const int lane = threadIdx.x & (HK_WAVE - 1);
    double th = 0.0;
    if (FROM_CALLER) {
        if (i < n) {
            th = theta[perm[i]];
            if (!(th >= 0.0) || !isfinite(th)) atomicOr(status, HK_ST_BADTHETA);
        }
        theta_s[i] = (float)th;
    } else {
        th = (double)theta_s[i];
    }
    const double dti = ts[i] - ts[i - lane];
    const bool precise = __any(i < n && dti > span_max);
    theta_v[i] = (!precise && th > 0.0) ? (float)(th * exp(omega * dti)) : (float)th;
    if (lane == 0) {
        chunk_precise[i / HK_WAVE] = precise;
        const int64_t nxt = i + HK_WAVE;
        tstep[i / HK_WAVE] = nxt < (int64_t)gridDim.x * blockDim.x ? exp(-omega * (ts[nxt] - ts[i])) : 0.0;
    }
}

// ------------------------------------------------------------------------------------
// 2^e for an FP64 exponent: exact integer part, FP32 fraction.  The term's
// relative error is then a few FP32 roundings whatever |e| (rounding the whole
// exponent to FP32 would give an error that grows with |e|).  e must be at
// least HK_EXP_FLOOR (the integer part stays inside int32).
__device__ __forceinline__ float exp2_split(double e) {
    const double n = rint(e);
    return __builtin_amdgcn_ldexpf(fexp2((float)(e - n)), (int)n);
}

// ------------------------------------------------------------------------------------
// The row pass sweeps a 64-column chunk in one of two forms, chosen per chunk.
//
// Fast form (a chunk whose events span at most min(HK_FACT_SPAN / omega,
// HK_COMPACT_TAU tau_t) in time; every chunk of the dense workloads).  The
// excitation's time factor is split at the chunk's first time T_c:
// exp(-omega (t_i - t_j)) = exp(-omega (t_i - T_c)) exp(omega (t_j - T_c)),
// both factors formed in FP64 once per event and chunk, so only the spatial
// part exp(-r^2 / 2h^2) goes through the FP32 exp2 of the pair loop.  Times
// enter relative to T_c, rounded to FP32: the rounding of the column's offset
// is at most 2^-25 of the chunk's span, and the row's relative to dt plus that
// span, so on a compact chunk dt is nearly as accurate as the FP64 difference.
//
// Precise form (every other chunk: sparse data).  dt is the FP64 difference of
// the times, both exponents are formed whole in FP64 and exponentiated by
// exp2_split, so a term's error does not grow with the size of its exponent or
// with the time span of the chunk.  It costs about a third more per pair and is
// taken only where the data is too sparse in time for the fast form.
//
// In both forms one sweep is 64 steps, each lane pairing its row with column
// (lane + s) mod 64 of the chunk.  The three sums lambda_i is built from
// (background row sum B0, background column sum, excitation X0) accumulate
// every term in FP64: a plain FP32 sum of positive terms rounds away every term
// below half an ulp of the running sum, which biases lambda low (by ~2e-8
// relative on clustered data).  The column sum goes through LDS: at step s lane
// l adds its term to its wavefront's slot l + s (column (l + s) mod 64 owns
// slots k and k + 64), one slot per lane and instruction and the wavefront's
// instructions in order, so the order of every sum is fixed.  The moments used
// only by derivatives stay in FP32 blocks.
//
// The spatial exponent of the background is formed in FP64 from coordinates
// pre-scaled by sqrt(-kbx) (two subtractions, a product and an FMA) and the
// fast form rounds it once to FP32, so it carries no rounded FP32 scale.
// The excitation's spatial exponent is that value times the ratio kex / kbx.
//
// Constants: times enter scaled by st = 1 / (tau_t sqrt(2 ln 2)) (in FP64,
// before any rounding), so the background's time exponent is exactly -dt'^2 and
// carries no rounded constant; the time moments are rescaled in FP64 by the
// finalisation.  The excitation's spatial exponent is the background's times
// the ratio rex = kex / kbx: in the log-likelihood-only mode the FP32 ratio is
// completed by its low part inside the loop (the fast form) or taken exact in
// FP64 (the precise form); the other modes use the FP32-rounded ratio in both
// forms and correct its rounding to first order through the moment X2.  (A low
// part added to an exactly representable FP32 value in a separate rounding
// would mostly be rounded away, one way: the earlier form of the background's
// time constant biased the log-likelihood-only pass's lambda by about 1e-9.)

// One pair's terms into the accumulators (b: background term, te: theta_j E_ij,
// ar, ae: spatial exponents of the two kernels in log2 units, dt = t_i - t_j).
template <int MODE>
__device__ __forceinline__ void row_accumulate(float b, float te, float ar, float ae, float dt, float dt2,
                                               float (&blk)[HK_NROW], float (&C)[HK_NCOL], double &B0d,
                                               double &X0c, double *__restrict__ acc0) {
#pragma clang fp contract(off)
    const double bd = (double)b;
    B0d += bd;
    // the column's FP64 sum: an LDS add into this step's slot (no return value)
    __hip_atomic_fetch_add(acc0, bd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    if (MODE >= HK_MODE_GRAD) {
        const float p1 = b * ar, p2 = b * dt2;
        blk[1] += p1;
        blk[2] += p2;
        C[1] = rot_next(C[1]) + p1;
        C[2] = rot_next(C[2]) + p2;
        if (MODE >= HK_MODE_HESS) {
            const float p11 = p1 * ar, p22 = p2 * dt2;
            blk[3] += p11;
            blk[4] += p22;
            C[3] = rot_next(C[3]) + p11;
            C[4] = rot_next(C[4]) + p22;
        }
    }
    X0c += (double)te;
    if (MODE >= HK_MODE_GRAD) {
        blk[6] = fmaf(te, dt, blk[6]);
        const float q = te * ae;
        blk[7] += q;
        if (MODE >= HK_MODE_HESS) {
            blk[8] = fmaf(te, dt2, blk[8]);
            blk[9] = fmaf(q, ae, blk[9]);
        }
    }
}

template <int MODE, bool MASK_BG, bool MASK_EX, bool FAST>
__device__ __forceinline__ void row_sweep(const float2 *__restrict__ rec, const double2 *__restrict__ rxy,
                                          const double *__restrict__ rtd,
                                          double tsi, int lane, float ti, double xr, double yr,
                                          int irow, int gr, int cbase, const PairConst kc,
                                          float (&blk)[HK_NROW], float (&C)[HK_NCOL], double &B0d, double &X0c,
                                          double *__restrict__ acc0) {
    // explicit FMAs only: a contracted (rotated + product) cannot take the DPP
    // operand, while a plain add of the shared product can
#pragma clang fp contract(off)
    const double rex_d = MODE == HK_MODE_LOGLIK ? kc.rex_x : (double)kc.rex;
#pragma unroll 16
    for (int s = 0; s < HK_WAVE; ++s) {
        const float2 r = rec[lane + s];
        const double2 pj = rxy[lane + s];
        const double dx = xr - pj.x, dy = yr - pj.y;
        float b, E, ar, ae, dt, dt2;
        if (FAST) {
            dt = ti - r.x;
            ar = (float)(-fma(dx, dx, dy * dy));
            dt2 = dt * dt;
            b = fexp2(ar - dt2);
            ae = MODE == HK_MODE_LOGLIK ? fmaf(ar, kc.rex, ar * kc.rex_lo) : ar * kc.rex;
            E = fexp2(ae);
        } else {
            const double dtd = tsi - rtd[lane + s];
            const double ard = -fma(dx, dx, dy * dy);
            const double aed = ard * rex_d;
            b = exp2_split(fmax(fma(-dtd, dtd, ard), HK_EXP_FLOOR));
            // a masked sweep also meets later columns (dt < 0, masked below): their
            // exponent is held at 2^128 so that its integer part stays in range
            double ee = fmax(fma(dtd, kc.kw_s, aed), HK_EXP_FLOOR);
            if (MASK_BG || MASK_EX) ee = fmin(ee, 128.0);
            E = exp2_split(ee);
            ar = (float)ard;
            ae = (float)aed;
            dt = (float)dtd;
            dt2 = dt * dt;
        }
        if (MASK_BG || MASK_EX) {
            const int j = cbase + ((lane + s) & (HK_WAVE - 1));
            if (MASK_BG && !(j < irow)) b = 0.0f;
            if (!(j < gr)) E = 0.0f;
        }
        row_accumulate<MODE>(b, E * r.y, ar, ae, dt, dt2, blk, C, B0d, X0c, acc0 + lane + s);
    }
}

template <int MODE, bool FAST>
__device__ __forceinline__ void row_sweep_masked(const float2 *__restrict__ rec, const double2 *__restrict__ rxy,
                                                 const double *__restrict__ rtd,
                                                 double tsi, int lane, float ti, double xr, double yr,
                                                 int irow, int gr, int c, int wave_chunk, int wave_gmin,
                                                 const PairConst kc, float (&blk)[HK_NROW],
                                                 float (&C)[HK_NCOL], double &B0d, double &X0c, double *__restrict__ acc0) {
    const int cbase = c * HK_WAVE;
    if (c == wave_chunk)
        row_sweep<MODE, true, true, FAST>(rec, rxy, rtd, tsi, lane, ti, xr, yr, irow, gr, cbase, kc, blk, C, B0d, X0c, acc0);
    else if (cbase + HK_WAVE - 1 >= wave_gmin)
        row_sweep<MODE, false, true, FAST>(rec, rxy, rtd, tsi, lane, ti, xr, yr, irow, gr, cbase, kc, blk, C, B0d, X0c, acc0);
    else
        row_sweep<MODE, false, false, FAST>(rec, rxy, rtd, tsi, lane, ti, xr, yr, irow, gr, cbase, kc, blk, C, B0d, X0c, acc0);
}

template <int MODE>
__global__ __launch_bounds__(HK_TILE, 4) void k_row(const double *__restrict__ ts, const double *__restrict__ xs,
                                                  const double *__restrict__ ys, const float *__restrict__ theta_v,
                                                  const int *__restrict__ chunk_precise, const double *__restrict__ tstep,
                                                  const int *__restrict__ g, const hk_item *__restrict__ items,
                                                  const int *__restrict__ block0,
                                                  const int64_t *__restrict__ colpart_off,
                                                  float *__restrict__ rowpart, float *__restrict__ colpart,
                                                  const PairConst kc) {
    // one LDS block with the staged chunk first: the sweep's loads then reach
    // every step's entry with an immediate offset from one address register
    struct Stage {
        float2 rec[2 * HK_WAVE];
        double rtd[2 * HK_WAVE];
        double2 rxy[2 * HK_WAVE];
        double colacc0[HK_WAVES][2 * HK_WAVE];  // column sums of the background, per wave
        float colbuf[HK_WAVES][HK_NCOL][HK_WAVE];
    };
    __shared__ Stage L;
    auto &rec = L.rec;
    auto &rxy = L.rxy;
    auto &rtd = L.rtd;
    auto &colacc0 = L.colacc0;
    auto &colbuf = L.colbuf;
    constexpr int NC = MODE == HK_MODE_LOGLIK ? 1 : (MODE == HK_MODE_GRAD ? 3 : 5);
    // the wavefront index is made visibly uniform, so that the per-wave chunk
    // bounds below live in scalar registers and select the sweep variant with
    // scalar branches
    const int tid = threadIdx.x, lane = tid & (HK_WAVE - 1), wv = __builtin_amdgcn_readfirstlane(tid / HK_WAVE);
    const int q_end = block0[blockIdx.x + 1];

    for (int q = block0[blockIdx.x]; q < q_end; ++q) {
        const hk_item it = items[q];
        const int I = it.tile;
        const int64_t row0 = (int64_t)I * HK_TILE;
        const int irow = (int)(row0 + tid);
        const double tsi = ts[irow];
        const double tsi_s = tsi * kc.st;  // scaled time (the precise form's FP64 differences)
        const double xr = xs[irow] * kc.sbx, yr = ys[irow] * kc.sbx;
        const int gr = g[irow];
        const int wave_chunk = I * HK_CHUNKS_PER_TILE + wv;
        const int wave_gmin = g[(int64_t)wave_chunk * HK_WAVE];  // g is non-decreasing
        const double wave_tmin = ts[(int64_t)wave_chunk * HK_WAVE];  // the wave's earliest row
        const int64_t stride = (int64_t)(I + 1) * HK_TILE;
        float *__restrict__ cp = colpart + colpart_off[I];

        double mom[HK_NROW];  // derivative moments, FP64 across chunks (slots 0 and 5 unused)
#pragma unroll
        for (int a = 0; a < HK_NROW; ++a) mom[a] = 0.0;
        double B0d = 0.0, X0d = 0.0;

        const double tile_tmin = ts[row0];
        // the row's split factor exp(-omega (t_i - T_c)) is evaluated at the first
        // split chunk that pairs with the wave and carried down to earlier chunks
        // by their step factors (it only decreases, so it cannot overflow); a wide
        // chunk breaks the chain
        double ui = 0.0;
        bool have_ui = false;
        for (int c = it.c_end - 1; c >= it.c_begin; --c) {
            if (have_ui) ui *= tstep[c];
            // under the cutoff a chunk that ends more than dt_cut before the
            // tile's first row is skipped by the whole block (nothing is staged
            // and no wave sweeps it): its column partials come out zero.  It
            // takes the same path as a swept chunk otherwise, which keeps the
            // accumulators in place across chunks.
            const double Tlast = ts[(int64_t)c * HK_WAVE + HK_WAVE - 1];
            const bool block_live = !(tile_tmin - Tlast > kc.dt_cut);
            // fast form: times relative to the chunk's first event, rounded to FP32
            const double Tc = ts[(int64_t)c * HK_WAVE];
            const float ti = (float)((tsi - Tc) * kc.st);  // scaled time
            const bool fact = chunk_precise[c] == 0;
            if (block_live && tid < HK_WAVE) {
                const int64_t j = (int64_t)c * HK_WAVE + tid;
                const double tj = ts[j];
                float2 r;
                r.x = (float)((tj - Tc) * kc.st);
                r.y = theta_v[j];  // theta_j, times exp(omega (t_j - T_c)) on a fast chunk
                rec[tid] = r;
                rec[tid + HK_WAVE] = r;
                const double2 pj = make_double2(xs[j] * kc.sbx, ys[j] * kc.sbx);
                rxy[tid] = pj;
                rxy[tid + HK_WAVE] = pj;
                rtd[tid] = rtd[tid + HK_WAVE] = tj * kc.st;  // the precise form's FP64 scaled time
            }
            __syncthreads();
            // the wave's column slots start at zero (the previous chunk's reads of
            // them ended before the barrier above)
            colacc0[wv][lane] = 0.0;
            colacc0[wv][lane + HK_WAVE] = 0.0;
            float blk[HK_NROW], C[HK_NCOL];
            double X0c = 0.0;
#pragma unroll
            for (int a = 0; a < HK_NROW; ++a) blk[a] = 0.0f;
#pragma unroll
            for (int a = 0; a < HK_NCOL; ++a) C[a] = 0.0f;
            // optional underflow cutoff: a chunk that ends more than dt_cut before
            // the wave's earliest row contributes only terms below 2^-160
            const bool live = block_live && c <= wave_chunk && !(wave_tmin - Tlast > kc.dt_cut);
            if (live) {
                if (fact)
                    row_sweep_masked<MODE, true>(rec, rxy, rtd, tsi_s, lane, ti, xr, yr, irow, gr, c, wave_chunk, wave_gmin,
                                                 kc, blk, C, B0d, X0c, colacc0[wv]);
                else
                    row_sweep_masked<MODE, false>(rec, rxy, rtd, tsi_s, lane, ti, xr, yr, irow, gr, c, wave_chunk, wave_gmin,
                                                  kc, blk, C, B0d, X0c, colacc0[wv]);
                // the row's time factor (t_i >= T_c here, so it is at most 1)
                if (fact) {
                    if (!have_ui) {
                        ui = exp(-kc.omega * (tsi - Tc));
                        have_ui = true;
                    }
                    X0d += ui * X0c;
                    const float uf = (float)ui;
#pragma unroll
                    for (int a = 6; a < HK_NROW; ++a) blk[a] *= uf;
                } else {
                    X0d += X0c;
                    have_ui = false;
                }
            }
            // after 64 rotation steps lane l holds the accumulators of column (l - 1) mod 64
            const int col = (lane + HK_WAVE - 1) & (HK_WAVE - 1);
#pragma unroll
            for (int a = 1; a < NC; ++a) colbuf[wv][a][col] = C[a];
            __syncthreads();
            // partial sums are stored rounded to FP32 once (unbiased, relative
            // 2^-24 each) and summed in FP64 by the finalisation
            for (int e = tid; e < NC * HK_WAVE; e += HK_TILE) {
                const int a = e / HK_WAVE, cc = e % HK_WAVE;
                float v;
                if (a == 0) {
                    double c0 = 0.0;
#pragma unroll
                    for (int w = 0; w < HK_WAVES; ++w) c0 += colacc0[w][cc] + colacc0[w][cc + HK_WAVE];
                    v = (float)c0;
                }
                else
                    v = ((colbuf[0][a][cc] + colbuf[1][a][cc]) + colbuf[2][a][cc]) + colbuf[3][a][cc];
                cp[a * stride + (int64_t)c * HK_WAVE + cc] = v;
            }
#pragma unroll
            for (int a = 0; a < HK_NROW; ++a) {
                const bool used = (MODE >= HK_MODE_GRAD && (a == 1 || a == 2 || a == 6 || a == 7)) ||
                                  (MODE >= HK_MODE_HESS && a != 0 && a != 5);
                if (used) mom[a] += (double)blk[a];
            }
        }
        float *__restrict__ rp = rowpart + (int64_t)q * HK_NROW * HK_TILE;
        rp[tid] = (float)B0d;
        rp[5 * HK_TILE + tid] = (float)X0d;
#pragma unroll
        for (int a = 0; a < HK_NROW; ++a) {
            const bool used = (MODE >= HK_MODE_GRAD && (a == 1 || a == 2 || a == 6 || a == 7)) ||
                              (MODE >= HK_MODE_HESS && a != 0 && a != 5);
            if (used) rp[a * HK_TILE + tid] = (float)mom[a];
        }
    }
}

// ------------------------------------------------------------------------------------
// Deterministic sums across a wavefront: DPP within 16-lane rows, then two
// cross-row exchanges.  Every lane ends with the same value.
__device__ __forceinline__ double dpp_f64(double v, int ctrl_sel) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    switch (ctrl_sel) {
        case 0:
            lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xf, 0xf, false);  // quad_perm [1,0,3,2]
            hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xf, 0xf, false);
            break;
        case 1:
            lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xf, 0xf, false);  // quad_perm [2,3,0,1]
            hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xf, 0xf, false);
            break;
        case 2:
            lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xf, 0xf, false);  // row_half_mirror
            hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xf, 0xf, false);
            break;
        default:
            lo = __builtin_amdgcn_mov_dpp(lo, 0x140, 0xf, 0xf, false);  // row_mirror
            hi = __builtin_amdgcn_mov_dpp(hi, 0x140, 0xf, 0xf, false);
            break;
    }
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_f64(v, 0);
    v += dpp_f64(v, 1);
    v += dpp_f64(v, 2);
    v += dpp_f64(v, 3);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

__device__ __forceinline__ double std_pdf(double u) { return 0.3989422804014327 * exp(-0.5 * u * u); }
__device__ __forceinline__ double std_cdf(double u) { return 0.5 * erfc(-u * 0.7071067811865476); }

// Knuth's TwoSum in FP64: the exact rounding error of a + b (independent of
// the order of the operands).
__device__ __forceinline__ double two_sum_err(double a, double b, double s) {
    const double bp = s - a;
    return (a - (s - bp)) + (b - bp);
}

// The per-block partials ([HK_NSUM][nblocks]) -> loglik and the hyperparameter
// derivatives, by HK_NSUM * HK_TOT_LANES threads of one block: lane l of sum k
// keeps a Neumaier sum over blocks l, l + HK_TOT_LANES, ... (coalesced loads,
// all in flight together), then the lanes of the sum combine by a butterfly of
// exact TwoSum steps, so that the result is fixed whatever the timing.
constexpr int HK_TOT_LANES = 32;

__device__ void fin_totals(const double *__restrict__ blockpart, int nblocks, double *__restrict__ loglik,
                           double *__restrict__ grad_hyper, double *__restrict__ negH_hyper,
                           int *__restrict__ status, double *tot) {
    const int l = threadIdx.x % HK_TOT_LANES, groups = (int)blockDim.x / HK_TOT_LANES;
    for (int k = threadIdx.x / HK_TOT_LANES; k < HK_NSUM; k += groups) {
        const double *part = blockpart + (int64_t)k * nblocks;
        double sum = 0.0, c = 0.0, plain = 0.0;
#pragma unroll 4
        for (int b = l; b < nblocks; b += HK_TOT_LANES) {
            const double v = part[b];
            const double t = sum + v;
            c += two_sum_err(sum, v, t);
            sum = t;
            plain += v;
        }
#pragma unroll
        for (int off = 1; off < HK_TOT_LANES; off <<= 1) {
            const double s2 = __shfl_xor(sum, off), c2 = __shfl_xor(c, off), p2 = __shfl_xor(plain, off);
            const double t = sum + s2;
            c = (c + c2) + two_sum_err(sum, s2, t);
            sum = t;
            plain += p2;
        }
        if (l == 0) tot[k] = isfinite(plain) ? sum + c : plain;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double ll = tot[0] - tot[13];
        if (loglik) loglik[0] = ll;
        if (isnan(ll)) atomicOr(status, HK_ST_NONFINITE);
        if (grad_hyper) {
            const double dL[6] = {tot[14], 0.0, tot[15], tot[16], tot[17], 0.0};
            for (int p = 0; p < 6; ++p) grad_hyper[p] = tot[1 + p] - dL[p];
        }
        if (negH_hyper) {
            const double d2L[6] = {0.0, 0.0, tot[18], 0.0, tot[19], 0.0};
            for (int p = 0; p < 6; ++p) negH_hyper[p] = -tot[7 + p] + d2L[p];
        }
    }
}

constexpr int HK_FIN_WAVES = 8;

// The first wavefront of a k_fin block: lambda_i, w_i, the per-event terms of
// the hyperparameter derivatives and the integral, and their block sums.
template <int MODE>
__device__ __forceinline__ void fin_events(const double *__restrict__ ts, const double *__restrict__ theta,
                                           const int *__restrict__ perm, int64_t n, const FinConst &fc,
                                           const double (*part)[HK_NROW][HK_WAVE],
                                           const double (*exact)[HK_WAVE], bool is_exact, int lane, int64_t i,
                                           double *__restrict__ lam, double *__restrict__ lw,
                                           double *__restrict__ a_out, double *__restrict__ blockpart,
                                           int *__restrict__ status) {
    double s[HK_NSUM];
#pragma unroll
    for (int k = 0; k < HK_NSUM; ++k) s[k] = 0.0;
    if (i < n) {
        // the ten sums in natural units: B0, B1 (r^2), B2 (dt^2), B11, B22,
        // X0, X1 (dt), X2 (r^2), X11, X22, from the pair passes' partials or,
        // for a row recomputed in FP64, from k_fin's exact sums
        double B0, B1, B2, B11, B22, X0, X1, X2, X11, X22;
        if (is_exact) {
            B0 = exact[0][lane];
            B1 = exact[1][lane];
            B2 = exact[2][lane];
            B11 = exact[3][lane];
            B22 = exact[4][lane];
            X0 = exact[5][lane];
            X1 = exact[6][lane];
            X2 = exact[7][lane];
            X11 = exact[8][lane];
            X22 = exact[9][lane];
        } else {
            double acc[HK_NROW];
#pragma unroll
            for (int k = 0; k < HK_NROW; ++k) {
                double v = part[0][k][lane];
                for (int q = 1; q < HK_FIN_WAVES; ++q) v += part[q][k][lane];
                acc[k] = v;
            }
            // moments corrected for the mean exp2 bias and, when the first moments
            // are present, for the rounding of the FP32 ratio rex
            double b0 = acc[0], x0 = acc[5];
            if (MODE >= HK_MODE_GRAD) {
                const double ln2 = 0.6931471805599453;
                x0 -= ln2 * fc.rho_ex * acc[7];
            }
            B0 = b0 * fc.corr;
            X0 = x0 * fc.corr;
            B1 = acc[1] * fc.corr * fc.Kx;
            B2 = acc[2] * fc.corr * fc.Kt;
            X1 = acc[6] * fc.corr * fc.inv_st;
            X2 = acc[7] * fc.corr * fc.Kh;
            B11 = acc[3] * fc.corr * fc.Kx * fc.Kx;
            B22 = acc[4] * fc.corr * fc.Kt * fc.Kt;
            X11 = acc[8] * fc.corr * fc.inv_st * fc.inv_st;
            X22 = acc[9] * fc.corr * fc.Kh * fc.Kh;
        }
        const double lamv = fc.c_b * B0 + fc.c_e * X0;
        lam[i] = lamv;
        if (!(lamv > 0.0)) {
            atomicOr(status, isnan(lamv) ? HK_ST_NONFINITE : HK_ST_ZERO);
        }
        s[0] = log(lamv);
        // the column pass's weight w_i = c_e / lambda_i as its log2 (FP64), which
        // enters the exponent of each term c_e E_ij / lambda_i
        lw[i] = lamv > 0.0 ? fmax(fc.log2_ce - s[0] * 1.4426950408889634, HK_EXP_FLOOR) : HK_EXP_FLOOR;
        const double inv = 1.0 / lamv;
        if (MODE >= HK_MODE_GRAD) {
            const double tx = fc.tau_x, tt = fc.tau_t, om = fc.omega, hh = fc.h;
            double d1[6];
            d1[0] = fc.cb1 * B0;
            d1[1] = fc.c_b * (-2.0 * B0 / tx + B1 / (tx * tx * tx));
            d1[2] = fc.c_b * (-B0 / tt + B2 / (tt * tt * tt));
            d1[3] = fc.ce1 * X0;
            d1[4] = fc.c_e * (X0 / om - X1);
            d1[5] = fc.c_e * (-2.0 * X0 / hh + X2 / (hh * hh * hh));
#pragma unroll
            for (int p = 0; p < 6; ++p) s[1 + p] = d1[p] * inv;
            if (MODE >= HK_MODE_HESS) {
                const double tx2 = tx * tx, tt2 = tt * tt, hh2 = hh * hh;
                double d2[6];
                d2[0] = 0.0;
                d2[1] = fc.c_b * (6.0 * B0 / tx2 - 7.0 * B1 / (tx2 * tx2) + B11 / (tx2 * tx2 * tx2));
                d2[2] = fc.c_b * (2.0 * B0 / tt2 - 5.0 * B2 / (tt2 * tt2) + B22 / (tt2 * tt2 * tt2));
                d2[3] = 0.0;
                d2[4] = fc.c_e * (X11 - 2.0 * X1 / om);
                d2[5] = fc.c_e * (6.0 * X0 / hh2 - 7.0 * X2 / (hh2 * hh2) + X22 / (hh2 * hh2 * hh2));
#pragma unroll
                for (int p = 0; p < 6; ++p) s[7 + p] = d2[p] * inv - s[1 + p] * s[1 + p];
            }
        }
        // integral term (App. A for the excitation; exact background integral)
        const double ti = ts[i];
        const double th = theta[perm[i]];
        const double sv = fc.t1 - ti;
        const double u1 = sv / fc.tau_t, u0 = (fc.t0 - ti) / fc.tau_t;
        const double Cn = std_cdf(u1) - std_cdf(u0);
        const double e = exp(-fc.omega * sv);
        const double one_m = -expm1(-fc.omega * sv);
        s[13] = fc.mu0 * Cn + fc.theta0 * th * one_m;
        a_out[i] = fc.theta0 * one_m;
        if (MODE >= HK_MODE_GRAD) {
            const double p1 = std_pdf(u1), p0 = std_pdf(u0);
            s[14] = Cn;
            s[15] = fc.mu0 * (-p1 * u1 + p0 * u0) / fc.tau_t;
            s[16] = th * one_m;
            s[17] = fc.theta0 * th * sv * e;
            s[18] = fc.mu0 * (p1 * (2.0 * u1 - u1 * u1 * u1) - p0 * (2.0 * u0 - u0 * u0 * u0)) / (fc.tau_t * fc.tau_t);
            s[19] = -fc.theta0 * th * sv * sv * e;
        }
    } else {
        lam[i] = 1.0;
        lw[i] = HK_EXP_FLOOR;
        a_out[i] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < HK_NSUM; ++k) {
        const double v = wave_sum_f64(s[k]);
        if (lane == k) blockpart[(int64_t)k * gridDim.x + blockIdx.x] = v;
    }
}


// The ten sums of row i straight from the definitions (Sec. 2.1): b_ij over
// every j != i, theta_j E_ij over the strictly earlier j, each term in FP64
// (the range of the oracle), this thread's share j = t, t + nt, ...
__device__ void exact_row_sums(const double *__restrict__ ts, const double *__restrict__ xs,
                               const double *__restrict__ ys, const double *__restrict__ theta,
                               const int *__restrict__ perm, const int *__restrict__ g, int64_t n,
                               const FinConst &fc, int64_t i, int t, int nt, double (&m)[HK_NROW]) {
    const double ti = ts[i], xi = xs[i], yi = ys[i];
    const int gi = g[i];
    const double kb = 0.5 / (fc.tau_x * fc.tau_x), kt = 0.5 / (fc.tau_t * fc.tau_t);
    const double kh = 0.5 / (fc.h * fc.h);
    for (int64_t j = t; j < n; j += nt) {
        if (j == i) continue;
        const double dx = xi - xs[j], dy = yi - ys[j];
        const double r2 = dx * dx + dy * dy;
        const double dt = ti - ts[j], dt2 = dt * dt;
        const double b = exp(-(r2 * kb) - dt2 * kt);
        m[0] += b;
        m[1] += b * r2;
        m[2] += b * dt2;
        m[3] += b * r2 * r2;
        m[4] += b * dt2 * dt2;
        if (j < gi) {
            const double te = theta[perm[j]] * exp(-fc.omega * dt - r2 * kh);
            m[5] += te;
            m[6] += te * dt;
            m[7] += te * r2;
            m[8] += te * dt2;
            m[9] += te * r2 * r2;
        }
    }
}

// Finalisation, one block per 64-event chunk.  The HK_FIN_WAVES wavefronts
// first split the partial sums of the chunk's events between them (row pieces
// and column partials of the later row tiles, round robin; these reads are the
// kernel's cost, so many are kept in flight), the partials are combined in a
// fixed order through LDS, and the first wavefront finishes the events.
template <int MODE>
__global__ __launch_bounds__(HK_FIN_WAVES * HK_WAVE) void k_fin(const double *__restrict__ ts, const double *__restrict__ xs,
                                             const double *__restrict__ ys, const int *__restrict__ g,
                                             const double *__restrict__ theta,
                                             const int *__restrict__ perm, int64_t n, int ntiles,
                                             const int *__restrict__ row_item0, const int *__restrict__ row_nseg,
                                             const float *__restrict__ rowpart, const float *__restrict__ colpart,
                                             const FinConst fc,
                                             double *__restrict__ lam, double *__restrict__ lw,
                                             double *__restrict__ a_out,
                                             double *__restrict__ blockpart, int *__restrict__ status) {
    __shared__ double part[HK_FIN_WAVES][HK_NROW][HK_WAVE];
    const int lane = threadIdx.x & (HK_WAVE - 1), wq = threadIdx.x / HK_WAVE;
    const int64_t i = (int64_t)blockIdx.x * HK_WAVE + lane;
    const int I = (int)(i / HK_TILE), r = (int)(i % HK_TILE);
    {
        double acc[HK_NROW];
#pragma unroll
        for (int k = 0; k < HK_NROW; ++k) acc[k] = 0.0;
        const int it0 = row_item0[I], ns = row_nseg[I];
        #pragma unroll 2
        for (int sg = wq; sg < ns; sg += HK_FIN_WAVES) {
            const float *rp = rowpart + (int64_t)(it0 + sg) * HK_NROW * HK_TILE + r;
            acc[0] += rp[0];
            acc[5] += rp[5 * HK_TILE];
            if (MODE >= HK_MODE_GRAD) {
                acc[1] += rp[1 * HK_TILE];
                acc[2] += rp[2 * HK_TILE];
                acc[6] += rp[6 * HK_TILE];
                acc[7] += rp[7 * HK_TILE];
            }
            if (MODE >= HK_MODE_HESS) {
                acc[3] += rp[3 * HK_TILE];
                acc[4] += rp[4 * HK_TILE];
                acc[8] += rp[8 * HK_TILE];
                acc[9] += rp[9 * HK_TILE];
            }
        }
        // background from later events: the column partials of row tiles J >= I
        // (region J starts at HK_NCOL HK_TILE J (J + 1) / 2)
        #pragma unroll 2
        for (int J = I + wq; J < ntiles; J += HK_FIN_WAVES) {
            const int64_t stride = (int64_t)(J + 1) * HK_TILE;
            const float *cp = colpart + (int64_t)HK_NCOL * HK_TILE * J * (J + 1) / 2 + i;
            acc[0] += (double)cp[0];
            if (MODE >= HK_MODE_GRAD) {
                acc[1] += (double)cp[stride];
                acc[2] += (double)cp[2 * stride];
            }
            if (MODE >= HK_MODE_HESS) {
                acc[3] += (double)cp[3 * stride];
                acc[4] += (double)cp[4 * stride];
            }
        }
#pragma unroll
        for (int k = 0; k < HK_NROW; ++k) part[wq][k][lane] = acc[k];
    }
    __syncthreads();
    // rows whose intensity from the partials is below fc.lam_exact (their FP32
    // terms may have lost more than 2^-30 of it) are recomputed here in FP64 by
    // the whole block, one row at a time; every wavefront derives the same mask
    __shared__ double exact[HK_NROW][HK_WAVE];
    __shared__ double red[HK_FIN_WAVES][HK_NROW];
    double b0 = part[0][0][lane], x0 = part[0][5][lane];
    for (int q = 1; q < HK_FIN_WAVES; ++q) {
        b0 += part[q][0][lane];
        x0 += part[q][5][lane];
    }
    const bool low = i < n && fc.c_b * b0 + fc.c_e * x0 < fc.lam_exact;
    const uint64_t low_mask = __ballot(low);
    for (uint64_t mk = low_mask; mk != 0; mk &= mk - 1) {
        const int rr = __ffsll((unsigned long long)mk) - 1;
        double m[HK_NROW];
#pragma unroll
        for (int k = 0; k < HK_NROW; ++k) m[k] = 0.0;
        exact_row_sums(ts, xs, ys, theta, perm, g, n, fc, (int64_t)blockIdx.x * HK_WAVE + rr, threadIdx.x,
                       HK_FIN_WAVES * HK_WAVE, m);
#pragma unroll
        for (int k = 0; k < HK_NROW; ++k) m[k] = wave_sum_f64(m[k]);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < HK_NROW; ++k) red[wq][k] = m[k];
        }
        __syncthreads();
        if (threadIdx.x < HK_NROW) {
            double v = red[0][threadIdx.x];
            for (int q = 1; q < HK_FIN_WAVES; ++q) v += red[q][threadIdx.x];
            exact[threadIdx.x][rr] = v;
        }
        __syncthreads();
    }
    if (wq == 0) fin_events<MODE>(ts, theta, perm, n, fc, part, exact, low, lane, i, lam, lw, a_out, blockpart,
                                  status);
}

// One block: the partials of every k_fin block -> the scalar results.
__global__ __launch_bounds__(HK_NSUM * HK_TOT_LANES) void k_fin2(const double *__restrict__ blockpart, int nblocks,
                                                                double *__restrict__ loglik,
                                                                double *__restrict__ grad_hyper,
                                                                double *__restrict__ negH_hyper,
                                                                int *__restrict__ status) {
    __shared__ double tot[HK_NSUM];
    fin_totals(blockpart, nblocks, loglik, grad_hyper, negH_hyper, status, tot);
}


// ------------------------------------------------------------------------------------
// Column pass.  G_j = sum_{t_i > t_j} T_ij and H_j = sum T_ij^2 with
// T_ij = c_e E_ij / lambda_i (Eq. 4 without theta0's integral term, and Eq. 5)
// for the lanes' columns j against a staged chunk of 64 later rows i.
//
// Each term is one exponential of its whole exponent in log2 units,
//   e_ij = lw_i - omega (t_i - t_j) / ln2 - |s (x_i - x_j)|^2,
// with lw_i = log2(c_e / lambda_i) from the finalisation and s = 1 / (h sqrt(2
// ln 2)), formed in FP64.  e_ij is split into its nearest integer n and a
// fraction f in [-1/2, 1/2]; only f is rounded to FP32 for the hardware exp2
// and 2^n is applied exactly (ldexp).  The term's relative error is then a few
// FP32 roundings whatever the size of e_ij: Eq. 5 squares the terms, and an
// error in the exponent's absolute value would become a relative error of the
// term that grows with |e_ij|.
//
// Eq. 4 alone (no Hessian) splits the row's weight instead: n_i =
// rint(lw_i) is applied exactly and the rest of the exponent, small for the
// terms that make up G_j, is rounded once to FP32 (relative error about 2^-24
// ln2 |e_ij - n_i| per term, larger only for terms negligible in the sum).
//
// The exponent is split into a row part (staged), a column part (per lane)
// and the cross term.  With DOT the spatial part is expanded,
//   -|u_i - u_j|^2 = 2 u_i . u_j - |u_i|^2 - |u_j|^2   (u = s x),
// which takes three FP64 operations per pair; it is used when every |u|^2 is
// at most HK_DOT_MAX2, where the cancellation costs at most ~2^-30 absolute.
// Otherwise the differences are formed (five operations).  Times enter
// relative to the column tile's first time, so that both parts stay small for
// the pairs whose terms are not negligible.
struct ColRow {     // one staged row
    double2 u;      // DOT: 2 u_i; else u_i
    double c;       // lw_i + kw (t_i - T_ref) (DOT: minus |u_i|^2), at least HK_EXP_FLOOR; Eq. 4 alone: minus n
    int n;          // Eq. 4 alone: rint(lw_i) (0 for a row at the floor), applied exactly
};

template <bool DOT>
__device__ __forceinline__ double col_exponent(const ColRow &r, double xj, double yj, double dj) {
    if (DOT) return fma(r.u.x, xj, fma(r.u.y, yj, r.c + dj));
    const double dx = r.u.x - xj, dy = r.u.y - yj;
    return fma(-dx, dx, fma(-dy, dy, r.c + dj));
}


template <bool SPLIT, bool MASKED, bool DOT>
__device__ __forceinline__ float col_term(const ColRow *__restrict__ rows, const int *__restrict__ rg, int s,
                                          int jcol, double xj, double yj, double dj) {
    const double e = col_exponent<DOT>(rows[s], xj, yj, dj);
    float T = SPLIT ? exp2_split(e) : __builtin_amdgcn_ldexpf(fexp2((float)e), rows[s].n);
    if (MASKED) {
        if (!(jcol < rg[s])) T = 0.0f;
    }
    return T;
}

// Two interleaved streams of steps (even and odd rows of the chunk) with their
// own accumulators: the FP64 exponent chains of neighbouring steps overlap.
// The loop is kept short (HK_COL_UNROLL pairs of steps per iteration): a
// deeper unroll hoists more LDS loads into registers and fits fewer
// wavefronts per SIMD.
#ifndef HK_COL_UNROLL
#define HK_COL_UNROLL 2
#endif
constexpr int kColUnroll = HK_COL_UNROLL;
template <bool WITH_H, bool SPLIT, bool MASKED, bool DOT>
__device__ __forceinline__ void col_sweep(const ColRow *__restrict__ rows, const int *__restrict__ rg, int jcol,
                                          double xj, double yj, double dj, float &G, float &H) {
#pragma clang fp contract(off)
    float G1 = 0.0f, H1 = 0.0f;
#pragma unroll kColUnroll
    for (int s = 0; s < HK_WAVE; s += 2) {
        const float e0 = col_term<SPLIT, MASKED, DOT>(rows, rg, s, jcol, xj, yj, dj);
        const float e1 = col_term<SPLIT, MASKED, DOT>(rows, rg, s + 1, jcol, xj, yj, dj);
        G += e0;
        G1 += e1;
        if (WITH_H) {
            H = fmaf(e0, e0, H);
            H1 = fmaf(e1, e1, H1);
        }
    }
    G += G1;
    H += H1;
}

template <bool WITH_H, bool DOT>
__global__ __launch_bounds__(HK_TILE) void k_col(const double *__restrict__ ts, const double *__restrict__ xs,
                                                  const double *__restrict__ ys, const double *__restrict__ lw,
                                                  const int *__restrict__ g, int64_t n,
                                                  const hk_item *__restrict__ items, const int *__restrict__ block0,
                                                  double *__restrict__ colG, const PairConst kc) {
    __shared__ ColRow rows[HK_WAVE];
    __shared__ int rg[HK_WAVE];
    __shared__ int chunk_split;  // Eq. 4 alone: the staged chunk splits every exponent exactly
    // uniform wavefront index: the per-wave bounds select the sweep with scalar branches
    const int tid = threadIdx.x, wvi = __builtin_amdgcn_readfirstlane(tid / HK_WAVE);
    const int q_end = block0[blockIdx.x + 1];

    for (int q = block0[blockIdx.x]; q < q_end; ++q) {
        const hk_item it = items[q];
        const int J = it.tile;
        const int64_t col0 = (int64_t)J * HK_TILE;
        const int jcol = (int)(col0 + tid);
        const double t_ref = ts[col0];
        const double uxj = xs[jcol] * kc.sx, uyj = ys[jcol] * kc.sx;
        // the column's part of the exponent: omega (t_j - T_ref) / ln2 (DOT:
        // minus |u_j|^2); a padding column's terms are never used
        double dj = -kc.kw_d * (ts[jcol] - t_ref);
        if (DOT) dj -= fma(uxj, uxj, uyj * uyj);
        if (jcol >= n) dj = HK_EXP_FLOOR;
        const int wave_first = (int)(col0 + wvi * HK_WAVE);
        const double wave_tmax = ts[(int64_t)wave_first + HK_WAVE - 1];  // the wave's latest column

        const double tile_tmax = ts[col0 + HK_TILE - 1];
        double Gd = 0.0, Hd = 0.0;
        for (int c = it.c_begin; c < it.c_end; ++c) {
            const double Tc = ts[(int64_t)c * HK_WAVE];
            // under the cutoff, rows starting more than dt_cut_ex after the
            // tile's latest column end the sweep (times are sorted)
            if (Tc - tile_tmax > kc.dt_cut_ex) break;
            if (tid < HK_WAVE) {
                const int64_t i = (int64_t)c * HK_WAVE + tid;
                const double ux = xs[i] * kc.sx, uy = ys[i] * kc.sx;
                const double lwi = lw[i];
                double cr = lwi + kc.kw_d * (ts[i] - t_ref);
                ColRow r;
                if (DOT) {
                    cr -= fma(ux, ux, uy * uy);
                    r.u = make_double2(2.0 * ux, 2.0 * uy);
                } else {
                    r.u = make_double2(ux, uy);
                }
                r.c = fmax(cr, HK_EXP_FLOOR);
                r.n = 0;
                // the staging wavefront holds the chunk's 64 rows
                const bool split = !WITH_H && __ballot(lwi > HK_LW_SPLIT_MAX) != 0;
                if (!WITH_H && !split && lwi > HK_EXP_FLOOR) {
                    const double nw = rint(lwi);
                    r.n = (int)nw;
                    r.c -= nw;
                }
                rows[tid] = r;
                rg[tid] = g[i];
                if (tid == 0) chunk_split = split;
            }
            __syncthreads();
            const int gmax = rg[HK_WAVE - 1], gmin = rg[0];
            const bool split = WITH_H || chunk_split != 0;
            // optional underflow cutoff: rows that all start more than dt_cut_ex
            // after the wave's latest column give excitation terms below 2^-160
            if (gmax > wave_first && !(Tc - wave_tmax > kc.dt_cut_ex)) {
                float G = 0.0f, H = 0.0f;
                if (gmin <= wave_first + HK_WAVE - 1) {
                    if (split)
                        col_sweep<WITH_H, true, true, DOT>(rows, rg, jcol, uxj, uyj, dj, G, H);
                    else
                        col_sweep<WITH_H, false, true, DOT>(rows, rg, jcol, uxj, uyj, dj, G, H);
                } else {
                    if (split)
                        col_sweep<WITH_H, true, false, DOT>(rows, rg, jcol, uxj, uyj, dj, G, H);
                    else
                        col_sweep<WITH_H, false, false, DOT>(rows, rg, jcol, uxj, uyj, dj, G, H);
                }
                Gd += (double)G;
                if (WITH_H) Hd += (double)H;
            }
            __syncthreads();
        }
        double *cg = colG + (int64_t)q * 2 * HK_TILE;
        cg[tid] = Gd;
        if (WITH_H) cg[HK_TILE + tid] = Hd;
    }
}

// Column finalisation, one block per 64-event chunk: the HK_FIN_WAVES
// wavefronts split the column pieces round robin (reads in flight), then the
// first combines them in a fixed order.
//
// With `totals` set, one block more (the last) reduces the row finalisation's
// block partials to the scalar results instead (the work of k_fin2, whose
// inputs are complete once the column pass runs): one launch fewer per
// evaluation.
__global__ __launch_bounds__(HK_FIN_WAVES * HK_WAVE) void k_colfin(const int *__restrict__ perm, int64_t n,
                                                const int *__restrict__ col_item0, const int *__restrict__ col_nseg,
                                                const double *__restrict__ colG, const double *__restrict__ a,
                                                const FinConst fc, double *__restrict__ grad_theta,
                                                double *__restrict__ negH_theta, int totals,
                                                const double *__restrict__ blockpart, int nfin,
                                                double *__restrict__ loglik, double *__restrict__ grad_hyper,
                                                double *__restrict__ negH_hyper, int *__restrict__ status) {
    __shared__ double part[HK_FIN_WAVES][2][HK_WAVE];
    if (totals && blockIdx.x == gridDim.x - 1) {
        __shared__ double tot[HK_NSUM];
        fin_totals(blockpart, nfin, loglik, grad_hyper, negH_hyper, status, tot);
        return;
    }
    const int lane = threadIdx.x & (HK_WAVE - 1), wv = threadIdx.x / HK_WAVE;
    const int64_t j = (int64_t)blockIdx.x * HK_WAVE + lane;
    const int J = (int)(j / HK_TILE), r = (int)(j % HK_TILE);
    const int it0 = col_item0[J], ns = col_nseg[J];
    double G = 0.0, H = 0.0;
    #pragma unroll 2
    for (int sg = wv; sg < ns; sg += HK_FIN_WAVES) {
        const double *cg = colG + (int64_t)(it0 + sg) * 2 * HK_TILE + r;
        G += cg[0];
        if (negH_theta) H += cg[HK_TILE];
    }
    part[wv][0][lane] = G;
    part[wv][1][lane] = H;
    __syncthreads();
    if (wv != 0 || j >= n) return;
    double Gs = part[0][0][lane], Hs = part[0][1][lane];
    for (int q = 1; q < HK_FIN_WAVES; ++q) {
        Gs += part[q][0][lane];
        Hs += part[q][1][lane];
    }
    const int dst = perm[j];
    if (grad_theta) grad_theta[dst] = Gs * fc.corr - a[j];
    if (negH_theta) negH_theta[dst] = Hs * fc.corr * fc.corr;
}

__global__ void k_scatter_lambda(const double *__restrict__ lam, const int *__restrict__ perm, int64_t n,
                                 double *__restrict__ out) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j < n) out[perm[j]] = lam[j];
}

}  // namespace

bool hk_hyper_ok(const hawkes_hyper *h) {
    if (!h) return false;
    const double v[6] = {h->mu0, h->tau_x, h->tau_t, h->theta0, h->omega, h->h};
    for (double x : v)
        if (!isfinite(x)) return false;
    return h->tau_x > 0 && h->tau_t > 0 && h->omega > 0 && h->h > 0 && h->mu0 >= 0 && h->theta0 >= 0;
}

// Constants shared by the evaluation entry points.
void hk_make_consts(const hawkes_plan p, const hawkes_hyper *hy, PairConst *kc, FinConst *fc) {
    const double ln2 = 0.6931471805599453;
    const double kbx = -1.0 / (2.0 * hy->tau_x * hy->tau_x * ln2);
    const double kbt = -1.0 / (2.0 * hy->tau_t * hy->tau_t * ln2);
    const double kex = -1.0 / (2.0 * hy->h * hy->h * ln2);
    const double kw = -hy->omega / ln2;
    kc->st = sqrt(-kbt);
    kc->omega = hy->omega;
    kc->kw_d = kw;
    kc->kw_s = kw / kc->st;
    // time gaps beyond which every background term (exponent <= kbt dt^2) and
    // every excitation term (exponent <= kw dt) is below 2^-160: exactly zero in
    // FP32, and below 1e-48 of a unit term in the split form
    if (p->cutoff) {
        kc->dt_cut_ex = -160.0 / kw;
        kc->dt_cut = fmax(sqrt(-160.0 / kbt), kc->dt_cut_ex);
    } else {
        kc->dt_cut = kc->dt_cut_ex = INFINITY;
    }
    kc->sx = sqrt(-kex);
    kc->sbx = sqrt(-kbx);
    {
        // largest |s x|^2 over the plan: the coordinates are centred, so |x| is
        // at most half the bounding box's larger side (with a margin for rounding)
        const double half = 0.5 * fmax(p->xmax - p->xmin, p->ymax - p->ymin) * (1.0 + 1e-12);
        const double umax = half * kc->sx;
        kc->dot = 2.0 * umax * umax <= HK_DOT_MAX2;
    }
    kc->rex = (float)(kex / kbx);
    kc->rex_x = kex / kbx;
    kc->span_max = fmin(HK_FACT_SPAN / hy->omega, HK_COMPACT_TAU * hy->tau_t);
    kc->rex_lo = (float)(kex / kbx - (double)kc->rex);
    fc->Kt = -1.0 / kbt;
    fc->inv_st = 1.0 / kc->st;
    fc->rho_ex = ((double)kc->rex - kex / kbx) / (double)kc->rex;
    const double corr = 1.0 / (1.0 + HK_EXP2_BIAS);
    const double two_pi = 6.283185307179586;
    fc->mu0 = hy->mu0; fc->tau_x = hy->tau_x; fc->tau_t = hy->tau_t;
    fc->theta0 = hy->theta0; fc->omega = hy->omega; fc->h = hy->h;
    fc->cb1 = 1.0 / (pow(two_pi, 1.5) * hy->tau_x * hy->tau_x * hy->tau_t);
    fc->ce1 = hy->omega / (two_pi * hy->h * hy->h);
    fc->c_b = fc->cb1 * hy->mu0;
    fc->c_e = fc->ce1 * hy->theta0;
    fc->log2_ce = log2(fc->c_e);
    // moments are accumulated in log2 units of the exponent: r^2 = -2 s^2 ln2 * a
    fc->Kx = -2.0 * hy->tau_x * hy->tau_x * ln2;
    fc->Kh = -2.0 * hy->h * hy->h * ln2;
    fc->corr = corr;
    fc->lam_exact = (fc->c_b + fc->c_e) * (double)p->n * 0x1p-96;
    fc->t0 = p->t0;
    fc->t1 = p->t1;
}

// Column pass and its finalisation on the plan's current w, a (Eq. 4, Eq. 5).
// With `totals`, the same launch as the column finalisation also reduces the
// row finalisation's block partials to d_loglik, d_grad_hyper, d_negH_hyper.
static void launch_col(hawkes_plan p, const PairConst &kc, const FinConst &fc, double *d_grad_theta,
                       double *d_negH_theta, hipStream_t stream, bool totals = false, double *d_loglik = nullptr,
                       double *d_grad_hyper = nullptr, double *d_negH_hyper = nullptr) {
    hk_prof_mark(p, HK_PROF_COL, true, stream);
#define HK_COL(H, D)                                                                                        \
    hipLaunchKernelGGL((k_col<H, D>), dim3(p->n_col_blocks), dim3(HK_TILE), 0, stream, p->ts, p->xs, p->ys, p->lw, \
                       p->g, p->n, p->col_items, p->col_block0, p->colG, kc)
    if (d_negH_theta) {
        if (kc.dot) HK_COL(true, true);
        else HK_COL(true, false);
    } else {
        if (kc.dot) HK_COL(false, true);
        else HK_COL(false, false);
    }
#undef HK_COL
    hk_prof_mark(p, HK_PROF_COL, false, stream);
    hipLaunchKernelGGL(k_colfin, dim3(p->nchunks + (totals ? 1 : 0)), dim3(HK_FIN_WAVES * HK_WAVE), 0, stream,
                       p->perm, p->n, p->col_item0, p->col_nseg, p->colG, p->a, fc, d_grad_theta, d_negH_theta,
                       totals ? 1 : 0, p->blockpart, p->nchunks, d_loglik, d_grad_hyper, d_negH_hyper, p->status);
}

extern "C" int64_t hawkes_plan_epoch(hawkes_plan p) { return p ? p->epoch : -1; }

extern "C" hawkes_status hawkes_plan_set_cutoff(hawkes_plan p, int enabled) {
    if (!p) return HAWKES_E_INVALID;
    p->cutoff = enabled != 0;
    return HAWKES_OK;
}

extern "C" hawkes_status hawkes_grad_theta_from_last(hawkes_plan p, const hawkes_hyper *hyper, int64_t epoch,
                                                     double *d_grad_theta, double *d_negH_theta,
                                                     hipStream_t stream) {
    if (!p || !hk_hyper_ok(hyper) || (!d_grad_theta && !d_negH_theta)) return HAWKES_E_INVALID;
    const hawkes_hyper &h = p->eval_hyper;
    const bool same = h.mu0 == hyper->mu0 && h.tau_x == hyper->tau_x && h.tau_t == hyper->tau_t &&
                      h.theta0 == hyper->theta0 && h.omega == hyper->omega && h.h == hyper->h;
    if (p->eval_epoch == 0 || epoch != p->eval_epoch || p->epoch != p->eval_epoch || !same) return HAWKES_E_STALE;
    p->last_stream = stream;
    PairConst kc;
    FinConst fc;
    hk_make_consts(p, hyper, &kc, &fc);
    launch_col(p, kc, fc, d_grad_theta, d_negH_theta, stream);
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}

extern "C" hawkes_status hawkes_eval(hawkes_plan p, const hawkes_hyper *hyper, const double *d_theta,
                                     double *d_loglik, double *d_grad_theta, double *d_grad_hyper,
                                     double *d_negH_theta, double *d_negH_hyper, hipStream_t stream) {
    if (!p || !d_theta || !hk_hyper_ok(hyper)) return HAWKES_E_INVALID;
    p->last_stream = stream;
    PairConst kc;
    FinConst fc;
    hk_make_consts(p, hyper, &kc, &fc);
    // the row pass carries the moments the requested hyperparameter derivatives
    // need: none for the log-likelihood and the rate derivatives (Eq. 4, Eq. 5
    // only need lambda), first moments for the hyperparameter gradient, second
    // moments for its Hessian diagonal
    const int mode = d_negH_hyper ? HK_MODE_HESS : (d_grad_hyper ? HK_MODE_GRAD : HK_MODE_LOGLIK);
    const int64_t npad = p->npad;

    hk_prof_mark(p, HK_PROF_EVAL, true, stream);
    hipLaunchKernelGGL(k_tfac<true>, dim3((unsigned)(npad / 256)), dim3(256), 0, stream, d_theta, p->perm, p->ts,
                       p->n, kc.omega, kc.span_max, p->theta_s, p->theta_v, p->chunk_precise, p->tstep, p->status);
    hk_prof_mark(p, HK_PROF_ROW, true, stream);
#define HK_ROW(M)                                                                                              \
    hipLaunchKernelGGL(k_row<M>, dim3(p->n_row_blocks), dim3(HK_TILE), 0, stream, p->ts, p->xs, p->ys,          \
                       p->theta_v, p->chunk_precise, p->tstep, p->g, p->row_items, p->row_block0, p->colpart_off,             \
                       p->rowpart, p->colpart, kc)
#define HK_FIN(M)                                                                                              \
    hipLaunchKernelGGL(k_fin<M>, dim3(p->nchunks), dim3(HK_FIN_WAVES * HK_WAVE), 0, stream, p->ts, p->xs, p->ys, \
                       p->g, d_theta,                                                                          \
                       p->perm, p->n, p->ntiles, p->row_item0, p->row_nseg, p->rowpart, p->colpart, fc,             \
                       p->lam, p->lw, p->a, p->blockpart, p->status)
    if (mode == HK_MODE_LOGLIK) HK_ROW(HK_MODE_LOGLIK);
    else if (mode == HK_MODE_GRAD) HK_ROW(HK_MODE_GRAD);
    else HK_ROW(HK_MODE_HESS);
    hk_prof_mark(p, HK_PROF_ROW, false, stream);
    if (mode == HK_MODE_LOGLIK) HK_FIN(HK_MODE_LOGLIK);
    else if (mode == HK_MODE_GRAD) HK_FIN(HK_MODE_GRAD);
    else HK_FIN(HK_MODE_HESS);
#undef HK_ROW
#undef HK_FIN
    // the scalar results come from the block partials: with a column pass, in
    // its finalisation's launch; without, in a launch of their own
    const bool col = d_grad_theta || d_negH_theta;
    if (!col)
        hipLaunchKernelGGL(k_fin2, dim3(1), dim3(HK_NSUM * HK_TOT_LANES), 0, stream, p->blockpart, p->nchunks,
                           d_loglik, d_grad_hyper, d_negH_hyper, p->status);
    p->epoch += 1;
    p->eval_epoch = p->epoch;
    p->eval_hyper = *hyper;
    if (col) launch_col(p, kc, fc, d_grad_theta, d_negH_theta, stream, true, d_loglik, d_grad_hyper, d_negH_hyper);
    hk_prof_mark(p, HK_PROF_EVAL, false, stream);
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}

void hk_launch_row_loglik(hawkes_plan p, const PairConst &kc, hipStream_t stream) {
    hipLaunchKernelGGL(k_tfac<false>, dim3((unsigned)(p->npad / 256)), dim3(256), 0, stream, (const double *)nullptr,
                       p->perm, p->ts, p->n, kc.omega, kc.span_max, p->theta_s, p->theta_v, p->chunk_precise, p->tstep, p->status);
    hipLaunchKernelGGL(k_row<HK_MODE_LOGLIK>, dim3(p->n_row_blocks), dim3(HK_TILE), 0, stream, p->ts, p->xs, p->ys,
                       p->theta_v, p->chunk_precise, p->tstep, p->g, p->row_items, p->row_block0, p->colpart_off, p->rowpart,
                       p->colpart, kc);
}

// Blocks per compute unit in the pair-pass schedules.  Eight blocks of four
// wavefronts fill a CU of gfx950 at the register footprints of k_row and k_col;
// two rounds of equal-weight blocks measured faster than one (the hardware
// dispatcher then evens out the blocks' run-time differences), while more
// rounds cost more partial-sum traffic than they gain.
#ifndef HK_BLOCKS_PER_CU
#define HK_BLOCKS_PER_CU 16
#endif

// From 65,536 (padded) events on, 20 row-pass and 32 column-pass blocks per CU:
// their shorter runs balance the larger passes better (N = 100,000 and 250,000:
// 2% per evaluation), while on smaller sets the extra partial sums cost as much
// as the balance gains.
#ifndef HK_LARGE_NPAD
#define HK_LARGE_NPAD 65536
#endif

int64_t hk_pass_slots(int device, int pass, int64_t npad) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1)
        cus = 256;
    if (npad >= HK_LARGE_NPAD) return (int64_t)cus * (pass == 1 ? 32 : 20);
    return (int64_t)cus * HK_BLOCKS_PER_CU;
}

extern "C" hawkes_status hawkes_loglik(hawkes_plan p, const hawkes_hyper *hyper, const double *d_theta,
                                       double *d_loglik, hipStream_t stream) {
    if (!d_loglik) return HAWKES_E_INVALID;
    return hawkes_eval(p, hyper, d_theta, d_loglik, nullptr, nullptr, nullptr, nullptr, stream);
}

extern "C" hawkes_status hawkes_grad(hawkes_plan p, const hawkes_hyper *hyper, const double *d_theta,
                                     double *d_loglik, double *d_grad_theta, double *d_grad_hyper,
                                     hipStream_t stream) {
    return hawkes_eval(p, hyper, d_theta, d_loglik, d_grad_theta, d_grad_hyper, nullptr, nullptr, stream);
}

extern "C" hawkes_status hawkes_hessdiag(hawkes_plan p, const hawkes_hyper *hyper, const double *d_theta,
                                         double *d_negH_theta, double *d_negH_hyper, hipStream_t stream) {
    if (!d_negH_theta && !d_negH_hyper) return HAWKES_E_INVALID;
    return hawkes_eval(p, hyper, d_theta, nullptr, nullptr, nullptr, d_negH_theta, d_negH_hyper, stream);
}

extern "C" hawkes_status hawkes_copy_lambda(hawkes_plan p, double *d_lambda, hipStream_t stream) {
    if (!p || !d_lambda) return HAWKES_E_INVALID;
    hipLaunchKernelGGL(k_scatter_lambda, dim3((unsigned)((p->n + 255) / 256)), dim3(256), 0, stream, p->lam,
                       p->perm, p->n, d_lambda);
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}
