// Evaluation of Eq. 1 (log-likelihood), Eq. 3 (rate gradient), Eq. 4 (rate
// Hessian diagonal) and the hyperparameter derivatives on gfx950.
//
// Kernels, in launch order:
//   k_gather   theta to sorted order (FP32), validity check
//   k_row      row pass over causal tile pairs: for each row i the background
//              moments over j < i and the excitation moments over t_j < t_i;
//              the background is symmetric, so each pair also adds its
//              background moments to column j through accumulators that rotate
//              one lane per step around the wavefront (DPP wave_rol)
//   k_fin      per event: partial sums -> lambda_i (FP64), log lambda_i,
//              w_i = c_e / lambda_i, integral term (App. A), hyperparameter
//              terms; fixed-order block reduction (DPP within the wavefront)
//   k_fin2     one block: block partials -> loglik, grad/negH of hyperparameters
//   k_col      column pass: G_j = sum_{t_i > t_j} E_ij w_i, H_j = sum (E_ij w_i)^2
//   k_colfin   G_j, H_j -> Eq. 3 / Eq. 4 in the caller's order
#include <hip/hip_runtime.h>
#include <math.h>

#include <vector>

#include "hawkes_internal.h"

struct hk_profile {
    std::vector<hipEvent_t> ev[HK_PROF_KINDS];  // start/stop pairs, in order
};

void hk_prof_mark(hawkes_plan p, int kind, bool start, hipStream_t stream) {
    if (!p->prof) return;
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
    if (!p) return HAWKES_E_INVALID;
    if (on && !p->prof) p->prof = new hk_profile();
    if (!on) hk_prof_free(p);
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
__global__ void k_gather(const double *__restrict__ theta, const int *__restrict__ perm, int64_t n,
                         int64_t npad, float *__restrict__ theta_s, int *__restrict__ status) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= npad) return;
    float v = 0.0f;
    if (i < n) {
        double th = theta[perm[i]];
        if (!(th >= 0.0) || !isfinite(th)) atomicOr(status, HK_ST_BADTHETA);
        v = (float)th;
    }
    theta_s[i] = v;
}

// ------------------------------------------------------------------------------------
// One sweep of a 64-column chunk by one wavefront: 64 steps, each lane pairing
// its row with column (lane + s) mod 64 of the chunk.
//
// The three sums lambda_i is built from (background row sum B0, background
// column sum, excitation X0) accumulate every term in FP64: a plain FP32 sum of
// positive terms rounds away every term below half an ulp of the running sum,
// which biases lambda low (by ~2e-8 relative on clustered data).  The moments
// used only by derivatives stay in FP32 blocks.
template <int MODE, bool MASK_BG, bool MASK_EX>
__device__ __forceinline__ void row_sweep(const float4 *__restrict__ rec, int lane, float ti, int xr, int yr,
                                          int irow, int gr, int cbase, const PairConst kc,
                                          float (&blk)[HK_NROW], float (&C)[HK_NCOL], double &B0d, double &X0d,
                                          double &C0d) {
    // explicit FMAs only: a contracted (rotated + product) cannot take the DPP
    // operand, while a plain add of the shared product can
#pragma clang fp contract(off)
#pragma unroll 16
    for (int s = 0; s < HK_WAVE; ++s) {
        const float4 r = rec[lane + s];
        const float dt = ti - r.x;
        const float dx = (float)(xr - __float_as_int(r.y));
        const float dy = (float)(yr - __float_as_int(r.z));
        const float r2 = fmaf(dx, dx, dy * dy);
        const float dt2 = dt * dt;
        const float ar = r2 * kc.kbx;
        float b = fexp2(fmaf(dt2, kc.kbt, ar));
        const float ae = r2 * kc.kex;
        float E = fexp2(fmaf(dt, kc.kw, ae));
        if (MASK_BG || MASK_EX) {
            const int j = cbase + ((lane + s) & (HK_WAVE - 1));
            if (MASK_BG && !(j < irow)) b = 0.0f;
            if (!(j < gr)) E = 0.0f;
        }
        const float te = E * r.w;
        B0d += (double)b;
        C0d = rot_next_d(C0d) + (double)b;
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
        X0d += (double)te;
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
}

template <int MODE>
__global__ __launch_bounds__(HK_TILE) void k_row(const double *__restrict__ ts, const int *__restrict__ xi,
                                                  const int *__restrict__ yi, const float *__restrict__ theta_s,
                                                  const int *__restrict__ g, const hk_item *__restrict__ items,
                                                  const int64_t *__restrict__ colpart_off,
                                                  double *__restrict__ rowpart, float *__restrict__ colpart,
                                                  double *__restrict__ colpart0, const PairConst kc) {
    __shared__ float4 rec[2 * HK_WAVE];
    __shared__ float colbuf[HK_WAVES][HK_NCOL][HK_WAVE];
    __shared__ double colbuf0[HK_WAVES][HK_WAVE];
    constexpr int NC = MODE == HK_MODE_LOGLIK ? 1 : (MODE == HK_MODE_GRAD ? 3 : 5);

    const hk_item it = items[blockIdx.x];
    const int I = it.tile;
    const int tid = threadIdx.x, lane = tid & (HK_WAVE - 1), wv = tid / HK_WAVE;
    const int64_t row0 = (int64_t)I * HK_TILE;
    const int irow = (int)(row0 + tid);
    const double tsi = ts[irow];
    const int xr = xi[irow], yr = yi[irow], gr = g[irow];
    const int wave_chunk = I * HK_CHUNKS_PER_TILE + wv;
    const int wave_gmin = g[(int64_t)wave_chunk * HK_WAVE];  // g is non-decreasing
    const int64_t stride = (int64_t)(I + 1) * HK_TILE;
    float *__restrict__ cp = colpart + colpart_off[I];
    double *__restrict__ cp0 = colpart0 + colpart_off[I] / HK_NCOL;

    float hi[HK_NROW], lo[HK_NROW];
#pragma unroll
    for (int a = 0; a < HK_NROW; ++a) hi[a] = lo[a] = 0.0f;
    double B0d = 0.0, X0d = 0.0;

    for (int c = it.c_begin; c < it.c_end; ++c) {
        // times relative to the chunk's first event: for the pairs that carry the
        // sums (close in time) both operands of dt are then small and exact to FP32
        const double Tc = ts[(int64_t)c * HK_WAVE];
        const float ti = (float)(tsi - Tc);
        if (tid < HK_WAVE) {
            const int64_t j = (int64_t)c * HK_WAVE + tid;
            float4 r;
            r.x = (float)(ts[j] - Tc);
            r.y = __int_as_float(xi[j]);
            r.z = __int_as_float(yi[j]);
            r.w = theta_s[j];
            rec[tid] = r;
            rec[tid + HK_WAVE] = r;
        }
        __syncthreads();
        float blk[HK_NROW], C[HK_NCOL];
        double C0d = 0.0;
#pragma unroll
        for (int a = 0; a < HK_NROW; ++a) blk[a] = 0.0f;
#pragma unroll
        for (int a = 0; a < HK_NCOL; ++a) C[a] = 0.0f;
        if (c <= wave_chunk) {
            const int cbase = c * HK_WAVE;
            if (c == wave_chunk)
                row_sweep<MODE, true, true>(rec, lane, ti, xr, yr, irow, gr, cbase, kc, blk, C, B0d, X0d, C0d);
            else if (cbase + HK_WAVE - 1 >= wave_gmin)
                row_sweep<MODE, false, true>(rec, lane, ti, xr, yr, irow, gr, cbase, kc, blk, C, B0d, X0d, C0d);
            else
                row_sweep<MODE, false, false>(rec, lane, ti, xr, yr, irow, gr, cbase, kc, blk, C, B0d, X0d, C0d);
        }
        // after 64 rotation steps lane l holds the accumulators of column (l - 1) mod 64
        const int col = (lane + HK_WAVE - 1) & (HK_WAVE - 1);
        colbuf0[wv][col] = C0d;
#pragma unroll
        for (int a = 1; a < NC; ++a) colbuf[wv][a][col] = C[a];
        __syncthreads();
        for (int q = tid; q < NC * HK_WAVE; q += HK_TILE) {
            const int a = q / HK_WAVE, cc = q % HK_WAVE;
            if (a == 0) {
                cp0[(int64_t)c * HK_WAVE + cc] = ((colbuf0[0][cc] + colbuf0[1][cc]) + colbuf0[2][cc]) + colbuf0[3][cc];
            } else {
                const float v = ((colbuf[0][a][cc] + colbuf[1][a][cc]) + colbuf[2][a][cc]) + colbuf[3][a][cc];
                cp[a * stride + (int64_t)c * HK_WAVE + cc] = v;
            }
        }
#pragma unroll
        for (int a = 0; a < HK_NROW; ++a) {
            const bool used = (MODE >= HK_MODE_GRAD && (a == 1 || a == 2 || a == 6 || a == 7)) ||
                              (MODE >= HK_MODE_HESS && a != 0 && a != 5);
            if (used) two_sum_acc(hi[a], lo[a], blk[a]);
        }
    }
    double *__restrict__ rp = rowpart + (int64_t)blockIdx.x * HK_NROW * HK_TILE;
    rp[tid] = B0d;
    rp[5 * HK_TILE + tid] = X0d;
#pragma unroll
    for (int a = 0; a < HK_NROW; ++a) {
        const bool used = (MODE >= HK_MODE_GRAD && (a == 1 || a == 2 || a == 6 || a == 7)) ||
                          (MODE >= HK_MODE_HESS && a != 0 && a != 5);
        if (used) rp[a * HK_TILE + tid] = (double)hi[a] + (double)lo[a];
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

template <int MODE>
__global__ __launch_bounds__(256) void k_fin(const double *__restrict__ ts, const double *__restrict__ theta,
                                             const int *__restrict__ perm, int64_t n, int ntiles,
                                             const int *__restrict__ row_item0, const int *__restrict__ row_nseg,
                                             const double *__restrict__ rowpart, const float *__restrict__ colpart,
                                             const double *__restrict__ colpart0,
                                             const int64_t *__restrict__ colpart_off, const FinConst fc,
                                             double *__restrict__ lam, float *__restrict__ w, float *__restrict__ wlo,
                                             double *__restrict__ a_out,
                                             double *__restrict__ blockpart, int *__restrict__ status) {
    __shared__ double sh[HK_WAVES][HK_NSUM];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double s[HK_NSUM];
#pragma unroll
    for (int k = 0; k < HK_NSUM; ++k) s[k] = 0.0;
    if (i < n) {
        const int I = (int)(i / HK_TILE), r = (int)(i % HK_TILE);
        double acc[HK_NROW];
#pragma unroll
        for (int k = 0; k < HK_NROW; ++k) acc[k] = 0.0;
        const int it0 = row_item0[I], ns = row_nseg[I];
        for (int sg = 0; sg < ns; ++sg) {
            const double *rp = rowpart + (int64_t)(it0 + sg) * HK_NROW * HK_TILE + r;
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
        // background from later events: the column partials of tiles I' >= I
        for (int J = I; J < ntiles; ++J) {
            const int64_t stride = (int64_t)(J + 1) * HK_TILE;
            const float *cp = colpart + colpart_off[J] + i;
            acc[0] += colpart0[colpart_off[J] / HK_NCOL + i];
            if (MODE >= HK_MODE_GRAD) {
                acc[1] += (double)cp[stride];
                acc[2] += (double)cp[2 * stride];
            }
            if (MODE >= HK_MODE_HESS) {
                acc[3] += (double)cp[3 * stride];
                acc[4] += (double)cp[4 * stride];
            }
        }
        // moments corrected for the mean exp2 bias and, when the first moments
        // are present, for the rounding of the FP32 exponent constants
        double b0 = acc[0], x0 = acc[5];
        if (MODE >= HK_MODE_GRAD) {
            const double ln2 = 0.6931471805599453;
            b0 -= ln2 * (fc.rho_bx * acc[1] + fc.dkbt * acc[2]);
            x0 -= ln2 * (fc.dkw * acc[6] + fc.rho_ex * acc[7]);
        }
        const double B0 = b0 * fc.corr, X0 = x0 * fc.corr;
        const double lamv = fc.c_b * B0 + fc.c_e * X0;
        lam[i] = lamv;
        if (!(lamv > 0.0)) {
            atomicOr(status, isnan(lamv) ? HK_ST_NONFINITE : HK_ST_ZERO);
        }
        {
            const double wd = lamv > 0.0 ? fc.c_e / lamv : 0.0;
            const float whi = (float)wd;
            w[i] = whi;
            wlo[i] = (float)(wd - (double)whi);
        }
        s[0] = log(lamv);
        const double inv = 1.0 / lamv;
        if (MODE >= HK_MODE_GRAD) {
            const double B1 = acc[1] * fc.corr * fc.Kx, B2 = acc[2] * fc.corr;
            const double X1 = acc[6] * fc.corr, X2 = acc[7] * fc.corr * fc.Kh;
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
                const double B11 = acc[3] * fc.corr * fc.Kx * fc.Kx, B22 = acc[4] * fc.corr;
                const double X11 = acc[8] * fc.corr, X22 = acc[9] * fc.corr * fc.Kh * fc.Kh;
                double d2[6];
                d2[0] = 0.0;
                d2[1] = fc.c_b * (6.0 * B0 / (tx * tx) - 7.0 * B1 / (tx * tx * tx * tx) + B11 / pow(tx, 6));
                d2[2] = fc.c_b * (2.0 * B0 / (tt * tt) - 5.0 * B2 / (tt * tt * tt * tt) + B22 / pow(tt, 6));
                d2[3] = 0.0;
                d2[4] = fc.c_e * (X11 - 2.0 * X1 / om);
                d2[5] = fc.c_e * (6.0 * X0 / (hh * hh) - 7.0 * X2 / (hh * hh * hh * hh) + X22 / pow(hh, 6));
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
    } else if (i < (int64_t)ntiles * HK_TILE) {
        lam[i] = 1.0;
        w[i] = 0.0f;
        wlo[i] = 0.0f;
        a_out[i] = 0.0;
    }
    const int lane = threadIdx.x & (HK_WAVE - 1), wv = threadIdx.x / HK_WAVE;
#pragma unroll
    for (int k = 0; k < HK_NSUM; ++k) {
        const double v = wave_sum_f64(s[k]);
        if (lane == 0) sh[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < HK_NSUM) {
        const int k = threadIdx.x;
        blockpart[(int64_t)blockIdx.x * HK_NSUM + k] = ((sh[0][k] + sh[1][k]) + sh[2][k]) + sh[3][k];
    }
}

__global__ void k_fin2(const double *__restrict__ blockpart, int nblocks, double *__restrict__ loglik,
                       double *__restrict__ grad_hyper, double *__restrict__ negH_hyper,
                       int *__restrict__ status) {
    __shared__ double tot[HK_NSUM];
    const int k = threadIdx.x;
    if (k < HK_NSUM) {
        double sum = 0.0, c = 0.0, plain = 0.0;  // Neumaier, fixed order
        for (int b = 0; b < nblocks; ++b) {
            const double v = blockpart[(int64_t)b * HK_NSUM + k];
            const double t = sum + v;
            plain += v;
            c += fabs(sum) >= fabs(v) ? (sum - t) + v : (v - t) + sum;
            sum = t;
        }
        tot[k] = isfinite(plain) ? sum + c : plain;
    }
    __syncthreads();
    if (k == 0) {
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

// ------------------------------------------------------------------------------------
// Column pass.  Each term E_ij w_i is formed to about FP32 rounding: w_i is a
// (hi, lo) pair, times are rebased per 64-row chunk, and Eq. 4 (squared terms)
// carries two extra moments, sum (E w)^2 dt and sum (E w)^2 a_e, from which the
// FP64 finalisation removes the bias of the rounded exponent constants.
template <bool WITH_H, bool MASKED>
__device__ __forceinline__ void col_sweep(const float4 *__restrict__ rrec, const float *__restrict__ rwlo,
                                          const int *__restrict__ rg, int jcol, float tj, int xj, int yj,
                                          const PairConst kc, float &G, float &H, float &Hdt, float &Hae) {
#pragma clang fp contract(off)
#pragma unroll 16
    for (int s = 0; s < HK_WAVE; ++s) {
        const float4 r = rrec[s];
        const float dt = r.x - tj;
        const float dx = (float)(__float_as_int(r.y) - xj);
        const float dy = (float)(__float_as_int(r.z) - yj);
        const float r2 = fmaf(dx, dx, dy * dy);
        const float ae = r2 * kc.kex;
        float E = fexp2(fmaf(dt, kc.kw, ae));
        if (MASKED) {
            if (!(jcol < rg[s])) E = 0.0f;
        }
        const float ew = fmaf(E, rwlo[s], E * r.w);
        G += ew;
        if (WITH_H) {
            const float e2 = ew * ew;
            H += e2;
            Hdt = fmaf(e2, dt, Hdt);
            Hae = fmaf(e2, ae, Hae);
        }
    }
}

template <bool WITH_H>
__global__ __launch_bounds__(HK_TILE) void k_col(const double *__restrict__ ts, const int *__restrict__ xi,
                                                  const int *__restrict__ yi, const float *__restrict__ w,
                                                  const float *__restrict__ wlo, const int *__restrict__ g,
                                                  const hk_item *__restrict__ items, double *__restrict__ colG,
                                                  const PairConst kc) {
    __shared__ float4 rrec[HK_WAVE];
    __shared__ float rwlo[HK_WAVE];
    __shared__ int rg[HK_WAVE];
    const hk_item it = items[blockIdx.x];
    const int J = it.tile;
    const int tid = threadIdx.x, wv = tid / HK_WAVE;
    const int64_t col0 = (int64_t)J * HK_TILE;
    const int jcol = (int)(col0 + tid);
    const double tsj = ts[jcol];
    const int xj = xi[jcol], yj = yi[jcol];
    const int wave_first = (int)(col0 + wv * HK_WAVE);

    float Gh = 0.0f, Gl = 0.0f, Hh = 0.0f, Hl = 0.0f, Hdt = 0.0f, Hae = 0.0f;
    for (int c = it.c_begin; c < it.c_end; ++c) {
        const double Tc = ts[(int64_t)c * HK_WAVE];
        if (tid < HK_WAVE) {
            const int64_t i = (int64_t)c * HK_WAVE + tid;
            float4 r;
            r.x = (float)(ts[i] - Tc);
            r.y = __int_as_float(xi[i]);
            r.z = __int_as_float(yi[i]);
            r.w = w[i];
            rrec[tid] = r;
            rwlo[tid] = wlo[i];
            rg[tid] = g[i];
        }
        __syncthreads();
        const int gmax = rg[HK_WAVE - 1], gmin = rg[0];
        if (gmax > wave_first) {
            const float tj = (float)(tsj - Tc);
            float G = 0.0f, H = 0.0f;
            if (gmin <= wave_first + HK_WAVE - 1)
                col_sweep<WITH_H, true>(rrec, rwlo, rg, jcol, tj, xj, yj, kc, G, H, Hdt, Hae);
            else
                col_sweep<WITH_H, false>(rrec, rwlo, rg, jcol, tj, xj, yj, kc, G, H, Hdt, Hae);
            two_sum_acc(Gh, Gl, G);
            if (WITH_H) two_sum_acc(Hh, Hl, H);
        }
        __syncthreads();
    }
    double *cg = colG + (int64_t)blockIdx.x * 4 * HK_TILE;
    cg[tid] = (double)Gh + (double)Gl;
    if (WITH_H) {
        cg[HK_TILE + tid] = (double)Hh + (double)Hl;
        cg[2 * HK_TILE + tid] = (double)Hdt;
        cg[3 * HK_TILE + tid] = (double)Hae;
    }
}

__global__ void k_colfin(const int *__restrict__ perm, int64_t n, const int *__restrict__ col_item0,
                         const int *__restrict__ col_nseg, const double *__restrict__ colG,
                         const double *__restrict__ a, const FinConst fc, double *__restrict__ grad_theta,
                         double *__restrict__ negH_theta) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int J = (int)(j / HK_TILE), r = (int)(j % HK_TILE);
    const int it0 = col_item0[J], ns = col_nseg[J];
    double G = 0.0, H = 0.0, Hdt = 0.0, Hae = 0.0;
    for (int sg = 0; sg < ns; ++sg) {
        const double *cg = colG + (int64_t)(it0 + sg) * 4 * HK_TILE + r;
        G += cg[0];
        if (negH_theta) {
            H += cg[HK_TILE];
            Hdt += cg[2 * HK_TILE];
            Hae += cg[3 * HK_TILE];
        }
    }
    const int dst = perm[j];
    if (grad_theta) grad_theta[dst] = G * fc.corr - a[j];
    if (negH_theta) {
        const double ln2 = 0.6931471805599453;
        H -= 2.0 * ln2 * (fc.dkw * Hdt + fc.rho_ex * Hae);
        negH_theta[dst] = H * fc.corr * fc.corr;
    }
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
    const double two_m2k = ldexp(1.0, -2 * p->fxk);
    const double kbx = -two_m2k / (2.0 * hy->tau_x * hy->tau_x * ln2);
    const double kbt = -1.0 / (2.0 * hy->tau_t * hy->tau_t * ln2);
    const double kex = -two_m2k / (2.0 * hy->h * hy->h * ln2);
    const double kw = -hy->omega / ln2;
    kc->kbx = (float)kbx;
    kc->kbt = (float)kbt;
    kc->kex = (float)kex;
    kc->kw = (float)kw;
    fc->rho_bx = ((double)kc->kbx - kbx) / (double)kc->kbx;
    fc->dkbt = (double)kc->kbt - kbt;
    fc->dkw = (double)kc->kw - kw;
    fc->rho_ex = ((double)kc->kex - kex) / (double)kc->kex;
    const double corr = 1.0 / (1.0 + HK_EXP2_BIAS);
    const double two_pi = 6.283185307179586;
    fc->mu0 = hy->mu0; fc->tau_x = hy->tau_x; fc->tau_t = hy->tau_t;
    fc->theta0 = hy->theta0; fc->omega = hy->omega; fc->h = hy->h;
    fc->cb1 = 1.0 / (pow(two_pi, 1.5) * hy->tau_x * hy->tau_x * hy->tau_t);
    fc->ce1 = hy->omega / (two_pi * hy->h * hy->h);
    fc->c_b = fc->cb1 * hy->mu0;
    fc->c_e = fc->ce1 * hy->theta0;
    // moments are accumulated in log2 units of the exponent: r^2 = -2 s^2 ln2 * a
    // (the fixed-point scale is already inside kbx / kex)
    fc->Kx = -2.0 * hy->tau_x * hy->tau_x * ln2;
    fc->Kh = -2.0 * hy->h * hy->h * ln2;
    fc->corr = corr;
    fc->t0 = p->t0;
    fc->t1 = p->t1;
}

extern "C" hawkes_status hawkes_eval(hawkes_plan p, const hawkes_hyper *hyper, const double *d_theta,
                                     double *d_loglik, double *d_grad_theta, double *d_grad_hyper,
                                     double *d_negH_theta, double *d_negH_hyper, hipStream_t stream) {
    if (!p || !d_theta || !hk_hyper_ok(hyper)) return HAWKES_E_INVALID;
    p->last_stream = stream;
    PairConst kc;
    FinConst fc;
    hk_make_consts(p, hyper, &kc, &fc);
    // the log-likelihood alone still needs the first moments: they carry the
    // correction for the rounded FP32 exponent constants
    const int mode = d_negH_hyper ? HK_MODE_HESS : HK_MODE_GRAD;
    const int64_t npad = p->npad;

    hk_prof_mark(p, HK_PROF_EVAL, true, stream);
    hipLaunchKernelGGL(k_gather, dim3((unsigned)(npad / 256)), dim3(256), 0, stream, d_theta, p->perm, p->n, npad,
                       p->theta_s, p->status);
    hk_prof_mark(p, HK_PROF_ROW, true, stream);
#define HK_ROW(M)                                                                                              \
    hipLaunchKernelGGL(k_row<M>, dim3(p->n_row_items), dim3(HK_TILE), 0, stream, p->ts, p->xi, p->yi, p->theta_s, \
                       p->g, p->row_items, p->colpart_off, p->rowpart, p->colpart, p->colpart0, kc)
#define HK_FIN(M)                                                                                              \
    hipLaunchKernelGGL(k_fin<M>, dim3(p->nfin_blocks), dim3(256), 0, stream, p->ts, d_theta, p->perm, p->n,      \
                       p->ntiles, p->row_item0, p->row_nseg, p->rowpart, p->colpart, p->colpart0, p->colpart_off, fc, \
                       p->lam, p->w, p->wlo, p->a, p->blockpart, p->status)
    if (mode == HK_MODE_GRAD) HK_ROW(HK_MODE_GRAD);
    else HK_ROW(HK_MODE_HESS);
    hk_prof_mark(p, HK_PROF_ROW, false, stream);
    if (mode == HK_MODE_GRAD) HK_FIN(HK_MODE_GRAD);
    else HK_FIN(HK_MODE_HESS);
#undef HK_ROW
#undef HK_FIN
    hipLaunchKernelGGL(k_fin2, dim3(1), dim3(64), 0, stream, p->blockpart, p->nfin_blocks, d_loglik, d_grad_hyper,
                       d_negH_hyper, p->status);
    if (d_grad_theta || d_negH_theta) {
        hk_prof_mark(p, HK_PROF_COL, true, stream);
        if (d_negH_theta)
            hipLaunchKernelGGL(k_col<true>, dim3(p->n_col_items), dim3(HK_TILE), 0, stream, p->ts, p->xi, p->yi,
                               p->w, p->wlo, p->g, p->col_items, p->colG, kc);
        else
            hipLaunchKernelGGL(k_col<false>, dim3(p->n_col_items), dim3(HK_TILE), 0, stream, p->ts, p->xi, p->yi,
                               p->w, p->wlo, p->g, p->col_items, p->colG, kc);
        hk_prof_mark(p, HK_PROF_COL, false, stream);
        hipLaunchKernelGGL(k_colfin, dim3((unsigned)((p->n + 255) / 256)), dim3(256), 0, stream, p->perm, p->n,
                           p->col_item0, p->col_nseg, p->colG, p->a, fc, d_grad_theta, d_negH_theta);
    }
    hk_prof_mark(p, HK_PROF_EVAL, false, stream);
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}

void hk_launch_row_loglik(hawkes_plan p, const PairConst &kc, hipStream_t stream) {
    hipLaunchKernelGGL(k_row<HK_MODE_GRAD>, dim3(p->n_row_items), dim3(HK_TILE), 0, stream, p->ts, p->xi, p->yi,
                       p->theta_s, p->g, p->row_items, p->colpart_off, p->rowpart, p->colpart, p->colpart0, kc);
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
