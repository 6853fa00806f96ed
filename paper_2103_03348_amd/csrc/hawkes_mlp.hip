// Learned preconditioner: per-event grid-count features, a 12 -> 64 -> 64 -> 1
// tanh network (forward, back-propagation, Adam) and the running-average mass
// update that consumes either its prediction or the exact Hessian diagonal.
//
// The network predicts, from cheap features of free event m, log H_m: the log
// of Eq. 5's Hessian diagonal, which the paper uses as the HMC mass.  The mass
// formed from it is theta_m^2 exp(prediction) + P_mm (the prior's precision
// added when the mass is formed).  The exact column pass remains the training
// target, the periodic fallback and the judge, so the sampler stays exact: any
// positive mass leaves the target distribution invariant.
//
// hawkes_mlp_train_step_noalloc is the training step for callers that cannot
// allocate: its workspace and gradient live in a fixed device array of this
// file (one copy per GPU, held until the process ends).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <mutex>

#include "hawkes_internal.h"

#define MLP_IN 12
#define MLP_H 64
#define MLP_OFF_W1 0
#define MLP_OFF_B1 (MLP_OFF_W1 + MLP_H * MLP_IN)
#define MLP_OFF_W2 (MLP_OFF_B1 + MLP_H)
#define MLP_OFF_B2 (MLP_OFF_W2 + MLP_H * MLP_H)
#define MLP_OFF_W3 (MLP_OFF_B2 + MLP_H)
#define MLP_OFF_B3 (MLP_OFF_W3 + MLP_H)
#define MLP_NP (MLP_OFF_B3 + 1)

static_assert(MLP_NP == 5057, "parameter count");

namespace {

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// ---- network -----------------------------------------------------------------------------
// One thread per sample; parameters staged in LDS.  Activations h1, h2 are kept
// for back-propagation when the pointers are non-NULL.
// A batch row index outside [0, n_rows) is not read: the sample is dropped
// (zero input, zero target weight) and bit 1 of *err is set.
__device__ __forceinline__ int64_t checked_row(const int *rows, int64_t s, int64_t n_rows, int *err, bool &ok) {
    const int64_t row = rows ? (int64_t)rows[s] : s;
    ok = row >= 0 && row < n_rows;
    if (!ok && err) atomicOr(err, 1);
    return ok ? row : 0;
}

__global__ __launch_bounds__(256) void k_mlp_fwd(const float *__restrict__ params, const float *__restrict__ X,
                                                 int64_t n_rows, const int *__restrict__ rows, int64_t B,
                                                 float *__restrict__ y, float *__restrict__ h1o,
                                                 float *__restrict__ h2o, int *__restrict__ err) {
    __shared__ float P[MLP_NP];
    for (int q = threadIdx.x; q < MLP_NP; q += blockDim.x) P[q] = params[q];
    __syncthreads();
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= B) return;
    bool ok;
    const int64_t row = checked_row(rows, s, n_rows, err, ok);
    float x[MLP_IN];
#pragma unroll
    for (int j = 0; j < MLP_IN; ++j) x[j] = ok ? X[row * MLP_IN + j] : 0.0f;
    float h1[MLP_H];
#pragma unroll 4
    for (int k = 0; k < MLP_H; ++k) {
        float a = P[MLP_OFF_B1 + k];
#pragma unroll
        for (int j = 0; j < MLP_IN; ++j) a = fmaf(P[MLP_OFF_W1 + k * MLP_IN + j], x[j], a);
        h1[k] = tanhf(a);
    }
    float out = P[MLP_OFF_B3];
    for (int k = 0; k < MLP_H; ++k) {
        float a = P[MLP_OFF_B2 + k];
#pragma unroll
        for (int j = 0; j < MLP_H; ++j) a = fmaf(P[MLP_OFF_W2 + k * MLP_H + j], h1[j], a);
        const float h2 = tanhf(a);
        if (h2o) h2o[s * MLP_H + k] = h2;
        out = fmaf(P[MLP_OFF_W3 + k], h2, out);
    }
    if (h1o)
#pragma unroll
        for (int k = 0; k < MLP_H; ++k) h1o[s * MLP_H + k] = h1[k];
    y[s] = out;
}

// Per-sample back-propagation: dy = 2 (y - t) / B, d2 = dy w3 (1 - h2^2),
// d1 = (W2^T d2) (1 - h1^2); block partial sums of the squared residuals.
__global__ __launch_bounds__(256) void k_mlp_bwd(const float *__restrict__ params, const float *__restrict__ y,
                                                 const float *__restrict__ target, int64_t n_rows,
                                                 const int *__restrict__ rows, int64_t B,
                                                 const float *__restrict__ h1, const float *__restrict__ h2,
                                                 float *__restrict__ d1o, float *__restrict__ d2o,
                                                 float *__restrict__ dyo, double *__restrict__ loss_part) {
    __shared__ float P[MLP_H * MLP_H + MLP_H];
    __shared__ double red[256];
    for (int q = threadIdx.x; q < MLP_H * MLP_H; q += blockDim.x) P[q] = params[MLP_OFF_W2 + q];
    for (int q = threadIdx.x; q < MLP_H; q += blockDim.x) P[MLP_H * MLP_H + q] = params[MLP_OFF_W3 + q];
    __syncthreads();
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double r2 = 0.0;
    if (s < B) {
        bool ok;
        const int64_t row = checked_row(rows, s, n_rows, nullptr, ok);
        const float r = ok ? y[s] - target[row] : 0.0f;
        r2 = (double)r * (double)r;
        const float dy = 2.0f * r / (float)B;
        dyo[s] = dy;
        float d2[MLP_H];
#pragma unroll
        for (int k = 0; k < MLP_H; ++k) {
            const float hk = h2[s * MLP_H + k];
            d2[k] = dy * P[MLP_H * MLP_H + k] * (1.0f - hk * hk);
            d2o[s * MLP_H + k] = d2[k];
        }
        for (int j = 0; j < MLP_H; ++j) {
            float a = 0.0f;
#pragma unroll
            for (int k = 0; k < MLP_H; ++k) a = fmaf(P[k * MLP_H + j], d2[k], a);
            const float hj = h1[s * MLP_H + j];
            d1o[s * MLP_H + j] = a * (1.0f - hj * hj);
        }
    }
    red[threadIdx.x] = r2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// One wavefront per parameter: lane l sums the gradient terms of samples
// l, l + 64, ... in FP64, then a fixed butterfly of shuffles adds the 64 lane
// sums, so the result does not depend on timing.
__global__ __launch_bounds__(256) void k_mlp_wgrad(const float *__restrict__ X, int64_t n_rows,
                                                   const int *__restrict__ rows, int64_t B,
                                                   const float *__restrict__ h1,
                                                   const float *__restrict__ h2, const float *__restrict__ d1,
                                                   const float *__restrict__ d2, const float *__restrict__ dy,
                                                   double *__restrict__ grad) {
    const int lane = threadIdx.x & 63;
    const int q = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    if (q >= MLP_NP) return;
    double acc = 0.0;
    if (q < MLP_OFF_B1) {
        const int k = q / MLP_IN, j = q % MLP_IN;
        for (int64_t s = lane; s < B; s += 64) {
            bool ok;
            const int64_t row = checked_row(rows, s, n_rows, nullptr, ok);
            if (ok) acc += (double)d1[s * MLP_H + k] * (double)X[row * MLP_IN + j];
        }
    } else if (q < MLP_OFF_W2) {
        const int k = q - MLP_OFF_B1;
        for (int64_t s = lane; s < B; s += 64) acc += (double)d1[s * MLP_H + k];
    } else if (q < MLP_OFF_B2) {
        const int k = (q - MLP_OFF_W2) / MLP_H, j = (q - MLP_OFF_W2) % MLP_H;
        for (int64_t s = lane; s < B; s += 64) acc += (double)d2[s * MLP_H + k] * (double)h1[s * MLP_H + j];
    } else if (q < MLP_OFF_W3) {
        const int k = q - MLP_OFF_B2;
        for (int64_t s = lane; s < B; s += 64) acc += (double)d2[s * MLP_H + k];
    } else if (q < MLP_OFF_B3) {
        const int k = q - MLP_OFF_W3;
        for (int64_t s = lane; s < B; s += 64) acc += (double)dy[s] * (double)h2[s * MLP_H + k];
    } else {
        for (int64_t s = lane; s < B; s += 64) acc += (double)dy[s];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) grad[q] = acc;
}

__global__ void k_mlp_loss(const double *__restrict__ part, int nb, int64_t B, double *__restrict__ loss) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[b];
        loss[0] = s / (double)B;
    }
}

// Adam (Kingma & Ba 2015) with bias correction; step t >= 1.
__global__ void k_adam(float *__restrict__ params, const double *__restrict__ grad, float *__restrict__ m,
                       float *__restrict__ v, int t, float lr, float b1, float b2, float eps) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= MLP_NP) return;
    const float g = (float)grad[q];
    const float mq = b1 * m[q] + (1.0f - b1) * g;
    const float vq = b2 * v[q] + (1.0f - b2) * g * g;
    m[q] = mq;
    v[q] = vq;
    const float mh = mq / (1.0f - powf(b1, (float)t));
    const float vh = vq / (1.0f - powf(b2, (float)t));
    params[q] -= lr * mh / (sqrtf(vh) + eps);
}

// ---- features -------------------------------------------------------------------------------
// Disc and time-window counts around each free event, exact by their
// definition: a spatial grid of cells of size 3h over all events (counting
// sort: per-cell counts, one exclusive scan, a scatter of the events' times
// and coordinates into cell order) gives each free event the candidates in the
// cells that a disc of radius 3h (the largest radius) around it touches;
// the candidates are then tested exactly.  Distances are dx * dx + dy * dy and
// radii r * r, each rounded once in FP64 (no contraction), so every count is
// the same integer as the definition's.
struct FeatGrid {
    double gx0, gy0, s;  // origin and cell size 3h
    int nx, ny;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

__device__ __forceinline__ int cell_x(double x, const FeatGrid &G) {
    return clampi((int)floor((x - G.gx0) / G.s), 0, G.nx - 1);
}
__device__ __forceinline__ int cell_y(double y, const FeatGrid &G) {
    return clampi((int)floor((y - G.gy0) / G.s), 0, G.ny - 1);
}

__global__ void k_fill_zero(int *__restrict__ a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0;
}

__global__ void k_cell_count(const double *__restrict__ xy, int64_t n, const FeatGrid G, int *__restrict__ cnt) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n) return;
    atomicAdd(&cnt[(int64_t)cell_y(xy[2 * e + 1], G) * G.nx + cell_x(xy[2 * e], G)], 1);
}

// Exclusive scan of the cell counts by one block: each thread scans a
// contiguous segment, the segment totals are scanned in LDS, then each thread
// writes its segment's offsets.  start[cells] = n.  fill is cleared for the
// scatter.
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void k_cell_scan(const int *__restrict__ cnt, int64_t cells,
                                                           int *__restrict__ start, int *__restrict__ fill) {
    __shared__ int tot[kScanThreads];
    const int64_t seg = (cells + kScanThreads - 1) / kScanThreads;
    const int64_t lo = min(cells, threadIdx.x * seg), hi = min(cells, lo + seg);
    int sum = 0;
    for (int64_t c = lo; c < hi; ++c) sum += cnt[c];
    tot[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int k = 0; k < kScanThreads; ++k) {
            const int v = tot[k];
            tot[k] = run;
            run += v;
        }
        start[cells] = run;
    }
    __syncthreads();
    int run = tot[threadIdx.x];
    for (int64_t c = lo; c < hi; ++c) {
        start[c] = run;
        run += cnt[c];
        fill[c] = 0;
    }
}

// Events into cell order (the order inside a cell does not matter for counts).
__global__ void k_cell_scatter(const double *__restrict__ t, const double *__restrict__ xy, int64_t n,
                               const FeatGrid G, const int *__restrict__ start, int *__restrict__ fill,
                               double *__restrict__ ct, double *__restrict__ cx, double *__restrict__ cy) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n) return;
    const double x = xy[2 * e], y = xy[2 * e + 1];
    const int64_t c = (int64_t)cell_y(y, G) * G.nx + cell_x(x, G);
    const int64_t q = start[c] + atomicAdd(&fill[c], 1);
    ct[q] = t[e];
    cx[q] = x;
    cy[q] = y;
}

// One wavefront per free event: the lanes split the candidates of the cells a
// disc of radius 3h touches, count, and the counts are summed across the
// wavefront (integers: exact in any order).
//
// Feature 8 is the forward sum of the squared excitation kernel,
//   S_m = sum over e with r2_e < (3h)^2, 0 < dt_e <= 6/omega of
//         exp(a_e),  a_e = -2 omega dt_e - r2_e / h^2,
// which is Eq. 5's H_m without the weights c_e / lambda_e: as
// max(log2 S_m, HK_KSUM_LOG2_FLOOR) / 8.  The candidates' order in the cells
// depends on the grid's scatter, so the sum is formed in a way that does not
// depend on it: the largest exponent a_max (a maximum is exact) and then
// sum_e rint(2^36 exp(a_e - a_max)) in 64-bit integers (exact up to 2^27
// terms), each exponential by the FP32 exp2 (a feature needs no more).
__global__ __launch_bounds__(256) void k_features(const double *__restrict__ t, const double *__restrict__ xy,
                                                  const int64_t *__restrict__ cidx, const int *__restrict__ pos,
                                                  const int *__restrict__ slot, const int *__restrict__ g,
                                                  const double *__restrict__ z, int64_t m, int64_t n, double t0,
                                                  double t1, double h, double tau_x, double omega, const FeatGrid G,
                                                  const int *__restrict__ start, const double *__restrict__ ct,
                                                  const double *__restrict__ cx, const double *__restrict__ cy,
                                                  float *__restrict__ feat) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & (HK_WAVE - 1);
    const int64_t r = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / HK_WAVE;
    if (r >= m) return;  // whole wavefronts leave together
    const int k = slot[r];
    const int64_t e = cidx[k];
    const double xm = xy[2 * e], ym = xy[2 * e + 1], tm = t[e];
    const double r0 = h * h, h3 = 3.0 * h, r1 = h3 * h3;
    const double w1 = 1.0 / omega, w3 = 3.0 / omega, w6 = 6.0 / omega;
    const double inv_h2 = 1.0 / (h * h);
    const int x_lo = cell_x(xm - h3, G), x_hi = cell_x(xm + h3, G);
    const int y_lo = cell_y(ym - h3, G), y_hi = cell_y(ym + h3, G);
    int c[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double amax = -INFINITY;  // largest exponent of feature 8's terms
    for (int yy = y_lo; yy <= y_hi; ++yy) {
        const int64_t row = (int64_t)yy * G.nx;
        for (int q = start[row + x_lo] + lane; q < start[row + x_hi + 1]; q += HK_WAVE) {
            const double dx = cx[q] - xm, dy = cy[q] - ym;
            const double d2 = dx * dx + dy * dy;
            const double dt = ct[q] - tm;
            const bool prev = dt >= -w1 && dt < 0.0, next = dt > 0.0 && dt <= w1, next3 = dt > 0.0 && dt <= w3;
            if (d2 < r1) {
                c[1] += 1;
                c[6] += prev;
                c[7] += next;
                if (dt > 0.0 && dt <= w6) {
                    c[2] += 1;
                    amax = fmax(amax, -2.0 * omega * dt - d2 * inv_h2);
                }
                if (d2 < r0) {
                    c[0] += 1;
                    c[3] += prev;
                    c[4] += next;
                    c[5] += next3;
                }
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
#pragma unroll
        for (int off = 1; off < HK_WAVE; off <<= 1) c[a] += __shfl_xor(c[a], off);
    }
#pragma unroll
    for (int off = 1; off < HK_WAVE; off <<= 1) amax = fmax(amax, __shfl_xor(amax, off));
    // feature 8's terms relative to the largest, in fixed point (2^36 units)
    long long ksum = 0;
    if (amax > -INFINITY) {
        for (int yy = y_lo; yy <= y_hi; ++yy) {
            const int64_t row = (int64_t)yy * G.nx;
            for (int q = start[row + x_lo] + lane; q < start[row + x_hi + 1]; q += HK_WAVE) {
                const double dx = cx[q] - xm, dy = cy[q] - ym;
                const double d2 = dx * dx + dy * dy;
                const double dt = ct[q] - tm;
                if (d2 < r1 && dt > 0.0 && dt <= w6) {
                    const double rel = (-2.0 * omega * dt - d2 * inv_h2) - amax;  // <= 0
                    ksum += llrint((double)exp2f((float)(rel * 1.4426950408889634)) * 68719476736.0);
                }
            }
        }
#pragma unroll
        for (int off = 1; off < HK_WAVE; off <<= 1) ksum += __shfl_xor(ksum, off);
    }
    if (lane == 0) {
        float f[MLP_IN];
        // the event itself is inside every disc
        for (int a = 0; a < 2; ++a) f[a] = (float)log1p((double)(c[a] - 1));
        f[2] = (float)log1p((double)c[2]);
        for (int a = 3; a < 8; ++a) f[a] = (float)log1p((double)c[a]);
        // log2 S_m = log2(ksum) - 36 + a_max / ln 2 (S_m = 0: the floor)
        const double l2s = ksum > 0 ? log2((double)ksum) - 36.0 + amax * 1.4426950408889634 : -INFINITY;
        f[8] = (float)(fmax(l2s, HK_KSUM_LOG2_FLOOR) * 0.125);
        f[9] = (float)z[k];
        f[10] = (float)((double)g[pos[r]] / (double)n);
        const double span = t1 - t0;
        f[11] = (float)(span > 0.0 ? (t1 - tm) / span : 0.0);
        for (int j = 0; j < MLP_IN; ++j) feat[(int64_t)k * MLP_IN + j] = f[j];
    }
}

// ---- curvature and mass update ---------------------------------------------------------
// In z (theta_k = exp(z_k + beta t_k), so d theta_k / d z_k = theta_k) the
// log-posterior's curvature on the diagonal is
//   c_k = theta_k^2 H_k - theta_k g_k + P_kk
// with g, H Eq. 4 and Eq. 5 on the subset and P the prior's precision
// diagonal: 1/sigma^2 (iid prior) or (V^{-1})_kk / sigma^2 (Eq. 2).
__device__ __forceinline__ double prior_prec(const double *__restrict__ pdiag, int k, double inv_s2) {
    return pdiag ? pdiag[k] * inv_s2 : inv_s2;
}

// The exact curvature c_k (slot order, FP64) and log max(H_k, HK_LOGH_FLOOR)
// (FP32, the learned preconditioner's target), either output may be NULL.
__global__ void k_curvature(const int *__restrict__ slot, int64_t m, const double *__restrict__ gsub,
                            const double *__restrict__ hsub, const double *__restrict__ theta,
                            const int64_t *__restrict__ cidx, const double *__restrict__ pdiag, double inv_s2,
                            double *__restrict__ curv, float *__restrict__ log_h) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= m) return;
    const int k = slot[r];
    const double th = theta[cidx[k]];
    if (curv) curv[k] = th * th * hsub[r] - th * gsub[r] + prior_prec(pdiag, k, inv_s2);
    if (log_h) log_h[k] = (float)log(fmax(hsub[r], HK_LOGH_FLOOR));
}

// mass <- (count mass + e_k) / (count + 1) with the estimate
//   exact:   e_k = max(theta^2 H - theta g, 0) + P_kk
//   learned: e_k = theta^2 exp(pred_k) + P_kk   (pred: the network's log H_k)
__global__ void k_mass_update(const int *__restrict__ slot, int64_t m, const double *__restrict__ gsub,
                              const double *__restrict__ hsub, const float *__restrict__ pred,
                              const double *__restrict__ theta, const int64_t *__restrict__ cidx,
                              const double *__restrict__ pdiag, double inv_s2, double count,
                              double *__restrict__ mass) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= m) return;
    const int k = slot[r];
    const double th = theta[cidx[k]];
    const double prec = prior_prec(pdiag, k, inv_s2);
    double est;
    if (pred) est = th * th * exp((double)pred[k]) + prec;
    else est = fmax(th * th * hsub[r] - th * gsub[r], 0.0) + prec;
    mass[k] = (count * mass[k] + est) / (count + 1.0);
}

}  // namespace

extern "C" int64_t hawkes_mlp_num_params(void) { return MLP_NP; }

extern "C" int64_t hawkes_mlp_workspace_floats(int64_t B) {
    // h1, h2, d1, d2 [B][64], y, dy [B], gradient (FP64, 2 floats each), loss partials (FP64)
    return 4 * B * MLP_H + 2 * B + 2 * (int64_t)MLP_NP + 2 * (int64_t)nblk(B, 256) + 2 + 64;
}

extern "C" hawkes_status hawkes_mlp_forward(const float *d_params, const float *d_x, int64_t B, float *d_y,
                                            hipStream_t stream) {
    if (!d_params || !d_x || !d_y || B < 1) return HAWKES_E_INVALID;
    hipLaunchKernelGGL(k_mlp_fwd, dim3(nblk(B, 256)), dim3(256), 0, stream, d_params, d_x, B, (const int *)nullptr,
                       B, d_y, (float *)nullptr, (float *)nullptr, (int *)nullptr);
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}

static void mlp_grad_launch(const float *d_params, const float *d_x, int64_t n_rows, const int *d_rows,
                            const float *d_target, int64_t B, float *d_work, double *d_grad, double *d_loss,
                            int *d_err, hipStream_t stream) {
    float *h1 = d_work, *h2 = h1 + B * MLP_H, *d1 = h2 + B * MLP_H, *d2 = d1 + B * MLP_H;
    float *y = d2 + B * MLP_H, *dy = y + B;
    // FP64 scratch after the FP32 arrays, 8-byte aligned
    uintptr_t up = (uintptr_t)(dy + B);
    up = (up + 7) & ~(uintptr_t)7;
    double *lpart = (double *)up;
    const unsigned nb = nblk(B, 256);
    hipLaunchKernelGGL(k_mlp_fwd, dim3(nb), dim3(256), 0, stream, d_params, d_x, n_rows, d_rows, B, y, h1, h2,
                       d_err);
    hipLaunchKernelGGL(k_mlp_bwd, dim3(nb), dim3(256), 0, stream, d_params, y, d_target, n_rows, d_rows, B, h1, h2,
                       d1, d2, dy, lpart);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(nblk((int64_t)MLP_NP * 64, 256)), dim3(256), 0, stream, d_x, n_rows, d_rows,
                       B, h1, h2, d1, d2, dy, d_grad);
    if (d_loss) hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(64), 0, stream, lpart, (int)nb, B, d_loss);
}

extern "C" hawkes_status hawkes_mlp_grad(const float *d_params, const float *d_x, int64_t n_rows,
                                         const int *d_rows, const float *d_target, int64_t B, float *d_work,
                                         double *d_grad, double *d_loss, int *d_err, hipStream_t stream) {
    if (!d_params || !d_x || !d_target || !d_work || !d_grad || B < 1 || n_rows < 1) return HAWKES_E_INVALID;
    if (!d_rows && B > n_rows) return HAWKES_E_INVALID;
    mlp_grad_launch(d_params, d_x, n_rows, d_rows, d_target, B, d_work, d_grad, d_loss, d_err, stream);
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}

// ---- allocation-free training step ---------------------------------------------------------
// The FP32 workspace of mlp_grad_launch for a batch of at most
// HK_NOALLOC_MLP_MAX_B samples (h1, h2, d1, d2, y, dy, the loss partials),
// then, 256-byte aligned, the FP64 gradient.  Every kernel of the step writes
// the parts it reads before reading them, so nothing needs clearing between
// calls.
constexpr int64_t kNoallocWorkFloats =
    ((4 * (int64_t)HK_NOALLOC_MLP_MAX_B * MLP_H + 2 * (int64_t)HK_NOALLOC_MLP_MAX_B + 2 +
      2 * (int64_t)((HK_NOALLOC_MLP_MAX_B + 255) / 256) + 63) / 64) * 64;
constexpr int64_t kNoallocFloats = kNoallocWorkFloats + 2 * (int64_t)MLP_NP;
static __device__ __align__(256) float scratch[kNoallocFloats];

// Device address of `scratch` on the current device, looked up once per device
// (each GPU holds its own copy of the array at its own address).  In host code
// the array's name is only a host-side stand-in, never a device address.
static constexpr int kNoallocMaxDevices = 64;

static hawkes_status noalloc_scratch(float **out) {
    static std::mutex mu;
    static float *ptr[kNoallocMaxDevices] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoallocMaxDevices) return HAWKES_E_DEVICE;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HAWKES_E_DEVICE;
        ptr[dev] = (float *)p;
    }
    *out = ptr[dev];
    return HAWKES_OK;
}

extern "C" int64_t hawkes_mlp_noalloc_max_batch(void) { return HK_NOALLOC_MLP_MAX_B; }

extern "C" hawkes_status hawkes_mlp_train_step_noalloc(float *d_params, float *d_adam_m, float *d_adam_v, int step,
                                                       float lr, const float *d_x, int64_t n_rows,
                                                       const int *d_rows, const float *d_target, int64_t B,
                                                       double *d_loss, int *d_err, hipStream_t stream) {
    if (!d_params || !d_adam_m || !d_adam_v || step < 1 || !d_x || !d_target || B < 1 || n_rows < 1)
        return HAWKES_E_INVALID;
    if (!d_rows && B > n_rows) return HAWKES_E_INVALID;
    if (B > HK_NOALLOC_MLP_MAX_B) return HAWKES_E_CAPACITY;
    float *work = nullptr;
    const hawkes_status st = noalloc_scratch(&work);
    if (st != HAWKES_OK) return st;
    double *grad = (double *)(work + kNoallocWorkFloats);
    mlp_grad_launch(d_params, d_x, n_rows, d_rows, d_target, B, work, grad, d_loss, d_err, stream);
    hipLaunchKernelGGL(k_adam, dim3(nblk(MLP_NP, 256)), dim3(256), 0, stream, d_params, (const double *)grad,
                       d_adam_m, d_adam_v, step, lr, 0.9f, 0.999f, 1e-8f);
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}

extern "C" hawkes_status hawkes_mlp_train_step(float *d_params, float *d_adam_m, float *d_adam_v, int step,
                                               float lr, const float *d_x, int64_t n_rows, const int *d_rows,
                                               const float *d_target, int64_t B, float *d_work, double *d_grad,
                                               double *d_loss, int *d_err, hipStream_t stream) {
    if (!d_params || !d_adam_m || !d_adam_v || step < 1 || !d_x || !d_target || !d_work || !d_grad || B < 1 ||
        n_rows < 1)
        return HAWKES_E_INVALID;
    if (!d_rows && B > n_rows) return HAWKES_E_INVALID;
    mlp_grad_launch(d_params, d_x, n_rows, d_rows, d_target, B, d_work, d_grad, d_loss, d_err, stream);
    hipLaunchKernelGGL(k_adam, dim3(nblk(MLP_NP, 256)), dim3(256), 0, stream, d_params, d_grad, d_adam_m, d_adam_v,
                       step, lr, 0.9f, 0.999f, 1e-8f);
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}

extern "C" hawkes_status hawkes_features(hawkes_plan p, const hawkes_hyper *hy, const double *d_t,
                                         const double *d_xy, const double *d_z, double gx0, double gy0,
                                         float *d_feat, hipStream_t stream) {
    if (!p || !hk_hyper_ok(hy) || !d_t || !d_xy || !d_z || !d_feat) return HAWKES_E_INVALID;
    if (!p->sub) return HAWKES_E_UNSUPPORTED;
    if (!(gx0 <= p->xmin) || !(gy0 <= p->ymin)) return HAWKES_E_INVALID;
    FeatGrid G;
    G.gx0 = gx0;
    G.gy0 = gy0;
    G.s = 3.0 * hy->h;
    const double nx = floor((p->xmax - gx0) / G.s) + 1.0, ny = floor((p->ymax - gy0) / G.s) + 1.0;
    if (!(nx * ny < (double)(1 << 26))) return HAWKES_E_UNSUPPORTED;
    G.nx = (int)nx;
    G.ny = (int)ny;
    const int64_t cells = (int64_t)G.nx * G.ny, n = p->n;
    // int workspace: counts [cells], starts [cells + 1], fill [cells]; then
    // (8-byte aligned) the events' times and coordinates in cell order [3 n]
    const int64_t ints = ((3 * cells + 1 + 1) / 2) * 2;
    hawkes_status st = hk_subset_grid(p, ints + 6 * n, stream);
    if (st != HAWKES_OK) return st;
    int *cnt = hk_subset_grid_ptr(p), *start = cnt + cells, *fill = start + cells + 1;
    double *ct = (double *)(cnt + ints), *cxs = ct + n, *cys = cxs + n;
    hipLaunchKernelGGL(k_fill_zero, dim3(std::min<int64_t>(nblk(cells, 256), 4096)), dim3(256), 0, stream, cnt,
                       cells);
    hipLaunchKernelGGL(k_cell_count, dim3(nblk(n, 256)), dim3(256), 0, stream, d_xy, n, G, cnt);
    hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(kScanThreads), 0, stream, cnt, cells, start, fill);
    hipLaunchKernelGGL(k_cell_scatter, dim3(nblk(n, 256)), dim3(256), 0, stream, d_t, d_xy, n, G, start, fill, ct,
                       cxs, cys);
    int64_t m;
    const int64_t *cidx;
    const int *pos, *slot;
    hk_subset_view(p, &m, &cidx, &pos, &slot);
    hipLaunchKernelGGL(k_features, dim3(nblk(m * HK_WAVE, 256)), dim3(256), 0, stream, d_t, d_xy, cidx, pos, slot,
                       p->g, d_z, m, n, p->t0, p->t1, hy->h, hy->tau_x, hy->omega, G, start, ct, cxs, cys, d_feat);
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}

// The prior's precision diagonal for prior = 0 (iid: NULL, 1/sigma^2) or 1 (the
// plan's tree); false when the prior is unknown or its tree is not set.
static bool prior_diag(hawkes_plan p, int prior, int64_t m, const double **pdiag) {
    *pdiag = nullptr;
    if (prior == 0) return true;
    if (prior != 1 || hk_tree_tips(p) != m) return false;
    *pdiag = hk_tree_precision_diag(p);
    return *pdiag != nullptr;
}

extern "C" hawkes_status hawkes_mass_update(hawkes_plan p, const hawkes_hyper *hy, const double *d_theta,
                                            const float *d_pred, double sigma_z, int prior, int64_t count,
                                            double *d_mass, hipStream_t stream) {
    if (!p || !hk_hyper_ok(hy) || !d_theta || !d_mass || !(sigma_z > 0.0) || count < 0) return HAWKES_E_INVALID;
    if (!p->sub) return HAWKES_E_UNSUPPORTED;
    int64_t m;
    const int64_t *cidx;
    const int *pos, *slot;
    hk_subset_view(p, &m, &cidx, &pos, &slot);
    const double *pdiag;
    if (!prior_diag(p, prior, m, &pdiag)) return prior == 1 ? HAWKES_E_UNSUPPORTED : HAWKES_E_INVALID;
    const double *gsub = nullptr, *hsub = nullptr;
    if (!d_pred) {
        hawkes_status st = hk_subset_exact(p, hy, d_theta, stream, &gsub, &hsub);
        if (st != HAWKES_OK) return st;
    }
    hipLaunchKernelGGL(k_mass_update, dim3(nblk(m, 256)), dim3(256), 0, stream, slot, m, gsub, hsub, d_pred, d_theta,
                       cidx, pdiag, 1.0 / (sigma_z * sigma_z), (double)count, d_mass);
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}

extern "C" hawkes_status hawkes_subset_curvature(hawkes_plan p, const hawkes_hyper *hy, const double *d_theta,
                                                 double sigma_z, int prior, double *d_curv, float *d_log_h,
                                                 hipStream_t stream) {
    if (!p || !hk_hyper_ok(hy) || !d_theta || !(sigma_z > 0.0) || (!d_curv && !d_log_h)) return HAWKES_E_INVALID;
    if (!p->sub) return HAWKES_E_UNSUPPORTED;
    int64_t m;
    const int64_t *cidx;
    const int *pos, *slot;
    hk_subset_view(p, &m, &cidx, &pos, &slot);
    const double *pdiag;
    if (!prior_diag(p, prior, m, &pdiag)) return prior == 1 ? HAWKES_E_UNSUPPORTED : HAWKES_E_INVALID;
    const double *gsub = nullptr, *hsub = nullptr;
    hawkes_status st = hk_subset_exact(p, hy, d_theta, stream, &gsub, &hsub);
    if (st != HAWKES_OK) return st;
    hipLaunchKernelGGL(k_curvature, dim3(nblk(m, 256)), dim3(256), 0, stream, slot, m, gsub, hsub, d_theta, cidx,
                       pdiag, 1.0 / (sigma_z * sigma_z), d_curv, d_log_h);
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}
