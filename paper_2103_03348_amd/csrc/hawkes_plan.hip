// Plan construction: stable time sort on the device, centred FP64 locations,
// tie groups, and the tile schedules of the two pair passes.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <algorithm>
#include <vector>

#include "hawkes_internal.h"

namespace {

// ---- input checks and bounding box -------------------------------------------------
// Block-wise min/max of t, x, y and a non-finite flag; one block finishes it.
__global__ void k_bbox(const double *__restrict__ t, const double *__restrict__ xy, int64_t n,
                       double *__restrict__ part /* [blocks][7] */) {
    __shared__ double sh[7][256];
    double v[7] = {INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY, 0.0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double tt = t[i], x = xy[2 * i], y = xy[2 * i + 1];
        if (!isfinite(tt) || !isfinite(x) || !isfinite(y)) v[6] = 1.0;
        v[0] = fmin(v[0], tt); v[1] = fmax(v[1], tt);
        v[2] = fmin(v[2], x);  v[3] = fmax(v[3], x);
        v[4] = fmin(v[4], y);  v[5] = fmax(v[5], y);
    }
    for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            for (int k = 0; k < 7; ++k) {
                double a = sh[k][threadIdx.x], b = sh[k][threadIdx.x + s];
                sh[k][threadIdx.x] = (k == 6) ? fmax(a, b) : ((k & 1) ? fmax(a, b) : fmin(a, b));
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 7) part[blockIdx.x * 7 + threadIdx.x] = sh[threadIdx.x][0];
}

// ---- stable sort: bitonic network on (time, caller index) pairs -----------------------
// Ordering by (time, index) lexicographically makes the result stable and unique.
__global__ void k_sort_init(const double *__restrict__ t, int64_t n, int64_t n2,
                            double *__restrict__ key, int *__restrict__ idx) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n2) return;
    key[i] = i < n ? t[i] : INFINITY;
    idx[i] = (int)i;
}

__device__ __forceinline__ bool pair_less(double ka, int ia, double kb, int ib) {
    return ka < kb || (ka == kb && ia < ib);
}

__global__ void k_bitonic_step(double *__restrict__ key, int *__restrict__ idx, int64_t n2,
                               int64_t k, int64_t j) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n2) return;
    int64_t p = i ^ j;
    if (p <= i) return;
    bool up = (i & k) == 0;
    double ki = key[i], kp = key[p];
    int ii = idx[i], ip = idx[p];
    bool swap = up ? pair_less(kp, ip, ki, ii) : pair_less(ki, ii, kp, ip);
    if (swap) {
        key[i] = kp; key[p] = ki;
        idx[i] = ip; idx[p] = ii;
    }
}

// ---- sorted structure-of-arrays --------------------------------------------------
__global__ void k_build_soa(const double *__restrict__ key, const int *__restrict__ idx,
                            const double *__restrict__ xy, int64_t n, int64_t npad, double t1,
                            double cx, double cy, double *__restrict__ ts,
                            double *__restrict__ xs, double *__restrict__ ys, int *__restrict__ perm) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= npad) return;
    if (i < n) {
        int src = idx[i];
        perm[i] = src;
        ts[i] = key[i];
        xs[i] = xy[2 * (int64_t)src] - cx;
        ys[i] = xy[2 * (int64_t)src + 1] - cy;
    } else {
        ts[i] = t1 + HK_PAD_DT;
        xs[i] = 0.0;
        ys[i] = 0.0;
    }
}

// Tie groups: g[i] = first sorted index whose time equals ts[i].  Computed as a
// prefix maximum of "i if a new time starts at i, else 0" in three steps.
__global__ void k_tie_local(const double *__restrict__ ts, int64_t npad, int *__restrict__ g,
                            int *__restrict__ bmax) {
    __shared__ int sh[1024];
    int64_t i = blockIdx.x * 1024 + threadIdx.x;
    int v = 0;
    if (i < npad) v = (i == 0 || ts[i] != ts[i - 1]) ? (int)i : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int o = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] = max(sh[threadIdx.x], o);
        __syncthreads();
    }
    if (i < npad) g[i] = sh[threadIdx.x];
    if (threadIdx.x == 1023) bmax[blockIdx.x] = sh[1023];
}

__global__ void k_tie_blocks(int *__restrict__ bmax, int nb) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int run = 0;
        for (int b = 0; b < nb; ++b) {
            int v = bmax[b];
            bmax[b] = run;  // exclusive prefix max
            run = max(run, v);
        }
    }
}

__global__ void k_tie_apply(int *__restrict__ g, const int *__restrict__ bmax, int64_t npad) {
    int64_t i = blockIdx.x * 1024 + threadIdx.x;
    if (i < npad) g[i] = max(g[i], bmax[blockIdx.x]);
}

}  // namespace

// Stable sort of n2 (power of two) (key, index) pairs in place, ordered by
// (key, index); enqueued on `stream`.
hipError_t hk_sort_pairs(double *key, int *idx, int64_t n2, hipStream_t stream) {
    const int thr = 256;
    const int64_t blocks = (n2 + thr - 1) / thr;
    for (int64_t kk = 2; kk <= n2; kk <<= 1)
        for (int64_t j = kk >> 1; j > 0; j >>= 1)
            hipLaunchKernelGGL(k_bitonic_step, dim3((unsigned)blocks), dim3(thr), 0, stream, key, idx, n2, kk, j);
    return hipGetLastError();
}

namespace {

template <class T>
hipError_t dalloc(T **p, size_t count) {
    return hipMalloc((void **)p, count * sizeof(T) + 16);
}

void free_plan(hawkes_plan p) {
    if (!p) return;
    hk_prof_free(p);
    hk_subset_free(p);
    hk_tree_free(p);
    void *ptrs[] = {p->ts, p->xs, p->ys, p->perm, p->g, p->row_items, p->row_block0, p->row_item0, p->row_nseg,
                    p->colpart_off, p->col_items, p->col_block0, p->col_item0, p->col_nseg, p->theta_s, p->theta_v, p->chunk_precise, p->tstep, p->lw, p->rowpart,
                    p->colpart, p->lam, p->a, p->colG, p->blockpart, p->status};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    delete p;
}

// Pair-pass schedule.  The sweeps of a pass -- (tile, chunk) pairs -- are laid
// out tile by tile and cut into `slots` runs of nearly equal weight, one run per
// block, so that every block resident on the chip finishes at about the same
// time (a second, partly filled round of blocks would run at low occupancy).
// A run is split into pieces at tile boundaries; the pieces of one tile are
// contiguous in the item table and in chunk order, and each piece owns one
// slice of the partial-sum buffers.  Weights count wavefront-sweeps: a chunk on
// the diagonal tile is swept by only some of the block's four wavefronts.
struct Schedule {
    std::vector<hk_item> items;
    std::vector<int> block0;  // [blocks + 1] first item of each block
    std::vector<int> item0;   // [tiles] first item of each tile
    std::vector<int> nseg;    // [tiles] items of each tile
};

template <class Lo, class Hi, class Wt>
Schedule make_schedule(int T, Lo lo, Hi hi, Wt weight, int64_t slots) {
    int64_t total = 0, nch = 0;
    for (int I = 0; I < T; ++I)
        for (int c = lo(I); c < hi(I); ++c) {
            total += weight(I, c);
            ++nch;
        }
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(slots, nch));
    auto target = [&](int64_t b) { return (total * (b + 1) + nb - 1) / nb; };
    Schedule s;
    s.item0.assign(T, 0);
    s.nseg.assign(T, 0);
    s.block0.push_back(0);
    int64_t cum = 0, b = 0;
    for (int I = 0; I < T; ++I) {
        s.item0[I] = (int)s.items.size();
        bool open = false;
        for (int c = lo(I); c < hi(I); ++c) {
            if (!open) {
                s.items.push_back({I, c, c, s.nseg[I]++});
                open = true;
            }
            s.items.back().c_end = c + 1;
            cum += weight(I, c);
            if (b < nb - 1 && cum >= target(b)) {
                open = false;
                s.block0.push_back((int)s.items.size());
                while (b < nb - 1 && cum >= target(b)) ++b;
            }
        }
    }
    if (s.block0.back() != (int)s.items.size()) s.block0.push_back((int)s.items.size());
    return s;
}

}  // namespace

extern "C" hawkes_status hawkes_plan_create(hawkes_plan *out, int64_t n, const double *d_t,
                                            const double *d_xy, double t_start, hipStream_t stream) {
    if (!out || !d_t || !d_xy || n < 1 || n > (int64_t)1 << 30) return HAWKES_E_INVALID;
    *out = nullptr;
    hawkes_plan p = new hawkes_plan_s();
    memset(p, 0, sizeof(*p));
    HK_CHECK(hipGetDevice(&p->device));
    p->n = n;
    p->npad = (n + HK_TILE - 1) / HK_TILE * HK_TILE;
    p->ntiles = (int)(p->npad / HK_TILE);
    p->nchunks = (int)(p->npad / HK_WAVE);
    p->t0 = t_start;
    p->last_stream = stream;

#define PC(call)                                   \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess) {                    \
            free_plan(p);                          \
            return e_ == hipErrorOutOfMemory ? HAWKES_E_NOMEM : HAWKES_E_DEVICE; \
        }                                          \
    } while (0)

    // bounding box and finiteness
    const int bb_blocks = 64;
    double *d_part = nullptr;
    PC(dalloc(&d_part, bb_blocks * 7));
    hipLaunchKernelGGL(k_bbox, dim3(bb_blocks), dim3(256), 0, stream, d_t, d_xy, n, d_part);
    PC(hipGetLastError());
    std::vector<double> hpart(bb_blocks * 7);
    PC(hipMemcpyAsync(hpart.data(), d_part, sizeof(double) * bb_blocks * 7, hipMemcpyDeviceToHost, stream));
    PC(hipStreamSynchronize(stream));
    (void)hipFree(d_part);
    double tmin = INFINITY, tmax = -INFINITY, xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY,
           ymax = -INFINITY, bad = 0;
    for (int b = 0; b < bb_blocks; ++b) {
        const double *v = &hpart[b * 7];
        tmin = fmin(tmin, v[0]); tmax = fmax(tmax, v[1]);
        xmin = fmin(xmin, v[2]); xmax = fmax(xmax, v[3]);
        ymin = fmin(ymin, v[4]); ymax = fmax(ymax, v[5]);
        bad = fmax(bad, v[6]);
    }
    if (bad != 0.0 || !(t_start <= tmin)) {
        free_plan(p);
        return HAWKES_E_INVALID;
    }
    p->t1 = tmax;
    p->xmin = xmin;
    p->xmax = xmax;
    p->ymin = ymin;
    p->ymax = ymax;
    p->cx = 0.5 * (xmin + xmax);
    p->cy = 0.5 * (ymin + ymax);

    // stable sort by time
    int64_t n2 = 1;
    while (n2 < n) n2 <<= 1;
    double *d_key = nullptr;
    int *d_idx = nullptr;
    PC(dalloc(&d_key, n2));
    PC(dalloc(&d_idx, n2));
    {
        int thr = 256;
        int64_t blocks = (n2 + thr - 1) / thr;
        hipLaunchKernelGGL(k_sort_init, dim3((unsigned)blocks), dim3(thr), 0, stream, d_t, n, n2, d_key, d_idx);
        PC(hk_sort_pairs(d_key, d_idx, n2, stream));
    }

    const int64_t npad = p->npad;
    PC(dalloc(&p->ts, npad));
    PC(dalloc(&p->xs, npad));
    PC(dalloc(&p->ys, npad));
    PC(dalloc(&p->perm, n));
    PC(dalloc(&p->g, npad));
    {
        int thr = 256;
        unsigned blocks = (unsigned)((npad + thr - 1) / thr);
        hipLaunchKernelGGL(k_build_soa, dim3(blocks), dim3(thr), 0, stream, d_key, d_idx, d_xy, n, npad, p->t1,
                           p->cx, p->cy, p->ts, p->xs, p->ys, p->perm);
        PC(hipGetLastError());
        int nb = (int)((npad + 1023) / 1024);
        int *d_bmax = nullptr;
        PC(dalloc(&d_bmax, nb));
        hipLaunchKernelGGL(k_tie_local, dim3(nb), dim3(1024), 0, stream, p->ts, npad, p->g, d_bmax);
        hipLaunchKernelGGL(k_tie_blocks, dim3(1), dim3(64), 0, stream, d_bmax, nb);
        hipLaunchKernelGGL(k_tie_apply, dim3(nb), dim3(1024), 0, stream, p->g, d_bmax, npad);
        PC(hipGetLastError());
        PC(hipStreamSynchronize(stream));
        (void)hipFree(d_bmax);
    }
    (void)hipFree(d_key);
    (void)hipFree(d_idx);

    // ---- schedules ----
    const int T = p->ntiles;
    const int C4 = HK_CHUNKS_PER_TILE;
    // row pass: row tile I sweeps column chunks [0, 4(I+1)); wavefront w of the
    // block stops at its own chunk 4I + w
    Schedule rs = make_schedule(
        T, [](int) { return 0; }, [&](int I) { return C4 * (I + 1); },
        [&](int I, int c) { return c < C4 * I ? C4 : C4 - (c - C4 * I); }, hk_pass_slots(p->device, 0, p->npad));
    // column pass: column tile J sweeps row chunks [4J, nchunks); wavefront w
    // starts at its own chunk 4J + w
    Schedule cs = make_schedule(
        T, [&](int J) { return C4 * J; }, [&](int) { return p->nchunks; },
        [&](int J, int c) { return c >= C4 * (J + 1) ? C4 : 1 + (c - C4 * J); }, hk_pass_slots(p->device, 1, p->npad));
    std::vector<int64_t> cpoff(T);
    int64_t cpl = 0;
    for (int I = 0; I < T; ++I) {
        cpoff[I] = cpl;
        cpl += (int64_t)HK_NCOL * (I + 1) * HK_TILE;
    }
    p->colpart_len = cpl;
    p->n_row_items = (int)rs.items.size();
    p->n_row_blocks = (int)rs.block0.size() - 1;
    p->n_col_items = (int)cs.items.size();
    p->n_col_blocks = (int)cs.block0.size() - 1;

    PC(dalloc(&p->row_items, rs.items.size()));
    PC(dalloc(&p->row_block0, rs.block0.size()));
    PC(dalloc(&p->row_item0, T));
    PC(dalloc(&p->row_nseg, T));
    PC(dalloc(&p->colpart_off, T));
    PC(dalloc(&p->col_items, cs.items.size()));
    PC(dalloc(&p->col_block0, cs.block0.size()));
    PC(dalloc(&p->col_item0, T));
    PC(dalloc(&p->col_nseg, T));
    PC(hipMemcpy(p->row_items, rs.items.data(), sizeof(hk_item) * rs.items.size(), hipMemcpyHostToDevice));
    PC(hipMemcpy(p->row_block0, rs.block0.data(), sizeof(int) * rs.block0.size(), hipMemcpyHostToDevice));
    PC(hipMemcpy(p->row_item0, rs.item0.data(), sizeof(int) * T, hipMemcpyHostToDevice));
    PC(hipMemcpy(p->row_nseg, rs.nseg.data(), sizeof(int) * T, hipMemcpyHostToDevice));
    PC(hipMemcpy(p->colpart_off, cpoff.data(), sizeof(int64_t) * T, hipMemcpyHostToDevice));
    PC(hipMemcpy(p->col_items, cs.items.data(), sizeof(hk_item) * cs.items.size(), hipMemcpyHostToDevice));
    PC(hipMemcpy(p->col_block0, cs.block0.data(), sizeof(int) * cs.block0.size(), hipMemcpyHostToDevice));
    PC(hipMemcpy(p->col_item0, cs.item0.data(), sizeof(int) * T, hipMemcpyHostToDevice));
    PC(hipMemcpy(p->col_nseg, cs.nseg.data(), sizeof(int) * T, hipMemcpyHostToDevice));

    // ---- per-evaluation scratch ----
    PC(dalloc(&p->theta_s, npad));
    PC(dalloc(&p->theta_v, npad));
    PC(dalloc(&p->chunk_precise, p->nchunks));
    PC(dalloc(&p->lw, npad));
    PC(dalloc(&p->tstep, p->nchunks));
    PC(dalloc(&p->rowpart, (size_t)p->n_row_items * HK_NROW * HK_TILE));
    PC(dalloc(&p->colpart, (size_t)cpl));
    PC(dalloc(&p->lam, npad));
    PC(dalloc(&p->a, npad));
    PC(dalloc(&p->colG, (size_t)p->n_col_items * 2 * HK_TILE));
    p->nfin_blocks = (int)(npad / 256);
    PC(dalloc(&p->blockpart, (size_t)p->nchunks * HK_NSUM));
    PC(dalloc(&p->status, 1));
    PC(hipMemsetAsync(p->status, 0, sizeof(int), stream));
    PC(hipStreamSynchronize(stream));
#undef PC
    *out = p;
    return HAWKES_OK;
}

extern "C" hawkes_status hawkes_plan_destroy(hawkes_plan p) {
    if (!p) return HAWKES_E_INVALID;
    (void)hipDeviceSynchronize();
    free_plan(p);
    return HAWKES_OK;
}

extern "C" int64_t hawkes_plan_size(hawkes_plan p) { return p ? p->n : -1; }

extern "C" hawkes_status hawkes_plan_status(hawkes_plan p) {
    if (!p) return HAWKES_E_INVALID;
    int h = 0;
    HK_CHECK(hipStreamSynchronize(p->last_stream));
    HK_CHECK(hipMemcpy(&h, p->status, sizeof(int), hipMemcpyDeviceToHost));
    HK_CHECK(hipMemset(p->status, 0, sizeof(int)));
    if (h & HK_ST_BADTHETA) return HAWKES_E_INVALID;
    if (h & HK_ST_NONFINITE) return HAWKES_E_NONFINITE;
    if (h & HK_ST_ZERO) return HAWKES_E_ZERO_INTENSITY;
    return HAWKES_OK;
}
