// Phylogenetic Brownian prior on the free log-rates (Sec. 2.2, Eq. 2).
//
// The log-rates z of the M tips of a bifurcating tree follow a Brownian
// diffusion: the root value is N(0, tau0 sigma^2), each child is its parent
// plus N(0, w sigma^2) for its branch length w, so z ~ N(0, sigma^2 V) with
// V_nm = tau0 + (length of the path from the root to the common ancestor of
// tips n and m).  Eq. 2 needs V^{-1}, O(M^3) dense; the tree structure gives
// log p(z) and its gradient in O(M) by message passing (the paper uses the
// dynamic programming of Pybus et al. 2012):
//
//  * post-order: a tip carries (m, v) = (z_k, 0).  An internal node a with
//    children b, c carries v_a = 1 / (1/(v_b + w_b) + 1/(v_c + w_c)) and
//    m_a = alpha_b m_b + alpha_c m_c, alpha_x = v_a / (v_x + w_x); the pair
//    contributes (m_b - m_c)^2 / s_a, s_a = v_b + w_b + v_c + w_c, to the
//    quadratic form, the root m_root^2 / (v_root + tau0);
//  * z^T V^{-1} z is the sum of those contributions and
//    log |V| = sum_a log s_a + log(v_root + tau0);
//  * V^{-1} z is the gradient of half the quadratic form: a pre-order pass
//    pushes the adjoint of each node to its children,
//    mbar_b = alpha_b mbar_a + d_a, mbar_c = alpha_c mbar_a - d_a,
//    d_a = (m_b - m_c) / s_a, starting from mbar_root = m_root / (v_root + tau0);
//  * the diagonal of V^{-1} (the prior's precision, used by the diagonal mass
//    matrix) is 1 / Var(z_k | every other tip): a pre-order pass carries the
//    variance u_a of what the rest of the tree says about node a, u_root =
//    tau0, u_b = (u_a (v_c + w_c)) / (u_a + v_c + w_c) + w_b for child b with
//    sibling c, and (V^{-1})_kk = 1 / u_k at tip k.
//
// The v, alpha, s depend on the tree only and are formed once on the host in
// FP64.  On the device one block walks the levels of the tree (nodes grouped by
// height, so that all children of a level are done before it), one thread per
// node of a level, with a barrier between levels.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <vector>

#include "hawkes_internal.h"

struct hk_tree {
    int64_t m;           // tips (= subset size)
    int64_t n_int;       // internal nodes (m - 1)
    int levels;          // height levels of internal nodes
    double logdet;       // log |V|
    // device arrays
    int *order;          // [n_int] internal nodes, grouped by level (increasing height)
    int *level0;         // [levels + 1] first entry of each level in order[]
    int *child;          // [2 (2m - 1)] children of each node (internal only)
    double *coef;        // [3 (2m - 1)] alpha_b, alpha_c, 1 / s_a per internal node
    double *mv;          // [2m - 1] node means (post-order), then adjoints
    double *dd;          // [2m - 1] d_a per internal node
    int root;
    double root_inv;     // 1 / (v_root + tau0)
    int *level0_h;       // host copy of level0 (launch loop bounds)
    double *pdiag;       // [m] diagonal of V^{-1}, tip (slot) order (device)
};

namespace {

constexpr int TREE_THREADS = 1024;

__global__ __launch_bounds__(TREE_THREADS) void k_tree_prior(const double *__restrict__ z, int64_t m,
                                                             const int *__restrict__ order,
                                                             const int *__restrict__ level0, int levels,
                                                             const int *__restrict__ child,
                                                             const double *__restrict__ coef, int root,
                                                             double root_inv, double *__restrict__ mv,
                                                             double *__restrict__ dd, double *__restrict__ vz,
                                                             double *__restrict__ quad) {
    __shared__ double red[TREE_THREADS];
    const int tid = threadIdx.x;
    double q = 0.0;
    for (int64_t k = tid; k < m; k += TREE_THREADS) mv[k] = z[k];
    __syncthreads();
    // post-order: level by level of increasing height
    for (int l = 0; l < levels; ++l) {
        for (int e = level0[l] + tid; e < level0[l + 1]; e += TREE_THREADS) {
            const int a = order[e];
            const int b = child[2 * a], c = child[2 * a + 1];
            const double mb = mv[b], mc = mv[c];
            const double ab = coef[3 * a], ac = coef[3 * a + 1], is = coef[3 * a + 2];
            mv[a] = ab * mb + ac * mc;
            const double d = mb - mc;
            q += d * d * is;
            dd[a] = d * is;
        }
        __syncthreads();
    }
    const double mroot = mv[root];
    if (tid == 0) q += mroot * mroot * root_inv;
    __syncthreads();
    // pre-order: adjoints of half the quadratic form, root level first (the
    // node means are no longer needed, so mv now holds adjoints)
    if (tid == 0) mv[root] = mroot * root_inv;
    __syncthreads();
    for (int l = levels - 1; l >= 0; --l) {
        for (int e = level0[l] + tid; e < level0[l + 1]; e += TREE_THREADS) {
            const int a = order[e];
            const int b = child[2 * a], c = child[2 * a + 1];
            const double ma = mv[a], d = dd[a];
            mv[b] = coef[3 * a] * ma + d;
            mv[c] = coef[3 * a + 1] * ma - d;
        }
        __syncthreads();
    }
    if (vz)
        for (int64_t k = tid; k < m; k += TREE_THREADS) vz[k] = mv[k];
    // fixed-order reduction of the quadratic form
    red[tid] = q;
    __syncthreads();
    for (int h = TREE_THREADS / 2; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0 && quad) quad[0] = red[0];
}

// log p(z) = -(m log(2 pi sigma^2) + log|V| + z^T V^{-1} z / sigma^2) / 2 and
// its gradient -V^{-1} z / sigma^2
__global__ void k_tree_logp(const double *__restrict__ quad, const double *__restrict__ vz, int64_t m,
                            double sigma2, double logdet, double *__restrict__ logp, double *__restrict__ grad) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k == 0 && logp)
        logp[0] = -0.5 * ((double)m * log(2.0 * 3.141592653589793 * sigma2) + logdet + quad[0] / sigma2);
    if (k < m && grad) grad[k] = -vz[k] / sigma2;
}

template <class T>
hipError_t dalloc(T **p, size_t count) {
    return hipMalloc((void **)p, count * sizeof(T) + 16);
}

}  // namespace

void hk_tree_free(hawkes_plan p) {
    hk_tree *t = p->tree;
    if (!t) return;
    void *ptrs[] = {t->order, t->level0, t->child, t->coef, t->mv, t->dd, t->pdiag};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    delete[] t->level0_h;
    delete t;
    p->tree = nullptr;
}

int64_t hk_tree_tips(hawkes_plan p) { return p->tree ? p->tree->m : 0; }

const double *hk_tree_precision_diag(hawkes_plan p) { return p->tree ? p->tree->pdiag : nullptr; }

hawkes_status hk_tree_launch(hawkes_plan p, const double *d_z, double *d_vz, double *d_quad, hipStream_t stream) {
    hk_tree *t = p->tree;
    if (!t) return HAWKES_E_UNSUPPORTED;
    hipLaunchKernelGGL(k_tree_prior, dim3(1), dim3(TREE_THREADS), 0, stream, d_z, t->m, t->order, t->level0,
                       t->levels, t->child, t->coef, t->root, t->root_inv, t->mv, t->dd, d_vz, d_quad);
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}

extern "C" hawkes_status hawkes_plan_set_tree(hawkes_plan p, int64_t n_nodes, const int64_t *parent,
                                              const double *length, double tau0) {
    if (!p || !parent || !length || n_nodes < 1 || n_nodes % 2 == 0 || !(tau0 > 0.0) || !isfinite(tau0))
        return HAWKES_E_INVALID;
    const int64_t m = (n_nodes + 1) / 2;
    if (m > (int64_t)1 << 30) return HAWKES_E_INVALID;
    // structure: nodes 0..m-1 are tips, exactly one root, every internal node
    // has two children, lengths finite and >= 0
    std::vector<int> nchild(n_nodes, 0), child(2 * n_nodes, -1);
    int64_t root = -1;
    for (int64_t v = 0; v < n_nodes; ++v) {
        const int64_t pa = parent[v];
        if (pa < 0) {
            if (root >= 0) return HAWKES_E_INVALID;
            root = v;
            continue;
        }
        if (pa >= n_nodes || pa < m || pa == v) return HAWKES_E_INVALID;
        if (!(length[v] >= 0.0) || !isfinite(length[v])) return HAWKES_E_INVALID;
        if (nchild[pa] >= 2) return HAWKES_E_INVALID;
        child[2 * pa + nchild[pa]++] = (int)v;
    }
    if (root < 0) return HAWKES_E_INVALID;
    if (m == 1 && root != 0) return HAWKES_E_INVALID;
    for (int64_t v = m; v < n_nodes; ++v)
        if (nchild[v] != 2) return HAWKES_E_INVALID;
    // heights by an explicit post-order from the root (also proves the graph is
    // one tree: every node must be reached exactly once)
    std::vector<int> height(n_nodes, -1), stack;
    std::vector<char> seen(n_nodes, 0);
    std::vector<int> post;
    post.reserve(n_nodes);
    stack.push_back((int)root);
    while (!stack.empty()) {
        const int v = stack.back();
        if (!seen[v]) {
            seen[v] = 1;
            if (v >= m) {
                for (int k = 0; k < 2; ++k) {
                    const int c = child[2 * v + k];
                    if (seen[c]) return HAWKES_E_INVALID;
                    stack.push_back(c);
                }
            }
        } else {
            stack.pop_back();
            post.push_back(v);
        }
    }
    if ((int64_t)post.size() != n_nodes) return HAWKES_E_INVALID;
    std::vector<double> var(n_nodes, 0.0), coef(3 * n_nodes, 0.0);
    double logdet = 0.0;
    for (int v : post) {
        if (v < m) {
            height[v] = 0;
            continue;
        }
        const int b = child[2 * v], c = child[2 * v + 1];
        height[v] = 1 + std::max(height[b], height[c]);
        const double vb = var[b] + length[b], vc = var[c] + length[c];
        const double s = vb + vc;
        if (!(s > 0.0)) return HAWKES_E_INVALID;  // two zero-variance children: V is singular
        const double va = vb * vc / s;
        var[v] = va;
        coef[3 * v] = vc / s;      // alpha_b = v_a / vb
        coef[3 * v + 1] = vb / s;  // alpha_c = v_a / vc
        coef[3 * v + 2] = 1.0 / s;
        logdet += log(s);
    }
    const double rv = var[root] + tau0;
    logdet += log(rv);
    // diagonal of V^{-1}: pre-order pass of the outside variances (reverse post-order)
    std::vector<double> outside(n_nodes, 0.0), pdiag(m, 0.0);
    outside[root] = tau0;
    for (auto it = post.rbegin(); it != post.rend(); ++it) {
        const int v = *it;
        if (v < m) {
            if (!(outside[v] > 0.0)) return HAWKES_E_INVALID;  // tip fixed by the others: V is singular
            pdiag[v] = 1.0 / outside[v];
            continue;
        }
        for (int k = 0; k < 2; ++k) {
            const int b = child[2 * v + k], c = child[2 * v + 1 - k];
            const double u = outside[v], vs = var[c] + length[c];
            const double x = u + vs > 0.0 ? u * vs / (u + vs) : 0.0;
            outside[b] = x + length[b];
        }
    }
    const int H = m > 1 ? height[root] : 0;
    std::vector<int> level0(H + 1, 0), order;
    for (int64_t v = m; v < n_nodes; ++v) level0[height[v]]++;  // heights 1..H
    // level l holds height l + 1
    std::vector<int> cnt(H + 1, 0);
    for (int l = 0; l < H; ++l) cnt[l] = level0[l + 1];
    std::vector<int> start(H + 1, 0);
    for (int l = 0; l < H; ++l) start[l + 1] = start[l] + cnt[l];
    order.assign(std::max<int64_t>(n_nodes - m, 1), 0);
    std::vector<int> fill(start.begin(), start.end());
    for (int64_t v = m; v < n_nodes; ++v) order[fill[height[v] - 1]++] = (int)v;

    hk_tree_free(p);
    hk_tree *t = new hk_tree();
    p->tree = t;
    t->m = m;
    t->n_int = n_nodes - m;
    t->levels = H;
    t->logdet = logdet;
    t->root = (int)root;
    t->root_inv = 1.0 / rv;
    t->level0_h = new int[H + 1];
    for (int l = 0; l <= H; ++l) t->level0_h[l] = start[l];
#define TC(call)                                                              \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) {                                               \
            hk_tree_free(p);                                                  \
            return e_ == hipErrorOutOfMemory ? HAWKES_E_NOMEM : HAWKES_E_DEVICE; \
        }                                                                     \
    } while (0)
    TC(dalloc(&t->order, order.size()));
    TC(dalloc(&t->level0, (size_t)H + 1));
    TC(dalloc(&t->child, child.size()));
    TC(dalloc(&t->coef, coef.size()));
    TC(dalloc(&t->mv, (size_t)n_nodes));
    TC(dalloc(&t->dd, (size_t)n_nodes));
    TC(dalloc(&t->pdiag, (size_t)m));
    TC(hipMemcpy(t->order, order.data(), sizeof(int) * order.size(), hipMemcpyHostToDevice));
    TC(hipMemcpy(t->level0, start.data(), sizeof(int) * (H + 1), hipMemcpyHostToDevice));
    TC(hipMemcpy(t->child, child.data(), sizeof(int) * child.size(), hipMemcpyHostToDevice));
    TC(hipMemcpy(t->coef, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice));
    TC(hipMemcpy(t->pdiag, pdiag.data(), sizeof(double) * m, hipMemcpyHostToDevice));
#undef TC
    return HAWKES_OK;
}

extern "C" hawkes_status hawkes_tree_prior(hawkes_plan p, const double *d_z, double sigma, double *d_logp,
                                           double *d_grad, double *d_quad, hipStream_t stream) {
    if (!p || !d_z || !(sigma > 0.0) || !isfinite(sigma) || !d_quad) return HAWKES_E_INVALID;
    hk_tree *t = p->tree;
    if (!t) return HAWKES_E_UNSUPPORTED;
    p->last_stream = stream;
    double *vz = t->mv;  // the adjoints of the tips are left in mv[0..m)
    hawkes_status st = hk_tree_launch(p, d_z, nullptr, d_quad, stream);
    if (st != HAWKES_OK) return st;
    if (d_logp || d_grad)
        hipLaunchKernelGGL(k_tree_logp, dim3((unsigned)((t->m + 255) / 256)), dim3(256), 0, stream, d_quad, vz, t->m,
                           sigma * sigma, t->logdet, d_logp, d_grad);
    HK_CHECK(hipGetLastError());
    return HAWKES_OK;
}
