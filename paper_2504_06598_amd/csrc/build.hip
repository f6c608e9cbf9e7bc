// Canonical records and BVH construction on the GPU.
//
// Sec. 3.1-3.2 of the paper: each Gaussian is bounded by the box of its
// k-sigma ellipsoid (eqn "cuboid") and a BVH is built over the boxes. The
// paper used Embree / OptiX builders; here the build is a GPU LBVH
// (63-bit Morton codes of box centres, radix sort, Karras' 2012 parallel
// binary hierarchy) collapsed top-down into W-wide nodes by greedily opening
// the child holding the most Gaussians, with subtrees of at most L Gaussians
// turned into leaves; wide-node boxes are then filled bottom-up, one level
// per launch, so no kernel needs cross-workgroup ordering of its writes. Records are then stored in leaf order
// so a leaf is one contiguous run of 64-B records.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "srt_internal.hpp"

using namespace srt;

namespace {

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Largest eigenvalue of A A^T (A 3x3 row-major) from the characteristic
// cubic (trigonometric solution), i.e. the squared largest singular value.
__device__ inline double lmax_sym3(const double A[9])
{
    double B[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            B[3 * i + j] = A[3 * i] * A[3 * j] + A[3 * i + 1] * A[3 * j + 1] + A[3 * i + 2] * A[3 * j + 2];
    const double p1 = B[1] * B[1] + B[2] * B[2] + B[5] * B[5];
    const double q = (B[0] + B[4] + B[8]) / 3.0;
    if (p1 <= 1e-300) return fmax(fmax(B[0], B[4]), B[8]);
    const double p2 = (B[0] - q) * (B[0] - q) + (B[4] - q) * (B[4] - q) + (B[8] - q) * (B[8] - q) +
                      2.0 * p1;
    const double p = sqrt(p2 / 6.0);
    double C[9];
    for (int i = 0; i < 9; ++i) C[i] = (B[i] - (i % 4 == 0 ? q : 0.0)) / p;
    const double detC = C[0] * (C[4] * C[8] - C[5] * C[7]) - C[1] * (C[3] * C[8] - C[5] * C[6]) +
                        C[2] * (C[3] * C[7] - C[4] * C[6]);
    const double rr = fmin(1.0, fmax(-1.0, detC / 2.0));
    const double phi = acos(rr) / 3.0;
    // the largest root, padded for the rounding of the iteration above
    return (q + 2.0 * p * cos(phi)) * (1.0 + 1e-9) + 1e-300;
}

// Canonical record: whitening matrix M = S^-1 R^T from the normalised
// quaternion and exp(log-scales), and opacity sigmoid(logit), computed in
// FP64 and rounded to nearest FP32. The box is that of the ellipsoid
// q <= 8 of the ROUNDED record: Sigma' = (M^T M)^-1 = M^-1 M^-T, half extent
// sqrt(8 Sigma'_ii), padded by 2^-20 relative and rounded outward to FP32.
__device__ void make_record(int64_t g, const float* __restrict__ means,
                            const float* __restrict__ log_scales, const float* __restrict__ quats,
                            const float* __restrict__ logits, Record& r, float* __restrict__ box_lo,
                            float* __restrict__ box_hi)
{
    double qw = quats[4 * g], qx = quats[4 * g + 1], qy = quats[4 * g + 2], qz = quats[4 * g + 3];
    const double nrm = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    if (nrm > 0.0) {
        qw /= nrm; qx /= nrm; qy /= nrm; qz /= nrm;
    } else {
        qw = 1.0; qx = qy = qz = 0.0;
    }
    // R maps the Gaussian's frame to the world (Hamilton convention).
    const double R[9] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz),
                         2.0 * (qx * qz + qw * qy),       2.0 * (qx * qy + qw * qz),
                         1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx),
                         2.0 * (qx * qz - qw * qy),       2.0 * (qy * qz + qw * qx),
                         1.0 - 2.0 * (qx * qx + qy * qy)};
    for (int i = 0; i < 3; ++i) {
        const double inv_s = exp(-(double)log_scales[3 * g + i]);
        for (int j = 0; j < 3; ++j) r.M[3 * i + j] = (float)(R[3 * j + i] * inv_s);
        r.mu[i] = means[3 * g + i];
    }
    r.opacity = (float)(1.0 / (1.0 + exp(-(double)logits[g])));
    r.gid = (int32_t)g;

    const double a = r.M[0], b = r.M[1], c = r.M[2];
    const double d = r.M[3], e = r.M[4], f = r.M[5];
    const double gg = r.M[6], h = r.M[7], k = r.M[8];
    const double c00 = e * k - f * h, c01 = -(d * k - f * gg), c02 = d * h - e * gg;
    const double det = a * c00 + b * c01 + c * c02;
    // rows of M^-1 = adj(M)^T / det
    const double inv[9] = {c00 / det, -(b * k - c * h) / det, (b * f - c * e) / det,
                           c01 / det, (a * k - c * gg) / det, -(a * f - c * d) / det,
                           c02 / det, -(a * h - b * gg) / det, (a * e - b * d) / det};
    for (int i = 0; i < 3; ++i) {
        const double s2 = inv[3 * i] * inv[3 * i] + inv[3 * i + 1] * inv[3 * i + 1] +
                          inv[3 * i + 2] * inv[3 * i + 2];
        const double hx = sqrt(kEllipsoidQ * s2) * (1.0 + 0x1p-20);
        box_lo[3 * g + i] = __double2float_rd((double)r.mu[i] - hx);
        box_hi[3 * g + i] = __double2float_ru((double)r.mu[i] + hx);
    }
    // radius of a sphere about mu holding the ellipsoid q <= 8 of the rounded
    // record: sqrt(8) times its largest semi-axis (largest singular value of
    // M^-1), padded and rounded up
    r.pad[0] = __double2float_ru(sqrt(kEllipsoidQ * lmax_sym3(inv)) * (1.0 + 0x1p-16));
    r.pad[1] = 0.0f;
}

__global__ void k_preprocess(int64_t G, const float* __restrict__ means,
                             const float* __restrict__ log_scales, const float* __restrict__ quats,
                             const float* __restrict__ logits, Record* __restrict__ recs,
                             float* __restrict__ box_lo, float* __restrict__ box_hi)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= G) return;
    Record r;
    make_record(g, means, log_scales, quats, logits, r, box_lo, box_hi);
    recs[g] = r;
}

// Refit: the record of the Gaussian at leaf position k, written in place
// (the tree keeps its leaf order; the boxes are refilled afterwards).
__global__ void k_refit_records(int64_t G, const int32_t* __restrict__ leaf_order,
                                const float* __restrict__ means,
                                const float* __restrict__ log_scales,
                                const float* __restrict__ quats, const float* __restrict__ logits,
                                Record* __restrict__ recs, float* __restrict__ box_lo,
                                float* __restrict__ box_hi)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= G) return;
    Record r;
    make_record(leaf_order[k], means, log_scales, quats, logits, r, box_lo, box_hi);
    recs[k] = r;
}

__device__ __forceinline__ uint32_t f2ord(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float ord2f(uint32_t o)
{
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

// Bounds of box centres: [0..2] min, [3..5] max, as order-preserving uints;
// [6] the largest bounding-sphere radius (positive float bits order as uints).
__global__ void k_centre_bounds(int64_t G, const float* __restrict__ lo, const float* __restrict__ hi,
                                const Record* __restrict__ recs, uint32_t* out)
{
    __shared__ uint32_t smin[3][256], smax[4][256];
    uint32_t mn[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, mx[4] = {0u, 0u, 0u, 0u};
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < G;
         g += (int64_t)gridDim.x * blockDim.x) {
        for (int i = 0; i < 3; ++i) {
            const uint32_t c = f2ord(0.5f * (lo[3 * g + i] + hi[3 * g + i]));
            mn[i] = min(mn[i], c);
            mx[i] = max(mx[i], c);
        }
        mx[3] = max(mx[3], __float_as_uint(recs[g].pad[0]));
    }
    for (int i = 0; i < 3; ++i) smin[i][threadIdx.x] = mn[i];
    for (int i = 0; i < 4; ++i) smax[i][threadIdx.x] = mx[i];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int i = 0; i < 3; ++i)
                smin[i][threadIdx.x] = min(smin[i][threadIdx.x], smin[i][threadIdx.x + s]);
            for (int i = 0; i < 4; ++i)
                smax[i][threadIdx.x] = max(smax[i][threadIdx.x], smax[i][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int i = 0; i < 3; ++i) {
            atomicMin(&out[i], smin[i][0]);
            atomicMax(&out[3 + i], smax[i][0]);
        }
        atomicMax(&out[6], smax[3][0]);
    }
}

__device__ __forceinline__ uint64_t spread3_21(uint32_t v)
{
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x1F00000000FFFFull;
    x = (x | (x << 16)) & 0x1F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// Sort key: the 63-bit Morton code of the box centre, or, with size_split
// k > 0, a 3-bit size class floor(log2(scene extent / box extent) / k)
// (largest Gaussians first) above a 60-bit Morton code, so Gaussians of very
// different sizes end up in subtrees of their own instead of inflating each
// other's boxes.
__global__ void k_morton(int64_t G, const float* __restrict__ lo, const float* __restrict__ hi,
                         const uint32_t* __restrict__ bounds, int32_t size_split,
                         uint64_t* __restrict__ keys, uint32_t* __restrict__ idx)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= G) return;
    uint32_t q[3];
    float scene_ext = 0.0f, box_ext = 0.0f;
    for (int i = 0; i < 3; ++i) {
        const float bmin = ord2f(bounds[i]), bmax = ord2f(bounds[3 + i]);
        const float ext = bmax - bmin;
        scene_ext = fmaxf(scene_ext, ext);
        box_ext = fmaxf(box_ext, hi[3 * g + i] - lo[3 * g + i]);
        const float c = 0.5f * (lo[3 * g + i] + hi[3 * g + i]);
        float t = ext > 0.0f ? (c - bmin) / ext : 0.0f;
        t = fminf(fmaxf(t, 0.0f), 1.0f);
        q[i] = min((uint32_t)(t * 2097152.0f), 2097151u);
    }
    uint64_t m = (spread3_21(q[0]) << 2) | (spread3_21(q[1]) << 1) | spread3_21(q[2]);
    if (size_split > 0) {
        int cls = 7;
        if (box_ext > 0.0f && scene_ext > 0.0f) {
            const float l = log2f(fmaxf(scene_ext, box_ext) / box_ext) / (float)size_split;
            cls = min(7, max(0, (int)l));
        }
        m = ((uint64_t)cls << 60) | (m >> 3);
    }
    keys[g] = m;
    idx[g] = (uint32_t)g;
}

// Length of the common prefix of sorted keys i and j (ties extended by the
// index), -1 outside the array.
__device__ __forceinline__ int prefix_len(const uint64_t* __restrict__ k, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    const uint64_t a = k[i], b = k[j];
    if (a == b) return 64 + __clz((uint32_t)(i ^ j));
    return __clzll(a ^ b);
}

// Karras (HPG 2012): internal node i covers a key range found by a doubling
// then binary search of common-prefix lengths, and splits where the prefix
// length of the range drops. Child refs: >= 0 internal, < 0 leaf ~k.
__global__ void k_karras(int n, const uint64_t* __restrict__ keys, int32_t* __restrict__ left,
                         int32_t* __restrict__ right, int32_t* __restrict__ parent,
                         int32_t* __restrict__ leaf_parent, int32_t* __restrict__ first,
                         int32_t* __restrict__ last)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (prefix_len(keys, n, i, i + 1) - prefix_len(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = prefix_len(keys, n, i, i - d);
    int lmax = 2;
    while (prefix_len(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = prefix_len(keys, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (prefix_len(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int split = i + s * d + min(d, 0);
    const int lo_i = min(i, j), hi_i = max(i, j);
    const int32_t lc = (lo_i == split) ? ~split : split;
    const int32_t rc = (hi_i == split + 1) ? ~(split + 1) : split + 1;
    left[i] = lc;
    right[i] = rc;
    first[i] = lo_i;
    last[i] = hi_i;
    if (lc < 0) leaf_parent[~lc] = i; else parent[lc] = i;
    if (rc < 0) leaf_parent[~rc] = i; else parent[rc] = i;
    if (i == 0) parent[0] = -1;
}

struct Task {
    int32_t bin;
    int32_t node;
};

struct BinTree {
    const int32_t *left, *right, *first, *last;
};

__device__ __forceinline__ int32_t bin_size(const BinTree& t, int32_t c)
{
    return c < 0 ? 1 : t.last[c] - t.first[c] + 1;
}

// One level of the top-down collapse into W-wide nodes: starting from the
// two children of the task's binary node, repeatedly open the child holding
// the most Gaussians until W children are collected or every child holds at
// most L (those become leaves). Internal children become the next level's
// tasks. Boxes are filled in afterwards, bottom-up (k_wide_boxes).
template <int W>
__global__ void k_collapse(BinTree t, int L, const Task* __restrict__ in, uint32_t* ctr,
                           Task* __restrict__ out, WideNode<W>* nodes,
                           int32_t* __restrict__ level_nodes)
{
    // ctr: [0] tasks of this level, [1] tasks of the next, [2] wide nodes made,
    // [3] where this level's node list starts in level_nodes
    uint32_t* n_out = ctr + 1;
    uint32_t* node_counter = ctr + 2;
    const uint32_t ti = blockIdx.x * blockDim.x + threadIdx.x;
    if (ti >= ctr[0]) return;
    const Task tk = in[ti];
    level_nodes[ctr[3] + ti] = tk.node;
    int32_t C[W];
    int32_t sz[W];
    int nc = 2;
    C[0] = t.left[tk.bin];
    C[1] = t.right[tk.bin];
    sz[0] = bin_size(t, C[0]);
    sz[1] = bin_size(t, C[1]);
    while (nc < W) {
        int best = -1;
        int32_t bs = L;
        for (int j = 0; j < nc; ++j)
            if (sz[j] > bs) {
                bs = sz[j];
                best = j;
            }
        if (best < 0) break;
        const int32_t c = C[best];
        C[best] = t.left[c];
        C[nc] = t.right[c];
        sz[best] = bin_size(t, C[best]);
        sz[nc] = bin_size(t, C[nc]);
        ++nc;
    }
    WideNode<W> nd;
    for (int s = 0; s < W; ++s) {
        for (int i = 0; i < 3; ++i) {
            nd.lo[i][s] = INFINITY;
            nd.hi[i][s] = -INFINITY;
        }
        nd.pad[s] = 0;
        if (s < nc) {
            const int32_t c = C[s];
            if (c < 0) {
                nd.child[s] = make_leaf((uint32_t)~c, 1u);
            } else if (sz[s] <= L) {
                nd.child[s] = make_leaf((uint32_t)t.first[c], (uint32_t)sz[s]);
            } else {
                const uint32_t idx = atomicAdd(node_counter, 1u);
                nd.child[s] = (int32_t)idx;
                out[atomicAdd(n_out, 1u)] = Task{c, (int32_t)idx};
            }
        } else {
            nd.child[s] = kEmptyChild;
        }
    }
    nodes[tk.node] = nd;
}

// Between two levels: record the level's size and start, then make the next
// level current (one thread; the next collapse launch sees the new counts).
__global__ void k_advance(uint32_t* ctr, uint32_t* lvl_cnt, uint32_t* lvl_base, int level)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    lvl_cnt[level] = ctr[0];
    lvl_base[level] = ctr[3];
    ctr[3] += ctr[0];
    ctr[0] = ctr[1];
    ctr[1] = 0u;
}

// Boxes of the wide nodes of one level, once the level below is complete:
// a leaf slot bounds its Gaussians' boxes, an internal slot bounds the slot
// boxes of its child node.
template <int W>
__global__ void k_wide_boxes(const int32_t* __restrict__ level_nodes, uint32_t count,
                             const uint32_t* __restrict__ order, const float* __restrict__ lo,
                             const float* __restrict__ hi, WideNode<W>* nodes)
{
    const uint32_t ti = blockIdx.x * blockDim.x + threadIdx.x;
    if (ti >= count) return;
    WideNode<W>& nd = nodes[level_nodes[ti]];
    for (int s = 0; s < W; ++s) {
        const int32_t c = nd.child[s];
        if (c == kEmptyChild) continue;
        float l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
        if (c < 0) {
            const uint32_t f = leaf_first(c), n = leaf_count(c);
            for (uint32_t p = f; p < f + n; ++p) {
                const uint32_t g = order[p];
                for (int i = 0; i < 3; ++i) {
                    l[i] = fminf(l[i], lo[3 * g + i]);
                    h[i] = fmaxf(h[i], hi[3 * g + i]);
                }
            }
        } else {
            const WideNode<W>& ch = nodes[c];
            for (int j = 0; j < W; ++j)
                for (int i = 0; i < 3; ++i) {
                    l[i] = fminf(l[i], ch.lo[i][j]);
                    h[i] = fmaxf(h[i], ch.hi[i][j]);
                }
        }
        for (int i = 0; i < 3; ++i) {
            nd.lo[i][s] = l[i];
            nd.hi[i][s] = h[i];
        }
    }
}

// A scene of at most L Gaussians: one root with a single leaf.
template <int W>
__global__ void k_single_leaf(int64_t G, const float* __restrict__ lo, const float* __restrict__ hi,
                              WideNode<W>* nodes)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    WideNode<W> nd;
    for (int s = 0; s < W; ++s) {
        for (int i = 0; i < 3; ++i) {
            nd.lo[i][s] = INFINITY;
            nd.hi[i][s] = -INFINITY;
        }
        nd.child[s] = kEmptyChild;
        nd.pad[s] = 0;
    }
    for (int64_t g = 0; g < G; ++g)
        for (int i = 0; i < 3; ++i) {
            nd.lo[i][0] = fminf(nd.lo[i][0], lo[3 * g + i]);
            nd.hi[i][0] = fmaxf(nd.hi[i][0], hi[3 * g + i]);
        }
    if (G > 0) nd.child[0] = make_leaf(0u, (uint32_t)G);
    nodes[0] = nd;
}

constexpr int32_t kStartLevels = 2;

// Parent of every wide node (-1 at the root) and the node whose slot holds
// each leaf position.
template <int W>
__global__ void k_node_parents(const WideNode<W>* __restrict__ nodes, int64_t num_nodes,
                               int32_t* __restrict__ parent, int32_t* __restrict__ leaf_node)
{
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= num_nodes) return;
    if (n == 0) parent[0] = -1;
    for (int c = 0; c < W; ++c) {
        const int32_t ch = nodes[n].child[c];
        if (ch == kEmptyChild) continue;
        if (ch >= 0) {
            parent[ch] = (int32_t)n;
        } else {
            const uint32_t f = leaf_first(ch), k = leaf_count(ch);
            for (uint32_t i = 0; i < k; ++i) leaf_node[f + i] = (int32_t)n;
        }
    }
}

__global__ void k_start_nodes(int64_t G, int32_t levels, const int32_t* __restrict__ leaf_pos,
                              const int32_t* __restrict__ leaf_node,
                              const int32_t* __restrict__ parent, int32_t* __restrict__ start)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= G) return;
    int32_t n = leaf_node[leaf_pos[g]];
    for (int32_t k = 0; k < levels && parent[n] >= 0; ++k) n = parent[n];
    start[g] = n;
}

__global__ void k_permute(int64_t G, const uint32_t* __restrict__ order, const Record* __restrict__ in,
                          Record* __restrict__ out, int32_t* __restrict__ leaf_order,
                          int32_t* __restrict__ leaf_pos)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= G) return;
    const uint32_t g = order[k];
    out[k] = in[g];
    leaf_order[k] = (int32_t)g;
    leaf_pos[g] = (int32_t)k;
}

__global__ void k_unpermute_records(int64_t G, const Record* __restrict__ recs, float* mu, float* M,
                                    float* op)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= G) return;
    const Record r = recs[k];
    const int64_t g = r.gid;
    if (mu)
        for (int i = 0; i < 3; ++i) mu[3 * g + i] = r.mu[i];
    if (M)
        for (int i = 0; i < 9; ++i) M[9 * g + i] = r.M[i];
    if (op) op[g] = r.opacity;
}

// Device allocations released on scope exit unless released to the caller.
// Device blocks for builds (temporaries) and handles (their buffers) are
// kept by the library when released and handed out again by later builds of
// the same size: hipMalloc and, above all, hipFree (which synchronises the
// device and measured ~0.5 ms per call) stay out of a rebuild. A block is
// released only when no work on it can be pending: temporaries after the
// build has synchronised its stream, a handle's buffers at destroy (whose
// contract says no work on the handle is pending). Blocks are kept per
// device and size class (64 KiB granules) up to 8 GiB in total; more is
// freed at once. An optional limit caps the bytes in use (handed out and not
// returned); a request beyond it fails as out of memory.
struct BlockCache {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<void*>> free_blocks;
    size_t kept = 0;
    size_t in_use = 0;
    size_t limit = 0;  // 0: none
    static constexpr size_t kGranule = size_t(1) << 16;
    static constexpr size_t kMaxKept = size_t(8) << 30;

    static size_t round(size_t bytes) { return (std::max<size_t>(bytes, 16) + kGranule - 1) / kGranule * kGranule; }

    hipError_t get(void** p, size_t bytes)
    {
        const size_t sz = round(bytes);
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        {
            std::lock_guard<std::mutex> lock(mu);
            if (limit > 0 && in_use + sz > limit) return hipErrorOutOfMemory;
            in_use += sz;  // reserved before the allocation
            auto it = free_blocks.find({dev, sz});
            if (it != free_blocks.end() && !it->second.empty()) {
                *p = it->second.back();
                it->second.pop_back();
                kept -= sz;
                return hipSuccess;
            }
        }
        e = hipMalloc(p, sz);
        if (e != hipSuccess) {
            std::lock_guard<std::mutex> lock(mu);
            in_use -= sz;
        }
        return e;
    }

    void put(void* p, size_t bytes)
    {
        if (!p) return;
        const size_t sz = round(bytes);
        {
            std::lock_guard<std::mutex> lock(mu);
            in_use -= std::min(in_use, sz);
        }
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            std::lock_guard<std::mutex> lock(mu);
            if (kept + sz <= kMaxKept) {
                free_blocks[{dev, sz}].push_back(p);
                kept += sz;
                return;
            }
        }
        (void)hipFree(p);
    }
};

BlockCache& block_cache()
{
    static BlockCache* c = new BlockCache();  // kept to process exit
    return *c;
}

// A handle's buffers, with their sizes so they can go back to the cache.
template <class T>
hipError_t handle_alloc(srt_bvh* b, T** p, size_t bytes)
{
    void* q = nullptr;
    const hipError_t e = block_cache().get(&q, bytes);
    *p = static_cast<T*>(e == hipSuccess ? q : nullptr);
    if (e == hipSuccess) b->blocks.push_back({q, bytes});
    return e;
}

struct DevAlloc {
    hipStream_t stream;
    std::vector<std::pair<void*, size_t>> blocks;
    explicit DevAlloc(hipStream_t s) : stream(s) {}
    template <class T>
    hipError_t get(T** p, size_t bytes)
    {
        void* q = nullptr;
        const hipError_t e = block_cache().get(&q, bytes);
        if (e == hipSuccess) blocks.push_back({q, bytes});
        *p = static_cast<T*>(q);
        return e;
    }
    ~DevAlloc()
    {
        // no kernel of the build may still use a block handed back (a no-op
        // wait on the success path, which has synchronised already)
        (void)hipStreamSynchronize(stream);
        for (auto& b : blocks) block_cache().put(b.first, b.second);
    }
};

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)std::max<int64_t>(1, (n + bs - 1) / bs); }

constexpr int kMaxLevels = 512;   // far above the depth of any tree of <= 2^28 Gaussians
constexpr int kLevelBatch = 8;    // levels launched between two host checks

template <int W>
srt_status collapse_all(hipStream_t s, DevAlloc& tmp, const BinTree& t, int64_t n, int L,
                        const uint32_t* order, const float* lo, const float* hi,
                        WideNode<W>* nodes, int64_t* num_nodes, int32_t* depth,
                        int32_t** level_nodes_out, std::vector<uint32_t>& level_off,
                        std::vector<uint32_t>& level_cnt)
{
    Task *qa = nullptr, *qb = nullptr;
    uint32_t* ctr = nullptr;  // see k_collapse
    uint32_t *lvl_cnt = nullptr, *lvl_base = nullptr;
    int32_t* level_nodes = nullptr;
    SRT_HIP_TRY(tmp.get(&qa, sizeof(Task) * (size_t)n));
    SRT_HIP_TRY(tmp.get(&qb, sizeof(Task) * (size_t)n));
    SRT_HIP_TRY(tmp.get(&ctr, 4 * sizeof(uint32_t)));
    SRT_HIP_TRY(tmp.get(&lvl_cnt, kMaxLevels * sizeof(uint32_t)));
    SRT_HIP_TRY(tmp.get(&lvl_base, kMaxLevels * sizeof(uint32_t)));
    SRT_HIP_TRY(tmp.get(&level_nodes, sizeof(int32_t) * (size_t)n));
    const Task root{0, 0};
    const uint32_t init[4] = {1u, 0u, 1u, 0u};
    SRT_HIP_TRY(hipMemcpyAsync(qa, &root, sizeof(Task), hipMemcpyHostToDevice, s));
    SRT_HIP_TRY(hipMemcpyAsync(ctr, init, sizeof(init), hipMemcpyHostToDevice, s));
    // Levels run back to back without a host round trip; the host looks at
    // the task count only every kLevelBatch levels (launches past the last
    // level find no tasks and return at once). A level holds at most W^l tasks.
    int levels = 0;
    int64_t bound = 1;
    for (;;) {
        if (levels + kLevelBatch > kMaxLevels) return SRT_ERR_HIP;  // not for a valid tree
        for (int b = 0; b < kLevelBatch; ++b, ++levels) {
            k_collapse<W><<<blocks_for(bound, 128), 128, 0, s>>>(t, L, qa, ctr, qb, nodes,
                                                                 level_nodes);
            SRT_HIP_TRY(hipGetLastError());
            k_advance<<<1, 1, 0, s>>>(ctr, lvl_cnt, lvl_base, levels);
            SRT_HIP_TRY(hipGetLastError());
            std::swap(qa, qb);
            bound = std::min<int64_t>(bound * W, n);
        }
        uint32_t pending = 0;
        SRT_HIP_TRY(hipMemcpyAsync(&pending, ctr, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        SRT_HIP_TRY(hipStreamSynchronize(s));
        if (pending == 0) break;
    }
    std::vector<uint32_t> cnt(levels), base(levels);
    uint32_t made = 0;
    SRT_HIP_TRY(hipMemcpyAsync(cnt.data(), lvl_cnt, sizeof(uint32_t) * levels,
                               hipMemcpyDeviceToHost, s));
    SRT_HIP_TRY(hipMemcpyAsync(base.data(), lvl_base, sizeof(uint32_t) * levels,
                               hipMemcpyDeviceToHost, s));
    SRT_HIP_TRY(hipMemcpyAsync(&made, ctr + 2, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SRT_HIP_TRY(hipStreamSynchronize(s));
    level_off.clear();
    level_cnt.clear();
    for (int l = 0; l < levels && cnt[l] > 0; ++l) {
        level_off.push_back(base[l]);
        level_cnt.push_back(cnt[l]);
    }
    *num_nodes = made;
    for (size_t lv = level_off.size(); lv-- > 0;) {
        k_wide_boxes<W><<<blocks_for(level_cnt[lv], 128), 128, 0, s>>>(
            level_nodes + level_off[lv], level_cnt[lv], order, lo, hi, nodes);
        SRT_HIP_TRY(hipGetLastError());
    }
    *depth = (int32_t)level_off.size();
    *level_nodes_out = level_nodes;
    return SRT_OK;
}

// Fill every wide node's boxes from the Gaussian boxes, deepest level first.
template <int W>
srt_status fill_boxes(const srt_bvh* b, hipStream_t s)
{
    WideNode<W>* nodes = static_cast<WideNode<W>*>(b->nodes);
    if (b->level_cnt.empty()) {
        k_single_leaf<W><<<1, 1, 0, s>>>(b->G, b->box_lo, b->box_hi, nodes);
        SRT_HIP_TRY(hipGetLastError());
        return SRT_OK;
    }
    const uint32_t* order = reinterpret_cast<const uint32_t*>(b->leaf_order);
    for (size_t lv = b->level_off.size(); lv-- > 0;) {
        k_wide_boxes<W><<<blocks_for(b->level_cnt[lv], 128), 128, 0, s>>>(
            b->level_nodes + b->level_off[lv], b->level_cnt[lv], order, b->box_lo, b->box_hi,
            nodes);
        SRT_HIP_TRY(hipGetLastError());
    }
    return SRT_OK;
}

// Largest bounding-sphere radius of the records (synchronises the stream).
srt_status read_r_max(srt_bvh* b, hipStream_t s)
{
    const uint32_t binit[8] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u, 0u, 0u};
    SRT_HIP_TRY(hipMemcpyAsync(b->bounds, binit, sizeof(binit), hipMemcpyHostToDevice, s));
    k_centre_bounds<<<std::min<unsigned>(blocks_for(b->G, 256), 1024u), 256, 0, s>>>(
        b->G, b->box_lo, b->box_hi, b->recs, b->bounds);
    SRT_HIP_TRY(hipGetLastError());
    uint32_t rmax_bits = 0;
    SRT_HIP_TRY(hipMemcpyAsync(&rmax_bits, b->bounds + 6, sizeof(uint32_t), hipMemcpyDeviceToHost,
                               s));
    SRT_HIP_TRY(hipStreamSynchronize(s));
    memcpy(&b->r_max, &rmax_bits, sizeof(float));
    return SRT_OK;
}

// Refit (same topology and leaf order): new records and Gaussian boxes from
// the scene's current parameters, then every node box bottom-up.
template <int W>
srt_status refit_impl(srt_bvh* b, const srt_scene* sc, hipStream_t s)
{
    const int64_t G = b->G;
    b->sh = sc->sh;
    if (G == 0) return SRT_OK;
    k_refit_records<<<blocks_for(G, 256), 256, 0, s>>>(G, b->leaf_order, sc->means,
                                                       sc->log_scales, sc->quats,
                                                       sc->opacity_logits, b->recs, b->box_lo,
                                                       b->box_hi);
    SRT_HIP_TRY(hipGetLastError());
    const srt_status st = fill_boxes<W>(b, s);
    if (st != SRT_OK) return st;
    return read_r_max(b, s);
}

template <int W>
srt_status build_impl(const srt_scene* sc, int L, int size_split, hipStream_t s, srt_bvh* b)
{
    const int64_t G = sc->num_gaussians;
    DevAlloc tmp(s);
    if (G == 0) {
        WideNode<W>* nodes = nullptr;
        SRT_HIP_TRY(handle_alloc(b, &nodes, sizeof(WideNode<W>)));
        b->nodes = nodes;
        k_single_leaf<W><<<1, 1, 0, s>>>(0, nullptr, nullptr, nodes);
        SRT_HIP_TRY(hipGetLastError());
        b->num_nodes = 1;
        b->depth = 1;
        b->bytes = sizeof(WideNode<W>);
        SRT_HIP_TRY(hipStreamSynchronize(s));
        return SRT_OK;
    }
    Record* recs_id = nullptr;
    SRT_HIP_TRY(tmp.get(&recs_id, sizeof(Record) * (size_t)G));
    SRT_HIP_TRY(handle_alloc(b, &b->box_lo, sizeof(float) * 3 * (size_t)G));
    SRT_HIP_TRY(handle_alloc(b, &b->box_hi, sizeof(float) * 3 * (size_t)G));
    SRT_HIP_TRY(handle_alloc(b, &b->recs, sizeof(Record) * (size_t)G));
    SRT_HIP_TRY(handle_alloc(b, &b->leaf_order, sizeof(int32_t) * (size_t)G));
    SRT_HIP_TRY(handle_alloc(b, &b->leaf_pos, sizeof(int32_t) * (size_t)G));
    b->bytes = (int64_t)(sizeof(float) * 6 + sizeof(Record) + 2 * sizeof(int32_t)) * G;

    k_preprocess<<<blocks_for(G, 256), 256, 0, s>>>(G, sc->means, sc->log_scales, sc->quats,
                                                    sc->opacity_logits, recs_id, b->box_lo,
                                                    b->box_hi);
    SRT_HIP_TRY(hipGetLastError());

    SRT_HIP_TRY(handle_alloc(b, &b->bounds, 8 * sizeof(uint32_t)));
    uint32_t* bounds = b->bounds;
    const uint32_t binit[8] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u, 0u, 0u};
    SRT_HIP_TRY(hipMemcpyAsync(bounds, binit, sizeof(binit), hipMemcpyHostToDevice, s));
    k_centre_bounds<<<std::min<unsigned>(blocks_for(G, 256), 1024u), 256, 0, s>>>(
        G, b->box_lo, b->box_hi, recs_id, bounds);
    SRT_HIP_TRY(hipGetLastError());

    uint64_t *keys = nullptr, *keys_sorted = nullptr;
    uint32_t *idx = nullptr, *order = nullptr;
    SRT_HIP_TRY(tmp.get(&keys, sizeof(uint64_t) * (size_t)G));
    SRT_HIP_TRY(tmp.get(&keys_sorted, sizeof(uint64_t) * (size_t)G));
    SRT_HIP_TRY(tmp.get(&idx, sizeof(uint32_t) * (size_t)G));
    SRT_HIP_TRY(tmp.get(&order, sizeof(uint32_t) * (size_t)G));
    k_morton<<<blocks_for(G, 256), 256, 0, s>>>(G, b->box_lo, b->box_hi, bounds, size_split, keys,
                                                idx);
    SRT_HIP_TRY(hipGetLastError());
    size_t sort_bytes = 0;
    SRT_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, keys, keys_sorted, idx,
                                                   order, (int)G, 0, 63, s));
    void* sort_tmp = nullptr;
    SRT_HIP_TRY(tmp.get(&sort_tmp, sort_bytes));
    SRT_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(sort_tmp, sort_bytes, keys, keys_sorted, idx,
                                                   order, (int)G, 0, 63, s));

    k_permute<<<blocks_for(G, 256), 256, 0, s>>>(G, order, recs_id, b->recs, b->leaf_order,
                                                 b->leaf_pos);
    SRT_HIP_TRY(hipGetLastError());

    WideNode<W>* nodes_max = nullptr;
    int64_t num_nodes = 1;
    int32_t depth = 1;
    if (G <= L) {
        SRT_HIP_TRY(tmp.get(&nodes_max, sizeof(WideNode<W>)));
        k_single_leaf<W><<<1, 1, 0, s>>>(G, b->box_lo, b->box_hi, nodes_max);
        SRT_HIP_TRY(hipGetLastError());
    } else {
        const int n = (int)G;
        int32_t *left, *right, *parent, *leaf_parent, *first, *last;
        SRT_HIP_TRY(tmp.get(&left, sizeof(int32_t) * (n - 1)));
        SRT_HIP_TRY(tmp.get(&right, sizeof(int32_t) * (n - 1)));
        SRT_HIP_TRY(tmp.get(&parent, sizeof(int32_t) * (n - 1)));
        SRT_HIP_TRY(tmp.get(&first, sizeof(int32_t) * (n - 1)));
        SRT_HIP_TRY(tmp.get(&last, sizeof(int32_t) * (n - 1)));
        SRT_HIP_TRY(tmp.get(&leaf_parent, sizeof(int32_t) * n));
        k_karras<<<blocks_for(n - 1, 256), 256, 0, s>>>(n, keys_sorted, left, right, parent,
                                                        leaf_parent, first, last);
        SRT_HIP_TRY(hipGetLastError());
        SRT_HIP_TRY(tmp.get(&nodes_max, sizeof(WideNode<W>) * (size_t)(n - 1)));
        const BinTree t{left, right, first, last};
        int32_t* lvl = nullptr;
        const srt_status st = collapse_all<W>(s, tmp, t, n, L, order, b->box_lo, b->box_hi,
                                              nodes_max, &num_nodes, &depth, &lvl, b->level_off,
                                              b->level_cnt);
        if (st != SRT_OK) return st;
        const size_t listed = (size_t)b->level_off.back() + b->level_cnt.back();
        SRT_HIP_TRY(handle_alloc(b, &b->level_nodes, sizeof(int32_t) * listed));
        SRT_HIP_TRY(hipMemcpyAsync(b->level_nodes, lvl, sizeof(int32_t) * listed,
                                   hipMemcpyDeviceToDevice, s));
        b->bytes += (int64_t)(sizeof(int32_t) * listed);
    }
    WideNode<W>* nodes = nullptr;
    SRT_HIP_TRY(handle_alloc(b, &nodes, sizeof(WideNode<W>) * (size_t)num_nodes));
    b->nodes = nodes;
    SRT_HIP_TRY(hipMemcpyAsync(nodes, nodes_max, sizeof(WideNode<W>) * (size_t)num_nodes,
                               hipMemcpyDeviceToDevice, s));
    // start subtrees two levels above each leaf: measured on the 1M mix's
    // shadow rays against 1, 3, 4 and 6 levels and against walks from the root
    b->start_levels = kStartLevels;
    if (G > L) {
        int32_t *parent = nullptr, *leaf_node = nullptr;
        SRT_HIP_TRY(tmp.get(&parent, sizeof(int32_t) * (size_t)num_nodes));
        SRT_HIP_TRY(tmp.get(&leaf_node, sizeof(int32_t) * (size_t)G));
        SRT_HIP_TRY(handle_alloc(b, &b->start_node, sizeof(int32_t) * (size_t)G));
        b->bytes += (int64_t)sizeof(int32_t) * G;
        k_node_parents<W><<<blocks_for(num_nodes, 256), 256, 0, s>>>(nodes, num_nodes, parent,
                                                                      leaf_node);
        SRT_HIP_TRY(hipGetLastError());
        k_start_nodes<<<blocks_for(G, 256), 256, 0, s>>>(G, b->start_levels, b->leaf_pos,
                                                         leaf_node, parent, b->start_node);
        SRT_HIP_TRY(hipGetLastError());
    }
    uint32_t rmax_bits = 0;
    SRT_HIP_TRY(hipMemcpyAsync(&rmax_bits, bounds + 6, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SRT_HIP_TRY(hipStreamSynchronize(s));
    memcpy(&b->r_max, &rmax_bits, sizeof(float));
    b->num_nodes = num_nodes;
    b->depth = depth;
    b->bytes += (int64_t)sizeof(WideNode<W>) * num_nodes;
    return SRT_OK;
}

}  // namespace

namespace srt {
void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s)
{
    if (n == 0) return;
    k_fill_u32<<<(unsigned)std::min<size_t>((n + 255) / 256, 1024), 256, 0, s>>>(p, v, n);
}
}  // namespace srt

extern "C" {

const char* srt_status_str(srt_status s)
{
    switch (s) {
    case SRT_OK: return "SRT_OK";
    case SRT_ERR_INVALID_ARG: return "SRT_ERR_INVALID_ARG";
    case SRT_ERR_OOM: return "SRT_ERR_OOM";
    case SRT_ERR_HIP: return "SRT_ERR_HIP";
    case SRT_ERR_UNSUPPORTED: return "SRT_ERR_UNSUPPORTED";
    case SRT_ERR_WORKSPACE: return "SRT_ERR_WORKSPACE";
    }
    return "SRT_ERR_UNKNOWN";
}

int32_t srt_version(void) { return 10000; }

srt_status srt_set_memory_limit(int64_t bytes)
{
    if (bytes < 0) return SRT_ERR_INVALID_ARG;
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    c.limit = (size_t)bytes;
    return SRT_OK;
}

srt_status srt_memory_stats(int64_t* in_use, int64_t* cached)
{
    if (!in_use && !cached) return SRT_ERR_INVALID_ARG;
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    if (in_use) *in_use = (int64_t)c.in_use;
    if (cached) *cached = (int64_t)c.kept;
    return SRT_OK;
}

srt_status srt_build_bvh(const srt_scene* sc, const srt_build_opts* opts, void* stream,
                         srt_bvh** out)
{
    const srt::Range range_("srt_build_bvh");
    if (!sc || !opts || !out) return SRT_ERR_INVALID_ARG;
    *out = nullptr;
    const int64_t G = sc->num_gaussians;
    if (G < 0 || G > (int64_t(1) << 28)) return SRT_ERR_INVALID_ARG;
    if (sc->sh_degree < 0 || sc->sh_degree > 3) return SRT_ERR_INVALID_ARG;
    if (G > 0 && (!sc->means || !sc->log_scales || !sc->quats || !sc->opacity_logits || !sc->sh))
        return SRT_ERR_INVALID_ARG;
    if (opts->width != 2 && opts->width != 4 && opts->width != 8) return SRT_ERR_INVALID_ARG;
    if (opts->leaf_size < 1 || opts->leaf_size > 8) return SRT_ERR_INVALID_ARG;
    if (opts->size_split < 0 || opts->size_split > 16) return SRT_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    srt_bvh* b = new srt_bvh();
    b->G = G;
    b->W = opts->width;
    b->L = opts->leaf_size;
    b->deg = sc->sh_degree;
    b->sh = sc->sh;
    srt_status st = SRT_ERR_INVALID_ARG;
    switch (b->W) {
    case 2: st = build_impl<2>(sc, b->L, opts->size_split, s, b); break;
    case 4: st = build_impl<4>(sc, b->L, opts->size_split, s, b); break;
    case 8: st = build_impl<8>(sc, b->L, opts->size_split, s, b); break;
    }
    if (st != SRT_OK) {
        (void)hipStreamSynchronize(s);
        srt_destroy_bvh(b);
        return st;
    }
    *out = b;
    return SRT_OK;
}

void srt_destroy_bvh(srt_bvh* b)
{
    if (!b) return;
    for (auto& blk : b->blocks) block_cache().put(blk.first, blk.second);
    delete b;
}

srt_status srt_refit_bvh(srt_bvh* b, const srt_scene* sc, void* stream)
{
    const srt::Range range_("srt_refit_bvh");
    if (!b || !sc) return SRT_ERR_INVALID_ARG;
    if (sc->num_gaussians != b->G || sc->sh_degree != b->deg) return SRT_ERR_INVALID_ARG;
    if (b->G > 0 && (!sc->means || !sc->log_scales || !sc->quats || !sc->opacity_logits || !sc->sh))
        return SRT_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (b->W) {
    case 2: return refit_impl<2>(b, sc, s);
    case 4: return refit_impl<4>(b, sc, s);
    case 8: return refit_impl<8>(b, sc, s);
    }
    return SRT_ERR_INVALID_ARG;
}

srt_status srt_bvh_get_info(const srt_bvh* b, srt_bvh_info* info)
{
    if (!b || !info) return SRT_ERR_INVALID_ARG;
    info->num_gaussians = b->G;
    info->num_nodes = b->num_nodes;
    info->width = b->W;
    info->leaf_size = b->L;
    info->depth = b->depth;
    info->sh_degree = b->deg;
    info->device_bytes = b->bytes;
    return SRT_OK;
}

srt_status srt_bvh_records(const srt_bvh* b, float* mu, float* M, float* opacity, float* box_lo,
                           float* box_hi, void* stream)
{
    if (!b) return SRT_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (b->G == 0) return SRT_OK;
    if (mu || M || opacity) {
        k_unpermute_records<<<blocks_for(b->G, 256), 256, 0, s>>>(b->G, b->recs, mu, M, opacity);
        SRT_HIP_TRY(hipGetLastError());
    }
    const size_t bytes = sizeof(float) * 3 * (size_t)b->G;
    if (box_lo) SRT_HIP_TRY(hipMemcpyAsync(box_lo, b->box_lo, bytes, hipMemcpyDeviceToDevice, s));
    if (box_hi) SRT_HIP_TRY(hipMemcpyAsync(box_hi, b->box_hi, bytes, hipMemcpyDeviceToDevice, s));
    return SRT_OK;
}

srt_status srt_bvh_nodes(const srt_bvh* b, void* nodes, int32_t* leaf_order, void* stream)
{
    if (!b) return SRT_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (nodes)
        SRT_HIP_TRY(hipMemcpyAsync(nodes, b->nodes, (size_t)b->num_nodes * 32 * (size_t)b->W,
                                   hipMemcpyDeviceToDevice, s));
    if (leaf_order && b->G > 0)
        SRT_HIP_TRY(hipMemcpyAsync(leaf_order, b->leaf_order, sizeof(int32_t) * (size_t)b->G,
                                   hipMemcpyDeviceToDevice, s));
    return SRT_OK;
}

}  // extern "C"
