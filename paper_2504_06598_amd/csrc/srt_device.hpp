// Device-side building blocks of libsrt (gfx950 / CDNA4).
//
// Data layout in HBM:
//   Record      64 B per Gaussian, leaf order: mu(3) M(9) opacity gid pad(2).
//               M = S^-1 R^T is the whitening matrix of the Gaussian
//               (eqn "gaussian"), so q(x) = |M (x - mu)|^2.
//   WideNode<W> 32*W bytes: lo_x[W] lo_y[W] lo_z[W] hi_x[W] hi_y[W] hi_z[W]
//               child[W], padded; W = 2/4/8 gives 64/128/256 B, one or two
//               128-B cache lines, loaded as 16-B vectors.
//   child >= 0: wide-node index; child < 0: leaf ~((first << 3) | (count-1))
//   over the leaf-ordered records; empty slots have an inverted box.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace srt {

// Squared k-sigma radius of the bounding ellipsoid, s = 2 sqrt 2 (eqn "cuboid").
constexpr double kEllipsoidQ = 8.0;

struct alignas(16) Record {
    float mu[3];
    float M[9];
    float opacity;
    int32_t gid;
    float pad[2];
};
static_assert(sizeof(Record) == 64, "record is one 64-B line");

template <int W>
struct alignas(16) WideNode {
    float lo[3][W];
    float hi[3][W];
    int32_t child[W];
    int32_t pad[W];
};
static_assert(sizeof(WideNode<4>) == 128, "BVH4 node is 128 B");

// Number of 16-B vectors that hold the used part of a node.
template <int W>
struct NodeVecs {
    static constexpr int value = (28 * W + 15) / 16;
};

template <int W>
struct NodeBuf {
    struct {
        float lo[3][W];
        float hi[3][W];
        int32_t child[W];
    } n;
};

template <int W>
__device__ __forceinline__ void load_node(const WideNode<W>* nodes, int32_t idx, NodeBuf<W>& b)
{
    constexpr int NV = NodeVecs<W>::value;
    const float4* p = reinterpret_cast<const float4*>(nodes + idx);
    float f[4 * NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const float4 v = p[i];
        f[4 * i] = v.x;
        f[4 * i + 1] = v.y;
        f[4 * i + 2] = v.z;
        f[4 * i + 3] = v.w;
    }
#pragma unroll
    for (int c = 0; c < W; ++c) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            b.n.lo[a][c] = f[a * W + c];
            b.n.hi[a][c] = f[(3 + a) * W + c];
        }
        b.n.child[c] = __float_as_int(f[6 * W + c]);
    }
}

// Child reference of slot `slot`, selected with bit masks: a select between
// two loads of the register-resident node can be folded by the compiler into
// a load through a selected address, which spills the node to scratch.
template <int W>
__device__ __forceinline__ int32_t child_at(const NodeBuf<W>& b, uint32_t slot)
{
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < W; ++j) c |= (uint32_t)b.n.child[j] & (0u - (uint32_t)(slot == (uint32_t)j));
    return (int32_t)c;
}

__device__ __forceinline__ bool ref_is_leaf(int32_t c) { return c < 0; }
__device__ __forceinline__ uint32_t leaf_first(int32_t c) { return ((uint32_t)~c) >> 3; }
__device__ __forceinline__ uint32_t leaf_count(int32_t c) { return (((uint32_t)~c) & 7u) + 1u; }
__host__ __device__ __forceinline__ int32_t make_leaf(uint32_t first, uint32_t count)
{
    return (int32_t)~((first << 3) | (count - 1u));
}
constexpr int32_t kEmptyChild = 0x7FFFFFFF;

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with Weyl-sequence key bumps between rounds.
// --------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 product each (a single v_mad_u64_u32 instead of a
        // separate low and high multiply)
        const uint64_t pa = (uint64_t)0xD2511F53u * c.x;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(pb >> 32) ^ c.y ^ k0, (uint32_t)pb,
                       (uint32_t)(pa >> 32) ^ c.w ^ k1, (uint32_t)pa);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ uint32_t word_of(const uint4& w, uint32_t i)
{
    return i == 0 ? w.x : i == 1 ? w.y : i == 2 ? w.z : w.w;
}

// u in [0, 1 - 2^-24], exact in FP32 and FP64.
__device__ __forceinline__ double u_of_word(uint32_t w) { return (double)(w >> 8) * 0x1p-24; }

// The paper's stateless trigonometric hash of a point (Sec. 4.2, eqns "hash"
// and "rng", its coefficients), in FP32 as a shader evaluates it:
// r1(q) = fract(b1 sin(a1 q)), r2(q) = fract(b2 sin(a2 . q)), xi(p) =
// r2(p_xy + r1(p_z)). Both components of b2 are equal, so r2's two outputs
// are equal and one is used. In FP32, b2 sin(.) ~ 4e4 leaves fract about 8
// fractional bits; the hash's statistics, not its bits, are what it offers.
__device__ __forceinline__ float fract(float v) { return v - floorf(v); }

__device__ __forceinline__ float trig_hash(float px, float py, float pz)
{
    const float r1 = fract(47453.5453f * sinf(91.3458f * pz));
    const float x = px + r1, y = py + r1;
    return fract(43758.5453f * sinf(12.9898f * x + 78.233f * y));
}

// The acceptance test u < alpha = opacity * exp(-q / 2) (eqn "rr") in FP64,
// for u from a Philox word (exact 24-bit) or a float. (An FP32 alpha with an
// exact FP64 fallback band measured slower on gfx950 than the FP64 exp.)
struct AlphaTest {
    double alpha;

    __device__ __forceinline__ AlphaTest(float op, double q) : alpha((double)op * exp(-0.5 * q)) {}

    __device__ __forceinline__ bool accepts(uint32_t word) const { return u_of_word(word) < alpha; }

    __device__ __forceinline__ bool accepts_u(float u) const { return (double)u < alpha; }
};

// --------------------------------------------------------------------------
// Real spherical harmonics up to degree 3 at a unit direction, orthonormal,
// Condon-Shortley phase, index l*l + l + m (m = -l..l).
// --------------------------------------------------------------------------
__device__ __forceinline__ void sh_eval(int deg, float x, float y, float z, float* Y)
{
    Y[0] = 0.28209479177387814f;
    if (deg < 1) return;
    const float k1 = 0.48860251190291987f;
    Y[1] = -k1 * y;
    Y[2] = k1 * z;
    Y[3] = -k1 * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    const float xy = x * y, yz = y * z, xz = x * z;
    Y[4] = 1.0925484305920792f * xy;
    Y[5] = -1.0925484305920792f * yz;
    Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);
    Y[7] = -1.0925484305920792f * xz;
    Y[8] = 0.54627421529603959f * (xx - yy);
    if (deg < 3) return;
    Y[9] = -0.59004358992664352f * y * (3.0f * xx - yy);
    Y[10] = 2.8906114426405538f * xy * z;
    Y[11] = -0.45704579946446577f * y * (4.0f * zz - xx - yy);
    Y[12] = 0.3731763325901154f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -0.45704579946446577f * x * (4.0f * zz - xx - yy);
    Y[14] = 1.4453057213202769f * z * (xx - yy);
    Y[15] = -0.59004358992664352f * x * (xx - 3.0f * yy);
}

// Makes x opaque to the optimiser so that code using it is not hoisted out
// of the loop it sits in (keeps e.g. the SH basis from living through a
// whole traversal and costing registers there).
__device__ __forceinline__ float opaque(float x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Unclamped SH colour sum of Gaussian gid (0.5 + sum k Y).
__device__ __forceinline__ float3 sh_colour_pre(const float* sh, int deg, int32_t gid, const float* Y)
{
    const int K = (deg + 1) * (deg + 1);
    const float* p = sh + (size_t)gid * (size_t)(3 * K);
    float r = 0.5f, g = 0.5f, b = 0.5f;
    for (int j = 0; j < K; ++j) {
        r = fmaf(p[3 * j + 0], Y[j], r);
        g = fmaf(p[3 * j + 1], Y[j], g);
        b = fmaf(p[3 * j + 2], Y[j], b);
    }
    return make_float3(r, g, b);
}

__device__ __forceinline__ float3 clamp0(float3 c)
{
    return make_float3(fmaxf(c.x, 0.0f), fmaxf(c.y, 0.0f), fmaxf(c.z, 0.0f));
}

// --------------------------------------------------------------------------
// Ray state and the conservative slab test.
// Node culling only has to be conservative: a box that contains a valid
// candidate's 1D-Gaussian mean must never be culled. The FP32 box contains
// the FP64 ellipsoid (rounded outward); Ize's robust factor 1 + 2*gamma_3 on
// the exit distance covers the slab arithmetic; the depth cut carries a
// 2^-20 relative slack, far above the few-ulp error of the entry distance.
// --------------------------------------------------------------------------
constexpr float kIzeFactor = 1.0000003576278687f;  // 1 + 2 gamma_3, gamma_3 = 3u/(1-3u)
constexpr float kCutSlack = 1.00000095367431641f;  // 1 + 2^-20

// One ray, all FP32 (the FP64 candidate test converts on use, so no FP64
// copy stays live during the traversal).
struct Ray {
    float ox, oy, oz;
    float dx, dy, dz;
    float ix, iy, iz;  // 1 / d, with |d_i| clamped away from 0
    float tmin;        // boxes exiting before it are culled: the ray's tmin,
                       // lowered by the depth slack in centre-depth mode
    float inv_dd;      // 1 / |d|^2
    float inv_len;     // 1 / |d|
};

__device__ __forceinline__ float safe_inv(float d)
{
    const float a = fabsf(d) < 1e-20f ? copysignf(1e-20f, d) : d;
    return 1.0f / a;
}

__device__ __forceinline__ Ray make_ray(float ox, float oy, float oz, float dx, float dy, float dz,
                                        float tmin)
{
    Ray r;
    r.ox = ox;
    r.oy = oy;
    r.oz = oz;
    r.dx = dx;
    r.dy = dy;
    r.dz = dz;
    r.ix = safe_inv(dx);
    r.iy = safe_inv(dy);
    r.iz = safe_inv(dz);
    r.tmin = tmin;
    const float dd = dx * dx + dy * dy + dz * dz;
    r.inv_dd = 1.0f / dd;
    r.inv_len = 1.0f / sqrtf(dd);
    return r;
}

// Hit mask and near-to-far sort keys of the W children of a node.
template <int W>
__device__ __forceinline__ void slab_keys(const NodeBuf<W>& b, const Ray& r, float tcut,
                                          uint32_t key[W])
{
#pragma unroll
    for (int c = 0; c < W; ++c) {
        const float ax = (b.n.lo[0][c] - r.ox) * r.ix, bx = (b.n.hi[0][c] - r.ox) * r.ix;
        const float ay = (b.n.lo[1][c] - r.oy) * r.iy, by = (b.n.hi[1][c] - r.oy) * r.iy;
        const float az = (b.n.lo[2][c] - r.oz) * r.iz, bz = (b.n.hi[2][c] - r.oz) * r.iz;
        const float t0 = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fminf(az, bz));
        const float t1 = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fmaxf(az, bz)) * kIzeFactor;
        const bool hit = (t0 <= t1) & (t0 <= tcut) & (t1 >= r.tmin) & (b.n.child[c] != kEmptyChild);
        const float tn = fmaxf(t0, 0.0f);
        key[c] = hit ? ((__float_as_uint(tn) & ~7u) | (uint32_t)c) : 0xFFFFFFFFu;
    }
}

// Entry depth of each child box (clamped at 0), or +inf where the ray misses
// it or enters beyond tcut; the same test as slab_keys.
template <int W>
__device__ __forceinline__ void slab_entry(const NodeBuf<W>& b, const Ray& r, float tcut,
                                           float te[W])
{
#pragma unroll
    for (int c = 0; c < W; ++c) {
        const float ax = (b.n.lo[0][c] - r.ox) * r.ix, bx = (b.n.hi[0][c] - r.ox) * r.ix;
        const float ay = (b.n.lo[1][c] - r.oy) * r.iy, by = (b.n.hi[1][c] - r.oy) * r.iy;
        const float az = (b.n.lo[2][c] - r.oz) * r.iz, bz = (b.n.hi[2][c] - r.oz) * r.iz;
        const float t0 = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fminf(az, bz));
        const float t1 = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fmaxf(az, bz)) * kIzeFactor;
        const bool hit = (t0 <= t1) & (t0 <= tcut) & (t1 >= r.tmin) & (b.n.child[c] != kEmptyChild);
        te[c] = hit ? fminf(fmaxf(t0, 0.0f), 0x1.fffffep127f) : INFINITY;
    }
}

__device__ __forceinline__ void cswap(uint32_t& a, uint32_t& b)
{
    const uint32_t lo = min(a, b), hi = max(a, b);
    a = lo;
    b = hi;
}

// Ascending sort of W keys (optimal networks for 2, 4 and 8 inputs).
template <int W>
__device__ __forceinline__ void sort_keys(uint32_t k[W]);

template <>
__device__ __forceinline__ void sort_keys<2>(uint32_t k[2])
{
    cswap(k[0], k[1]);
}

template <>
__device__ __forceinline__ void sort_keys<4>(uint32_t k[4])
{
    cswap(k[0], k[1]);
    cswap(k[2], k[3]);
    cswap(k[0], k[2]);
    cswap(k[1], k[3]);
    cswap(k[1], k[2]);
}

template <>
__device__ __forceinline__ void sort_keys<8>(uint32_t k[8])
{
    cswap(k[0], k[2]); cswap(k[1], k[3]); cswap(k[4], k[6]); cswap(k[5], k[7]);
    cswap(k[0], k[4]); cswap(k[1], k[5]); cswap(k[2], k[6]); cswap(k[3], k[7]);
    cswap(k[0], k[1]); cswap(k[2], k[3]); cswap(k[4], k[5]); cswap(k[6], k[7]);
    cswap(k[2], k[4]); cswap(k[3], k[5]);
    cswap(k[1], k[4]); cswap(k[3], k[6]);
    cswap(k[1], k[2]); cswap(k[3], k[4]); cswap(k[5], k[6]);
}

// --------------------------------------------------------------------------
// Candidate test in FP64 (Sec. 3.1 and eqn "cuboid"): the ray x(t) = o + t d
// cuts the Gaussian in a 1D Gaussian with mean t* = -(o'.d')/(d'.d'), where
// o' = M (o - mu) and d' = M d; q = |o' + t* d'|^2 and alpha = o exp(-q/2).
// --------------------------------------------------------------------------
struct Isect {
    double t, q;
    double p[3];  // whitened position at t*
};

// t*, q and the whitened position p = M (x(t*) - mu).
__device__ __forceinline__ void isect_tqp(const Record& r, const Ray& ray, double& t_out,
                                          double& q_out, double p[3])
{
    const double wx = (double)ray.ox - (double)r.mu[0];
    const double wy = (double)ray.oy - (double)r.mu[1];
    const double wz = (double)ray.oz - (double)r.mu[2];
    const double dx = ray.dx, dy = ray.dy, dz = ray.dz;
    double op[3], dp[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double m0 = r.M[3 * i], m1 = r.M[3 * i + 1], m2 = r.M[3 * i + 2];
        op[i] = fma(m2, wz, fma(m1, wy, m0 * wx));
        dp[i] = fma(m2, dz, fma(m1, dy, m0 * dx));
    }
    const double dd = fma(dp[2], dp[2], fma(dp[1], dp[1], dp[0] * dp[0]));
    const double od = fma(op[2], dp[2], fma(op[1], dp[1], op[0] * dp[0]));
    const double t = -od / dd;
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] = fma(t, dp[i], op[i]);
    t_out = t;
    q_out = fma(p[2], p[2], fma(p[1], p[1], p[0] * p[0]));
}

// Only t and q (the forward needs nothing else).
__device__ __forceinline__ void isect_tq(const Record& r, const Ray& ray, double& t_out,
                                         double& q_out)
{
    double p[3];
    isect_tqp(r, ray, t_out, q_out, p);
}

__device__ __forceinline__ Record load_record(const Record* recs, uint32_t i)
{
    const float4* p = reinterpret_cast<const float4*>(recs + i);
    const float4 a = p[0], b = p[1], c = p[2], d = p[3];
    Record r;
    r.mu[0] = a.x; r.mu[1] = a.y; r.mu[2] = a.z; r.M[0] = a.w;
    r.M[1] = b.x; r.M[2] = b.y; r.M[3] = b.z; r.M[4] = b.w;
    r.M[5] = c.x; r.M[6] = c.y; r.M[7] = c.z; r.M[8] = c.w;
    r.opacity = d.x; r.gid = __float_as_int(d.y); r.pad[0] = d.z; r.pad[1] = d.w;
    return r;
}

// True when the record cannot hold a valid candidate of depth in
// [tmin, tcut]: the 1D mean of a valid candidate lies inside the ellipsoid,
// hence inside the sphere of radius pad[0] about mu, so its depth lies
// within radius / |d| of the closest approach tc to mu and the ray passes
// within the radius. FP32 with slack far above its rounding error; a pure
// prefilter of the FP64 test.
__device__ __forceinline__ bool sphere_reject(const Record& r, const Ray& ray, float tmin,
                                              float tcut)
{
    const float wx = r.mu[0] - ray.ox, wy = r.mu[1] - ray.oy, wz = r.mu[2] - ray.oz;
    const float tc = (wx * ray.dx + wy * ray.dy + wz * ray.dz) * ray.inv_dd;
    const float rad = r.pad[0];
    const float rt = rad * ray.inv_len;
    const float slack = 1e-5f * (fabsf(tc) + rt + 1.0f);
    if (tc - rt - slack > tcut || tc + rt + slack < tmin) return true;
    const float cx = wy * ray.dz - wz * ray.dy;
    const float cy = wz * ray.dx - wx * ray.dz;
    const float cz = wx * ray.dy - wy * ray.dx;
    const float c2 = (cx * cx + cy * cy + cz * cz) * ray.inv_dd;  // (distance to mu)^2
    const float rr = rad * 1.0001f + 1e-5f * (fabsf(wx) + fabsf(wy) + fabsf(wz) + 1.0f);
    return c2 > rr * rr;
}

// (t, gid) lexicographic order of depth keys.
__device__ __forceinline__ bool key_less(float ta, int32_t ga, float tb, int32_t gb)
{
    return ta < tb || (ta == tb && ga < gb);
}

// Wave-level sum, then one atomic per wave.
__device__ __forceinline__ void wave_add_u64(unsigned long long* dst, unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, v);
}

// Workgroups of a launch are dispatched to the 8 XCDs in turn (b -> XCD b % 8).
// Renumber them so that each XCD runs one contiguous range of logical
// workgroups: neighbouring rays then share that XCD's L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb)
{
    const uint32_t x = b & 7u, i = b >> 3, q = nb >> 3, r = nb & 7u;
    return x * q + (x < r ? x : r) + i;
}

// Thread t of an image launch -> pixel index in a row-major w x h image, with
// each group of 64 threads on one 8x8 tile (tiles in row-major order); -1 for
// the threads of a partial tile that fall outside the image.
__device__ __forceinline__ int64_t tile_pixel(int64_t t, int32_t w, int64_t h)
{
    const int64_t tiles_x = (w + 7) / 8;
    const int64_t tile = t >> 6;
    const int32_t lane = (int32_t)(t & 63);
    const int64_t x = (tile % tiles_x) * 8 + (lane & 7);
    const int64_t y = (tile / tiles_x) * 8 + (lane >> 3);
    return (x < w && y < h) ? y * w + x : -1;
}

// Threads an image launch needs for w x h pixels.
__host__ __device__ __forceinline__ int64_t tile_threads(int32_t w, int64_t h)
{
    return (int64_t)((w + 7) / 8) * ((h + 7) / 8) * 64;
}

}  // namespace srt
