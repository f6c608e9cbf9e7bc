// The traversal core shared by every kernel of libsrt: a depth-first walk of
// the W-wide BVH that visits hit children near to far and hands each Gaussian
// of a reached leaf to a visitor. Boxes entering beyond the depth cut `tcut`
// (which the visitor may lower) are skipped: the clipping that the paper's
// ReportIntersection applies to the ray (Alg. "intersect").
#pragma once

#include "srt_device.hpp"

namespace srt {

// Per-lane stack with entry i at base[i * stride] (LDS with stride = block
// size keeps the 64 lanes of a wave on distinct banks).
struct FlatStack {
    int32_t* base;
    int stride;
    int cap;
    __device__ __forceinline__ void store(int i, int32_t v) { base[i * stride] = v; }
    __device__ __forceinline__ int32_t load(int i) const { return base[i * stride]; }
};

// Two tiers: the first `lds_cap` entries in LDS, the rest in global memory.
struct TwoTierStack {
    int32_t* lds;
    int lds_stride;
    int lds_cap;
    int32_t* glb;
    int glb_stride;
    int cap;
    __device__ __forceinline__ void store(int i, int32_t v)
    {
        if (i < lds_cap)
            lds[i * lds_stride] = v;
        else
            glb[(i - lds_cap) * glb_stride] = v;
    }
    __device__ __forceinline__ int32_t load(int i) const
    {
        return i < lds_cap ? lds[i * lds_stride] : glb[(i - lds_cap) * glb_stride];
    }
};

enum WalkResult { kWalkDone = 0, kWalkOverflow = 1, kWalkStopped = 2 };

// visit(record_index) -> true stops the walk (any-hit termination). Boxes
// are culled against tcut + slack (slack > 0 when keys are not bounded below
// by box entry; see DepthCtx).
template <int W, class Stack, class Visit>
__device__ __forceinline__ int walk(const WideNode<W>* __restrict__ nodes, const Ray& rf,
                                    float& tcut, float slack, Stack& stk, int64_t max_steps,
                                    uint32_t& n_nodes, uint32_t& n_prims, Visit&& visit)
{
    int sp = 0;
    int32_t node = 0;
    for (int64_t step = 0;; ++step) {
        if (step > max_steps) return kWalkOverflow;
        if (node >= 0) {
            ++n_nodes;
            NodeBuf<W> b;
            load_node<W>(nodes, node, b);
            uint32_t key[W];
            slab_keys<W>(b, rf, tcut + slack, key);
            sort_keys<W>(key);
            int nh = 0;
#pragma unroll
            for (int c = 0; c < W; ++c) nh += key[c] != 0xFFFFFFFFu;
            if (nh > 0) {
                if (sp + nh - 1 > stk.cap) return kWalkOverflow;
#pragma unroll
                for (int c = W - 1; c >= 1; --c)
                    if (key[c] != 0xFFFFFFFFu) {
                        stk.store(sp, child_at<W>(b, key[c] & 7u));
                        ++sp;
                    }
                node = child_at<W>(b, key[0] & 7u);
                continue;
            }
        } else {
            const uint32_t first = leaf_first(node), count = leaf_count(node);
            for (uint32_t i = 0; i < count; ++i) {
                ++n_prims;
                if (visit(first + i)) return kWalkStopped;
            }
        }
        if (sp == 0) return kWalkDone;
        --sp;
        node = stk.load(sp);
    }
}

// Stack of a walk shared by the 64 lanes of a wave. Node ids are uniform:
// entry i sits in lane i % 64 of register ids[i / 64] (so cap <= 128). Each
// lane's entry depth of entry i sits in LDS at lds[i * 64 + lane] for
// i < lds_cap, beyond that in global memory at glb[(i - lds_cap) * stride]
// (a per-lane base, as TwoTierStack; null when there is no second tier).
struct WaveStack {
    float* lds;
    int lds_cap;
    float* glb;
    int64_t glb_stride;
    int cap;
    int32_t ids[2] = {0, 0};

    __device__ __forceinline__ void push(int i, int32_t id, float t, int lane)
    {
        if (i < 64)
            ids[0] = lane == i ? id : ids[0];
        else
            ids[1] = lane == i - 64 ? id : ids[1];
        if (i < lds_cap)
            lds[i * 64 + lane] = t;
        else
            glb[(int64_t)(i - lds_cap) * glb_stride] = t;
    }
    __device__ __forceinline__ int32_t id(int i) const
    {
        return i < 64 ? __builtin_amdgcn_readlane(ids[0], i)
                      : __builtin_amdgcn_readlane(ids[1], i - 64);
    }
    __device__ __forceinline__ float depth(int i, int lane) const
    {
        return i < lds_cap ? lds[i * 64 + lane] : glb[(int64_t)(i - lds_cap) * glb_stride];
    }
};

// One walk shared by the 64 rays of a wave (the rays of an 8x8 pixel tile
// are coherent, so they need nearly the same nodes). The wave pops one node
// at a time, in uniform control flow; a lane takes part when its ray entered
// the node's box no farther than its own depth cut (plus slack), so each lane
// sees only nodes and leaves its own walk would reach, in another order
// (results do not depend on the order). Children go on the stack when any
// lane hit them, in the near-to-far order of the first lane that takes part
// (+inf entry depth for the lanes that missed them). Node and record
// addresses are uniform, so they are fetched once per wave. visit(record
// index, on) is called by every lane for each record of a reached leaf; only
// lanes with `on` may act on it. ANY: visit returns true when the lane's ray
// is resolved (any-hit), and the lane takes part in nothing after that; the
// walk ends once every lane is resolved. Returns kWalkDone, kWalkStopped (ANY)
// or kWalkOverflow (wave-uniform).
template <int W, bool ANY = false, class Visit>
__device__ __forceinline__ int walk_wave(const WideNode<W>* __restrict__ nodes, const Ray& rf,
                                         bool live, float& tcut, float slack, WaveStack& stk,
                                         int64_t max_steps, uint32_t& n_nodes,
                                         uint32_t& n_prims, Visit&& visit)
{
    const int lane = (int)__lane_id();
    int sp = 0;
    int32_t node = 0;
    float t_in = -INFINITY;
    for (int64_t step = 0;; ++step) {
        if (step > max_steps) return kWalkOverflow;
        const bool on = live && t_in <= tcut + slack;
        const uint64_t act = __ballot(on);
        if (act != 0) {
            if (node >= 0) {
                n_nodes += on ? 1u : 0u;
                NodeBuf<W> b;
                load_node<W>(nodes, node, b);
                float te[W];
                slab_entry<W>(b, rf, tcut + slack, te);
                const int rep = __builtin_ctzll(act);
                uint32_t key[W];
#pragma unroll
                for (int c = 0; c < W; ++c) {
                    const bool hit = on && te[c] != INFINITY;
                    if (!on) te[c] = INFINITY;
                    const uint32_t k =
                        (uint32_t)__builtin_amdgcn_readlane((int)__float_as_uint(te[c]), rep);
                    key[c] = __ballot(hit) != 0 ? ((k & ~7u) | (uint32_t)c) : 0xFFFFFFFFu;
                }
                sort_keys<W>(key);
                int nh = 0;
#pragma unroll
                for (int c = 0; c < W; ++c) nh += key[c] != 0xFFFFFFFFu;
                if (nh > 0) {
                    if (sp + nh - 1 > stk.cap) return kWalkOverflow;
#pragma unroll
                    for (int c = W - 1; c >= 1; --c)
                        if (key[c] != 0xFFFFFFFFu) {
                            const uint32_t slot = key[c] & 7u;
                            float tv = te[0];
#pragma unroll
                            for (int j = 1; j < W; ++j) tv = slot == (uint32_t)j ? te[j] : tv;
                            stk.push(sp, child_at<W>(b, slot), tv, lane);
                            ++sp;
                        }
                    const uint32_t s0 = key[0] & 7u;
                    float tv = te[0];
#pragma unroll
                    for (int j = 1; j < W; ++j) tv = s0 == (uint32_t)j ? te[j] : tv;
                    t_in = tv;
                    node = child_at<W>(b, s0);
                    continue;
                }
            } else {
                const uint32_t first = leaf_first(node), count = leaf_count(node);
                bool lon = on;
                for (uint32_t i = 0; i < count; ++i) {
                    n_prims += lon ? 1u : 0u;
                    if (visit(first + i, lon) && ANY) {
                        lon = false;
                        live = false;
                    }
                }
                if (ANY && __ballot(live) == 0) return kWalkStopped;
            }
        }
        if (sp == 0) return kWalkDone;
        --sp;
        node = stk.id(sp);
        t_in = stk.depth(sp, lane);
    }
}

// Depth cut just beyond the key depth t: the entry distance of a box that
// holds a candidate of depth <= t is computed within a few ulps of it.
__device__ __forceinline__ float cut_after(float t)
{
    return t + fabsf(t) * 0x1p-20f + 1e-30f;
}

// Depth of a candidate (Sec. 3.1, Sec. 4.1). Mode 0: the mean t* of the 1D
// Gaussian along the ray. Mode 1: the centre projected onto a viewing axis a,
// as the ray parameter of the same depth along a, t = ((mu - o) . a) / (d . a)
// (a = the ray's direction when none is given); the opacity stays at the 1D
// peak. Because x(t*) lies in the bounding sphere of radius r about mu,
// |t - t*| <= r / (d . a_hat), so boxes are culled against the cut plus that
// slack (r = the largest radius in the scene), and a box is kept when it
// exits after tmin minus that slack: a Gaussian whose centre depth is past
// tmin can be crossed before tmin.
struct DepthCtx {
    int mode;         // uniform
    bool own_axis;    // uniform: the axis is each ray's direction
    float ax, ay, az; // uniform axis (when !own_axis)
    double inv_den;   // per ray: 1 / (d . a)
    float node_slack; // per ray
};

// In mode 1 also lowers ray.tmin (the box-exit bound) by the slack.
__device__ __forceinline__ DepthCtx make_depth(int mode, const float axis[3], Ray& ray,
                                               float r_max)
{
    DepthCtx c;
    c.mode = mode;
    c.own_axis = axis[0] == 0.0f && axis[1] == 0.0f && axis[2] == 0.0f;
    c.ax = axis[0];
    c.ay = axis[1];
    c.az = axis[2];
    c.node_slack = 0.0f;
    c.inv_den = 0.0;
    if (mode != 0) {
        double den, alen;
        if (c.own_axis) {
            den = (double)ray.dx * ray.dx + (double)ray.dy * ray.dy + (double)ray.dz * ray.dz;
            alen = sqrt(den);
        } else {
            den = (double)ray.dx * c.ax + (double)ray.dy * c.ay + (double)ray.dz * c.az;
            alen = sqrt((double)c.ax * c.ax + (double)c.ay * c.ay + (double)c.az * c.az);
        }
        c.inv_den = 1.0 / den;
        const double cosd = den / alen;  // d . a_hat
        c.node_slack = cosd > 0.0 ? (float)((double)r_max * (1.0 + 0x1p-12) / cosd) * 1.0001f
                                  : INFINITY;
        ray.tmin = ray.tmin - c.node_slack;
    }
    return c;
}

// DM: the depth mode fixed at compile time (0 mean, 1 centre), or -1 to read
// it from the context (one kernel for both modes, at some register cost).
template <int DM>
__device__ __forceinline__ int depth_mode_of(const DepthCtx& c)
{
    return DM < 0 ? c.mode : DM;
}

template <int DM = -1>
__device__ __forceinline__ double depth_of(const DepthCtx& c, const Record& r, const Ray& ray,
                                           double t_mean)
{
    if (depth_mode_of<DM>(c) == 0) return t_mean;
    const double wx = (double)r.mu[0] - (double)ray.ox;
    const double wy = (double)r.mu[1] - (double)ray.oy;
    const double wz = (double)r.mu[2] - (double)ray.oz;
    const double num = c.own_axis ? wx * ray.dx + wy * ray.dy + wz * ray.dz
                                  : wx * c.ax + wy * c.ay + wz * c.az;
    return num * c.inv_den;
}

// Forward resolution state of N samples sharing one walk (eqns "rr",
// "cloest", "multisample"): sample k keeps the smallest (t, gid) key among
// the valid candidates its Philox number accepts; (wt, wg) is the largest of
// the N keys and tcut the depth cut it implies.
template <int N>
struct FwdSamples {
    float bt[N];
    int32_t bg[N];
    float wt, tcut, tmax_f;
    int32_t wg;
    int n_act;

    __device__ __forceinline__ void reset(int n, float tmax)
    {
        n_act = n;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            bt[k] = k < n ? INFINITY : -INFINITY;
            bg[k] = 0x7FFFFFFF;
        }
        tmax_f = tmax;
        tcut = tmax;
        wt = INFINITY;
        wg = 0x7FFFFFFF;
    }
};

struct ForwardCtx {
    const Record* recs;
    uint32_t purpose, k0, k1;
};

// Hash-mode number of sample s for a candidate whose mean lies at depth t:
// the hit position p = o + t d, moved by s along (1, 1, 1) so the samples of
// one walk draw different numbers (the paper walks one sample per ray).
__device__ __forceinline__ float hash_u(const Ray& ray, float t, uint32_t s)
{
    const float fs = (float)s;
    return trig_hash((ray.ox + t * ray.dx) + fs, (ray.oy + t * ray.dy) + fs,
                     (ray.oz + t * ray.dz) + fs);
}

struct FwdCounts {
    uint32_t cands = 0, philox = 0;
};

// Validity of record r as a candidate of the ray (Sec. 3.1): the ray passes
// within the Gaussian's k-sigma ellipsoid (q <= k^2) and the candidate's
// depth t lies in (tmin, tmax), r not being the ignored Gaussian. In mean
// depth mode a bounding-sphere test against [ray.tmin, tcut] rejects records
// first (tcut: no candidate past it can change a result); the centre-depth
// depth is not bounded by the sphere's span, so there only a sphere the ray
// misses is rejected. tm: the 1D mean along the ray.
template <int DM>
__device__ __forceinline__ bool valid_candidate(const Record& r, const Ray& ray,
                                                const DepthCtx& dc, double tmin, double tmax,
                                                float tcut, int32_t ign, double& t, double& tm,
                                                double& q)
{
    if (depth_mode_of<DM>(dc) == 0) {
        if (sphere_reject(r, ray, ray.tmin, tcut)) return false;
    } else if (sphere_reject(r, ray, -INFINITY, INFINITY)) {
        return false;
    }
    isect_tq(r, ray, tm, q);
    t = depth_of<DM>(dc, r, ray, tm);
    if (!(q <= kEllipsoidQ && t > tmin && t < tmax) || r.gid == ign) return false;
    return true;
}

// Offer record r to the samples; true when an any-hit walk may stop. HASH:
// acceptance numbers from the trigonometric hash of the hit position instead
// of Philox.
template <int N, bool ANY, bool HASH = false, int DM = -1>
__device__ __forceinline__ bool fwd_offer(FwdSamples<N>& st, const Record& r, const Ray& ray,
                                          const DepthCtx& dc, double tmin, double tmax,
                                          int32_t ign, uint32_t rid, uint32_t s0,
                                          const ForwardCtx& fc, FwdCounts& cnt)
{
    double t, tm, q;
    if (!valid_candidate<DM>(r, ray, dc, tmin, tmax, st.tcut, ign, t, tm, q)) return false;
    ++cnt.cands;
    const float t32 = (float)t;
    if (!key_less(t32, r.gid, st.wt, st.wg)) return false;
    AlphaTest at(r.opacity, q);
    uint4 w = make_uint4(0, 0, 0, 0);
    uint32_t grp = 0xFFFFFFFFu;
    bool changed = false;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        if (k < st.n_act && key_less(t32, r.gid, st.bt[k], st.bg[k])) {
            const uint32_t s = s0 + (uint32_t)k;
            bool acc;
            if constexpr (!HASH) {
                if ((s >> 2) != grp) {
                    grp = s >> 2;
                    w = philox4x32_10(make_uint4(rid, grp, (uint32_t)r.gid, fc.purpose), fc.k0,
                                      fc.k1);
                    ++cnt.philox;
                }
                acc = at.accepts(word_of(w, s & 3u));
            } else {
                acc = at.accepts_u(hash_u(ray, (float)tm, s));
            }
            if (acc) {
                st.bt[k] = t32;
                st.bg[k] = r.gid;
                changed = true;
            }
        }
    }
    if (!changed) return false;
    if (ANY) return true;
    st.wt = -INFINITY;
    st.wg = (int32_t)0x80000000;
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (k < st.n_act && key_less(st.wt, st.wg, st.bt[k], st.bg[k])) {
            st.wt = st.bt[k];
            st.wg = st.bg[k];
        }
    st.tcut = fminf(cut_after(st.wt), st.tmax_f);
    return false;
}

// Offer record r to a group of identical any-hit rays that differ only in
// their sample indices (bit j of `pending`: sample s0 + j still unoccluded).
// The validity test is fwd_offer's for an any-hit ray with cut tmax; each
// pending sample then draws its own Philox number (one block per four
// consecutive samples) and is occluded iff u < alpha. Returns the samples r
// occludes.
template <int DM>
__device__ __forceinline__ uint64_t group_offer(const Record& r, const Ray& ray,
                                                const DepthCtx& dc, double tmin, double tmax,
                                                float tcut, int32_t ign, uint32_t rid,
                                                uint32_t s0, uint64_t pending,
                                                const ForwardCtx& fc, FwdCounts& cnt)
{
    double t, tm, q;
    if (!valid_candidate<DM>(r, ray, dc, tmin, tmax, tcut, ign, t, tm, q)) return 0;
    ++cnt.cands;
    const AlphaTest at(r.opacity, q);
    uint64_t occ = 0, m = pending;
    uint4 w = make_uint4(0, 0, 0, 0);
    uint32_t grp = 0xFFFFFFFFu;
    while (m) {
        const int j = __builtin_ctzll(m);
        m &= m - 1;
        const uint32_t s = s0 + (uint32_t)j;
        if ((s >> 2) != grp) {
            grp = s >> 2;
            w = philox4x32_10(make_uint4(rid, grp, (uint32_t)r.gid, fc.purpose), fc.k0, fc.k1);
            ++cnt.philox;
        }
        if (at.accepts(word_of(w, s & 3u))) occ |= 1ull << j;
    }
    return occ;
}

// (t, gid) key as one unsigned 64-bit value whose integer order is
// key_less's order: the depth's bits mapped monotonically (-0 taken as +0),
// then the id with its sign bit flipped.
__device__ __forceinline__ uint64_t pack_key(float t, int32_t gid)
{
    uint32_t b = __float_as_uint(t + 0.0f);
    b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ((uint64_t)b << 32) | ((uint32_t)gid ^ 0x80000000u);
}

__device__ __forceinline__ void unpack_key(uint64_t k, float& t, int32_t& gid)
{
    uint32_t b = (uint32_t)(k >> 32);
    b = (b & 0x80000000u) ? (b & 0x7FFFFFFFu) : ~b;
    t = __uint_as_float(b);
    gid = (int32_t)((uint32_t)k ^ 0x80000000u);
}

// fwd_offer for samples whose keys live in LDS (key of sample k at
// keys[64 k]) and may be lowered by other lanes in the same step: the
// validity test, then each of the n_act samples whose key the candidate's
// beats draws its number and on acceptance lowers the key with an LDS atomic
// minimum. (wt, wg) and tcut may lag the keys: a larger bound only tests more
// records, and each sample's result is the minimum over its accepted
// candidates whatever the order they are offered in. True when a key fell.
template <int N, int DM>
__device__ __forceinline__ bool keyed_offer(const Record& r, const Ray& ray, const DepthCtx& dc,
                                            double tmin, double tmax, float tcut, float wt,
                                            int32_t wg, uint32_t rid, uint32_t s0, int n_act,
                                            uint32_t purpose, uint32_t k0, uint32_t k1,
                                            unsigned long long* keys, FwdCounts& cnt)
{
    double t, tm, q;
    if (!valid_candidate<DM>(r, ray, dc, tmin, tmax, tcut, -1, t, tm, q)) return false;
    ++cnt.cands;
    const float t32 = (float)t;
    if (!key_less(t32, r.gid, wt, wg)) return false;
    const unsigned long long key = pack_key(t32, r.gid);
    const AlphaTest at(r.opacity, q);
    uint4 w = make_uint4(0, 0, 0, 0);
    uint32_t grp = 0xFFFFFFFFu;
    bool changed = false;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        if (k < n_act && key < keys[64 * k]) {
            const uint32_t s = s0 + (uint32_t)k;
            if ((s >> 2) != grp) {
                grp = s >> 2;
                w = philox4x32_10(make_uint4(rid, grp, (uint32_t)r.gid, purpose), k0, k1);
                ++cnt.philox;
            }
            if (at.accepts(word_of(w, s & 3u))) {
                atomicMin(keys + 64 * k, key);
                changed = true;
            }
        }
    }
    return changed;
}

template <int W, int N, bool ANY, class Stack, bool HASH = false, int DM = -1>
__device__ __forceinline__ int resolve_samples(const WideNode<W>* __restrict__ nodes,
                                               const ForwardCtx& fc, const DepthCtx& dc,
                                               const Ray& ray, double tmin,
                                               double tmax, int32_t ign, uint32_t rid, uint32_t s0,
                                               int n_act, Stack& stk, int64_t max_steps,
                                               float (&bt)[N], int32_t (&bg)[N],
                                               uint32_t& n_nodes, uint32_t& n_prims,
                                               uint32_t& n_cands, uint32_t& n_philox)
{
    FwdSamples<N> st;
    st.reset(n_act, (float)tmax);
    FwdCounts fcnt;
    auto visit = [&](uint32_t ri) -> bool {
        const Record r = load_record(fc.recs, ri);
        return fwd_offer<N, ANY, HASH, DM>(st, r, ray, dc, tmin, tmax, ign, rid, s0, fc, fcnt);
    };
    const float slack = DM == 0 ? 0.0f : dc.node_slack;
    const int res = walk<W>(nodes, ray, st.tcut, slack, stk, max_steps, n_nodes, n_prims, visit);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        bt[k] = st.bt[k];
        bg[k] = st.bg[k];
    }
    n_cands += fcnt.cands;
    n_philox += fcnt.philox;
    return res;
}

// resolve_samples over a walk shared by the wave (closest-hit only); lanes
// that are not live take part in the control flow and keep no hits.
template <int W, int N, int DM = -1>
__device__ __forceinline__ int resolve_samples_wave(const WideNode<W>* __restrict__ nodes,
                                                    const Record* __restrict__ recs,
                                                    const ForwardCtx& fc, const DepthCtx& dc,
                                                    const Ray& ray, bool live, double tmin,
                                                    double tmax, int32_t ign, uint32_t rid,
                                                    uint32_t s0, int n_act, WaveStack& stk,
                                                    int64_t max_steps, float (&bt)[N],
                                                    int32_t (&bg)[N], uint32_t& n_nodes,
                                                    uint32_t& n_prims, uint32_t& n_cands,
                                                    uint32_t& n_philox)
{
    FwdSamples<N> st;
    st.reset(n_act, (float)tmax);
    FwdCounts fcnt;
    auto visit = [&](uint32_t ri, bool on) -> bool {
        const Record r = load_record(recs, ri);
        if (on) fwd_offer<N, false, false, DM>(st, r, ray, dc, tmin, tmax, ign, rid, s0, fc, fcnt);
        return false;
    };
    const float slack = DM == 0 ? 0.0f : dc.node_slack;
    const int res = walk_wave<W>(nodes, ray, live, st.tcut, slack, stk, max_steps, n_nodes,
                                 n_prims, visit);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        bt[k] = st.bt[k];
        bg[k] = st.bg[k];
    }
    n_cands += fcnt.cands;
    n_philox += fcnt.philox;
    return res;
}

}  // namespace srt
