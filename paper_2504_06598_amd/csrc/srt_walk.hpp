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

// visit(record_index) -> true stops the walk (any-hit termination).
template <int W, class Stack, class Visit>
__device__ __forceinline__ int walk(const WideNode<W>* __restrict__ nodes, const RayF& rf,
                                    float& tcut, Stack& stk, int64_t max_steps,
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
            slab_keys<W>(b, rf, tcut, key);
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

// Depth cut just beyond the key depth t: the entry distance of a box that
// holds a candidate of depth <= t is computed within a few ulps of it.
__device__ __forceinline__ float cut_after(float t)
{
    return t + fabsf(t) * 0x1p-20f + 1e-30f;
}

// Forward resolution of N samples in one walk (eqns "rr", "cloest",
// "multisample"): sample k keeps the smallest (t, gid) key among the valid
// candidates its Philox number accepts.
struct ForwardCtx {
    const Record* recs;
    uint32_t purpose, k0, k1;
};

template <int W, int N, bool ANY, class Stack>
__device__ __forceinline__ int resolve_samples(const WideNode<W>* __restrict__ nodes,
                                               const ForwardCtx& fc, const RayF& rf,
                                               const RayD& rd, double tmin, double tmax,
                                               int32_t ign, uint32_t rid, uint32_t s0, int n_act,
                                               Stack& stk, int64_t max_steps, float (&bt)[N],
                                               int32_t (&bg)[N], uint32_t& n_nodes,
                                               uint32_t& n_prims, uint32_t& n_cands,
                                               uint32_t& n_philox)
{
#pragma unroll
    for (int k = 0; k < N; ++k) {
        bt[k] = k < n_act ? INFINITY : -INFINITY;
        bg[k] = 0x7FFFFFFF;
    }
    const float tmax_f = (float)tmax;
    float tcut = tmax_f;
    float wt = INFINITY;
    int32_t wg = 0x7FFFFFFF;
    const RayS rs = make_rays((float)rd.dx, (float)rd.dy, (float)rd.dz);
    auto visit = [&](uint32_t ri) -> bool {
        const Record r = load_record(fc.recs, ri);
        if (sphere_reject(r, rf, rs, rf.tmin, tcut)) return false;
        double t, q;
        isect_tq(r, rd, t, q);
        if (!(q <= kEllipsoidQ && t > tmin && t < tmax) || r.gid == ign) return false;
        ++n_cands;
        const float t32 = (float)t;
        if (!key_less(t32, r.gid, wt, wg)) return false;
        const double alpha = (double)r.opacity * exp(-0.5 * q);
        uint4 w = make_uint4(0, 0, 0, 0);
        uint32_t grp = 0xFFFFFFFFu;
        bool changed = false;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            if (k < n_act && key_less(t32, r.gid, bt[k], bg[k])) {
                const uint32_t s = s0 + (uint32_t)k;
                if ((s >> 2) != grp) {
                    grp = s >> 2;
                    w = philox4x32_10(make_uint4(rid, grp, (uint32_t)r.gid, fc.purpose), fc.k0,
                                      fc.k1);
                    ++n_philox;
                }
                if (u_of_word(word_of(w, s & 3u)) < alpha) {
                    bt[k] = t32;
                    bg[k] = r.gid;
                    changed = true;
                }
            }
        }
        if (!changed) return false;
        if (ANY) return true;
        wt = -INFINITY;
        wg = (int32_t)0x80000000;
#pragma unroll
        for (int k = 0; k < N; ++k)
            if (k < n_act && key_less(wt, wg, bt[k], bg[k])) {
                wt = bt[k];
                wg = bg[k];
            }
        tcut = fminf(cut_after(wt), tmax_f);
        return false;
    };
    return walk<W>(nodes, rf, tcut, stk, max_steps, n_nodes, n_prims, visit);
}

__device__ __forceinline__ RayF make_rayf(float ox, float oy, float oz, float dx, float dy,
                                          float dz, float tmin)
{
    RayF rf;
    rf.ox = ox;
    rf.oy = oy;
    rf.oz = oz;
    rf.ix = safe_inv(dx);
    rf.iy = safe_inv(dy);
    rf.iz = safe_inv(dz);
    rf.tmin = tmin;
    return rf;
}

}  // namespace srt
