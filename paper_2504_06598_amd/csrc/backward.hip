// Backward pass: gradients of the expected pixel colour.
//
// The paper leaves differentiable rendering to future work (Sec. 7) and only
// notes that a gradient applied to the selected Gaussian alone is easy but
// not the whole story. The expected colour is the exact composite
// L = sum_k T_k alpha_k c_k + T_end bg (eqn "accumulated"), whose partials are
// dL/dalpha_k = T_k (c_k - B_k) (B_k: expected colour behind k) and
// dL/dc_k = T_k alpha_k. Per sample with result a (colour X = c_a, or bg on a
// miss), every valid candidate k in front of a was rejected, which happens
// with probability T_k (1 - alpha_k) and leaves E[X | that] = B_k; so the
// estimate <g, c_k - X> / (1 - alpha_k) for alpha_k is unbiased, and the
// result a receives the colour gradient g. Each sample weighs 1/spp
// (eqn "multisample").
//
// Kernel 1 re-traverses every ray with the depth cut at the farthest of the
// pass's accepted hits (no per-ray hit lists are stored) and evaluates each
// front candidate in FP64. With alpha = o exp(-q/2), q = |p|^2 and
// p = M (x* - mu) = S^-1 R^T (x* - mu) at the 1D mean x* (dq/dt* = 0), a
// candidate's opacity weight s contributes through sa = s * alpha only via
//   dloss/dlogit = (1 - o) sa,  dloss/dmu = M^T (sa p),
//   dloss/dlog_s_i = sa p_i^2,  dloss/dR_ji = -(1/s_i) sum_k R_jk s_k sa p_i p_k,
// so each Gaussian accumulates ten numbers: sum sa, sum sa p, sum sa p p^T.
// The grid holds as many workgroups as stay resident; each takes tiles of 128
// neighbouring rays from a per-XCD band of the image with one atomic per
// tile. It pre-sums these ten numbers in an LDS hash table keyed by Gaussian
// id, and the accepted hits' SH colour gradients in a second one, flushing
// both to global memory with FP32 atomics after each tile (coherent rays
// share most Gaussians, so this removes most global atomic traffic; a
// Gaussian that finds no free slot goes straight to global memory). Kernel 2
// maps each Gaussian's sums to the raw parameters.
#include <algorithm>
#include <climits>

#include "srt_internal.hpp"
#include "srt_walk.hpp"

using namespace srt;

namespace {

constexpr int kBlock = 128;
constexpr int kLdsEntries = 16;  // on-chip stack entries per lane (deeper ones in global memory)
constexpr int kAccStride = 16;  // floats per Gaussian: sa, sa p (3), sa p p^T (6), pad (6)
constexpr int kAccVals = 10;
constexpr int kTableSlots = 128;  // LDS table of the alpha sums (a 128-ray tile of the
                                  // 1M scene's views holds 40-70 distinct front Gaussians)
constexpr int kShSlots = 64;      // LDS table of SH colour gradients (28-44 distinct
                                  // accepted Gaussians per such tile, of 512 samples)
constexpr int kShVals = 48;       // (deg + 1)^2 * 3 at degree 3
constexpr int kProbes = 8;

struct BwdArgs {
    const void* nodes;
    const Record* recs;
    const float* sh;
    int32_t deg;
    int64_t R;
    const float* o;
    const float* d;
    const float* tmin;
    const float* tmax;
    const int32_t* ign;
    const uint32_t* rid;
    const uint32_t* sid;
    uint32_t purpose, k0, k1;
    int32_t spp;
    uint32_t soff;
    float bg[3];
    const float* grad_rgb;
    const int32_t* hit_gid;
    const float* hit_t;
    float* acc;
    float* g_sh;
    int32_t* glb_stack;
    int32_t glb_stride;
    int32_t lds_cap;  // stack entries kept in LDS (<= kLdsEntries); the rest in glb_stack
    int32_t cap;
    int64_t max_steps;
    unsigned long long* counters;
    int32_t depth_mode;
    float depth_axis[3];
    float r_max;
    int32_t img_w;  // > 0: rays are a row-major image of this width, walked in 8x8 tiles
    const int32_t* leaf_pos;  // leaf position of each Gaussian id
    uint32_t* tile_ctr;       // [8 * 16]: tiles taken from each XCD band (64 B apart)
};

__device__ __forceinline__ void atomic_add_f32(float* p, float v)
{
    if (v != 0.0f) atomicAdd(p, v);
}

// x of a lane 16 * r + (i <op> j) of the same row of 16, by a DPP move
// (a vector-ALU operand modifier, where a lane shuffle goes through LDS).
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// x + (x of lane i ^ 16) and x + (x of lane i ^ 32): the CDNA4 lane-swap
// instructions exchange rows 1 and 3 with rows 0 and 2 (resp. the wave's
// halves) of two registers; swapping a register with itself gives both
// values of every pair in the two results.
__device__ __forceinline__ float add_xor16(float x)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(x), __float_as_int(x), false,
                                                    false);
    return __int_as_float(r[0]) + __int_as_float(r[1]);
}

__device__ __forceinline__ float add_xor32(float x)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(x), __float_as_int(x), false,
                                                    false);
    return __int_as_float(r[0]) + __int_as_float(r[1]);
}

// Sum of x over the wave's 64 lanes, held by every lane (each lane may add
// in its own order, so the lanes' values can differ in the last bits):
// within quads and rows of 16 by DPP, across rows by lane swaps; no LDS.
__device__ __forceinline__ float wave_sum(float x)
{
    x += dpp_move<0xB1>(x);   // quad_perm [1,0,3,2]
    x += dpp_move<0x4E>(x);   // quad_perm [2,3,0,1]
    x += dpp_move<0x124>(x);  // row_ror:4
    x += dpp_move<0x128>(x);  // row_ror:8
    return add_xor32(add_xor16(x));
}

struct Table {
    int32_t* keys;  // [kTableSlots], -1 = empty
    float* vals;    // [kAccVals][kTableSlots]
};

// Slot of `gid` in an open-addressing LDS table of `slots` keys (a power of
// two; -1 = empty), claimed with a compare-and-swap; -1 when no slot within
// kProbes probes holds or takes it.
template <int SLOTS>
__device__ __forceinline__ int lds_slot(int32_t* keys, int32_t gid)
{
    constexpr int bits = __builtin_ctz(SLOTS);
    uint32_t h = ((uint32_t)gid * 2654435761u) >> (32 - bits);
#pragma unroll 1
    for (int p = 0; p < kProbes; ++p) {
        const int32_t k = keys[h];
        if (k == gid) return (int)h;
        if (k == -1) {
            const int32_t old = atomicCAS(&keys[h], -1, gid);
            if (old == -1 || old == gid) return (int)h;
        }
        h = (h + 1) & (SLOTS - 1);
    }
    return -1;
}

// Add one candidate's ten sums to the workgroup table (global atomics when
// the table has no room for it).
__device__ __forceinline__ void table_add(Table& t, float* acc, int32_t gid, const float v[kAccVals])
{
    const int slot = lds_slot<kTableSlots>(t.keys, gid);
    if (slot >= 0) {
#pragma unroll
        for (int c = 0; c < kAccVals; ++c) atomicAdd(&t.vals[c * kTableSlots + slot], v[c]);
    } else {
        float* g = acc + (size_t)gid * kAccStride;
#pragma unroll
        for (int c = 0; c < kAccVals; ++c) atomic_add_f32(g + c, v[c]);
    }
}

// WV: the 64 rays of each 8x8 tile re-traverse together (walk_wave; image
// launches), else each lane walks for its own ray. Registers are capped for 3
// waves per SIMD (a few spill to scratch; measured faster than 2 waves).
template <int W, int N, bool COUNT, bool RB, int DM, bool WV>
__global__ __launch_bounds__(kBlock, 3) void k_backward(BwdArgs a, const void* __restrict__ nodes_v,
                                                     const Record* __restrict__ recs_r,
                                                     const float* __restrict__ sh_r)
{
    __shared__ int32_t lds[kLdsEntries * kBlock];
    __shared__ int32_t tkeys[kTableSlots];
    __shared__ float tvals[kAccVals * kTableSlots];
    __shared__ int32_t shkeys[kShSlots];
    __shared__ float shvals[kShVals * kShSlots];
    Table table{tkeys, tvals};
    for (int i = threadIdx.x; i < kTableSlots; i += kBlock) {
        tkeys[i] = -1;
        for (int c = 0; c < kAccVals; ++c) tvals[c * kTableSlots + i] = 0.0f;
    }
    for (int i = threadIdx.x; i < kShSlots; i += kBlock) {
        shkeys[i] = -1;
        for (int c = 0; c < kShVals; ++c) shvals[c * kShSlots + i] = 0.0f;
    }
    __syncthreads();
    const int64_t gt = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    TwoTierStack stk{lds + threadIdx.x, kBlock, a.lds_cap, a.glb_stack + gt, a.glb_stride, a.cap};
    // wave-shared stack: entry depths in this wave's half of the same LDS, then
    // in the lane's global stack
    WaveStack wstk{reinterpret_cast<float*>(lds) + (threadIdx.x >> 6) * (kLdsEntries * 64),
                   a.lds_cap, reinterpret_cast<float*>(a.glb_stack + gt), a.glb_stride,
                   min(128, a.cap)};
    const WideNode<W>* nodes = static_cast<const WideNode<W>*>(a.nodes);
    const WideNode<W>* __restrict__ wnodes = static_cast<const WideNode<W>*>(nodes_v);
    const int K = (a.deg + 1) * (a.deg + 1);
    const float inv_spp = 1.0f / (float)a.spp;
    uint32_t n_trav = 0, n_nodes = 0, n_prims = 0, n_front = 0, n_samples = 0, n_lost = 0,
             n_philox = 0, n_fwd_cands = 0;
    const int64_t n_threads = a.img_w > 0 ? tile_threads(a.img_w, a.R / a.img_w) : a.R;
    const int64_t n_tiles = (n_threads + kBlock - 1) / kBlock;

    // Tiles are handed out dynamically: the image is cut into 8 bands, one per
    // XCD (workgroups are dispatched to the XCDs in turn, so workgroup b runs
    // on XCD b % 8); a workgroup takes the next tile of its own band with one
    // atomic, and once its band is used up, of the next bands in turn. Every
    // thread of the workgroup runs the same tiles (the tile is broadcast
    // through LDS), so the barriers below are reached by all of them.
    __shared__ int64_t s_tile;
    int band = blockIdx.x & 7;
    int bands_left = 8;
    for (;;) {
        if (threadIdx.x == 0) {
            int64_t t = -1;
            while (bands_left > 0) {
                const int64_t b0 = n_tiles * band / 8, b1 = n_tiles * (band + 1) / 8;
                const int64_t k = (int64_t)atomicAdd(&a.tile_ctr[16 * band], 1u);
                if (b0 + k < b1) {
                    t = b0 + k;
                    break;
                }
                band = (band + 1) & 7;
                --bands_left;
            }
            s_tile = t;
        }
        __syncthreads();
        const int64_t tile = s_tile;
        if (tile < 0) break;  // uniform: every thread read the same value
        const int64_t t = tile * kBlock + threadIdx.x;
        const int64_t ray = a.img_w > 0 ? tile_pixel(t, a.img_w, a.R / a.img_w) : t;
        const bool valid = ray >= 0 && ray < a.R;
        float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
        float tmin_f = 0.0f, tmax_f = 0.0f;
        if (valid) {
            g0 = a.grad_rgb[3 * ray];
            g1 = a.grad_rgb[3 * ray + 1];
            g2 = a.grad_rgb[3 * ray + 2];
            tmin_f = a.tmin ? a.tmin[ray] : 0.0f;
            tmax_f = a.tmax ? a.tmax[ray] : INFINITY;
        }
        const bool work = valid && (g0 != 0.0f || g1 != 0.0f || g2 != 0.0f) && tmax_f > tmin_f;
        // WV: lanes without work take part in the shared walks with no samples
        if (WV || work) {
            const int64_t rq = work ? ray : 0;
            const float ox = a.o[3 * rq], oy = a.o[3 * rq + 1], oz = a.o[3 * rq + 2];
            const float dx = a.d[3 * rq], dy = a.d[3 * rq + 1], dz = a.d[3 * rq + 2];
            const int32_t ign = a.ign ? a.ign[rq] : -1;
            const uint32_t rid = a.rid ? a.rid[rq] : (uint32_t)rq;
            const uint32_t sbase = (a.sid ? a.sid[rq] : 0u) + a.soff;
            Ray rr = make_ray(ox, oy, oz, dx, dy, dz, tmin_f);
            const double tmin = tmin_f, tmax = tmax_f;
            const DepthCtx dc = make_depth(a.depth_mode, a.depth_axis, rr, a.r_max);
            float Y[16];
            sh_eval(a.deg, dx * rr.inv_len, dy * rr.inv_len, dz * rr.inv_len, Y);
            for (int pass = 0; pass * N < a.spp; ++pass) {
                const int n_act = work ? min(N, a.spp - pass * N) : 0;
                float ta[N];
                int32_t ga[N];
                if (a.hit_gid) {
#pragma unroll
                    for (int k = 0; k < N; ++k) {
                        if (k < n_act) {
                            const int64_t o = ray * a.spp + pass * N + k;
                            const int32_t g = a.hit_gid[o];
                            ga[k] = g >= 0 ? g : 0x7FFFFFFF;
                            ta[k] = g >= 0 ? a.hit_t[o] : INFINITY;
                        } else {
                            ga[k] = 0x7FFFFFFF;
                            ta[k] = -INFINITY;
                        }
                    }
                } else {
                    const ForwardCtx fc{WV ? recs_r : a.recs, a.purpose, a.k0, a.k1};
                    uint32_t dummy_nodes = 0, dummy_prims = 0;
                    int res;
                    if constexpr (WV)
                        res = resolve_samples_wave<W, N, DM>(
                            wnodes, recs_r, fc, dc, rr, work, tmin, tmax, ign, rid,
                            sbase + (uint32_t)(pass * N), n_act, wstk, a.max_steps, ta, ga,
                            dummy_nodes, dummy_prims, n_fwd_cands, n_philox);
                    else
                        res = resolve_samples<W, N, false, TwoTierStack, false, DM>(
                            nodes, fc, dc, rr, tmin, tmax, ign, rid, sbase + (uint32_t)(pass * N),
                            n_act, stk, a.max_steps, ta, ga, dummy_nodes, dummy_prims,
                            n_fwd_cands, n_philox);
                    if (res == kWalkOverflow) {  // wave-uniform under WV
                        n_lost += work ? 1u : 0u;
                        continue;
                    }
                }
                // <g, X> of each sample's result colour X (bg on a miss), and the
                // farthest key the walk has to reach; only scalars are live during it.
                // RB: a hit sample also searches its second accepted candidate
                // (tb, gb) behind its first, so its far key is that one; a miss
                // sample's front is every candidate.
                float gx[N];
                float tb[RB ? N : 1];
                int32_t gb[RB ? N : 1];
                float wt = -INFINITY;
                int32_t wg = INT_MIN;
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    gx[k] = 0.0f;
                    if constexpr (RB) {
                        tb[k] = -INFINITY;
                        gb[k] = INT_MIN;
                    }
                    if (k >= n_act) continue;
                    if (ga[k] != 0x7FFFFFFF) {
                        const float3 c = clamp0(sh_colour_pre(a.sh, a.deg, ga[k], Y));
                        gx[k] = g0 * c.x + g1 * c.y + g2 * c.z;
                        if constexpr (RB) {
                            tb[k] = INFINITY;
                            gb[k] = 0x7FFFFFFF;
                        }
                    } else {
                        gx[k] = g0 * a.bg[0] + g1 * a.bg[1] + g2 * a.bg[2];
                    }
                    const float fk = RB && ga[k] != 0x7FFFFFFF ? tb[k] : ta[k];
                    const int32_t fg = RB && ga[k] != 0x7FFFFFFF ? gb[k] : ga[k];
                    if (key_less(wt, wg, fk, fg)) {
                        wt = fk;
                        wg = fg;
                    }
                }
                n_samples += (uint32_t)n_act;
                n_trav += work ? 1u : 0u;
                float tcut = fminf(cut_after(wt), tmax_f);
                const uint32_t s0 = sbase + (uint32_t)(pass * N);
                // the ten sums' terms of record r for this lane's samples; false
                // when r is no valid candidate in front of them
                auto front_terms = [&](const Record& r, float (&v)[kAccVals]) -> bool {
                    if (depth_mode_of<DM>(dc) == 0 ? sphere_reject(r, rr, tmin_f, tcut)
                                                   : sphere_reject(r, rr, -INFINITY, INFINITY))
                        return false;
                    double tm, q, p[3];
                    isect_tqp(r, rr, tm, q, p);
                    const double t = depth_of<DM>(dc, r, rr, tm);
                    if (!(q <= kEllipsoidQ && t > tmin && t < tmax) || r.gid == ign) return false;
                    const float t32 = (float)t;
                    if (!key_less(t32, r.gid, wt, wg)) return false;
                    int nf = 0, na = 0;
                    float xs = 0.0f;
                    bool found = false;
                    uint4 w = make_uint4(0, 0, 0, 0);
                    uint32_t grp = 0xFFFFFFFFu;
                    double alpha64 = -1.0;  // formed only if some sample needs a test
#pragma unroll
                    for (int k = 0; k < N; ++k) {
                        if (k >= n_act) continue;
                        if (key_less(t32, r.gid, ta[k], ga[k])) {
                            ++nf;
                            xs += gx[k];
                        } else if constexpr (RB) {
                            if (r.gid == ga[k] && t32 == ta[k]) {
                                ++na;  // the sample's first accepted candidate
                            } else if (key_less(t32, r.gid, tb[k], gb[k])) {
                                // behind the first accepted: is it a nearer second one?
                                const uint32_t smp = s0 + (uint32_t)k;
                                if ((smp >> 2) != grp) {
                                    grp = smp >> 2;
                                    w = philox4x32_10(
                                        make_uint4(rid, grp, (uint32_t)r.gid, a.purpose), a.k0,
                                        a.k1);
                                    ++n_philox;
                                }
                                if (alpha64 < 0.0) alpha64 = (double)r.opacity * exp(-0.5 * q);
                                if (u_of_word(word_of(w, smp & 3u)) < alpha64) {
                                    tb[k] = t32;
                                    gb[k] = r.gid;
                                    found = true;
                                }
                            }
                        }
                    }
                    if constexpr (RB) {
                        if (found) {
                            wt = -INFINITY;
                            wg = INT_MIN;
#pragma unroll
                            for (int k = 0; k < N; ++k) {
                                if (k >= n_act) continue;
                                const float fk = ga[k] != 0x7FFFFFFF ? tb[k] : ta[k];
                                const int32_t fg = ga[k] != 0x7FFFFFFF ? gb[k] : ga[k];
                                if (key_less(wt, wg, fk, fg)) {
                                    wt = fk;
                                    wg = fg;
                                }
                            }
                            tcut = fminf(cut_after(wt), tmax_f);
                        }
                    }
                    if (nf == 0 && na == 0) return false;
                    ++n_front;
                    // alpha only weights FP32 sums here: FP32 precision suffices
                    const float alpha = r.opacity * expf(-0.5f * (float)q);
                    // WV: r.gid is the same on every lane, so its SH row is fetched once
                    const float3 c = clamp0(sh_colour_pre(WV ? sh_r : a.sh, a.deg, r.gid, Y));
                    const float gc = g0 * c.x + g1 * c.y + g2 * c.z;
                    // plain: <g, c_k - X> / (1 - alpha_k) per front sample; RB: the
                    // same without the division, and <g, c_a> for a sample's first
                    // accepted a (its -<g, X2> part is added after the walk)
                    const float s_alpha = RB ? ((float)(nf + na) * gc - xs) * inv_spp
                                             : ((float)nf * gc - xs) * inv_spp / (1.0f - alpha);
                    const float sa = s_alpha * alpha;
                    const float p0 = (float)p[0], p1 = (float)p[1], p2 = (float)p[2];
                    v[0] = sa;
                    v[1] = sa * p0;
                    v[2] = sa * p1;
                    v[3] = sa * p2;
                    v[4] = sa * p0 * p0;
                    v[5] = sa * p1 * p1;
                    v[6] = sa * p2 * p2;
                    v[7] = sa * p0 * p1;
                    v[8] = sa * p0 * p2;
                    v[9] = sa * p1 * p2;
                    return true;
                };
                const float slack = DM == 0 ? 0.0f : dc.node_slack;
                int res;
                if constexpr (WV) {
                    // every lane of the walk handles the same record: the lanes' terms
                    // are summed across the wave and one lane adds them to the table
                    // (instead of up to 64 atomics on one LDS slot)
                    auto visit = [&](uint32_t ri, bool on) -> bool {
                        const Record r = load_record(recs_r, ri);
                        float v[kAccVals] = {};
                        const bool c = on && front_terms(r, v);
                        const uint64_t m = __ballot(c);
                        if (m != 0) {
#pragma unroll
                            for (int j = 0; j < kAccVals; ++j) v[j] = wave_sum(c ? v[j] : 0.0f);
                            if ((int)__lane_id() == __builtin_ctzll(m))
                                table_add(table, a.acc, r.gid, v);
                        }
                        return false;
                    };
                    res = walk_wave<W>(wnodes, rr, work, tcut, slack, wstk, a.max_steps, n_nodes,
                                       n_prims, visit);
                } else {
                    auto visit = [&](uint32_t ri) -> bool {
                        const Record r = load_record(a.recs, ri);
                        float v[kAccVals];
                        if (front_terms(r, v)) table_add(table, a.acc, r.gid, v);
                        return false;
                    };
                    res = walk<W>(nodes, rr, tcut, slack, stk, a.max_steps, n_nodes, n_prims, visit);
                }
                if (res == kWalkOverflow) n_lost += work ? 1u : 0u;
                if constexpr (RB) {
                    // -<g, X2> on the alpha of each sample's first accepted a (X2 the
                    // colour of its second accepted, bg if none), samples sharing a merged
                    if (res != kWalkOverflow) {
#pragma unroll
                        for (int k = 0; k < N; ++k) {
                            if (k >= n_act || ga[k] == 0x7FFFFFFF) continue;
                            bool first = true;
                            float s2 = 0.0f;
#pragma unroll
                            for (int j = 0; j < N; ++j) {
                                if (j >= n_act || ga[j] != ga[k]) continue;
                                if (j < k) first = false;
                                float x2;
                                if (gb[j] != 0x7FFFFFFF) {
                                    const float3 c2 = clamp0(sh_colour_pre(a.sh, a.deg, gb[j], Y));
                                    x2 = g0 * c2.x + g1 * c2.y + g2 * c2.z;
                                } else {
                                    x2 = g0 * a.bg[0] + g1 * a.bg[1] + g2 * a.bg[2];
                                }
                                s2 -= x2;
                            }
                            if (!first) continue;
                            const Record r = load_record(a.recs, (uint32_t)a.leaf_pos[ga[k]]);
                            double tm, q, p[3];
                            isect_tqp(r, rr, tm, q, p);
                            const float alpha = r.opacity * expf(-0.5f * (float)q);
                            const float sa = s2 * inv_spp * alpha;
                            const float p0 = (float)p[0], p1 = (float)p[1], p2 = (float)p[2];
                            const float v[kAccVals] = {sa,           sa * p0,      sa * p1,
                                                       sa * p2,      sa * p0 * p0, sa * p1 * p1,
                                                       sa * p2 * p2, sa * p0 * p1, sa * p0 * p2,
                                                       sa * p1 * p2};
                            table_add(table, a.acc, r.gid, v);
                        }
                    }
                }
                // colour gradient of each accepted result, samples sharing a Gaussian merged
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    if (k >= n_act || ga[k] == 0x7FFFFFFF) continue;
                    bool first = true;
                    int mult = 0;
#pragma unroll
                    for (int j = 0; j < N; ++j) {
                        if (j >= n_act || ga[j] != ga[k]) continue;
                        if (j < k) first = false;
                        ++mult;
                    }
                    if (!first) continue;
                    const float3 pre = sh_colour_pre(a.sh, a.deg, ga[k], Y);
                    const float f = (float)mult * inv_spp;
                    // the clamp passes the gradient only where the colour is positive
                    const float f0 = pre.x > 0.0f ? g0 * f : 0.0f;
                    const float f1 = pre.y > 0.0f ? g1 * f : 0.0f;
                    const float f2 = pre.z > 0.0f ? g2 * f : 0.0f;
                    if (f0 == 0.0f && f1 == 0.0f && f2 == 0.0f) continue;
                    const int slot = lds_slot<kShSlots>(shkeys, ga[k]);
                    if (slot >= 0) {
                        for (int j = 0; j < K; ++j) {
                            atomicAdd(&shvals[(3 * j + 0) * kShSlots + slot], Y[j] * f0);
                            atomicAdd(&shvals[(3 * j + 1) * kShSlots + slot], Y[j] * f1);
                            atomicAdd(&shvals[(3 * j + 2) * kShSlots + slot], Y[j] * f2);
                        }
                    } else {
                        float* gs = a.g_sh + (size_t)ga[k] * (size_t)(3 * K);
                        for (int j = 0; j < K; ++j) {
                            atomic_add_f32(gs + 3 * j + 0, Y[j] * f0);
                            atomic_add_f32(gs + 3 * j + 1, Y[j] * f1);
                            atomic_add_f32(gs + 3 * j + 2, Y[j] * f2);
                        }
                    }
                }
            }
        }
        // flush the tile's sums and clear the table
        __syncthreads();
        for (int i = threadIdx.x; i < kTableSlots; i += kBlock) {
            const int32_t gid = tkeys[i];
            if (gid >= 0) {
                float* g = a.acc + (size_t)gid * kAccStride;
                for (int c = 0; c < kAccVals; ++c) {
                    atomic_add_f32(g + c, tvals[c * kTableSlots + i]);
                    tvals[c * kTableSlots + i] = 0.0f;
                }
                tkeys[i] = -1;
            }
        }
        for (int i = threadIdx.x; i < kShSlots; i += kBlock) {
            const int32_t gid = shkeys[i];
            if (gid >= 0) {
                float* gs = a.g_sh + (size_t)gid * (size_t)(3 * K);
                for (int c = 0; c < 3 * K; ++c) {
                    atomic_add_f32(gs + c, shvals[c * kShSlots + i]);
                    shvals[c * kShSlots + i] = 0.0f;
                }
                shkeys[i] = -1;
            }
        }
        __syncthreads();
    }
    if (COUNT && a.counters) {
        wave_add_u64(a.counters + SRT_CNT_TRAVERSALS, n_trav);
        wave_add_u64(a.counters + SRT_CNT_NODES, n_nodes);
        wave_add_u64(a.counters + SRT_CNT_PRIMS, n_prims);
        wave_add_u64(a.counters + SRT_CNT_CANDIDATES, n_front + n_fwd_cands);
        wave_add_u64(a.counters + SRT_CNT_PHILOX, n_philox);
        wave_add_u64(a.counters + SRT_CNT_RAY_SAMPLES, n_samples);
        wave_add_u64(a.counters + SRT_CNT_LOST, n_lost);
    }
}

// Per Gaussian: the ten sums -> gradients of the raw parameters, added to the
// caller's buffers. With A = sum sa, v = sum sa p, P = sum sa p p^T:
//   dlogit = (1 - o) A,  dmu = M^T v = R S^-1 v,  dlog_s_i = P_ii,
//   dR_ji = -(1/s_i) sum_k R_jk s_k P_ik, then through R(q / |q|).
__global__ void k_chain(int64_t G, const float* __restrict__ acc, const float* __restrict__ ls,
                        const float* __restrict__ quats, const float* __restrict__ logits,
                        float* g_means, float* g_ls, float* g_quats, float* g_logits)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= G) return;
    const float4* p4 = reinterpret_cast<const float4*>(acc + g * kAccStride);
    const float4 u0 = p4[0], u1 = p4[1], u2 = p4[2];
    const double A = u0.x;
    const double v[3] = {u0.y, u0.z, u0.w};
    const double P[9] = {u1.x, u1.w, u2.x, u1.w, u1.y, u2.y, u2.x, u2.y, u1.z};
    if (A == 0.0 && v[0] == 0.0 && v[1] == 0.0 && v[2] == 0.0 && P[0] == 0.0 && P[4] == 0.0 &&
        P[8] == 0.0 && P[1] == 0.0 && P[2] == 0.0 && P[5] == 0.0)
        return;
    double w = quats[4 * g], x = quats[4 * g + 1], y = quats[4 * g + 2], z = quats[4 * g + 3];
    const double qn = sqrt(w * w + x * x + y * y + z * z);
    if (!(qn > 0.0)) return;
    w /= qn; x /= qn; y /= qn; z /= qn;
    const double R[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
                         2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                         2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)};
    double s[3];
    for (int i = 0; i < 3; ++i) s[i] = exp((double)ls[3 * g + i]);
    const double o = 1.0 / (1.0 + exp(-(double)logits[g]));
    double GR[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc_ji = 0.0;
            for (int k = 0; k < 3; ++k) acc_ji += R[3 * j + k] * s[k] * P[3 * i + k];
            GR[3 * j + i] = -acc_ji / s[i];
        }
    // dR/dq of the unit quaternion contracted with GR (row-major R)
    const double dw = 2.0 * (-z * GR[1] + y * GR[2] + z * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
    const double dx = 2.0 * (y * GR[1] + z * GR[2] + y * GR[3] - 2.0 * x * GR[4] - w * GR[5] +
                             z * GR[6] + w * GR[7] - 2.0 * x * GR[8]);
    const double dy = 2.0 * (-2.0 * y * GR[0] + x * GR[1] + w * GR[2] + x * GR[3] + z * GR[5] -
                             w * GR[6] + z * GR[7] - 2.0 * y * GR[8]);
    const double dz = 2.0 * (-2.0 * z * GR[0] - w * GR[1] + x * GR[2] + w * GR[3] - 2.0 * z * GR[4] +
                             y * GR[5] + x * GR[6] + y * GR[7]);
    const double dot = dw * w + dx * x + dy * y + dz * z;
    g_quats[4 * g + 0] += (float)((dw - w * dot) / qn);
    g_quats[4 * g + 1] += (float)((dx - x * dot) / qn);
    g_quats[4 * g + 2] += (float)((dy - y * dot) / qn);
    g_quats[4 * g + 3] += (float)((dz - z * dot) / qn);
    for (int j = 0; j < 3; ++j) {
        double mu_j = 0.0;
        for (int i = 0; i < 3; ++i) mu_j += R[3 * j + i] * v[i] / s[i];
        g_means[3 * g + j] += (float)mu_j;
    }
    for (int i = 0; i < 3; ++i) g_ls[3 * g + i] += (float)P[4 * i];
    g_logits[g] += (float)((1.0 - o) * A);
}

using BwdFn = void (*)(BwdArgs, const void*, const Record*, const float*);

template <int W, bool C, bool RB, int DM, bool WV>
BwdFn pick_n(int N)
{
    switch (N) {
    case 1: return k_backward<W, 1, C, RB, DM, WV>;
    case 2: return k_backward<W, 2, C, RB, DM, WV>;
    case 4: return k_backward<W, 4, C, RB, DM, WV>;
    case 8: return k_backward<W, 8, C, RB, DM, WV>;
    }
    return nullptr;
}

template <int W, int DM, bool WV>
BwdFn pick_w(int N, bool count, bool rb)
{
    if (rb) return count ? pick_n<W, true, true, DM, WV>(N) : pick_n<W, false, true, DM, WV>(N);
    return count ? pick_n<W, true, false, DM, WV>(N) : pick_n<W, false, false, DM, WV>(N);
}

template <int DM, bool WV>
BwdFn pick_dm(int W, int N, bool count, bool rb)
{
    switch (W) {
    case 2: return pick_w<2, DM, WV>(N, count, rb);
    case 4: return pick_w<4, DM, WV>(N, count, rb);
    case 8: return pick_w<8, DM, WV>(N, count, rb);
    }
    return nullptr;
}

BwdFn pick(int W, int N, bool count, bool rb, int depth_mode, bool wave)
{
    if (wave)
        return depth_mode == 0 ? pick_dm<0, true>(W, N, count, rb)
                               : pick_dm<1, true>(W, N, count, rb);
    return depth_mode == 0 ? pick_dm<0, false>(W, N, count, rb)
                           : pick_dm<1, false>(W, N, count, rb);
}

constexpr int64_t kMaxBwdBlocks = 2048;

struct BwdWs {
    uint32_t* tile_ctr;  // [128]
    float* acc;
    int32_t* stack;
    int32_t threads;
    size_t bytes;
};

BwdWs bwd_ws(const srt_bvh* b, int64_t R, void* base)
{
    BwdWs w{};
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((R + kBlock - 1) / kBlock,
                                                                  kMaxBwdBlocks));
    w.threads = (int32_t)(blocks * kBlock);
    char* p = static_cast<char*>(base);
    size_t off = 0;
    w.tile_ctr = reinterpret_cast<uint32_t*>(p ? p + off : nullptr);
    off = align_up(off + 128 * sizeof(uint32_t), 256);
    w.acc = reinterpret_cast<float*>(p ? p + off : nullptr);
    off = align_up(off + sizeof(float) * kAccStride * (size_t)std::max<int64_t>(b->G, 1), 256);
    // a whole stack per thread, so that any split between LDS and global fits
    w.stack = reinterpret_cast<int32_t*>(p ? p + off : nullptr);
    off = align_up(off + sizeof(int32_t) * (size_t)w.threads * (size_t)deep_stack_cap(b), 256);
    w.bytes = off;
    return w;
}

}  // namespace

extern "C" {

size_t srt_backward_workspace_size(const srt_bvh* b, int64_t num_rays)
{
    if (!b || num_rays < 0) return 0;
    return bwd_ws(b, num_rays, nullptr).bytes;
}

srt_status srt_trace_backward(const srt_bvh* b, const srt_scene* scene, const srt_rays* rays,
                              const srt_trace_opts* opts, const float* grad_rgb,
                              const int32_t* hit_gid, const float* hit_t, float* g_means,
                              float* g_log_scales, float* g_quats, float* g_opacity_logits,
                              float* g_sh, uint64_t* counters, void* workspace,
                              size_t workspace_bytes, void* stream)
{
    const srt::Range range_("srt_trace_backward");
    if (!b || !rays || !opts || !scene) return SRT_ERR_INVALID_ARG;
    if (opts->spp < 1 || opts->any_hit) return SRT_ERR_INVALID_ARG;
    if (opts->depth_mode != 0 && opts->depth_mode != 1) return SRT_ERR_INVALID_ARG;
    if (opts->image_width < 0) return SRT_ERR_INVALID_ARG;
    if (opts->image_width > 0 && rays->count % opts->image_width != 0) return SRT_ERR_INVALID_ARG;
    if (opts->estimator != 0 && opts->estimator != 1) return SRT_ERR_INVALID_ARG;
    if (opts->rng != 0 && opts->rng != 1) return SRT_ERR_INVALID_ARG;
    if (opts->walk < 0 || opts->walk > 2) return SRT_ERR_INVALID_ARG;
    if (opts->stack_limit < 0) return SRT_ERR_INVALID_ARG;
    // wave-shared walks need an image launch (tiles of neighbouring rays)
    if (opts->walk == 2 && opts->image_width == 0) return SRT_ERR_UNSUPPORTED;
    // the backward draws numbers only to recompute results or to find second
    // hits; with the hash those are not provided here
    if (opts->rng == 1 && (hit_gid == nullptr || opts->estimator == 1))
        return SRT_ERR_UNSUPPORTED;
    const int N = opts->n_per_traversal;
    if (N != 1 && N != 2 && N != 4 && N != 8) return SRT_ERR_INVALID_ARG;
    if (rays->count < 0 || rays->count > (int64_t)UINT32_MAX) return SRT_ERR_INVALID_ARG;
    if (rays->count > 0 && (!rays->origins || !rays->dirs || !grad_rgb)) return SRT_ERR_INVALID_ARG;
    if ((hit_gid == nullptr) != (hit_t == nullptr)) return SRT_ERR_INVALID_ARG;
    if (scene->num_gaussians != b->G || scene->sh_degree != b->deg) return SRT_ERR_INVALID_ARG;
    if (b->G > 0 && (!g_means || !g_log_scales || !g_quats || !g_opacity_logits || !g_sh ||
                     !scene->log_scales || !scene->quats || !scene->opacity_logits))
        return SRT_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < srt_backward_workspace_size(b, rays->count))
        return SRT_ERR_WORKSPACE;
    if (b->G == 0 || rays->count == 0) return SRT_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const BwdWs ws = bwd_ws(b, rays->count, workspace);
    const bool wave = opts->walk != 1 && opts->image_width > 0;
    BwdFn fn = pick(b->W, N, counters != nullptr, opts->estimator == 1, opts->depth_mode, wave);
    if (!fn) return SRT_ERR_UNSUPPORTED;
    // as many workgroups as stay resident (tiles are handed out dynamically),
    // at most the number the workspace holds stacks for
    int dev = 0, n_cu = 0, per_cu = 0;
    SRT_HIP_TRY(hipGetDevice(&dev));
    SRT_HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    SRT_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(fn), kBlock, 0));
    const unsigned blocks = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>(ws.threads / kBlock, (int64_t)n_cu * std::max(1, per_cu)));
    fill_u32(reinterpret_cast<uint32_t*>(ws.acc), 0u, (size_t)kAccStride * (size_t)b->G, s);
    BwdArgs a{};
    a.nodes = b->nodes;
    a.recs = b->recs;
    a.sh = b->sh;
    a.deg = b->deg;
    a.R = rays->count;
    a.o = rays->origins;
    a.d = rays->dirs;
    a.tmin = rays->tmin;
    a.tmax = rays->tmax;
    a.ign = rays->ignore_gid;
    a.rid = rays->ray_ids;
    a.sid = rays->sample_ids;
    a.purpose = rays->purpose;
    a.k0 = (uint32_t)opts->seed;
    a.k1 = (uint32_t)(opts->seed >> 32);
    a.spp = opts->spp;
    a.soff = opts->sample_offset;
    for (int i = 0; i < 3; ++i) a.bg[i] = opts->bg[i];
    a.grad_rgb = grad_rgb;
    a.hit_gid = hit_gid;
    a.hit_t = hit_t;
    a.acc = ws.acc;
    a.g_sh = g_sh;
    a.glb_stack = ws.stack;
    a.glb_stride = ws.threads;
    a.lds_cap = opts->stack_limit > 0 ? std::min(kLdsEntries, opts->stack_limit) : kLdsEntries;
    a.cap = std::max(a.lds_cap, deep_stack_cap(b));
    a.max_steps = 2 * b->num_nodes + 2 * b->G + 64;
    a.counters = reinterpret_cast<unsigned long long*>(counters);
    a.depth_mode = opts->depth_mode;
    for (int i = 0; i < 3; ++i) a.depth_axis[i] = opts->depth_axis[i];
    a.r_max = b->r_max;
    a.img_w = opts->image_width;
    a.leaf_pos = b->leaf_pos;
    a.tile_ctr = ws.tile_ctr;
    fill_u32(ws.tile_ctr, 0u, 128, s);
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(kBlock), 0, s, a, static_cast<const void*>(b->nodes),
                       static_cast<const Record*>(b->recs), static_cast<const float*>(b->sh));
    SRT_HIP_TRY(hipGetLastError());
    k_chain<<<(unsigned)((b->G + 255) / 256), 256, 0, s>>>(
        b->G, ws.acc, scene->log_scales, scene->quats, scene->opacity_logits, g_means, g_log_scales,
        g_quats, g_opacity_logits);
    SRT_HIP_TRY(hipGetLastError());
    return SRT_OK;
}

}  // extern "C"
