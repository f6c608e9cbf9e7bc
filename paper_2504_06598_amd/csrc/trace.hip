// Forward stochastic ray tracing on gfx950.
//
// One lane per ray. For an image launch of closest-hit rays the 64 rays of
// an 8x8 pixel tile walk the BVH together (k_trace_wave: one shared stack,
// node and record fetches once per wave, each lane acting only on the nodes
// and Gaussians its own walk would reach); when a pixel needs 2 or 4 passes,
// each pass gets its own lane and a wave covers 8x4 or 4x4 pixels. Otherwise each lane walks the
// W-wide BVH with a per-lane stack in LDS (stride = block size, so the 64
// lanes of a wave hit 64 distinct banks whatever their depths), visiting hit
// children near to far. Each Gaussian of
// a reached leaf is tested in FP64 (Sec. 3.1, eqn "cuboid"); a valid one
// draws u from Philox per sample and is accepted iff u < alpha (eqn "rr");
// each of the N samples of the traversal keeps its closest accepted
// (depth, id) (eqns "cloest", "multisample"). Once every sample holds a hit,
// boxes entering beyond the farthest of them are culled (the clipping of the
// paper's ReportIntersection). A lane whose stack overflows abandons the ray
// and queues it; a second launch reruns queued rays with a stack in global
// memory sized by the tree depth.
#include <algorithm>
#include <climits>
#include <mutex>

#include "srt_internal.hpp"
#include "srt_walk.hpp"

using namespace srt;

namespace {

constexpr int kBlock = 128;

template <int W>
struct LdsStack {
    static constexpr int value = (W == 8) ? 48 : 32;
};

struct TraceArgs {
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
    uint32_t purpose;
    uint32_t k0, k1;
    int32_t spp;
    uint32_t soff;
    float bg[3];
    int32_t stack_cap;
    float* rgb;
    int32_t* hit_gid;
    float* hit_t;
    unsigned long long* counters;
    uint32_t* ctrl;  // [0] overflow count, [1] rays lost by the deep pass
    uint32_t* ovf_list;
    int32_t* deep_stack;
    int32_t deep_cap;
    int64_t max_steps;  // bound on loop iterations of one traversal (a tree visits
                        // each node once); exceeding it marks the ray as lost
    int32_t depth_mode;
    float depth_axis[3];
    float r_max;
    int32_t img_w;  // > 0: rays are a row-major image of this width, traced in tiles
    unsigned long long* work;  // persistent launch: next ray (item) to hand out
    int32_t threshold;         // persistent launch: idle lanes that trigger a refill
    int32_t phases;            // wave-shared image launch: lanes per pixel (1, 2 or 4)
    const int32_t* start;      // per Gaussian: node whose subtree a ray leaving it
                               // walks first (null: every walk starts at the root)
};

struct Counts {
    uint32_t trav = 0, nodes = 0, prims = 0, cands = 0, philox = 0, samples = 0;
};

// Trace every pass of one ray, shade and write its outputs. Returns false on
// a stack overflow (nothing is written then).
template <int W, int N, bool ANY, bool HASH, int DM>
__device__ __forceinline__ bool trace_ray(const TraceArgs& a, int64_t ray, int32_t* stk, int stride,
                                          int cap, Counts& cnt)
{
    const float ox = a.o[3 * ray], oy = a.o[3 * ray + 1], oz = a.o[3 * ray + 2];
    const float dx = a.d[3 * ray], dy = a.d[3 * ray + 1], dz = a.d[3 * ray + 2];
    const float tmin_f = a.tmin ? a.tmin[ray] : 0.0f;
    const float tmax_f = a.tmax ? a.tmax[ray] : INFINITY;
    const int32_t ign = a.ign ? a.ign[ray] : -1;
    const uint32_t rid = a.rid ? a.rid[ray] : (uint32_t)ray;
    const uint32_t sbase = (a.sid ? a.sid[ray] : 0u) + a.soff;
    const bool live = tmax_f > tmin_f;

    Ray rd = make_ray(ox, oy, oz, dx, dy, dz, tmin_f);
    const ForwardCtx fc{a.recs, a.purpose, a.k0, a.k1};
    const DepthCtx dc = make_depth(a.depth_mode, a.depth_axis, rd, a.r_max);
    const WideNode<W>* nodes = static_cast<const WideNode<W>*>(a.nodes);
    FlatStack stack{stk, stride, cap};

    const bool shade = a.rgb != nullptr && !ANY;
    uint32_t samples = 0;  // counted once the whole ray has completed
    float acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
    for (int pass = 0; pass * N < a.spp; ++pass) {
        const int n_act = min(N, a.spp - pass * N);
        float bt[N];
        int32_t bgid[N];
        if (live) {
            ++cnt.trav;
            const int res = resolve_samples<W, N, ANY, FlatStack, HASH, DM>(
                nodes, fc, dc, rd, (double)tmin_f, (double)tmax_f, ign, rid,
                sbase + (uint32_t)(pass * N), n_act, stack, a.max_steps, bt, bgid, cnt.nodes,
                cnt.prims, cnt.cands, cnt.philox);
            if (res == kWalkOverflow) return false;
            samples += (uint32_t)n_act;
        } else {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                bt[k] = INFINITY;
                bgid[k] = INT_MAX;
            }
        }
        // the SH basis is formed after the traversal so it is not live during it
        float Y[16];
        if (shade) {
            const float ex = opaque(dx), ey = opaque(dy), ez = opaque(dz);
            const float n = sqrtf(ex * ex + ey * ey + ez * ez);
            sh_eval(a.deg, ex / n, ey / n, ez / n, Y);
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            if (k >= n_act) continue;
            const bool hit = bgid[k] != INT_MAX;
            const int64_t o = ray * a.spp + pass * N + k;
            if (a.hit_gid) a.hit_gid[o] = hit ? bgid[k] : -1;
            if (a.hit_t) a.hit_t[o] = hit ? bt[k] : INFINITY;
            if (ANY) {
                const float v = hit ? 0.0f : 1.0f;
                acc0 += v; acc1 += v; acc2 += v;
            } else if (shade) {
                if (hit) {
                    const float3 c = clamp0(sh_colour_pre(a.sh, a.deg, bgid[k], Y));
                    acc0 += c.x; acc1 += c.y; acc2 += c.z;
                } else {
                    acc0 += a.bg[0]; acc1 += a.bg[1]; acc2 += a.bg[2];
                }
            }
        }
    }
    if (a.rgb) {
        const float inv = 1.0f / (float)a.spp;
        a.rgb[3 * ray] = acc0 * inv;
        a.rgb[3 * ray + 1] = acc1 * inv;
        a.rgb[3 * ray + 2] = acc2 * inv;
    }
    cnt.samples += samples;
    return true;
}

// COUNT: accumulate the statistics counters (a launch without a counters
// buffer compiles them away, which frees their registers).
template <int W, int N, bool ANY, bool DEEP, bool COUNT, bool HASH, int DM>
__global__ __launch_bounds__(kBlock) void k_trace(TraceArgs a)
{
    __shared__ int32_t lds[DEEP ? 1 : LdsStack<W>::value * kBlock];
    int32_t* stk;
    int stride, cap;
    const int64_t gt = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (DEEP) {
        stk = a.deep_stack + gt;
        stride = kDeepThreads;
        cap = a.deep_cap;
    } else {
        stk = lds + threadIdx.x;
        stride = kBlock;
        cap = min(LdsStack<W>::value, a.stack_cap);
    }
    Counts cnt;
    uint32_t deep_runs = 0, lost = 0;
    if (DEEP) {
        const int64_t n = (int64_t)a.ctrl[0];
        for (int64_t it = gt; it < n; it += (int64_t)gridDim.x * kBlock) {
            const int64_t ray = a.ovf_list[it];
            ++deep_runs;
            if (!trace_ray<W, N, ANY, HASH, DM>(a, ray, stk, stride, cap, cnt)) {
                atomicAdd(&a.ctrl[1], 1u);
                ++lost;
            }
        }
    } else {
        const int64_t t = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
        const int64_t ray = a.img_w > 0 ? tile_pixel(t, a.img_w, a.R / a.img_w) : t;
        if (ray >= 0 && ray < a.R && !trace_ray<W, N, ANY, HASH, DM>(a, ray, stk, stride, cap, cnt)) {
            const uint32_t slot = atomicAdd(&a.ctrl[0], 1u);
            a.ovf_list[slot] = (uint32_t)ray;
        }
    }
    if (COUNT && a.counters) {
        // every lane of the wave reaches this point (no early return above)
        wave_add_u64(a.counters + SRT_CNT_TRAVERSALS, cnt.trav);
        wave_add_u64(a.counters + SRT_CNT_NODES, cnt.nodes);
        wave_add_u64(a.counters + SRT_CNT_PRIMS, cnt.prims);
        wave_add_u64(a.counters + SRT_CNT_CANDIDATES, cnt.cands);
        wave_add_u64(a.counters + SRT_CNT_PHILOX, cnt.philox);
        wave_add_u64(a.counters + SRT_CNT_DEEP, deep_runs);
        wave_add_u64(a.counters + SRT_CNT_RAY_SAMPLES, cnt.samples);
        wave_add_u64(a.counters + SRT_CNT_LOST, lost);
    }
}

// Persistent work-stealing variant (same outputs as k_trace, bit for bit):
// each workgroup is one wave that loops until the rays run out. A lane walks
// its ray one node or one leaf per iteration and runs all passes of the ray
// before it goes idle; when at least `threshold` lanes are idle, the wave
// takes that many rays with one atomic on the work counter. Lanes that
// finish early no longer wait for the longest walk of their wave. A ray
// whose stack overflows is queued for the deep pass (k_trace with DEEP),
// which reruns all its passes.
constexpr int kPersistBlock = 64;
constexpr int kDefaultRefill = 16;

template <int W, int N, bool ANY, bool COUNT, int DM>
__global__ __launch_bounds__(kPersistBlock) void k_trace_persist(TraceArgs a)
{
    __shared__ int32_t lds[LdsStack<W>::value * kPersistBlock];
    const int lane = threadIdx.x;
    const int cap = min(LdsStack<W>::value, a.stack_cap);
    const WideNode<W>* nodes = static_cast<const WideNode<W>*>(a.nodes);
    const int64_t n_items = a.img_w > 0 ? tile_threads(a.img_w, a.R / a.img_w) : a.R;
    const bool shade = a.rgb != nullptr && !ANY;
    Counts cnt;

    bool active = false, exhausted = false;
    int64_t ray = 0;
    int32_t pass = 0, n_act = 0;
    float tmin_f = 0.0f, tmax_f = 0.0f;
    int32_t ign = -1;
    uint32_t rid = 0, sbase = 0, samples = 0;
    Ray lr;
    DepthCtx dc;
    FwdSamples<N> st;
    int32_t node = 0;
    int sp = 0;
    int64_t steps = 0;
    float acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
    const ForwardCtx fc{a.recs, a.purpose, a.k0, a.k1};

    for (;;) {
        // ---- refill idle lanes (wave-uniform decision) ----
        const unsigned long long idle = __ballot(!active);
        const int n_idle = __popcll(idle);
        if (n_idle == 64 && exhausted) break;
        if (!exhausted && (n_idle >= a.threshold || n_idle == 64)) {
            const int leader = __ffsll((long long)idle) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(a.work, (unsigned long long)n_idle);
            base = __shfl(base, leader, 64);
            if (base + (unsigned long long)n_idle >= (unsigned long long)n_items) exhausted = true;
            if (!active) {
                const unsigned long long below = idle & ((1ull << lane) - 1ull);
                const int64_t it = (int64_t)(base + (unsigned long long)__popcll(below));
                const int64_t r = it >= n_items ? -1
                                  : a.img_w > 0 ? tile_pixel(it, a.img_w, a.R / a.img_w)
                                                : it;
                if (r >= 0 && r < a.R) {
                    ray = r;
                    tmin_f = a.tmin ? a.tmin[ray] : 0.0f;
                    tmax_f = a.tmax ? a.tmax[ray] : INFINITY;
                    if (tmax_f > tmin_f) {
                        ign = a.ign ? a.ign[ray] : -1;
                        rid = a.rid ? a.rid[ray] : (uint32_t)ray;
                        sbase = (a.sid ? a.sid[ray] : 0u) + a.soff;
                        lr = make_ray(a.o[3 * ray], a.o[3 * ray + 1], a.o[3 * ray + 2],
                                      a.d[3 * ray], a.d[3 * ray + 1], a.d[3 * ray + 2], tmin_f);
                        dc = make_depth(a.depth_mode, a.depth_axis, lr, a.r_max);
                        pass = 0;
                        n_act = min(N, a.spp);
                        st.reset(n_act, tmax_f);
                        node = 0;
                        sp = 0;
                        steps = 0;
                        samples = 0;
                        acc0 = acc1 = acc2 = 0.0f;
                        active = true;
                        ++cnt.trav;
                    } else {
                        // an empty ray: every sample misses, nothing to walk
                        for (int32_t k = 0; k < a.spp; ++k) {
                            const int64_t o = ray * a.spp + k;
                            if (a.hit_gid) a.hit_gid[o] = -1;
                            if (a.hit_t) a.hit_t[o] = INFINITY;
                        }
                        if (a.rgb) {  // the same sum as a walked ray's, term by term
                            float e0 = 0.0f, e1 = 0.0f, e2 = 0.0f;
                            for (int32_t k = 0; k < a.spp; ++k) {
                                e0 += ANY ? 1.0f : a.bg[0];
                                e1 += ANY ? 1.0f : a.bg[1];
                                e2 += ANY ? 1.0f : a.bg[2];
                            }
                            const float inv = 1.0f / (float)a.spp;
                            a.rgb[3 * ray] = e0 * inv;
                            a.rgb[3 * ray + 1] = e1 * inv;
                            a.rgb[3 * ray + 2] = e2 * inv;
                        }
                    }
                }
            }
        }
        if (!active) continue;

        // ---- one traversal step: one node or one leaf ----
        bool done = false, overflow = false;
        if (++steps > a.max_steps) {
            overflow = true;
        } else if (node >= 0) {
            ++cnt.nodes;
            NodeBuf<W> nb;
            load_node<W>(nodes, node, nb);
            uint32_t key[W];
            slab_keys<W>(nb, lr, st.tcut + (DM == 0 ? 0.0f : dc.node_slack), key);
            sort_keys<W>(key);
            int nh = 0;
#pragma unroll
            for (int c = 0; c < W; ++c) nh += key[c] != 0xFFFFFFFFu;
            if (nh > 0) {
                if (sp + nh - 1 > cap) {
                    overflow = true;
                } else {
#pragma unroll
                    for (int c = W - 1; c >= 1; --c)
                        if (key[c] != 0xFFFFFFFFu) {
                            lds[sp * kPersistBlock + lane] = child_at<W>(nb, key[c] & 7u);
                            ++sp;
                        }
                    node = child_at<W>(nb, key[0] & 7u);
                }
            } else if (sp == 0) {
                done = true;
            } else {
                --sp;
                node = lds[sp * kPersistBlock + lane];
            }
        } else {
            const uint32_t first = leaf_first(node), count = leaf_count(node);
            FwdCounts fcnt;
            const uint32_t s0 = sbase + (uint32_t)(pass * N);
            bool stop = false;
            for (uint32_t i = 0; i < count && !stop; ++i) {
                ++cnt.prims;
                const Record r = load_record(a.recs, first + i);
                stop = fwd_offer<N, ANY, false, DM>(st, r, lr, dc, (double)tmin_f,
                                                    (double)tmax_f, ign, rid, s0, fc, fcnt);
            }
            cnt.cands += fcnt.cands;
            cnt.philox += fcnt.philox;
            if (stop || sp == 0) {
                done = true;
            } else {
                --sp;
                node = lds[sp * kPersistBlock + lane];
            }
        }
        if (overflow) {
            const uint32_t slot = atomicAdd(&a.ctrl[0], 1u);
            a.ovf_list[slot] = (uint32_t)ray;
            active = false;
        } else if (done) {
            // the pass is resolved: write its samples, shade, then the next pass
            float Y[16];
            if (shade) {
                const float ex = opaque(lr.dx), ey = opaque(lr.dy), ez = opaque(lr.dz);
                const float n = sqrtf(ex * ex + ey * ey + ez * ez);
                sh_eval(a.deg, ex / n, ey / n, ez / n, Y);
            }
#pragma unroll
            for (int k = 0; k < N; ++k) {
                if (k >= n_act) continue;
                const bool hit = st.bg[k] != INT_MAX;
                const int64_t o = ray * a.spp + pass * N + k;
                if (a.hit_gid) a.hit_gid[o] = hit ? st.bg[k] : -1;
                if (a.hit_t) a.hit_t[o] = hit ? st.bt[k] : INFINITY;
                if (ANY) {
                    const float v = hit ? 0.0f : 1.0f;
                    acc0 += v; acc1 += v; acc2 += v;
                } else if (shade) {
                    if (hit) {
                        const float3 c = clamp0(sh_colour_pre(a.sh, a.deg, st.bg[k], Y));
                        acc0 += c.x; acc1 += c.y; acc2 += c.z;
                    } else {
                        acc0 += a.bg[0]; acc1 += a.bg[1]; acc2 += a.bg[2];
                    }
                }
            }
            samples += (uint32_t)n_act;
            if ((pass + 1) * N < a.spp) {
                ++pass;
                n_act = min(N, a.spp - pass * N);
                st.reset(n_act, tmax_f);
                node = 0;
                sp = 0;
                steps = 0;
                ++cnt.trav;
            } else {
                if (a.rgb) {
                    const float inv = 1.0f / (float)a.spp;
                    a.rgb[3 * ray] = acc0 * inv;
                    a.rgb[3 * ray + 1] = acc1 * inv;
                    a.rgb[3 * ray + 2] = acc2 * inv;
                }
                cnt.samples += samples;
                active = false;
            }
        }
    }
    if (COUNT && a.counters) {
        wave_add_u64(a.counters + SRT_CNT_TRAVERSALS, cnt.trav);
        wave_add_u64(a.counters + SRT_CNT_NODES, cnt.nodes);
        wave_add_u64(a.counters + SRT_CNT_PRIMS, cnt.prims);
        wave_add_u64(a.counters + SRT_CNT_CANDIDATES, cnt.cands);
        wave_add_u64(a.counters + SRT_CNT_PHILOX, cnt.philox);
        wave_add_u64(a.counters + SRT_CNT_RAY_SAMPLES, cnt.samples);
    }
}

// Wave-shared walks (same outputs as k_trace, bit for bit, except which
// accepted id an any-hit ray reports): each wave is one workgroup and takes
// one 8x8 pixel tile of an image launch, else 64 consecutive rays, and its
// rays traverse the BVH together (walk_wave), so the wave never diverges
// between node steps and leaf tests and reads each node and record once
// instead of once per lane. Lanes keep their own samples, depth cuts and
// candidate tests. When the shared stack would exceed kWaveCap the whole
// group is queued for the deep pass (k_trace with DEEP), which reruns all
// passes of its rays.
constexpr int kWaveCap = 48;

// Image launches whose rays need Q = 2 or 4 passes give each pixel Q lanes,
// lane q running pass q, so a wave covers 64 / Q pixels (8x4 or 4x4): fewer
// distinct rays share each walk. Thread t -> pixel of a w x h image (or -1)
// and its phase q.
__host__ __device__ __forceinline__ void wave_tile_dims(int32_t Q, int32_t& tw, int32_t& th)
{
    tw = Q == 4 ? 4 : 8;
    th = 64 / Q / tw;
}

__host__ __device__ __forceinline__ int64_t wave_tiles(int32_t w, int64_t h, int32_t Q)
{
    int32_t tw, th;
    wave_tile_dims(Q, tw, th);
    return (int64_t)((w + tw - 1) / tw) * ((h + th - 1) / th);
}

__device__ __forceinline__ int64_t wave_pixel(int64_t t, int32_t w, int64_t h, int32_t Q,
                                              int32_t& phase)
{
    int32_t tw, th;
    wave_tile_dims(Q, tw, th);
    const int32_t per = 64 / Q;
    const int32_t lane = (int32_t)(t & 63);
    phase = lane / per;
    const int32_t j = lane % per;
    const int64_t tiles_x = (w + tw - 1) / tw;
    const int64_t tile = t >> 6;
    const int64_t x = (tile % tiles_x) * tw + j % tw;
    const int64_t y = (tile / tiles_x) * th + j / tw;
    return (x < w && y < h) ? y * w + x : -1;
}

// PH: the pixels of an image launch get a.phases (2 or 4) lanes, one per
// pass; otherwise one lane per ray (no registers for the colour hand-over).
// Registers are capped for 3 waves per SIMD: the walk waits on its node and
// record fetches, and at 8 samples per traversal the kernel would otherwise
// hold 233 VGPRs and 2 waves (measured: camera rays of the path-tracer mix
// 12.3 -> 10.4 ms with the spills; a cap for 4 waves was slower, 15.5 ms).
// SH: false for launches without colour output (ids and depths only; the
// path-tracer mix's camera rays), whose registers then hold no colours.
template <int W, int N, bool ANY, bool COUNT, int DM, bool PH, bool SH = true>
__global__ __launch_bounds__(64, 3) void k_trace_wave(TraceArgs a, const void* __restrict__ nodes_v,
                                                   const Record* __restrict__ recs)
{
    __shared__ float lds_t[kWaveCap * 64];
    const WideNode<W>* __restrict__ nodes = static_cast<const WideNode<W>*>(nodes_v);
    const int64_t t = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 64 + threadIdx.x;
    const int32_t Q = PH ? a.phases : 1;  // lanes per pixel; phase q runs passes q, q + Q, ...
    int32_t phase = 0;
    const int64_t ray =
        a.img_w > 0 ? (PH ? wave_pixel(t, a.img_w, a.R / a.img_w, Q, phase)
                          : tile_pixel(t, a.img_w, a.R / a.img_w))
                    : (t < a.R ? t : -1);
    const bool valid = ray >= 0;
    const int64_t rr = valid ? ray : 0;
    const float ox = a.o[3 * rr], oy = a.o[3 * rr + 1], oz = a.o[3 * rr + 2];
    const float dx = a.d[3 * rr], dy = a.d[3 * rr + 1], dz = a.d[3 * rr + 2];
    const float tmin_f = a.tmin ? a.tmin[rr] : 0.0f;
    const float tmax_f = a.tmax ? a.tmax[rr] : INFINITY;
    const int32_t ign = a.ign ? a.ign[rr] : -1;
    const uint32_t rid = a.rid ? a.rid[rr] : (uint32_t)rr;
    const uint32_t sbase = (a.sid ? a.sid[rr] : 0u) + a.soff;
    const bool live = valid && tmax_f > tmin_f;

    Ray rd = make_ray(ox, oy, oz, dx, dy, dz, tmin_f);
    const ForwardCtx fc{recs, a.purpose, a.k0, a.k1};
    const DepthCtx dc = make_depth(a.depth_mode, a.depth_axis, rd, a.r_max);
    const float slack = DM == 0 ? 0.0f : dc.node_slack;
    const bool shade = SH && a.rgb != nullptr && !ANY;
    const int cap = min(kWaveCap, a.stack_cap);

    Counts cnt;
    uint32_t samples = 0;
    float acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
    float col[PH ? N : 1][3];  // PH: this lane's sample colours (of its one pass)
    int my_n = 0;
    bool overflow = false;
    const int P = (a.spp + N - 1) / N;
    for (int it = 0; it * Q < P; ++it) {  // uniform
        const int pass = it * Q + phase;
        const bool has = pass < P;
        const int n_act = has ? min(N, a.spp - pass * N) : 0;
        const bool lv = live && has;
        const uint32_t s0 = sbase + (uint32_t)(pass * N);
        FwdSamples<N> st;
        st.reset(n_act, tmax_f);
        FwdCounts fcnt;
        auto visit = [&](uint32_t ri, bool on) -> bool {
            const Record r = load_record(recs, ri);
            return on && fwd_offer<N, ANY, false, DM>(st, r, rd, dc, (double)tmin_f,
                                                      (double)tmax_f, ign, rid, s0, fc, fcnt);
        };
        uint32_t n_nodes = 0, n_prims = 0;
        WaveStack stk{lds_t, kWaveCap, nullptr, 0, cap};
        const int res = walk_wave<W, ANY>(nodes, rd, lv, st.tcut, slack, stk, a.max_steps,
                                          n_nodes, n_prims, visit);
        if (lv) {
            ++cnt.trav;
            cnt.nodes += n_nodes;
            cnt.prims += n_prims;
            cnt.cands += fcnt.cands;
            cnt.philox += fcnt.philox;
        }
        if (res == kWalkOverflow) {
            overflow = true;
            break;
        }
        if (!valid || !has) continue;
        samples += live ? (uint32_t)n_act : 0u;
        my_n = n_act;
        float Y[16];
        if (shade) {
            const float ex = opaque(dx), ey = opaque(dy), ez = opaque(dz);
            const float n = sqrtf(ex * ex + ey * ey + ez * ez);
            sh_eval(a.deg, ex / n, ey / n, ez / n, Y);
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            if (k >= n_act) continue;
            const bool hit = st.bg[k] != INT_MAX;
            const int64_t o = ray * a.spp + pass * N + k;
            if (a.hit_gid) a.hit_gid[o] = hit ? st.bg[k] : -1;
            if (a.hit_t) a.hit_t[o] = hit ? st.bt[k] : INFINITY;
            if constexpr (!SH) continue;
            float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
            if (ANY) {
                c0 = c1 = c2 = hit ? 0.0f : 1.0f;
            } else if (shade) {
                if (hit) {
                    const float3 c = clamp0(sh_colour_pre(a.sh, a.deg, st.bg[k], Y));
                    c0 = c.x; c1 = c.y; c2 = c.z;
                } else {
                    c0 = a.bg[0]; c1 = a.bg[1]; c2 = a.bg[2];
                }
            }
            if constexpr (PH) {
                col[k][0] = c0; col[k][1] = c1; col[k][2] = c2;
            } else {
                acc0 += c0; acc1 += c1; acc2 += c2;
            }
        }
    }
    if (PH && SH && !overflow) {
        // the pixel's colour sums its samples in sample order, as one lane
        // would: phase 0's samples, then phase 1's, ...; the running sum moves
        // to the pixel's lane of the next phase
        const int per = 64 / Q;
        for (int q = 0; q < Q; ++q) {  // uniform
            if (phase == q) {
#pragma unroll
                for (int k = 0; k < (PH ? N : 1); ++k) {
                    if (k >= my_n) continue;
                    acc0 += col[k][0]; acc1 += col[k][1]; acc2 += col[k][2];
                }
            }
            const float u0 = __shfl_up(acc0, per, 64);
            const float u1 = __shfl_up(acc1, per, 64);
            const float u2 = __shfl_up(acc2, per, 64);
            if (phase == q + 1) {
                acc0 = u0; acc1 = u1; acc2 = u2;
            }
        }
    }
    if (overflow) {
        if (valid && phase == 0) {  // once per pixel
            const uint32_t slot = atomicAdd(&a.ctrl[0], 1u);
            a.ovf_list[slot] = (uint32_t)ray;
        }
    } else if (valid) {
        if (SH && a.rgb && phase == Q - 1) {
            const float inv = 1.0f / (float)a.spp;
            a.rgb[3 * ray] = acc0 * inv;
            a.rgb[3 * ray + 1] = acc1 * inv;
            a.rgb[3 * ray + 2] = acc2 * inv;
        }
        cnt.samples += samples;
    }
    if (COUNT && a.counters) {
        wave_add_u64(a.counters + SRT_CNT_TRAVERSALS, cnt.trav);
        wave_add_u64(a.counters + SRT_CNT_NODES, cnt.nodes);
        wave_add_u64(a.counters + SRT_CNT_PRIMS, cnt.prims);
        wave_add_u64(a.counters + SRT_CNT_CANDIDATES, cnt.cands);
        wave_add_u64(a.counters + SRT_CNT_PHILOX, cnt.philox);
        wave_add_u64(a.counters + SRT_CNT_RAY_SAMPLES, cnt.samples);
    }
}

using WaveFn = void (*)(TraceArgs, const void*, const Record*);

template <int W, int N, bool ANY, int DM, bool PH, bool SH = true>
WaveFn wave_c(bool count)
{
    return count ? k_trace_wave<W, N, ANY, true, DM, PH, SH>
                 : k_trace_wave<W, N, ANY, false, DM, PH, SH>;
}

// shade = false: the launch writes no colours (instantiated without them for
// the pass-per-lane layouts at 4 and 8 samples per traversal)
template <int W, int DM>
WaveFn wave_w(int N, bool any, bool count, bool ph, bool shade)
{
    if (any) return N == 1 && !ph ? wave_c<W, 1, true, DM, false>(count) : nullptr;
    switch (N) {
    case 1: return ph ? wave_c<W, 1, false, DM, true>(count) : wave_c<W, 1, false, DM, false>(count);
    case 2: return ph ? wave_c<W, 2, false, DM, true>(count) : wave_c<W, 2, false, DM, false>(count);
    case 4:
        if (ph) return shade ? wave_c<W, 4, false, DM, true>(count)
                             : wave_c<W, 4, false, DM, true, false>(count);
        return wave_c<W, 4, false, DM, false>(count);
    case 8:
        if (ph) return shade ? wave_c<W, 8, false, DM, true>(count)
                             : wave_c<W, 8, false, DM, true, false>(count);
        return wave_c<W, 8, false, DM, false>(count);
    }
    return nullptr;
}

template <int DM>
WaveFn wave_dm(int W, int N, bool any, bool count, bool ph, bool shade)
{
    switch (W) {
    case 2: return wave_w<2, DM>(N, any, count, ph, shade);
    case 4: return wave_w<4, DM>(N, any, count, ph, shade);
    case 8: return wave_w<8, DM>(N, any, count, ph, shade);
    }
    return nullptr;
}

WaveFn pick_wave(int W, int N, bool any, bool count, int depth_mode, bool ph, bool shade)
{
    return depth_mode == 0 ? wave_dm<0>(W, N, any, count, ph, shade)
                           : wave_dm<1>(W, N, any, count, ph, shade);
}

using KernelFn = void (*)(TraceArgs);

template <int W, int N, bool ANY, bool H, int DM>
void pick(bool count, KernelFn* fast, KernelFn* deep)
{
    *fast = count ? k_trace<W, N, ANY, false, true, H, DM> : k_trace<W, N, ANY, false, false, H, DM>;
    *deep = count ? k_trace<W, N, ANY, true, true, H, DM> : k_trace<W, N, ANY, true, false, H, DM>;
}

template <int W, bool H, int DM>
bool pick_w(int N, bool any, bool count, KernelFn* f, KernelFn* d)
{
    if (any) {
        if (N != 1) return false;
        pick<W, 1, true, H, DM>(count, f, d);
        return true;
    }
    switch (N) {
    case 1: pick<W, 1, false, H, DM>(count, f, d); return true;
    case 2: pick<W, 2, false, H, DM>(count, f, d); return true;
    case 4: pick<W, 4, false, H, DM>(count, f, d); return true;
    case 8: pick<W, 8, false, H, DM>(count, f, d); return true;
    }
    return false;
}

template <bool H, int DM>
bool pick_h(int W, int N, bool any, bool count, KernelFn* f, KernelFn* d)
{
    switch (W) {
    case 2: return pick_w<2, H, DM>(N, any, count, f, d);
    case 4: return pick_w<4, H, DM>(N, any, count, f, d);
    case 8: return pick_w<8, H, DM>(N, any, count, f, d);
    }
    return false;
}

// Philox kernels come with the depth mode fixed at compile time (fewer
// registers); the hash kernels read it at run time.
bool pick_kernels(int W, int N, bool any, bool count, bool hash, int depth_mode, KernelFn* f,
                  KernelFn* d)
{
    if (hash) return pick_h<true, -1>(W, N, any, count, f, d);
    return depth_mode == 0 ? pick_h<false, 0>(W, N, any, count, f, d)
                           : pick_h<false, 1>(W, N, any, count, f, d);
}

template <int W, int N, bool ANY, int DM>
KernelFn persist_fn(bool count)
{
    return count ? k_trace_persist<W, N, ANY, true, DM> : k_trace_persist<W, N, ANY, false, DM>;
}

template <int W, int DM>
KernelFn persist_w(int N, bool any, bool count)
{
    if (any) return N == 1 ? persist_fn<W, 1, true, DM>(count) : nullptr;
    switch (N) {
    case 1: return persist_fn<W, 1, false, DM>(count);
    case 2: return persist_fn<W, 2, false, DM>(count);
    case 4: return persist_fn<W, 4, false, DM>(count);
    case 8: return persist_fn<W, 8, false, DM>(count);
    }
    return nullptr;
}

template <int DM>
KernelFn persist_dm(int W, int N, bool any, bool count)
{
    switch (W) {
    case 2: return persist_w<2, DM>(N, any, count);
    case 4: return persist_w<4, DM>(N, any, count);
    case 8: return persist_w<8, DM>(N, any, count);
    }
    return nullptr;
}

KernelFn pick_persistent(int W, int N, bool any, bool count, int depth_mode)
{
    return depth_mode == 0 ? persist_dm<0>(W, N, any, count)
                           : persist_dm<1>(W, N, any, count);
}

// Waves a persistent launch keeps resident: its occupancy on every CU.
template <class Fn>
srt_status persistent_grid(Fn fn, unsigned* blocks)
{
    int dev = 0, n_cu = 0, per_cu = 0;
    SRT_HIP_TRY(hipGetDevice(&dev));
    SRT_HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    SRT_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(fn), kPersistBlock, 0));
    *blocks = (unsigned)std::max(1, n_cu * std::max(1, per_cu));
    return SRT_OK;
}

srt_status validate_opts(const srt_trace_opts* o)
{
    if (!o) return SRT_ERR_INVALID_ARG;
    if (o->spp < 1) return SRT_ERR_INVALID_ARG;
    const int N = o->n_per_traversal;
    if (N != 1 && N != 2 && N != 4 && N != 8) return SRT_ERR_INVALID_ARG;
    if (o->any_hit && N != 1) return SRT_ERR_INVALID_ARG;
    if (o->stack_limit < 0) return SRT_ERR_INVALID_ARG;
    if (o->depth_mode != 0 && o->depth_mode != 1) return SRT_ERR_INVALID_ARG;
    if (o->image_width < 0) return SRT_ERR_INVALID_ARG;
    if (o->persistent != 0 && o->persistent != 1) return SRT_ERR_INVALID_ARG;
    if (o->refill_threshold < 0 || o->refill_threshold > 64) return SRT_ERR_INVALID_ARG;
    if (o->rng != 0 && o->rng != 1) return SRT_ERR_INVALID_ARG;
    if (o->walk < 0 || o->walk > 2) return SRT_ERR_INVALID_ARG;
    return SRT_OK;
}

// Kernel arguments of a trace launch over `rays`.
void fill_args(const srt_bvh* b, const srt_rays* rays, const srt_trace_opts* o, float* rgb,
               int32_t* hit_gid, float* hit_t, uint64_t* counters, const TraceWorkspace& ws,
               TraceArgs& a)
{
    a = TraceArgs{};
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
    a.k0 = (uint32_t)o->seed;
    a.k1 = (uint32_t)(o->seed >> 32);
    a.spp = o->spp;
    a.soff = o->sample_offset;
    for (int i = 0; i < 3; ++i) a.bg[i] = o->bg[i];
    a.stack_cap = o->stack_limit > 0 ? o->stack_limit : INT_MAX;
    a.rgb = rgb;
    a.hit_gid = hit_gid;
    a.hit_t = hit_t;
    a.counters = reinterpret_cast<unsigned long long*>(counters);
    a.ctrl = ws.ctrl;
    a.ovf_list = ws.ovf_list;
    a.deep_stack = ws.deep_stack;
    a.deep_cap = deep_stack_cap(b);
    a.max_steps = 2 * b->num_nodes + 2 * b->G + 64;
    a.depth_mode = o->depth_mode;
    for (int i = 0; i < 3; ++i) a.depth_axis[i] = o->depth_axis[i];
    a.r_max = b->r_max;
    a.img_w = o->image_width;
    // ctrl[0] overflow count, ctrl[1] rays lost, ctrl[2..3] the persistent work counter
    a.work = reinterpret_cast<unsigned long long*>(ws.ctrl + 2);
    a.threshold = o->refill_threshold > 0 ? o->refill_threshold : kDefaultRefill;
    a.start = b->start_node;
}

// Enqueue the fast and deep traversal launches for an explicit ray set.
srt_status launch_trace(const srt_bvh* b, const srt_rays* rays, const srt_trace_opts* o,
                        float* rgb, int32_t* hit_gid, float* hit_t, uint64_t* counters,
                        void* workspace, hipStream_t s)
{
    KernelFn fast = nullptr, deep = nullptr;
    if (!pick_kernels(b->W, o->n_per_traversal, o->any_hit != 0, counters != nullptr,
                      o->rng == 1, o->depth_mode, &fast, &deep))
        return SRT_ERR_UNSUPPORTED;
    if (o->rng == 1 && o->persistent) return SRT_ERR_UNSUPPORTED;  // Philox only
    const TraceWorkspace ws = trace_workspace(b, rays->count, workspace);
    TraceArgs a;
    fill_args(b, rays, o, rgb, hit_gid, hit_t, counters, ws, a);
    if (a.img_w > 0 && rays->count % a.img_w != 0) return SRT_ERR_INVALID_ARG;
    // wave-shared walks: Philox rays, not persistent; chosen automatically for
    // image launches of closest-hit rays
    const bool wave_ok = o->rng == 0 && !o->persistent;
    if (o->walk == 2 && !wave_ok) return SRT_ERR_UNSUPPORTED;
    WaveFn wf = nullptr;
    a.phases = 1;
    if (o->walk == 2 || (o->walk == 0 && wave_ok && a.img_w > 0 && !o->any_hit)) {
        // 2 or 4 passes per pixel: one lane per pass (see wave_pixel)
        const int passes = (o->spp + o->n_per_traversal - 1) / o->n_per_traversal;
        if (a.img_w > 0 && !o->any_hit && (passes == 2 || passes == 4)) a.phases = passes;
        wf = pick_wave(b->W, o->n_per_traversal, o->any_hit != 0, counters != nullptr,
                       o->depth_mode, a.phases > 1, rgb != nullptr);
        if (!wf) return SRT_ERR_UNSUPPORTED;
    }
    KernelFn pf = nullptr;
    unsigned blocks = 0;
    if (o->persistent && rays->count > 0) {
        pf = pick_persistent(b->W, o->n_per_traversal, o->any_hit != 0, counters != nullptr,
                             o->depth_mode);
        if (!pf) return SRT_ERR_UNSUPPORTED;
        const srt_status gs = persistent_grid(pf, &blocks);
        if (gs != SRT_OK) return gs;
    }
    fill_u32(ws.ctrl, 0u, 4, s);
    if (rays->count > 0) {
        if (pf) {
            hipLaunchKernelGGL(pf, dim3(blocks), dim3(kPersistBlock), 0, s, a);
        } else if (wf) {
            const int64_t tiles = a.img_w > 0 ? wave_tiles(a.img_w, rays->count / a.img_w, a.phases)
                                              : (rays->count + 63) / 64;
            hipLaunchKernelGGL(wf, dim3((unsigned)tiles), dim3(64), 0, s, a,
                               static_cast<const void*>(b->nodes), b->recs);
        } else {
            const int64_t threads =
                a.img_w > 0 ? tile_threads(a.img_w, rays->count / a.img_w) : rays->count;
            const unsigned grid = (unsigned)((threads + kBlock - 1) / kBlock);
            hipLaunchKernelGGL(fast, dim3(grid), dim3(kBlock), 0, s, a);
        }
        SRT_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(deep, dim3(kDeepThreads / kBlock), dim3(kBlock), 0, s, a);
        SRT_HIP_TRY(hipGetLastError());
    }
    return SRT_OK;
}

// --------------------------------------------------------------------------
// Camera rays (canonical FP32; this translation unit is compiled without
// floating-point contraction, and FP32 division and square root are
// correctly rounded).
// --------------------------------------------------------------------------
__device__ __forceinline__ void camera_ray(const srt_camera& c, int32_t x, int32_t y, float o[3],
                                           float d[3])
{
    const float aspect = (float)c.width / (float)c.height;
    const float px = (((float)x + 0.5f) + c.jitter[0]) / (float)c.width;
    const float sx = ((px * 2.0f) - 1.0f) * c.tan_half * aspect;
    const float py = (((float)y + 0.5f) + c.jitter[1]) / (float)c.height;
    const float sy = (1.0f - (py * 2.0f)) * c.tan_half;
    float v[3];
    for (int i = 0; i < 3; ++i) {
        const float a = sx * c.right[i];
        const float b = sy * c.up[i];
        v[i] = (c.forward[i] + a) + b;
    }
    const float xx = v[0] * v[0];
    const float yy = v[1] * v[1];
    const float zz = v[2] * v[2];
    const float n = sqrtf((xx + yy) + zz);
    for (int i = 0; i < 3; ++i) {
        d[i] = v[i] / n;
        o[i] = c.eye[i];
    }
}

__global__ void k_camera_rays(srt_camera c, float* __restrict__ o, float* __restrict__ d)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t R = (int64_t)c.width * c.height;
    if (p >= R) return;
    float oo[3], dd[3];
    camera_ray(c, (int32_t)(p % c.width), (int32_t)(p / c.width), oo, dd);
    for (int i = 0; i < 3; ++i) {
        o[3 * p + i] = oo[i];
        d[3 * p + i] = dd[i];
    }
}

// --------------------------------------------------------------------------
// Path-tracer mix: spawn secondaries from camera hits, then compose.
// --------------------------------------------------------------------------
struct SecRays {
    float *o, *d, *tmin, *tmax;
    int32_t* ign;
    uint32_t *rid, *sid;
};

__global__ void k_spawn(int64_t R, int32_t spp, uint32_t rid_base, const float* __restrict__ co,
                        const float* __restrict__ cd, const int32_t* __restrict__ cam_gid,
                        const float* __restrict__ cam_t, srt_pathmix_opts pm, SecRays sh,
                        SecRays mr)
{
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= R * spp) return;
    const int64_t p = idx / spp;
    const uint32_t s = (uint32_t)(idx % spp);
    const float o[3] = {co[3 * p], co[3 * p + 1], co[3 * p + 2]};
    const float d[3] = {cd[3 * p], cd[3 * p + 1], cd[3 * p + 2]};
    const int32_t g = cam_gid[idx];
    const float tg = g >= 0 ? cam_t[idx] : INFINITY;
    float tp = INFINITY;
    if (d[1] < 0.0f) {
        const float num = pm.plane_y - o[1];
        const float tt = num / d[1];
        if (tt > 0.0f) tp = tt;
    }
    const bool on_gauss = g >= 0 && tg <= tp;
    const bool on_plane = !on_gauss && tp < INFINITY;
    const uint32_t rid = rid_base + (uint32_t)p;
    // empty slots: tmin = 1 > tmax = 0; the kernels that read these rays
    // skip them, and nothing reads an empty slot's other fields
    if (!on_plane) {
        mr.tmin[idx] = 1.0f;
        mr.tmax[idx] = 0.0f;
    }
    if (!on_gauss && !on_plane) {
        sh.tmin[idx] = 1.0f;
        sh.tmax[idx] = 0.0f;
        sh.ign[idx] = -1;
        return;
    }
    const float t = on_gauss ? tg : tp;
    float P[3];
    for (int i = 0; i < 3; ++i) {
        const float prod = t * d[i];
        P[i] = o[i] + prod;
    }
    if (on_plane) P[1] = pm.plane_y;
    const float v[3] = {pm.light[0] - P[0], pm.light[1] - P[1], pm.light[2] - P[2]};
    const float vx2 = v[0] * v[0];
    const float vy2 = v[1] * v[1];
    const float vz2 = v[2] * v[2];
    const float len = sqrtf((vx2 + vy2) + vz2);
    for (int i = 0; i < 3; ++i) {
        sh.o[3 * idx + i] = P[i];
        sh.d[3 * idx + i] = v[i] / len;
    }
    sh.tmin[idx] = pm.tmin_secondary;
    sh.tmax[idx] = len;
    sh.ign[idx] = on_gauss ? g : -1;
    sh.rid[idx] = rid;
    sh.sid[idx] = s;
    if (on_plane) {
        for (int i = 0; i < 3; ++i) mr.o[3 * idx + i] = P[i];
        mr.d[3 * idx] = d[0];
        mr.d[3 * idx + 1] = -d[1];
        mr.d[3 * idx + 2] = d[2];
        mr.tmin[idx] = pm.tmin_secondary;
        mr.tmax[idx] = INFINITY;
        mr.ign[idx] = -1;
        mr.rid[idx] = rid;
        mr.sid[idx] = s;
    }
}

// One thread per pixel, 64 pixels per workgroup. The per-sample inputs are
// staged through LDS 16 samples of each pixel at a time, loaded by
// consecutive threads from consecutive samples (a thread reading its own
// pixel's samples would touch a different cache line per lane on every
// load); the per-sample outputs are written from the same coalesced pass.
constexpr int kComposePix = 64;
constexpr int kComposeChunk = 16;

__global__ __launch_bounds__(kComposePix) void k_compose(
    int64_t R, int32_t spp, int32_t deg, const float* __restrict__ sh,
    const float* __restrict__ cd, const int32_t* __restrict__ cam_gid, SecRays shr, SecRays mrr,
    const int32_t* __restrict__ sh_hit, const int32_t* __restrict__ mr_hit, float bg0, float bg1,
    float bg2, float* __restrict__ rgb, uint8_t* __restrict__ vis_out,
    int32_t* __restrict__ mirror_out)
{
    // sample k of pixel t of the chunk at [t * (kComposeChunk + 1) + k]
    constexpr int kRow = kComposeChunk + 1;
    __shared__ uint8_t s_flag[kComposePix * kRow];  // 1 shadow ray, 2 mirror ray, 4 unoccluded
    __shared__ int32_t s_gid[kComposePix * kRow];   // camera hit, or mirror hit
    __shared__ float s_nl[kComposePix * kRow];      // max(light direction y, 0)
    const int t = threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * kComposePix;
    const int64_t p = p0 + t;
    const bool in = p < R;
    float Yc[16], Ym[16];
    if (in) {
        const float dx = cd[3 * p], dy = cd[3 * p + 1], dz = cd[3 * p + 2];
        const float n = sqrtf(dx * dx + dy * dy + dz * dz);
        sh_eval(deg, dx / n, dy / n, dz / n, Yc);
        sh_eval(deg, dx / n, -dy / n, dz / n, Ym);
    }
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
    // a pixel's samples often shade the same Gaussian: the last colour of
    // each kind is kept (the same inputs give the same bits)
    int32_t last_g = -1, last_m = -1;
    float3 col_g = make_float3(0.0f, 0.0f, 0.0f), col_m = col_g;
    for (int32_t c0 = 0; c0 < spp; c0 += kComposeChunk) {
        const int n_c = min(kComposeChunk, spp - c0);
        __syncthreads();
        for (int e = t; e < kComposePix * kComposeChunk; e += kComposePix) {
            const int px = e / kComposeChunk, k = e % kComposeChunk;
            if (k >= n_c || p0 + px >= R) continue;
            const int64_t i = (p0 + px) * spp + c0 + k;
            const bool has_shadow = shr.tmax[i] > shr.tmin[i];
            const bool has_mirror = mrr.tmax[i] > mrr.tmin[i];
            uint8_t f = 0;
            int32_t g = 0;
            float nl = 0.0f;
            uint8_t vis = 255;
            int32_t mg = -2;
            if (has_shadow) {
                const bool unocc = sh_hit[i] < 0;
                vis = unocc ? 1 : 0;
                f = (uint8_t)(1 | (unocc ? 4 : 0));
                if (!has_mirror) {
                    g = cam_gid[i];
                } else {
                    f |= 2;
                    g = mg = mr_hit[i];
                    nl = fmaxf(shr.d[3 * i + 1], 0.0f);
                }
            }
            s_flag[px * kRow + k] = f;
            s_gid[px * kRow + k] = g;
            s_nl[px * kRow + k] = nl;
            if (vis_out) vis_out[i] = vis;
            if (mirror_out) mirror_out[i] = mg;
        }
        __syncthreads();
        if (!in) continue;
        for (int k = 0; k < n_c; ++k) {
            const uint8_t f = s_flag[t * kRow + k];
            float c0_ = bg0, c1_ = bg1, c2_ = bg2;
            if (f & 1) {
                const float V = (f & 4) ? 1.0f : 0.0f;
                const int32_t g = s_gid[t * kRow + k];
                if (!(f & 2)) {
                    if (g != last_g) {
                        col_g = clamp0(sh_colour_pre(sh, deg, g, Yc));
                        last_g = g;
                    }
                    const float3 c = col_g;
                    const float fv = 0.3f + 0.7f * V;
                    c0_ = c.x * fv; c1_ = c.y * fv; c2_ = c.z * fv;
                } else {
                    float3 Lm = make_float3(bg0, bg1, bg2);
                    if (g >= 0) {
                        if (g != last_m) {
                            col_m = clamp0(sh_colour_pre(sh, deg, g, Ym));
                            last_m = g;
                        }
                        Lm = col_m;
                    }
                    const float lit = 0.5f * V * s_nl[t * kRow + k];
                    c0_ = lit + 0.5f * Lm.x; c1_ = lit + 0.5f * Lm.y; c2_ = lit + 0.5f * Lm.z;
                }
            }
            a0 += c0_; a1 += c1_; a2 += c2_;
        }
    }
    if (!in) return;
    const float inv = 1.0f / (float)spp;
    rgb[3 * p] = a0 * inv;
    rgb[3 * p + 1] = a1 * inv;
    rgb[3 * p + 2] = a2 * inv;
}

// --------------------------------------------------------------------------
// Shadow-ray groups of the path-tracer mix. Samples of one pixel whose
// shading points coincide (the same accepted Gaussian, whose depth key fixes
// the point on the camera ray, or the ground plane, met at the camera ray's
// plane distance) spawn shadow rays that are identical except for their
// sample index, i.e. their acceptance numbers. One walk resolves such a
// group: at each valid candidate every still-unoccluded sample draws its own
// number, and the walk ends once all of them are occluded. Visibility (is
// any candidate accepted) does not depend on the visiting order, so each
// sample's result equals that of its own any-hit walk.
// --------------------------------------------------------------------------
struct ShadowGroups {
    uint32_t* rep;    // [groups] per-sample index of the group's first sample
    uint64_t* mask;   // [groups] bit j: sample j of the pixel belongs to the group
    uint32_t* count;  // number of groups (device)
    int32_t spp;      // samples per pixel (<= 64)
};

// Groups of pixel p, one call per group in sample order; returns the count.
template <class Emit>
__device__ __forceinline__ int pixel_groups(int64_t p, int32_t spp, const SecRays& sh, Emit&& emit)
{
    int n = 0;
    uint64_t done = 0;
    for (int32_t s = 0; s < spp; ++s) {
        const int64_t i = p * spp + s;
        if (((done >> s) & 1ull) || !(sh.tmax[i] > sh.tmin[i])) continue;
        const int32_t key = sh.ign[i];
        uint64_t m = 1ull << s;
        for (int32_t s2 = s + 1; s2 < spp; ++s2) {
            const int64_t i2 = p * spp + s2;
            if (sh.tmax[i2] > sh.tmin[i2] && sh.ign[i2] == key) m |= 1ull << s2;
        }
        done |= m;
        emit(n, (uint32_t)i, m);
        ++n;
    }
    return n;
}

// One thread per pixel; a wave's groups are stored contiguously (pixel
// order within the wave) at an offset taken with one atomic per wave.
__global__ __launch_bounds__(256) void k_shadow_groups(int64_t R, SecRays sh, ShadowGroups g)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool in = p < R;
    const int n = in ? pixel_groups(p, g.spp, sh, [](int, uint32_t, uint64_t) {}) : 0;
    int incl = n;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    const int total = __shfl(incl, 63, 64);
    uint32_t base = 0;
    if (lane == 63 && total > 0) base = atomicAdd(g.count, (uint32_t)total);
    base = __shfl(base, 63, 64) + (uint32_t)(incl - n);
    if (in && n > 0)
        pixel_groups(p, g.spp, sh, [&](int k, uint32_t rep, uint64_t m) {
            g.rep[base + k] = rep;
            g.mask[base + k] = m;
        });
}

// The same groups when spp divides 64: one thread per sample, a pixel's
// samples in consecutive lanes of one wave, keys compared by lane shuffles;
// the first sample of each group stores it. A block's groups (1024 samples)
// are stored contiguously (pixel order) at an offset taken with one atomic
// per block.
constexpr int kGroupBlock = 1024;

__global__ __launch_bounds__(kGroupBlock) void k_shadow_groups_wave(int64_t n, SecRays sh,
                                                                   ShadowGroups g)
{
    constexpr int kWaves = kGroupBlock / 64;
    __shared__ uint32_t wave_n[kWaves], wave_base[kWaves];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int spp = g.spp;
    const bool has = i < n && sh.tmax[i] > sh.tmin[i];
    // a sample without a shadow ray takes a key no shadow ray has (-1 plane, ids >= 0)
    const int32_t key = has ? sh.ign[i] : INT_MIN;
    const int seg = lane - lane % spp;
    const int s = lane - seg;
    uint64_t m = 0;
    for (int j = 0; j < spp; ++j)
        if (__shfl(key, seg + j, 64) == key) m |= 1ull << j;
    const bool leader = has && (m & ((1ull << s) - 1ull)) == 0;
    const uint64_t lead = __ballot(leader);
    if (lane == 0) wave_n[wave] = (uint32_t)__popcll(lead);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int k = 0; k < kWaves; ++k) {
            wave_base[k] = tot;
            tot += wave_n[k];
        }
        const uint32_t b0 = tot ? atomicAdd(g.count, tot) : 0u;
        for (int k = 0; k < kWaves; ++k) wave_base[k] += b0;
    }
    __syncthreads();
    if (leader) {
        const uint32_t at = wave_base[wave] + (uint32_t)__popcll(lead & ((1ull << lane) - 1ull));
        g.rep[at] = (uint32_t)i;
        g.mask[at] = m;
    }
}

// Work-stealing waves over the groups (the refill scheme of k_trace_persist),
// with the record tests taken off the lanes' walks. A lane walks one group's
// ray. Each iteration every walking lane hands up to kRecPerStep records of
// the leaf it is at (and of a leaf it pops right after) to a wave-wide queue in
// LDS, then takes one node step; the wave then tests the queued records one
// per lane, reading the owner's ray from the owner's registers with lane
// shuffles, and occludes samples of the owner's group through a per-lane
// mask in LDS (64-bit LDS atomics). So the node code and the record code do
// not run for different lanes of one step one after the other, and a leaf's
// records are tested side by side.
// `a` describes the per-sample shadow rays (spp 1, any-hit); hit_gid of each
// occluded sample receives a Gaussian that occluded it, -1 if none did. A
// group whose stack overflows queues each of its samples for the deep pass.
template <int W, bool COUNT, int DM>
__global__ __launch_bounds__(kPersistBlock, W == 8 ? 3 : 4) void k_shadow_queue(TraceArgs a,
                                                                                ShadowGroups g)
{
    // width 4: a 28-entry stack leaves LDS for 7 queued records per lane at
    // 4 waves per SIMD (stack 28 + 7 records: 9.9 KB per wave); the extra
    // groups a shorter stack sends to the deep pass are few at leaf size 4
    constexpr int kRecPerStep = W == 4 ? 7 : 4;
    // leaves a lane may take records from per step (a third: 19.4 -> 19.8 ms)
    constexpr int kLeafPerStep = 2;
    constexpr int kStack = W == 4 ? 28 : LdsStack<W>::value;
    __shared__ int32_t lds[kStack * kPersistBlock];
    __shared__ uint32_t q_rec[kPersistBlock * kRecPerStep];
    __shared__ uint8_t q_lane[kPersistBlock * kRecPerStep];
    __shared__ unsigned long long s_pend[kPersistBlock];
    const int lane = threadIdx.x;
    const int cap = min(kStack, a.stack_cap);
    const WideNode<W>* nodes = static_cast<const WideNode<W>*>(a.nodes);
    const int64_t n_items = (int64_t)*g.count;
    const uint32_t spp = (uint32_t)g.spp;
    Counts cnt;

    bool active = false, walking = false, exhausted = false;
    uint32_t pix = 0;
    uint64_t all = 0;
    float tmin_f = 0.0f, tmax_f = 0.0f;
    int32_t ign = -1;
    uint32_t rid = 0;
    Ray lr = make_ray(0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 1.0f, 0.0f);
    DepthCtx dc = make_depth(0, a.depth_axis, lr, a.r_max);
    int32_t node = 0, skip = -1;
    bool phase2 = true;
    int sp = 0;
    int64_t steps = 0;
    const ForwardCtx fc{a.recs, a.purpose, a.k0, a.k1};
    s_pend[lane] = 0;

    for (;;) {
        // ---- refill idle lanes (wave-uniform decision) ----
        const unsigned long long idle = __ballot(!active);
        const int n_idle = __popcll(idle);
        if (n_idle == 64 && exhausted) break;
        if (!exhausted && (n_idle >= a.threshold || n_idle == 64)) {
            const int leader = __ffsll((long long)idle) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(a.work, (unsigned long long)n_idle);
            base = __shfl(base, leader, 64);
            if (base + (unsigned long long)n_idle >= (unsigned long long)n_items) exhausted = true;
            if (!active) {
                const unsigned long long below = idle & ((1ull << lane) - 1ull);
                const int64_t it = (int64_t)(base + (unsigned long long)__popcll(below));
                if (it < n_items) {
                    const int64_t ray = g.rep[it];
                    all = g.mask[it];
                    s_pend[lane] = all;
                    pix = (uint32_t)(ray / spp);
                    tmin_f = a.tmin[ray];
                    tmax_f = a.tmax[ray];
                    ign = a.ign[ray];
                    rid = a.rid[ray];
                    lr = make_ray(a.o[3 * ray], a.o[3 * ray + 1], a.o[3 * ray + 2],
                                  a.d[3 * ray], a.d[3 * ray + 1], a.d[3 * ray + 2], tmin_f);
                    dc = make_depth(a.depth_mode, a.depth_axis, lr, a.r_max);
                    // a ray leaving a Gaussian first walks the subtree around
                    // it, then the whole tree without that subtree
                    node = (a.start && ign >= 0) ? a.start[ign] : 0;
                    phase2 = node == 0;
                    skip = phase2 ? -1 : node;
                    sp = 0;
                    steps = 0;
                    active = walking = true;
                    ++cnt.trav;
                }
            }
        }
        __syncthreads();

        // ---- one step of every walking lane: the records of the leaf it is
        // at go to the queue (up to kRecPerStep, from at most two leaves met
        // one after the other), then it takes one node step ----
        uint32_t q_first[kLeafPerStep];
        int q_n[kLeafPerStep];
#pragma unroll
        for (int l = 0; l < kLeafPerStep; ++l) {
            q_first[l] = 0;
            q_n[l] = 0;
        }
        int q_all = 0;
        if (active && walking) {
            bool ended = false;
            // the next stack entry, or the whole tree after the start
            // subtree; false when the walk is over
            auto next_entry = [&]() -> bool {
                if (sp > 0) {
                    --sp;
                    node = lds[sp * kPersistBlock + lane];
                    return true;
                }
                if (!phase2) {
                    phase2 = true;
                    node = 0;
                    return true;
                }
                return false;
            };
            if (s_pend[lane] == 0) {
                walking = false;  // every sample occluded
            } else if (++steps > a.max_steps) {
                ended = true;
            } else {
                // leaves met one after the other, while queue slots remain
#pragma unroll
                for (int l = 0; l < kLeafPerStep; ++l) {
                    if (node >= 0 || q_all == kRecPerStep) break;
                    const uint32_t first = leaf_first(node), count = leaf_count(node);
                    const int take = (int)min(count, (uint32_t)(kRecPerStep - q_all));
                    q_first[l] = first;
                    q_n[l] = take;
                    q_all += take;
                    if (count > (uint32_t)take) {
                        node = make_leaf(first + (uint32_t)take, count - (uint32_t)take);
                        break;
                    }
                    if (!next_entry()) {
                        walking = false;
                        break;
                    }
                }
                if (walking && node >= 0) {
                    ++cnt.nodes;
                    NodeBuf<W> nb;
                    load_node<W>(nodes, node, nb);
                    uint32_t key[W];
                    slab_keys<W>(nb, lr, tmax_f + (DM == 0 ? 0.0f : dc.node_slack), key);
                    if (phase2 && skip >= 0) {
#pragma unroll
                        for (int c = 0; c < W; ++c)
                            if (nb.n.child[c] == skip) key[c] = 0xFFFFFFFFu;
                    }
                    sort_keys<W>(key);
                    int nh = 0;
#pragma unroll
                    for (int c = 0; c < W; ++c) nh += key[c] != 0xFFFFFFFFu;
                    if (nh > 0) {
                        if (sp + nh - 1 > cap) {
                            ended = true;
                        } else {
#pragma unroll
                            for (int c = W - 1; c >= 1; --c)
                                if (key[c] != 0xFFFFFFFFu) {
                                    lds[sp * kPersistBlock + lane] = child_at<W>(nb, key[c] & 7u);
                                    ++sp;
                                }
                            node = child_at<W>(nb, key[0] & 7u);
                        }
                    } else if (sp > 0) {
                        --sp;
                        node = lds[sp * kPersistBlock + lane];
                    } else if (!phase2) {
                        phase2 = true;
                        node = 0;
                    } else {
                        walking = false;
                    }
                }
            }
            if (ended) {
                // stack or step bound exceeded: the deep pass reruns every
                // sample of the group on its own (the leaf records queued in
                // this step are dropped with the mask)
                for (uint64_t m = all; m; m &= m - 1) {
                    const uint32_t slot = atomicAdd(&a.ctrl[0], 1u);
                    a.ovf_list[slot] = pix * spp + (uint32_t)__builtin_ctzll(m);
                }
                s_pend[lane] = 0;
                active = walking = false;
            }
        }

        // ---- queue the records (wave prefix sum of the counts, bit by bit:
        // a lane queues at most kRecPerStep) ----
        constexpr int kCountBits = kRecPerStep < 8 ? 3 : 4;
        static_assert(kRecPerStep < 16, "at most four bits per count");
        const unsigned long long below = (1ull << lane) - 1ull;
        int excl = 0, total = 0;
#pragma unroll
        for (int bit = 0; bit < kCountBits; ++bit) {
            const unsigned long long m = __ballot((q_all >> bit) & 1);
            excl += __popcll(m & below) << bit;
            total += __popcll(m) << bit;
        }
        {
            int at = excl;
#pragma unroll
            for (int l = 0; l < kLeafPerStep; ++l)
                for (int i = 0; i < q_n[l]; ++i, ++at) {
                    q_rec[at] = q_first[l] + (uint32_t)i;
                    q_lane[at] = (uint8_t)lane;
                }
        }
        __syncthreads();

        // ---- test the queued records, one per lane ----
        for (int b0 = 0; b0 < total; b0 += 64) {
            const int e = b0 + lane;
            const bool has = e < total;
            const int owner = has ? (int)q_lane[e] : lane;
            const float rox = __shfl(lr.ox, owner, 64), roy = __shfl(lr.oy, owner, 64),
                        roz = __shfl(lr.oz, owner, 64);
            const float rdx = __shfl(lr.dx, owner, 64), rdy = __shfl(lr.dy, owner, 64),
                        rdz = __shfl(lr.dz, owner, 64);
            const float r_cull = __shfl(lr.tmin, owner, 64);
            const float r_idd = __shfl(lr.inv_dd, owner, 64);
            const float r_il = __shfl(lr.inv_len, owner, 64);
            const float r_tmin = __shfl(tmin_f, owner, 64), r_tmax = __shfl(tmax_f, owner, 64);
            const int32_t r_ign = __shfl(ign, owner, 64);
            const uint32_t r_rid = (uint32_t)__shfl((int32_t)rid, owner, 64);
            const uint32_t r_pix = (uint32_t)__shfl((int32_t)pix, owner, 64);
            double r_den = 0.0;
            if (DM != 0) r_den = __shfl(dc.inv_den, owner, 64);
            if (has) {
                ++cnt.prims;
                Ray rr;
                rr.ox = rox; rr.oy = roy; rr.oz = roz;
                rr.dx = rdx; rr.dy = rdy; rr.dz = rdz;
                rr.ix = rr.iy = rr.iz = 0.0f;  // not used by the record test
                rr.tmin = r_cull;
                rr.inv_dd = r_idd;
                rr.inv_len = r_il;
                DepthCtx rdc = dc;
                rdc.inv_den = r_den;
                const uint64_t pend_o = s_pend[owner];
                if (pend_o) {
                    const Record rec = load_record(a.recs, q_rec[e]);
                    FwdCounts fcnt;
                    const uint64_t occ =
                        group_offer<DM>(rec, rr, rdc, (double)r_tmin, (double)r_tmax, r_tmax,
                                        r_ign, r_rid, a.soff, pend_o, fc, fcnt);
                    cnt.cands += fcnt.cands;
                    cnt.philox += fcnt.philox;
                    if (occ) {
                        const uint64_t old = atomicAnd(&s_pend[owner], ~occ);
                        for (uint64_t m = old & occ; m; m &= m - 1)
                            a.hit_gid[(int64_t)r_pix * spp + __builtin_ctzll(m)] = rec.gid;
                    }
                }
            }
        }
        __syncthreads();

        // ---- finish lanes whose walk ended or whose samples are all occluded ----
        if (active && (!walking || s_pend[lane] == 0)) {
            for (uint64_t m = s_pend[lane]; m; m &= m - 1)
                a.hit_gid[(int64_t)pix * spp + __builtin_ctzll(m)] = -1;
            cnt.samples += (uint32_t)__popcll(all);
            s_pend[lane] = 0;
            active = walking = false;
        }
    }
    if (COUNT && a.counters) {
        wave_add_u64(a.counters + SRT_CNT_TRAVERSALS, cnt.trav);
        wave_add_u64(a.counters + SRT_CNT_NODES, cnt.nodes);
        wave_add_u64(a.counters + SRT_CNT_PRIMS, cnt.prims);
        wave_add_u64(a.counters + SRT_CNT_CANDIDATES, cnt.cands);
        wave_add_u64(a.counters + SRT_CNT_PHILOX, cnt.philox);
        wave_add_u64(a.counters + SRT_CNT_RAY_SAMPLES, cnt.samples);
    }
}

using KernelFnG = void (*)(TraceArgs, ShadowGroups);

template <int W, int DM>
KernelFnG shadow_fn_w(bool count)
{
    return count ? k_shadow_queue<W, true, DM> : k_shadow_queue<W, false, DM>;
}

KernelFnG pick_shadow(int W, bool count, int depth_mode)
{
    if (depth_mode == 0) {
        switch (W) {
        case 2: return shadow_fn_w<2, 0>(count);
        case 4: return shadow_fn_w<4, 0>(count);
        case 8: return shadow_fn_w<8, 0>(count);
        }
    } else {
        switch (W) {
        case 2: return shadow_fn_w<2, 1>(count);
        case 4: return shadow_fn_w<4, 1>(count);
        case 8: return shadow_fn_w<8, 1>(count);
        }
    }
    return nullptr;
}

__global__ void k_iota(uint32_t* p, uint32_t base, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = base + (uint32_t)i;
}

struct PathmixWs {
    float *co, *cd;
    int32_t* cam_gid;
    float* cam_t;
    SecRays sh, mr;
    int32_t *sh_hit, *mr_hit;
    uint32_t* grp_count;
    uint32_t* grp_rep;
    uint64_t* grp_mask;
    void* trace_ws;
    size_t bytes;
};

PathmixWs pathmix_ws(const srt_bvh* b, int64_t R, int32_t spp, void* base)
{
    PathmixWs w{};
    char* p = static_cast<char*>(base);
    size_t off = 0;
    const int64_t n = R * spp;
    auto take = [&](size_t bytes) {
        void* q = p ? p + off : nullptr;
        off = align_up(off + bytes, 256);
        return q;
    };
    w.co = static_cast<float*>(take(12 * (size_t)R));
    w.cd = static_cast<float*>(take(12 * (size_t)R));
    w.cam_gid = static_cast<int32_t*>(take(4 * (size_t)n));
    w.cam_t = static_cast<float*>(take(4 * (size_t)n));
    for (SecRays* s : {&w.sh, &w.mr}) {
        s->o = static_cast<float*>(take(12 * (size_t)n));
        s->d = static_cast<float*>(take(12 * (size_t)n));
        s->tmin = static_cast<float*>(take(4 * (size_t)n));
        s->tmax = static_cast<float*>(take(4 * (size_t)n));
        s->ign = static_cast<int32_t*>(take(4 * (size_t)n));
        s->rid = static_cast<uint32_t*>(take(4 * (size_t)n));
        s->sid = static_cast<uint32_t*>(take(4 * (size_t)n));
    }
    w.sh_hit = static_cast<int32_t*>(take(4 * (size_t)n));
    w.mr_hit = static_cast<int32_t*>(take(4 * (size_t)n));
    w.grp_count = static_cast<uint32_t*>(take(4));
    w.grp_rep = static_cast<uint32_t*>(take(4 * (size_t)n));
    w.grp_mask = static_cast<uint64_t*>(take(8 * (size_t)n));
    TraceWorkspace tw = trace_workspace(b, n, nullptr);
    w.trace_ws = take(tw.bytes);
    w.bytes = off;
    return w;
}

// Groups of identical shadow rays of a path-tracer mix (see k_shadow_groups).
srt_status build_shadow_groups(int64_t R, int32_t spp, const PathmixWs& w, hipStream_t s)
{
    fill_u32(w.grp_count, 0u, 1, s);
    if (R == 0) return SRT_OK;
    const ShadowGroups g{w.grp_rep, w.grp_mask, w.grp_count, spp};
    if (64 % spp == 0) {
        const int64_t n = R * spp;
        k_shadow_groups_wave<<<(unsigned)((n + kGroupBlock - 1) / kGroupBlock), kGroupBlock, 0,
                               s>>>(n, w.sh, g);
    } else {
        k_shadow_groups<<<(unsigned)((R + 255) / 256), 256, 0, s>>>(R, w.sh, g);
    }
    SRT_HIP_TRY(hipGetLastError());
    return SRT_OK;
}

// The any-hit shadow rays of a path-tracer mix (`rr`: one per sample, spp
// 1) traced as the groups build_shadow_groups made, with the deep pass for
// groups whose stack overflows.
srt_status launch_shadow_groups(const srt_bvh* b, const srt_rays* rr, const srt_trace_opts* so,
                                int64_t R, int32_t spp, const PathmixWs& w, uint64_t* counters,
                                hipStream_t s)
{
    KernelFn fast = nullptr, deep = nullptr;
    if (!pick_kernels(b->W, 1, true, counters != nullptr, false, so->depth_mode, &fast, &deep))
        return SRT_ERR_UNSUPPORTED;
    const KernelFnG gf = pick_shadow(b->W, counters != nullptr, so->depth_mode);
    if (!gf) return SRT_ERR_UNSUPPORTED;
    const TraceWorkspace ws = trace_workspace(b, rr->count, w.trace_ws);
    TraceArgs a;
    fill_args(b, rr, so, nullptr, w.sh_hit, nullptr, counters, ws, a);
    const ShadowGroups g{w.grp_rep, w.grp_mask, w.grp_count, spp};
    unsigned blocks = 0;
    const srt_status gs = persistent_grid(gf, &blocks);
    if (gs != SRT_OK) return gs;
    fill_u32(ws.ctrl, 0u, 4, s);  // overflow count, lost, work counter
    if (R == 0) return SRT_OK;
    hipLaunchKernelGGL(gf, dim3(blocks), dim3(kPersistBlock), 0, s, a, g);
    SRT_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(deep, dim3(kDeepThreads / kBlock), dim3(kBlock), 0, s, a);
    SRT_HIP_TRY(hipGetLastError());
    return SRT_OK;
}

// Scratch of srt_trace_forward_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends. Host code never uses the array's name
// as an address; each device's address comes from hipGetSymbolAddress, taken
// once per device at that device's first call, with the device current.
}  // namespace

constexpr size_t kStaticScratchBytes = (size_t)SRT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the device that runs work on `s`.
srt_status static_scratch(hipStream_t s, void** out)
{
    int dev = -1;
    if (s) {
        hipDevice_t d = -1;
        SRT_HIP_TRY(hipStreamGetDevice(s, &d));
        dev = (int)d;
    } else {
        SRT_HIP_TRY(hipGetDevice(&dev));
    }
    if (dev < 0 || dev >= kMaxDevices) return SRT_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        SRT_HIP_TRY(hipGetDevice(&cur));
        if (cur != dev) SRT_HIP_TRY(hipSetDevice(dev));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) SRT_HIP_TRY(hipSetDevice(cur));
        if (e != hipSuccess || !p) return SRT_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SRT_OK;
}

}  // namespace

extern "C" {

size_t srt_trace_workspace_size(const srt_bvh* b, int64_t num_rays)
{
    if (!b || num_rays < 0) return 0;
    return trace_workspace(b, num_rays, nullptr).bytes;
}

srt_status srt_trace_forward(const srt_bvh* b, const srt_rays* rays, const srt_trace_opts* opts,
                             float* rgb, int32_t* hit_gid, float* hit_t, uint64_t* counters,
                             void* workspace, size_t workspace_bytes, void* stream)
{
    const srt::Range range_("srt_trace_forward");
    if (!b || !rays) return SRT_ERR_INVALID_ARG;
    const srt_status vs = validate_opts(opts);
    if (vs != SRT_OK) return vs;
    if (rays->count < 0 || rays->count > (int64_t)UINT32_MAX) return SRT_ERR_INVALID_ARG;
    if (rays->count > 0 && (!rays->origins || !rays->dirs)) return SRT_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < srt_trace_workspace_size(b, rays->count))
        return SRT_ERR_WORKSPACE;
    return launch_trace(b, rays, opts, rgb, hit_gid, hit_t, counters, workspace,
                        static_cast<hipStream_t>(stream));
}

srt_status srt_trace_forward_noalloc(const srt_bvh* b, const srt_rays* rays,
                                     const srt_trace_opts* opts, float* rgb, int32_t* hit_gid,
                                     float* hit_t, uint64_t* counters, void* stream)
{
    const srt::Range range_("srt_trace_forward_noalloc");
    if (!b || !rays) return SRT_ERR_INVALID_ARG;
    const srt_status vs = validate_opts(opts);
    if (vs != SRT_OK) return vs;
    if (rays->count < 0 || rays->count > (int64_t)UINT32_MAX) return SRT_ERR_INVALID_ARG;
    if (rays->count > 0 && (!rays->origins || !rays->dirs)) return SRT_ERR_INVALID_ARG;
    if (srt_trace_workspace_size(b, rays->count) > kStaticScratchBytes) return SRT_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* ws = nullptr;
    const srt_status ss = static_scratch(s, &ws);
    if (ss != SRT_OK) return ss;
    return launch_trace(b, rays, opts, rgb, hit_gid, hit_t, counters, ws, s);
}

srt_status srt_camera_rays(const srt_camera* cam, float* origins, float* dirs, void* stream)
{
    if (!cam || !origins || !dirs || cam->width < 1 || cam->height < 1) return SRT_ERR_INVALID_ARG;
    const int64_t R = (int64_t)cam->width * cam->height;
    hipStream_t s = static_cast<hipStream_t>(stream);
    k_camera_rays<<<(unsigned)((R + 255) / 256), 256, 0, s>>>(*cam, origins, dirs);
    SRT_HIP_TRY(hipGetLastError());
    return SRT_OK;
}

size_t srt_pathmix_workspace_size(const srt_bvh* b, const srt_camera* cam, int32_t spp)
{
    if (!b || !cam || spp < 1 || cam->width < 1 || cam->height < 1) return 0;
    return pathmix_ws(b, (int64_t)cam->width * cam->height, spp, nullptr).bytes;
}

srt_status srt_trace_pathmix(const srt_bvh* b, const srt_camera* cam, uint32_t ray_id_base,
                             const srt_trace_opts* opts, const srt_pathmix_opts* pm, float* rgb,
                             int32_t* cam_gid, float* cam_t, uint8_t* shadow_vis,
                             int32_t* mirror_gid, uint64_t* counters, void* workspace,
                             size_t workspace_bytes, void* stream)
{
    const srt::Range range_("srt_trace_pathmix");
    if (!b || !cam || !pm || !rgb) return SRT_ERR_INVALID_ARG;
    const srt_status vs = validate_opts(opts);
    if (vs != SRT_OK) return vs;
    if (opts->any_hit) return SRT_ERR_INVALID_ARG;
    if (cam->width < 1 || cam->height < 1) return SRT_ERR_INVALID_ARG;
    const int64_t R = (int64_t)cam->width * cam->height;
    if (R * opts->spp > (int64_t)UINT32_MAX) return SRT_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < srt_pathmix_workspace_size(b, cam, opts->spp))
        return SRT_ERR_WORKSPACE;
    if (pm->stages < 0 || pm->stages > 15) return SRT_ERR_INVALID_ARG;
    const int stages = pm->stages == 0 ? 15 : pm->stages;
    hipStream_t s = static_cast<hipStream_t>(stream);
    PathmixWs w = pathmix_ws(b, R, opts->spp, workspace);
    int32_t* cg = cam_gid ? cam_gid : w.cam_gid;
    float* ct = cam_t ? cam_t : w.cam_t;
    const int64_t n = R * opts->spp;
    // shadow rays resolved per group of identical rays (Philox numbers only)
    const bool grouped = opts->rng == 0 && opts->spp <= 64;
    srt_status st = SRT_OK;

    if (stages & SRT_PATHMIX_CAMERA) {
        const Range r("srt_trace_pathmix: camera rays");
        k_camera_rays<<<(unsigned)((R + 255) / 256), 256, 0, s>>>(*cam, w.co, w.cd);
        SRT_HIP_TRY(hipGetLastError());
        srt_rays cr{};
        cr.count = R;
        cr.origins = w.co;
        cr.dirs = w.cd;
        // camera ray ids: base + pixel
        // (ray_ids null means the index; a nonzero base is added via a table)
        uint32_t* rid_tab = nullptr;
        if (ray_id_base != 0) {
            rid_tab = w.sh.rid;  // scratch: overwritten later by the spawn kernel
            k_iota<<<(unsigned)((R + 255) / 256), 256, 0, s>>>(rid_tab, ray_id_base, R);
            SRT_HIP_TRY(hipGetLastError());
            cr.ray_ids = rid_tab;
        }
        cr.purpose = 0;
        srt_trace_opts co = *opts;
        co.image_width = cam->width;
        st = launch_trace(b, &cr, &co, nullptr, cg, ct, counters, w.trace_ws, s);
        if (st != SRT_OK) return st;
        k_spawn<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(R, opts->spp, ray_id_base, w.co, w.cd,
                                                            cg, ct, *pm, w.sh, w.mr);
        SRT_HIP_TRY(hipGetLastError());
        if (grouped) {
            st = build_shadow_groups(R, opts->spp, w, s);
            if (st != SRT_OK) return st;
        }
    }

    srt_trace_opts so = *opts;
    so.spp = 1;
    so.n_per_traversal = 1;
    so.sample_offset = opts->sample_offset;
    so.image_width = 0;
    so.walk = opts->walk == 1 ? 1 : 0;  // secondary rays are not an image: automatic
                                        // choice gives lane walks
    for (int pass = 0; pass < 2; ++pass) {
        if (!(stages & (pass == 0 ? SRT_PATHMIX_SHADOW : SRT_PATHMIX_MIRROR))) continue;
        const Range r(pass == 0 ? "srt_trace_pathmix: shadow rays" : "srt_trace_pathmix: mirror rays");
        const SecRays& sr = pass == 0 ? w.sh : w.mr;
        srt_rays rr{};
        rr.count = n;
        rr.origins = sr.o;
        rr.dirs = sr.d;
        rr.tmin = sr.tmin;
        rr.tmax = sr.tmax;
        rr.ignore_gid = sr.ign;
        rr.ray_ids = sr.rid;
        rr.sample_ids = sr.sid;
        rr.purpose = pass == 0 ? 2u : 3u;
        so.any_hit = pass == 0 ? 1 : 0;
        // shadow rays (walks of very uneven length: many end at a neighbour of
        // their start, the unoccluded ones cross the whole scene) always run on
        // work-stealing waves, which measured faster for them than one lane per
        // ray and than wave-shared walks (a shared walk lasts as long as its
        // longest ray); camera and mirror rays follow the caller's choice
        so.persistent = pass == 0 && opts->rng == 0 ? 1 : opts->persistent;
        if (pass == 0 && grouped)
            st = launch_shadow_groups(b, &rr, &so, R, opts->spp, w, counters, s);
        else
            st = launch_trace(b, &rr, &so, nullptr, pass == 0 ? w.sh_hit : w.mr_hit, nullptr,
                              counters, w.trace_ws, s);
        if (st != SRT_OK) return st;
    }
    if (stages & SRT_PATHMIX_COMPOSE) {
        k_compose<<<(unsigned)((R + kComposePix - 1) / kComposePix), kComposePix, 0, s>>>(
            R, opts->spp, b->deg, b->sh, w.cd, cg, w.sh, w.mr, w.sh_hit, w.mr_hit, opts->bg[0],
            opts->bg[1], opts->bg[2], rgb, shadow_vis, mirror_gid);
        SRT_HIP_TRY(hipGetLastError());
    }
    return SRT_OK;
}

}  // extern "C"
