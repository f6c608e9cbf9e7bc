// Batched forward: many views with uneven samples per pixel plus extra
// (incoherent) rays in one launch, captured in a HIP graph.
//
// Work is a flat list of items. A camera item is one pass of N samples of one
// pixel of one view; pixels are enumerated in 8x8 tiles, so the 64 items a
// wave fetches together are one tile at one pass (maximally coherent rays).
// An extra-ray item is one pass of one extra ray. Item order: views in
// order, then the extra rays.
//
// Two kernels compute the same per-sample results:
//  * plain: one lane per ray (pixel or extra ray), looping over its passes;
//  * persistent: a grid sized to the machine; every wave keeps stepping its
//    lanes' traversals one node at a time, and whenever at least
//    `refill_threshold` of its 64 lanes are idle it claims that many new items
//    with a single atomic on a global counter (ballot + prefix count hand them
//    out), so lanes whose rays finish early are refilled instead of idling
//    until the longest ray of the wave is done. The records of the leaves the
//    lanes reach go to a wave-wide queue in LDS and are tested one per lane.
//    Colour accumulates into the image with FP32 atomics (each item adds its
//    samples' colours / spp).
// With wave-shared walks (srt_trace_opts.walk != 1) the camera pixels go to
// tile kernels instead: plain, one wave per 8x8 tile looping over its
// passes; persistent, after the extra rays' work-stealing grid, a second
// persistent grid claims one (tile, pass) group of 64 items per atomic on a
// second counter and walks it with its 64 rays together (walk_wave).
// Items whose stack overflows (the lane kernel keeps entries beyond its LDS
// part in global memory, so there only a walk past the tree's depth bound
// does) are queued; a deep pass with a global-memory stack reruns them (an
// item contributes only once complete).
#include <algorithm>
#include <climits>
#include <vector>

#include "srt_internal.hpp"
#include "srt_walk.hpp"

using namespace srt;

namespace {

constexpr int kTile = 8;
constexpr int kPersistBlock = 64;  // one wave per workgroup
constexpr int kPlainBlock = 128;

struct Segment {
    // a camera view (width > 0) or the extra rays (width == 0)
    srt_camera cam;
    int64_t item_begin;   // first item of the segment (persistent numbering)
    int64_t enum_begin;   // first lane of the segment (plain numbering, tile-padded)
    int64_t ray_begin;    // first output row (pixel or extra ray) in the outputs
    int64_t sample_begin; // first sample index in the per-sample outputs
    int32_t width, height, tiles_x;
    int32_t spp, passes;
    int32_t n;            // samples per pass (per traversal)
    uint32_t ray_id_base;
    int64_t rays;         // pixels or extra rays
};

struct BatchArgs {
    int64_t first;        // plain: enumerated index of lane 0 of the grid
    int64_t n_cam;        // camera items (persistent) or camera lanes (plain), a multiple of 64
    unsigned long long* groups;  // persistent wave kernel: next (tile, pass) group
    const void* nodes;
    const Record* recs;
    const float* sh;
    int32_t deg;
    const Segment* segs;
    int32_t n_segs;
    int64_t n_items;      // total items (persistent) or rays (plain)
    // extra rays
    const float* eo;
    const float* ed;
    const float* etmin;
    const float* etmax;
    const uint32_t* erid;
    uint32_t epurpose;
    uint32_t k0, k1;
    uint32_t soff;
    float bg[3];
    int32_t stack_cap;
    float* rgb;           // [rows, 3]: views' pixels, then extra rays
    int32_t* hit_gid;     // [samples] or null
    unsigned long long* counters;
    unsigned long long* work;  // persistent work counter
    uint32_t* ctrl;       // [0] overflow count, [1] lost
    uint64_t* ovf_list;   // queued items (persistent) or rays (plain)
    int32_t* deep_stack;
    int32_t deep_cap;
    int32_t* lane_stack;     // persistent lane kernel: stack entries beyond LDS
    int32_t lane_stack_cap;  // entries per lane there
    int32_t lds_stack;       // entries per lane kept in LDS (<= kQueueStack)
    int32_t threshold;
    int64_t max_steps;
    int32_t N;
    int32_t depth_mode;
    float depth_axis[3];
    float r_max;
};

// Segment of an item (by_item) or plain lane index by binary search.
__device__ __forceinline__ int find_seg(const BatchArgs& a, int64_t idx, bool by_item)
{
    int lo = 0, hi = a.n_segs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t b = by_item ? a.segs[mid].item_begin : a.segs[mid].enum_begin;
        if (b <= idx) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Canonical camera ray (FP32, single rounded operations in a fixed order;
// this translation unit is compiled without contraction).
__device__ __forceinline__ void cam_ray(const srt_camera& c, int32_t x, int32_t y, float o[3], float d[3])
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

// A ray of the batch: row (output index), geometry and Philox identity.
struct BRay {
    int64_t row;          // output row in rgb
    int64_t sample0;      // per-sample output index of sample 0 of this ray
    float o[3], d[3];
    float tmin, tmax;
    uint32_t rid, purpose;
    int32_t spp, npass;   // samples, samples per pass
    bool valid;
};

// Ray number r (within segment s) of the batch.
__device__ __forceinline__ BRay seg_ray(const BatchArgs& a, const Segment& S, int64_t r)
{
    BRay b;
    b.spp = S.spp;
    b.npass = S.n;
    for (int i = 0; i < 3; ++i) {
        b.o[i] = 0.0f;
        b.d[i] = 0.0f;
    }
    if (S.width > 0) {
        // 8x8 tiles, row-major tiles; pixels outside the image are not rays
        const int64_t tile = r / (kTile * kTile);
        const int32_t in = (int32_t)(r % (kTile * kTile));
        const int32_t x = (int32_t)(tile % S.tiles_x) * kTile + (in % kTile);
        const int32_t y = (int32_t)(tile / S.tiles_x) * kTile + (in / kTile);
        b.valid = x < S.width && y < S.height;
        const int64_t pix = (int64_t)y * S.width + x;
        b.row = S.ray_begin + pix;
        b.sample0 = S.sample_begin + pix * S.spp;
        b.rid = S.ray_id_base + (uint32_t)pix;
        b.purpose = 0;
        b.tmin = 0.0f;
        b.tmax = INFINITY;
        if (b.valid) cam_ray(S.cam, x, y, b.o, b.d);
    } else {
        b.valid = r < S.rays;
        const int64_t rr = b.valid ? r : 0;
        b.row = S.ray_begin + r;
        b.sample0 = S.sample_begin + r * S.spp;
        b.rid = a.erid ? a.erid[rr] : S.ray_id_base + (uint32_t)r;
        b.purpose = a.epurpose;
        b.tmin = a.etmin ? a.etmin[rr] : 0.0f;
        b.tmax = a.etmax ? a.etmax[rr] : INFINITY;
        if (b.valid)
            for (int i = 0; i < 3; ++i) {
                b.o[i] = a.eo[3 * r + i];
                b.d[i] = a.ed[3 * r + i];
            }
    }
    return b;
}

// Rays a segment enumerates (camera views: whole 8x8 tiles).
__host__ __device__ inline int64_t seg_rays_enumerated(const Segment& S)
{
    if (S.width > 0) {
        const int64_t ty = (S.height + kTile - 1) / kTile;
        return (int64_t)S.tiles_x * ty * kTile * kTile;
    }
    return S.rays;
}

struct LaneCounts {
    uint32_t trav = 0, nodes = 0, prims = 0, cands = 0, philox = 0, samples = 0;
};

// Resolve samples [pass*N, pass*N + n_act) of ray b, shade them and add their
// colours / spp to the output (atomically when `atomic`). Returns false on a
// stack overflow (nothing was written).
template <int W, int N, int DM, class Stack>
__device__ __forceinline__ bool run_pass(const BatchArgs& a, const BRay& b, int pass, Stack& stk,
                                         LaneCounts& cnt, bool atomic, float acc[3])
{
    const int n_act = min(b.npass, b.spp - pass * b.npass);
    Ray ray = make_ray(b.o[0], b.o[1], b.o[2], b.d[0], b.d[1], b.d[2], b.tmin);
    const ForwardCtx fc{a.recs, b.purpose, a.k0, a.k1};
    const DepthCtx dc = make_depth(a.depth_mode, a.depth_axis, ray, a.r_max);
    float bt[N];
    int32_t bg[N];
    ++cnt.trav;
    const int res = resolve_samples<W, N, false, Stack, false, DM>(
        static_cast<const WideNode<W>*>(a.nodes), fc, dc, ray, (double)b.tmin, (double)b.tmax, -1,
        b.rid, a.soff + (uint32_t)(pass * b.npass), n_act, stk, a.max_steps, bt, bg, cnt.nodes,
        cnt.prims, cnt.cands, cnt.philox);
    if (res == kWalkOverflow) return false;
    float Y[16];
    const float n = sqrtf(b.d[0] * b.d[0] + b.d[1] * b.d[1] + b.d[2] * b.d[2]);
    sh_eval(a.deg, b.d[0] / n, b.d[1] / n, b.d[2] / n, Y);
    float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        if (k >= n_act) continue;
        const bool hit = bg[k] != 0x7FFFFFFF;
        if (a.hit_gid) a.hit_gid[b.sample0 + pass * b.npass + k] = hit ? bg[k] : -1;
        if (hit) {
            const float3 c = clamp0(sh_colour_pre(a.sh, a.deg, bg[k], Y));
            c0 += c.x; c1 += c.y; c2 += c.z;
        } else {
            c0 += a.bg[0]; c1 += a.bg[1]; c2 += a.bg[2];
        }
    }
    const float w = 1.0f / (float)b.spp;
    if (atomic) {
        // an item counts its samples when it completes (items are atomic units)
        cnt.samples += (uint32_t)n_act;
        atomicAdd(a.rgb + 3 * b.row, c0 * w);
        atomicAdd(a.rgb + 3 * b.row + 1, c1 * w);
        atomicAdd(a.rgb + 3 * b.row + 2, c2 * w);
    } else {
        acc[0] += c0; acc[1] += c1; acc[2] += c2;
    }
    return true;
}

// run_pass over a walk shared by the wave's 64 rays (all lanes call it, with
// the same pass; lanes whose ray is not valid take part without samples).
// Returns false (wave-uniform) on a stack overflow; nothing was written then.
template <int W, int N, int DM>
__device__ __forceinline__ bool wave_pass(const BatchArgs& a, const WideNode<W>* __restrict__ nodes,
                                          const Record* __restrict__ recs, const BRay& b, int pass,
                                          WaveStack& stk, LaneCounts& cnt, bool atomic,
                                          float acc[3])
{
    const bool live = b.valid && b.tmax > b.tmin;
    const int n_act = live ? min(b.npass, b.spp - pass * b.npass) : 0;
    Ray ray = make_ray(b.o[0], b.o[1], b.o[2], b.d[0], b.d[1], b.d[2], b.tmin);
    const ForwardCtx fc{recs, b.purpose, a.k0, a.k1};
    const DepthCtx dc = make_depth(a.depth_mode, a.depth_axis, ray, a.r_max);
    float bt[N];
    int32_t bg[N];
    uint32_t n_nodes = 0, n_prims = 0;
    const int res = resolve_samples_wave<W, N, DM>(
        nodes, recs, fc, dc, ray, live, (double)b.tmin, (double)b.tmax, -1, b.rid,
        a.soff + (uint32_t)(pass * b.npass), n_act, stk, a.max_steps, bt, bg, n_nodes, n_prims,
        cnt.cands, cnt.philox);
    if (live) {
        ++cnt.trav;
        cnt.nodes += n_nodes;
        cnt.prims += n_prims;
    }
    if (res == kWalkOverflow) return false;
    if (!b.valid) return true;
    float Y[16];
    const float n = sqrtf(b.d[0] * b.d[0] + b.d[1] * b.d[1] + b.d[2] * b.d[2]);
    sh_eval(a.deg, b.d[0] / n, b.d[1] / n, b.d[2] / n, Y);
    float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    const int n_out = min(b.npass, b.spp - pass * b.npass);  // an empty ray's samples are misses
#pragma unroll
    for (int k = 0; k < N; ++k) {
        if (k >= n_out) continue;
        const bool hit = k < n_act && bg[k] != 0x7FFFFFFF;
        if (a.hit_gid) a.hit_gid[b.sample0 + pass * b.npass + k] = hit ? bg[k] : -1;
        if (hit) {
            const float3 c = clamp0(sh_colour_pre(a.sh, a.deg, bg[k], Y));
            c0 += c.x; c1 += c.y; c2 += c.z;
        } else {
            c0 += a.bg[0]; c1 += a.bg[1]; c2 += a.bg[2];
        }
    }
    const float w = 1.0f / (float)b.spp;
    if (atomic) {
        cnt.samples += (uint32_t)n_out;
        atomicAdd(a.rgb + 3 * b.row, c0 * w);
        atomicAdd(a.rgb + 3 * b.row + 1, c1 * w);
        atomicAdd(a.rgb + 3 * b.row + 2, c2 * w);
    } else {
        acc[0] += c0; acc[1] += c1; acc[2] += c2;
    }
    return true;
}

template <bool COUNT>
__device__ __forceinline__ void flush_counts(const BatchArgs& a, const LaneCounts& c, uint32_t deep,
                                             uint32_t lost)
{
    if (!COUNT || !a.counters) return;
    wave_add_u64(a.counters + SRT_CNT_TRAVERSALS, c.trav);
    wave_add_u64(a.counters + SRT_CNT_NODES, c.nodes);
    wave_add_u64(a.counters + SRT_CNT_PRIMS, c.prims);
    wave_add_u64(a.counters + SRT_CNT_CANDIDATES, c.cands);
    wave_add_u64(a.counters + SRT_CNT_PHILOX, c.philox);
    wave_add_u64(a.counters + SRT_CNT_DEEP, deep);
    wave_add_u64(a.counters + SRT_CNT_RAY_SAMPLES, c.samples);
    wave_add_u64(a.counters + SRT_CNT_LOST, lost);
}

// ---------------------------------------------------------------------------
// Plain: one lane per ray.
// ---------------------------------------------------------------------------
template <int W, int N, bool COUNT, int DM>
__global__ __launch_bounds__(kPlainBlock) void k_plain(BatchArgs a)
{
    __shared__ int32_t lds[32 * kPlainBlock];
    const int64_t r = a.first + blockIdx.x * (int64_t)kPlainBlock + threadIdx.x;
    FlatStack stk{lds + threadIdx.x, kPlainBlock, min(32, a.stack_cap)};
    LaneCounts cnt;
    if (r < a.n_items) {
        const Segment& S = a.segs[find_seg(a, r, false)];
        const BRay b = seg_ray(a, S, r - S.enum_begin);
        if (b.valid) {
            float acc[3] = {0.0f, 0.0f, 0.0f};
            bool ok = true;
            for (int pass = 0; pass * b.npass < b.spp && ok; ++pass)
                ok = run_pass<W, N, DM>(a, b, pass, stk, cnt, false, acc);
            if (ok) {
                cnt.samples += (uint32_t)b.spp;
                const float w = 1.0f / (float)b.spp;
                a.rgb[3 * b.row] = acc[0] * w;
                a.rgb[3 * b.row + 1] = acc[1] * w;
                a.rgb[3 * b.row + 2] = acc[2] * w;
            } else {
                const uint32_t slot = atomicAdd(&a.ctrl[0], 1u);
                a.ovf_list[slot] = (uint64_t)r;
            }
        }
    }
    flush_counts<COUNT>(a, cnt, 0, 0);
}

// Plain deep pass: queued rays with the global-memory stack.
template <int W, int N, bool COUNT, int DM>
__global__ __launch_bounds__(kPlainBlock) void k_plain_deep(BatchArgs a)
{
    const int64_t gt = blockIdx.x * (int64_t)kPlainBlock + threadIdx.x;
    FlatStack stk{a.deep_stack + gt, kDeepThreads, a.deep_cap};
    LaneCounts cnt;
    uint32_t deep = 0, lost = 0;
    const int64_t n = a.ctrl[0];
    for (int64_t it = gt; it < n; it += (int64_t)gridDim.x * kPlainBlock) {
        const int64_t r = (int64_t)a.ovf_list[it];
        const Segment& S = a.segs[find_seg(a, r, false)];
        const BRay b = seg_ray(a, S, r - S.enum_begin);
        float acc[3] = {0.0f, 0.0f, 0.0f};
        bool ok = true;
        ++deep;
        for (int pass = 0; pass * b.npass < b.spp && ok; ++pass)
            ok = run_pass<W, N, DM>(a, b, pass, stk, cnt, false, acc);
        if (!ok) {
            ++lost;
            atomicAdd(&a.ctrl[1], 1u);
            continue;
        }
        cnt.samples += (uint32_t)b.spp;
        const float w = 1.0f / (float)b.spp;
        a.rgb[3 * b.row] = acc[0] * w;
        a.rgb[3 * b.row + 1] = acc[1] * w;
        a.rgb[3 * b.row + 2] = acc[2] * w;
    }
    flush_counts<COUNT>(a, cnt, deep, lost);
}

// ---------------------------------------------------------------------------
// Persistent work stealing.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void decode_item(const BatchArgs& a, int64_t item, int32_t& seg,
                                            int64_t& ray, int32_t& pass)
{
    seg = find_seg(a, item, true);
    const Segment& S = a.segs[seg];
    const int64_t local = item - S.item_begin;
    if (S.width > 0) {
        // tile-major: each tile runs its passes back to back, 64 items per pass
        const int64_t per_tile = (int64_t)S.passes * kTile * kTile;
        const int64_t tile = local / per_tile;
        const int64_t rem = local % per_tile;
        pass = (int32_t)(rem / (kTile * kTile));
        ray = tile * kTile * kTile + rem % (kTile * kTile);
    } else {
        ray = local / S.passes;
        pass = (int32_t)(local % S.passes);
    }
}

// Records a walking lane hands to the wave's queue per step.
constexpr int kQueueRecs = 8;

// Lane stack entries of the queued lane refilling kept in LDS; deeper ones
// go to the lane's part of a global-memory stack (BatchArgs::lane_stack).
constexpr int kQueueStack = 24;

// LDS of the queued lane refilling: the lane stacks, the N sample keys of
// each lane, the record queue (record index, owner lane).
template <int N>
struct QueueLds {
    int32_t stack[kQueueStack * kPersistBlock];
    unsigned long long keys[N * kPersistBlock];
    uint32_t q_rec[kQueueRecs * kPersistBlock];
    uint8_t q_lane[kQueueRecs * kPersistBlock];
    unsigned long long dirty;  // bit l: a key of lane l fell in this step
};

// The lane-refilling loop over items numbered from the work counter's
// starting value up to n_items, with the record tests taken off the lanes'
// walks (the scheme of the queued shadow kernel, for closest hits). Each step a walking lane hands up to kQueueRecs records of the leaf it is
// at to a wave-wide queue in LDS and then takes one node step; the wave tests
// the queued records one per lane with the owner's ray read through lane
// shuffles, and lowers the owner's sample keys (kept in LDS) with atomic
// minima. An owner's depth cut follows its keys one step later, which only
// tests more records. A lane whose walk has ended shades its samples once
// the records it queued in its last step are tested.
template <int W, int N, bool COUNT, int DM>
__device__ __forceinline__ void persist_queue(const BatchArgs& a, QueueLds<N>& L, LaneCounts& cnt)
{
    const int lane = threadIdx.x;
    const int n_lds = a.lds_stack;
    const int cap = min(n_lds + a.lane_stack_cap, a.stack_cap);
    const WideNode<W>* nodes = static_cast<const WideNode<W>*>(a.nodes);
    unsigned long long* keys = L.keys + lane;
    // entry e >= n_lds of this lane's stack: glb[(e - n_lds) * gstride]
    const int64_t gstride = (int64_t)gridDim.x * kPersistBlock;
    int32_t* glb = a.lane_stack ? a.lane_stack + (int64_t)blockIdx.x * kPersistBlock + lane
                                : nullptr;
    const unsigned long long miss_key = pack_key(INFINITY, 0x7FFFFFFF);

    bool active = false, walking = false, exhausted = false;
    BRay b{};
    int32_t pass = 0, n_act = 0;
    int64_t item_id = 0;
    uint32_t s0 = 0;
    Ray lr = make_ray(0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 1.0f, 0.0f);
    DepthCtx dc = make_depth(0, a.depth_axis, lr, a.r_max);
    float wt = INFINITY, tcut = 0.0f;
    int32_t wg = 0x7FFFFFFF;
    int32_t node = 0;
    int sp = 0;
    int64_t steps = 0;
    auto push = [&](int32_t v) {
        if (sp < n_lds)
            L.stack[sp * kPersistBlock + lane] = v;
        else
            glb[(int64_t)(sp - n_lds) * gstride] = v;
        ++sp;
    };
    auto pop = [&]() -> int32_t {
        --sp;
        return sp < n_lds ? L.stack[sp * kPersistBlock + lane]
                          : glb[(int64_t)(sp - n_lds) * gstride];
    };

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
            if (base + (unsigned long long)n_idle >= (unsigned long long)a.n_items) exhausted = true;
            if (!active) {
                const unsigned long long below = idle & ((1ull << lane) - 1ull);
                const int64_t it = (int64_t)(base + (unsigned long long)__popcll(below));
                if (it < a.n_items) {
                    int32_t seg;
                    int64_t ray;
                    decode_item(a, it, seg, ray, pass);
                    b = seg_ray(a, a.segs[seg], ray);
                    if (b.valid) {
                        item_id = it;
                        n_act = min(b.npass, b.spp - pass * b.npass);
                        s0 = a.soff + (uint32_t)(pass * b.npass);
                        lr = make_ray(b.o[0], b.o[1], b.o[2], b.d[0], b.d[1], b.d[2], b.tmin);
                        dc = make_depth(a.depth_mode, a.depth_axis, lr, a.r_max);
#pragma unroll
                        for (int k = 0; k < N; ++k) keys[64 * k] = miss_key;
                        wt = INFINITY;
                        wg = 0x7FFFFFFF;
                        tcut = b.tmax;
                        node = 0;
                        sp = 0;
                        steps = 0;
                        active = walking = true;
                        ++cnt.trav;
                    }
                }
            }
        }
        __syncthreads();

        // ---- one step of every walking lane: up to kQueueRecs records of
        // the leaf it is at go to the queue, then it takes one node step ----
        uint32_t q_first = 0;
        int q_n = 0;
        if (active && walking) {
            bool ended = false;
            if (++steps > a.max_steps) {
                ended = true;
            } else {
                if (node < 0) {
                    const uint32_t first = leaf_first(node), count = leaf_count(node);
                    q_first = first;
                    q_n = (int)min(count, (uint32_t)kQueueRecs);
                    if (count > (uint32_t)q_n) {
                        node = make_leaf(first + (uint32_t)q_n, count - (uint32_t)q_n);
                    } else if (sp > 0) {
                        node = pop();
                    } else {
                        walking = false;
                    }
                }
                if (walking && node >= 0) {
                    ++cnt.nodes;
                    NodeBuf<W> nb;
                    load_node<W>(nodes, node, nb);
                    uint32_t key[W];
                    slab_keys<W>(nb, lr, tcut + (DM == 0 ? 0.0f : dc.node_slack), key);
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
                                if (key[c] != 0xFFFFFFFFu) push(child_at<W>(nb, key[c] & 7u));
                            node = child_at<W>(nb, key[0] & 7u);
                        }
                    } else if (sp > 0) {
                        node = pop();
                    } else {
                        walking = false;
                    }
                }
            }
            if (ended) {
                // stack or step bound exceeded: the deep pass reruns the item
                const uint32_t slot = atomicAdd(&a.ctrl[0], 1u);
                a.ovf_list[slot] = (uint64_t)item_id;
                q_n = 0;
                active = walking = false;
            }
        }

        // ---- queue the records (wave prefix sum of the counts, bit by
        // bit: a lane queues at most kQueueRecs <= 8) ----
        static_assert(kQueueRecs <= 8, "four bits per count");
        const unsigned long long below = (1ull << lane) - 1ull;
        int excl = 0, total = 0;
#pragma unroll
        for (int bit = 0; bit < 4; ++bit) {
            const unsigned long long m = __ballot((q_n >> bit) & 1);
            excl += __popcll(m & below) << bit;
            total += __popcll(m) << bit;
        }
        for (int i = 0; i < q_n; ++i) {
            L.q_rec[excl + i] = q_first + (uint32_t)i;
            L.q_lane[excl + i] = (uint8_t)lane;
        }
        if (lane == 0) L.dirty = 0ull;
        __syncthreads();

        // ---- test the queued records, one per lane ----
        for (int e0 = 0; e0 < total; e0 += 64) {
            const int e = e0 + lane;
            const bool has = e < total;
            const int owner = has ? (int)L.q_lane[e] : lane;
            Ray rr;
            rr.ox = __shfl(lr.ox, owner, 64);
            rr.oy = __shfl(lr.oy, owner, 64);
            rr.oz = __shfl(lr.oz, owner, 64);
            rr.dx = __shfl(lr.dx, owner, 64);
            rr.dy = __shfl(lr.dy, owner, 64);
            rr.dz = __shfl(lr.dz, owner, 64);
            rr.ix = rr.iy = rr.iz = 0.0f;  // not used by the record test
            rr.tmin = __shfl(lr.tmin, owner, 64);
            rr.inv_dd = __shfl(lr.inv_dd, owner, 64);
            rr.inv_len = __shfl(lr.inv_len, owner, 64);
            const float r_tmin = __shfl(b.tmin, owner, 64), r_tmax = __shfl(b.tmax, owner, 64);
            const float r_tcut = __shfl(tcut, owner, 64), r_wt = __shfl(wt, owner, 64);
            const int32_t r_wg = __shfl(wg, owner, 64);
            const uint32_t r_rid = (uint32_t)__shfl((int32_t)b.rid, owner, 64);
            const uint32_t r_pur = (uint32_t)__shfl((int32_t)b.purpose, owner, 64);
            const uint32_t r_s0 = (uint32_t)__shfl((int32_t)s0, owner, 64);
            const int r_nact = __shfl(n_act, owner, 64);
            DepthCtx rdc = dc;
            if (DM != 0) rdc.inv_den = __shfl(dc.inv_den, owner, 64);
            if (has) {
                ++cnt.prims;
                const Record rec = load_record(a.recs, L.q_rec[e]);
                FwdCounts fcnt;
                if (keyed_offer<N, DM>(rec, rr, rdc, (double)r_tmin, (double)r_tmax, r_tcut, r_wt,
                                       r_wg, r_rid, r_s0, r_nact, r_pur, a.k0, a.k1,
                                       L.keys + owner, fcnt))
                    atomicOr(&L.dirty, 1ull << owner);
                cnt.cands += fcnt.cands;
                cnt.philox += fcnt.philox;
            }
        }
        __syncthreads();

        if (!active) continue;
        // ---- the depth cut follows the keys; an ended walk shades ----
        if ((L.dirty >> lane) & 1ull) {
            wt = -INFINITY;
            wg = (int32_t)0x80000000;
#pragma unroll
            for (int k = 0; k < N; ++k) {
                if (k >= n_act) continue;
                float t;
                int32_t g;
                unpack_key(keys[64 * k], t, g);
                if (key_less(wt, wg, t, g)) {
                    wt = t;
                    wg = g;
                }
            }
            tcut = fminf(cut_after(wt), b.tmax);
        }
        if (!walking) {
            cnt.samples += (uint32_t)n_act;
            float Y[16];
            const float nn = sqrtf(b.d[0] * b.d[0] + b.d[1] * b.d[1] + b.d[2] * b.d[2]);
            sh_eval(a.deg, b.d[0] / nn, b.d[1] / nn, b.d[2] / nn, Y);
            float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
            for (int k = 0; k < N; ++k) {
                if (k >= n_act) continue;
                float t;
                int32_t g;
                unpack_key(keys[64 * k], t, g);
                const bool hit = g != 0x7FFFFFFF;
                if (a.hit_gid) a.hit_gid[b.sample0 + pass * b.npass + k] = hit ? g : -1;
                if (hit) {
                    const float3 c = clamp0(sh_colour_pre(a.sh, a.deg, g, Y));
                    c0 += c.x; c1 += c.y; c2 += c.z;
                } else {
                    c0 += a.bg[0]; c1 += a.bg[1]; c2 += a.bg[2];
                }
            }
            const float wgt = 1.0f / (float)b.spp;
            atomicAdd(a.rgb + 3 * b.row, c0 * wgt);
            atomicAdd(a.rgb + 3 * b.row + 1, c1 * wgt);
            atomicAdd(a.rgb + 3 * b.row + 2, c2 * wgt);
            active = false;
        }
    }
}

template <int W, int N, bool COUNT, int DM>
__global__ __launch_bounds__(kPersistBlock) void k_persistent(BatchArgs a)
{
    __shared__ QueueLds<N> q;
    LaneCounts cnt;
    persist_queue<W, N, COUNT, DM>(a, q, cnt);
    flush_counts<COUNT>(a, cnt, 0, 0);
}

// Wave-uniform copy of a value every lane holds.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

constexpr int kWaveCap = 48;  // wave-shared stack entries (12 KB of LDS per wave)

// Persistent with wave-shared walks for the camera pixels: each wave claims
// camera (tile, pass) groups, one per atomic, and walks each with its 64
// rays together. (The extra rays go to k_persistent, launched before it at
// its own occupancy: its lane walks need fewer registers than these.)
// Registers are capped for 3 waves per SIMD (views at 16 samples per
// traversal, 3.3M Gaussians: 1.57 -> 1.40 s with the spills; the plain tile
// kernel lost with the same cap, 2.04 -> 2.17 s, and keeps 2).
template <int W, int N, bool COUNT, int DM>
__global__ __launch_bounds__(kPersistBlock, 3) void k_persistent_wave(BatchArgs a,
                                                                   const void* __restrict__ nodes_v,
                                                                   const Record* __restrict__ recs)
{
    __shared__ float lds[kWaveCap * 64];
    const WideNode<W>* __restrict__ nodes = static_cast<const WideNode<W>*>(nodes_v);
    const int lane = threadIdx.x;
    LaneCounts cnt;
    WaveStack stk{lds, kWaveCap, nullptr, 0, min(kWaveCap, a.stack_cap)};
    for (;;) {
        unsigned long long g = 0;
        if (lane == 0) g = atomicAdd(a.groups, 1ull);
        g = uniform_u64(__shfl(g, 0, 64));
        const int64_t it0 = (int64_t)g * 64;
        if (it0 >= a.n_cam) break;
        const int64_t item = it0 + lane;
        int32_t seg, pass;
        int64_t ray;
        decode_item(a, item, seg, ray, pass);
        const BRay b = seg_ray(a, a.segs[seg], ray);
        if (!wave_pass<W, N, DM>(a, nodes, recs, b, pass, stk, cnt, true, nullptr) && b.valid) {
            const uint32_t slot = atomicAdd(&a.ctrl[0], 1u);
            a.ovf_list[slot] = (uint64_t)item;
        }
    }
    flush_counts<COUNT>(a, cnt, 0, 0);
}

// Plain with wave-shared walks: one wave per 8x8 tile of a view, over all
// passes of its pixels (the camera lanes [0, n_cam) of the plain numbering).
template <int W, int N, bool COUNT, int DM>
__global__ __launch_bounds__(64, 2) void k_plain_wave(BatchArgs a, const void* __restrict__ nodes_v,
                                                   const Record* __restrict__ recs)
{
    __shared__ float lds[kWaveCap * 64];
    const WideNode<W>* __restrict__ nodes = static_cast<const WideNode<W>*>(nodes_v);
    const int64_t r = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 64 + threadIdx.x;
    const Segment& S = a.segs[find_seg(a, r, false)];
    const BRay b = seg_ray(a, S, r - S.enum_begin);
    WaveStack stk{lds, kWaveCap, nullptr, 0, min(kWaveCap, a.stack_cap)};
    LaneCounts cnt;
    float acc[3] = {0.0f, 0.0f, 0.0f};
    bool ok = true;
    const int passes = __builtin_amdgcn_readfirstlane(S.passes);  // one view per tile
    for (int pass = 0; pass < passes && ok; ++pass)
        ok = wave_pass<W, N, DM>(a, nodes, recs, b, pass, stk, cnt, false, acc);
    if (b.valid) {
        if (ok) {
            cnt.samples += (uint32_t)b.spp;
            const float w = 1.0f / (float)b.spp;
            a.rgb[3 * b.row] = acc[0] * w;
            a.rgb[3 * b.row + 1] = acc[1] * w;
            a.rgb[3 * b.row + 2] = acc[2] * w;
        } else {
            const uint32_t slot = atomicAdd(&a.ctrl[0], 1u);
            a.ovf_list[slot] = (uint64_t)r;
        }
    }
    flush_counts<COUNT>(a, cnt, 0, 0);
}

// Persistent deep pass: queued items with the global-memory stack.
template <int W, int N, bool COUNT, int DM>
__global__ __launch_bounds__(kPlainBlock) void k_persistent_deep(BatchArgs a)
{
    const int64_t gt = blockIdx.x * (int64_t)kPlainBlock + threadIdx.x;
    FlatStack stk{a.deep_stack + gt, kDeepThreads, a.deep_cap};
    LaneCounts cnt;
    uint32_t deep = 0, lost = 0;
    const int64_t n = a.ctrl[0];
    for (int64_t it = gt; it < n; it += (int64_t)gridDim.x * kPlainBlock) {
        int32_t seg, pass;
        int64_t ray;
        decode_item(a, (int64_t)a.ovf_list[it], seg, ray, pass);
        const BRay b = seg_ray(a, a.segs[seg], ray);
        ++deep;
        if (!run_pass<W, N, DM>(a, b, pass, stk, cnt, true, nullptr)) {
            ++lost;
            atomicAdd(&a.ctrl[1], 1u);
        }
    }
    flush_counts<COUNT>(a, cnt, deep, lost);
}

__global__ void k_zero_f32(float* p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// work[0]: next item of the lane refilling (from `start`); work[1]: next
// camera group of the persistent wave kernel.
__global__ void k_reset(unsigned long long* work, uint32_t* ctrl, unsigned long long start)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        work[0] = start;
        work[1] = 0ull;
        ctrl[0] = 0u;
        ctrl[1] = 0u;
    }
}

using BatchFn = void (*)(BatchArgs);
using WaveBatchFn = void (*)(BatchArgs, const void*, const Record*);

struct Kernels {
    BatchFn plain, plain_deep, persistent, persistent_deep;
    WaveBatchFn plain_wave, persistent_wave;
};

// Samples per pass of lane walks (their per-lane state lives in registers
// or, queued, in LDS): larger passes go to wave-shared walks only.
constexpr int kLaneMaxN = 8;

template <int W, int N, bool C, int DM>
void pick_all(Kernels& k)
{
    constexpr int NL = N < kLaneMaxN ? N : kLaneMaxN;
    k.plain = k_plain<W, NL, C, DM>;
    k.plain_deep = k_plain_deep<W, N, C, DM>;
    k.persistent = k_persistent<W, NL, C, DM>;
    k.persistent_deep = k_persistent_deep<W, N, C, DM>;
    k.plain_wave = k_plain_wave<W, N, C, DM>;
    k.persistent_wave = k_persistent_wave<W, N, C, DM>;
}

template <int W, bool C, int DM>
bool pick_w(int N, Kernels& k)
{
    switch (N) {
    case 1: pick_all<W, 1, C, DM>(k); return true;
    case 2: pick_all<W, 2, C, DM>(k); return true;
    case 4: pick_all<W, 4, C, DM>(k); return true;
    case 8: pick_all<W, 8, C, DM>(k); return true;
    case 16: pick_all<W, 16, C, DM>(k); return true;
    }
    return false;
}

template <int DM>
bool pick_dm(int W, int N, bool count, Kernels& k)
{
    switch (W) {
    case 2: return count ? pick_w<2, true, DM>(N, k) : pick_w<2, false, DM>(N, k);
    case 4: return count ? pick_w<4, true, DM>(N, k) : pick_w<4, false, DM>(N, k);
    case 8: return count ? pick_w<8, true, DM>(N, k) : pick_w<8, false, DM>(N, k);
    }
    return false;
}

// kernels with the depth mode fixed at compile time (fewer registers)
bool pick(int W, int N, bool count, int depth_mode, Kernels& k)
{
    return depth_mode == 0 ? pick_dm<0>(W, N, count, k) : pick_dm<1>(W, N, count, k);
}

}  // namespace

struct srt_batch_plan {
    const srt_bvh* bvh = nullptr;
    srt_trace_opts opts{};
    srt_tuning tuning{};
    std::vector<Segment> segs;
    Segment* d_segs = nullptr;
    int64_t n_items = 0, n_rays = 0, n_samples = 0, rows = 0;
    int64_t n_cam_items = 0, n_cam_rays = 0;  // camera part (multiples of 64)
    srt_rays extra{};
    unsigned long long* work = nullptr;
    uint32_t* ctrl = nullptr;
    uint64_t* ovf = nullptr;
    int32_t* deep_stack = nullptr;
    int32_t* lane_stack = nullptr;  // persistent lane kernel's stack entries beyond LDS
    int32_t lane_stack_cap = 0;
    int64_t ovf_cap = 0;
    int32_t n_cu = 0;
    int32_t resident[2][2] = {{1, 1}, {1, 1}};  // [counters][lane, wave]: workgroups per CU
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    float* g_rgb = nullptr;
    int32_t* g_hits = nullptr;
    uint64_t* g_counters = nullptr;
};

namespace {

void plan_free(srt_batch_plan* p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    (void)hipFree(p->d_segs);
    (void)hipFree(p->work);
    (void)hipFree(p->ctrl);
    (void)hipFree(p->ovf);
    (void)hipFree(p->deep_stack);
    (void)hipFree(p->lane_stack);
    delete p;
}

srt_status enqueue(srt_batch_plan* p, float* rgb, int32_t* hits, uint64_t* counters, hipStream_t s)
{
    const srt_bvh* b = p->bvh;
    Kernels k{};
    if (!pick(b->W, p->opts.n_per_traversal, counters != nullptr, p->opts.depth_mode, k))
        return SRT_ERR_UNSUPPORTED;
    const bool wave = p->opts.walk != 1 && p->n_cam_rays > 0;
    BatchArgs a{};
    a.nodes = b->nodes;
    a.recs = b->recs;
    a.sh = b->sh;
    a.deg = b->deg;
    a.segs = p->d_segs;
    a.n_segs = (int32_t)p->segs.size();
    a.eo = p->extra.origins;
    a.ed = p->extra.dirs;
    a.etmin = p->extra.tmin;
    a.etmax = p->extra.tmax;
    a.erid = p->extra.ray_ids;
    a.epurpose = p->extra.purpose;
    a.k0 = (uint32_t)p->opts.seed;
    a.k1 = (uint32_t)(p->opts.seed >> 32);
    a.soff = p->opts.sample_offset;
    for (int i = 0; i < 3; ++i) a.bg[i] = p->opts.bg[i];
    a.stack_cap = p->opts.stack_limit > 0 ? p->opts.stack_limit : INT_MAX;
    a.rgb = rgb;
    a.hit_gid = hits;
    a.counters = reinterpret_cast<unsigned long long*>(counters);
    a.work = p->work;
    a.ctrl = p->ctrl;
    a.ovf_list = p->ovf;
    a.deep_stack = p->deep_stack;
    a.deep_cap = deep_stack_cap(b);
    a.lane_stack = p->lane_stack;
    a.lane_stack_cap = p->lane_stack ? p->lane_stack_cap : 0;
    a.lds_stack = p->tuning.lds_stack > 0 ? p->tuning.lds_stack : kQueueStack;
    a.threshold = std::max(1, std::min(64, p->tuning.refill_threshold));
    a.max_steps = 2 * b->num_nodes + 2 * b->G + 64;
    a.N = p->opts.n_per_traversal;
    a.depth_mode = p->opts.depth_mode;
    for (int i = 0; i < 3; ++i) a.depth_axis[i] = p->opts.depth_axis[i];
    a.r_max = b->r_max;
    a.groups = p->work + 1;
    const bool persistent = p->tuning.persistent != 0;
    a.n_cam = wave ? (persistent ? p->n_cam_items : p->n_cam_rays) : 0;
    k_reset<<<1, 64, 0, s>>>(p->work, p->ctrl, (unsigned long long)a.n_cam);
    SRT_HIP_TRY(hipGetLastError());
    const void* nodes = b->nodes;
    const Record* recs = b->recs;
    if (persistent) {
        k_zero_f32<<<1024, 256, 0, s>>>(rgb, 3 * p->rows);
        SRT_HIP_TRY(hipGetLastError());
        a.n_items = p->n_items;
        // a persistent grid beyond what stays resident only adds waves that
        // start when the work is gone
        const int wpc = std::max(1, p->tuning.waves_per_cu);
        const int ci = counters ? 1 : 0;
        if (p->n_items > a.n_cam) {  // lane items: all (lane walks) or the extra rays
            const int g = p->n_cu * std::min(wpc, p->resident[ci][0]);
            hipLaunchKernelGGL(k.persistent, dim3((unsigned)g), dim3(kPersistBlock), 0, s, a);
            SRT_HIP_TRY(hipGetLastError());
        }
        if (wave) {
            const int g = p->n_cu * std::min(wpc, p->resident[ci][1]);
            hipLaunchKernelGGL(k.persistent_wave, dim3((unsigned)g), dim3(kPersistBlock), 0, s, a,
                               nodes, recs);
            SRT_HIP_TRY(hipGetLastError());
        }
        hipLaunchKernelGGL(k.persistent_deep, dim3(kDeepThreads / kPlainBlock), dim3(kPlainBlock),
                           0, s, a);
        SRT_HIP_TRY(hipGetLastError());
    } else {
        a.n_items = p->n_rays;
        if (wave) {
            hipLaunchKernelGGL(k.plain_wave, dim3((unsigned)(p->n_cam_rays / 64)), dim3(64), 0, s,
                               a, nodes, recs);
            SRT_HIP_TRY(hipGetLastError());
        }
        a.first = a.n_cam;
        const int64_t lanes = p->n_rays - a.first;
        if (lanes > 0) {
            hipLaunchKernelGGL(k.plain, dim3((unsigned)((lanes + kPlainBlock - 1) / kPlainBlock)),
                               dim3(kPlainBlock), 0, s, a);
            SRT_HIP_TRY(hipGetLastError());
        }
        hipLaunchKernelGGL(k.plain_deep, dim3(kDeepThreads / kPlainBlock), dim3(kPlainBlock), 0, s,
                           a);
        SRT_HIP_TRY(hipGetLastError());
    }
    return SRT_OK;
}

}  // namespace

extern "C" {

srt_status srt_batch_plan_create(const srt_bvh* b, const srt_batch* batch,
                                 const srt_trace_opts* opts, const srt_tuning* tuning, void* stream,
                                 srt_batch_plan** out)
{
    const srt::Range range_("srt_batch_plan_create");
    if (!b || !batch || !opts || !tuning || !out) return SRT_ERR_INVALID_ARG;
    *out = nullptr;
    const int N = opts->n_per_traversal;
    if (N != 1 && N != 2 && N != 4 && N != 8 && N != 16) return SRT_ERR_INVALID_ARG;
    // passes of the views' pixels on wave-shared walks take N samples, lane
    // walks at most kLaneMaxN
    const int n_lane = std::min(N, kLaneMaxN);
    const int n_cam = opts->walk == 1 ? n_lane : N;
    if (opts->any_hit || opts->stack_limit < 0) return SRT_ERR_INVALID_ARG;
    if (opts->depth_mode != 0 && opts->depth_mode != 1) return SRT_ERR_INVALID_ARG;
    if (opts->rng != 0 && opts->rng != 1) return SRT_ERR_INVALID_ARG;
    if (opts->rng == 1) return SRT_ERR_UNSUPPORTED;  // batched plans draw Philox numbers
    if (opts->walk < 0 || opts->walk > 2) return SRT_ERR_INVALID_ARG;
    if (batch->num_views < 0 || (batch->num_views > 0 && (!batch->cameras || !batch->spp)))
        return SRT_ERR_INVALID_ARG;
    if (batch->extra.count < 0 || batch->extra_spp < 0) return SRT_ERR_INVALID_ARG;
    if (batch->extra.count > 0 &&
        (!batch->extra.origins || !batch->extra.dirs || batch->extra_spp < 1))
        return SRT_ERR_INVALID_ARG;
    if (tuning->refill_threshold < 1 || tuning->refill_threshold > 64 || tuning->waves_per_cu < 1 ||
        tuning->lds_stack < 0 || tuning->lds_stack > kQueueStack)
        return SRT_ERR_INVALID_ARG;
    srt_batch_plan* p = new srt_batch_plan();
    p->bvh = b;
    p->opts = *opts;
    p->tuning = *tuning;
    p->extra = batch->extra;
    int64_t items = 0, rows = 0, samples = 0, rays = 0;
    for (int v = 0; v < batch->num_views; ++v) {
        const srt_camera& c = batch->cameras[v];
        const int32_t spp = batch->spp[v];
        if (c.width < 1 || c.height < 1 || spp < 1) {
            plan_free(p);
            return SRT_ERR_INVALID_ARG;
        }
        Segment S{};
        S.cam = c;
        S.width = c.width;
        S.height = c.height;
        S.tiles_x = (c.width + kTile - 1) / kTile;
        S.spp = spp;
        S.n = n_cam;
        S.passes = (spp + n_cam - 1) / n_cam;
        S.rays = (int64_t)c.width * c.height;
        S.item_begin = items;
        S.enum_begin = rays;
        S.ray_begin = rows;
        S.sample_begin = samples;
        S.ray_id_base = batch->ray_id_base + (uint32_t)rows;
        const int64_t en = seg_rays_enumerated(S);
        items += en * S.passes;
        rows += S.rays;
        samples += S.rays * spp;
        rays += en;
        p->segs.push_back(S);
    }
    p->n_cam_items = items;
    p->n_cam_rays = rays;
    if (batch->extra.count > 0) {
        Segment S{};
        S.width = 0;
        S.spp = batch->extra_spp;
        S.n = n_lane;
        S.passes = (batch->extra_spp + n_lane - 1) / n_lane;
        S.rays = batch->extra.count;
        S.item_begin = items;
        S.enum_begin = rays;
        S.ray_begin = rows;
        S.sample_begin = samples;
        S.ray_id_base = batch->ray_id_base + (uint32_t)rows;
        items += S.rays * S.passes;
        rows += S.rays;
        samples += S.rays * S.spp;
        rays += S.rays;
        p->segs.push_back(S);
    }
    p->n_items = items;
    p->rows = rows;
    p->n_samples = samples;
    p->n_rays = rays;
    srt_status st = SRT_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        plan_free(p);
        return SRT_ERR_HIP;
    }
    p->n_cu = prop.multiProcessorCount;
    for (int c = 0; c < 2; ++c) {
        Kernels k{};
        if (!pick(b->W, N, c == 1, opts->depth_mode, k)) {
            plan_free(p);
            return SRT_ERR_UNSUPPORTED;
        }
        int nl = 0, nw = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nl, reinterpret_cast<const void*>(k.persistent), kPersistBlock, 0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nw, reinterpret_cast<const void*>(k.persistent_wave), kPersistBlock, 0) !=
                hipSuccess) {
            plan_free(p);
            return SRT_ERR_HIP;
        }
        p->resident[c][0] = std::max(1, nl);
        p->resident[c][1] = std::max(1, nw);
    }
    p->ovf_cap = std::max<int64_t>(items, rays) + 1;
    if (hipMalloc(&p->d_segs, sizeof(Segment) * std::max<size_t>(1, p->segs.size())) != hipSuccess ||
        hipMalloc(&p->work, 2 * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&p->ctrl, 4 * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&p->ovf, sizeof(uint64_t) * (size_t)p->ovf_cap) != hipSuccess ||
        hipMalloc(&p->deep_stack, sizeof(int32_t) * (size_t)kDeepThreads * (size_t)deep_stack_cap(b)) !=
            hipSuccess) {
        plan_free(p);
        return SRT_ERR_OOM;
    }
    if (tuning->persistent) {
        // every lane of the largest lane-kernel grid gets the entries a walk
        // can need beyond its LDS part
        const int n_lds = tuning->lds_stack > 0 ? tuning->lds_stack : kQueueStack;
        p->lane_stack_cap = std::max(0, deep_stack_cap(b) - n_lds);
        const size_t lanes = (size_t)p->n_cu *
                             (size_t)std::max(p->resident[0][0], p->resident[1][0]) * kPersistBlock;
        if (p->lane_stack_cap > 0 &&
            hipMalloc(&p->lane_stack, sizeof(int32_t) * lanes * (size_t)p->lane_stack_cap) !=
                hipSuccess) {
            plan_free(p);
            return SRT_ERR_OOM;
        }
    }
    if (!p->segs.empty() &&
        hipMemcpyAsync(p->d_segs, p->segs.data(), sizeof(Segment) * p->segs.size(),
                       hipMemcpyHostToDevice, s) != hipSuccess)
        st = SRT_ERR_HIP;
    if (st == SRT_OK && hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
        st = SRT_ERR_HIP;
    if (st == SRT_OK && hipStreamSynchronize(s) != hipSuccess) st = SRT_ERR_HIP;
    if (st != SRT_OK) {
        plan_free(p);
        return st;
    }
    *out = p;
    return SRT_OK;
}

void srt_batch_plan_destroy(srt_batch_plan* p) { plan_free(p); }

srt_status srt_batch_plan_info(const srt_batch_plan* p, int64_t* rows, int64_t* samples,
                               int64_t* items)
{
    if (!p) return SRT_ERR_INVALID_ARG;
    if (rows) *rows = p->rows;
    if (samples) *samples = p->n_samples;
    if (items) *items = p->tuning.persistent ? p->n_items : p->n_rays;
    return SRT_OK;
}

srt_status srt_batch_plan_execute(srt_batch_plan* p, float* rgb, int32_t* hit_gid,
                                  uint64_t* counters, void* stream)
{
    const srt::Range range_("srt_batch_plan_execute");
    if (!p || (!rgb && p->rows > 0)) return SRT_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!p->exec || p->g_rgb != rgb || p->g_hits != hit_gid || p->g_counters != counters) {
        // (re)capture: the graph holds the output pointers it was captured with
        if (p->exec) {
            (void)hipGraphExecDestroy(p->exec);
            p->exec = nullptr;
        }
        if (p->graph) {
            (void)hipGraphDestroy(p->graph);
            p->graph = nullptr;
        }
        SRT_HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        const srt_status st = enqueue(p, rgb, hit_gid, counters, p->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
        if (st != SRT_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        SRT_HIP_TRY(e);
        p->graph = g;
        SRT_HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
        p->g_rgb = rgb;
        p->g_hits = hit_gid;
        p->g_counters = counters;
    }
    SRT_HIP_TRY(hipGraphLaunch(p->exec, s));
    return SRT_OK;
}

srt_status srt_batch_plan_execute_eager(srt_batch_plan* p, float* rgb, int32_t* hit_gid,
                                        uint64_t* counters, void* stream)
{
    if (!p || (!rgb && p->rows > 0)) return SRT_ERR_INVALID_ARG;
    return enqueue(p, rgb, hit_gid, counters, static_cast<hipStream_t>(stream));
}

}  // extern "C"
