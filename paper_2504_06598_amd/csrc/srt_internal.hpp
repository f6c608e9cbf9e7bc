// Host-side internals shared by the translation units of libsrt.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <utility>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "srt.h"
#include "srt_device.hpp"

struct srt_bvh {
    int64_t G = 0;
    int32_t W = 4, L = 4, depth = 0, deg = 0;
    int64_t num_nodes = 0;
    void* nodes = nullptr;           // WideNode<W>[num_nodes]
    srt::Record* recs = nullptr;     // leaf order
    int32_t* leaf_order = nullptr;   // Gaussian id at each leaf position
    int32_t* leaf_pos = nullptr;     // leaf position of each Gaussian id
    float* box_lo = nullptr;         // [G,3], Gaussian-id order
    float* box_hi = nullptr;
    const float* sh = nullptr;       // borrowed from the scene
    float r_max = 0.0f;              // largest bounding-sphere radius
    int64_t bytes = 0;
    // topology kept for refits: node indices grouped by level (root level
    // first; empty when the tree is a single leaf), and a small device
    // buffer for the scene bounds
    int32_t* level_nodes = nullptr;
    std::vector<uint32_t> level_off, level_cnt;
    uint32_t* bounds = nullptr;      // [8]
    // start_node[gid]: the node start_levels levels above the leaf that holds
    // Gaussian gid (the root when the leaf is shallower); null when absent.
    // A ray that starts inside that Gaussian can walk this subtree first.
    int32_t* start_node = nullptr;
    int32_t start_levels = 0;
    std::vector<std::pair<void*, size_t>> blocks;  // device buffers owned (pointer, bytes)
};

namespace srt {

// A roctx range over a host call (it covers the enqueueing, shown on the CPU
// timeline of `rocprofv3 --marker-trace`); free when no tool listens.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

#define SRT_HIP_TRY(expr)                              \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return map_hip_error(e_); \
    } while (0)

inline srt_status map_hip_error(hipError_t e)
{
    return e == hipErrorOutOfMemory ? SRT_ERR_OOM : SRT_ERR_HIP;
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Deep-stack fallback: fixed grid of lanes that rerun rays whose on-chip
// stack overflowed, each with a stack in global memory.
constexpr int kDeepThreads = 16384;

inline int32_t deep_stack_cap(const srt_bvh* b)
{
    // a wide traversal pushes at most W-1 entries per level below the root
    return (b->depth + 2) * b->W + 8;
}

// Trace workspace layout.
struct TraceWorkspace {
    uint32_t* ctrl;        // [64]: [0] overflow count
    uint32_t* ovf_list;    // [R]
    int32_t* deep_stack;   // [kDeepThreads * cap]
    size_t bytes;
};

inline TraceWorkspace trace_workspace(const srt_bvh* b, int64_t R, void* base)
{
    TraceWorkspace w{};
    size_t off = 0;
    char* p = static_cast<char*>(base);
    w.ctrl = reinterpret_cast<uint32_t*>(p + off);
    off += 256;
    w.ovf_list = reinterpret_cast<uint32_t*>(p + off);
    off = align_up(off + (size_t)(R > 0 ? R : 1) * 4, 256);
    w.deep_stack = reinterpret_cast<int32_t*>(p + off);
    off = align_up(off + (size_t)kDeepThreads * (size_t)deep_stack_cap(b) * 4, 256);
    w.bytes = off;
    return w;
}

// Fill a device array with a 32-bit value (used instead of a memset so the
// work is capturable in graphs).
void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);

}  // namespace srt
