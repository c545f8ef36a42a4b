// Kernel launch interface of libpt (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pt_internal.h"

namespace pt {

// Scene as the kernels see it (device pointers into the caller's arena).
struct DevScene {
    const float4* nodes;     // [nnodes][4]  child-pair nodes
    const float4* nodes4;    // [nnodes4][8] four-wide nodes of the same tree
    const float4* nodes4q;   // [nnodes4][4] the four-wide nodes with quantized child boxes
    uint32_t quant;          // the quantized nodes are usable (every step 2^e has e <= 60)
    uint32_t wide;           // traverse the four-wide nodes
    const float4* btris;     // [ntri][3]    BVH order; v0.w = original triangle id (int bits)
    const float4* otris;     // [ntri][3]    original order
    const uint32_t* tri_mat; // [ntri]
    const pt_material* mats; // [nmat]
    const uint32_t* emit;    // [nemit] emissive triangles, original order
    uint32_t ntri, nmat, nemit;
    float env[3];
    float lo[3], hi[3];
};

// One frame's launch constants.
struct Frame {
    int w, h, spp, B, mode;
    int W, H, K, WH, reuse_max;
    int SW, SH, TS, cols;     // super tile (one workgroup of the shade kernel)
    int nstx, nsty, ntx;      // super tiles per row/column, reuse tiles per row
    uint32_t nslots;
    uint64_t seed;
    float cpos[3], cfwd[3], cright[3], cup[3];
    float th, thx;
    int nee;                  // next-event estimation at Lambert points
    int frame_groups;         // one tile shuffle per sample (drawn at bounce 0), not one per bounce
    uint32_t region;          // compacted queues: ray slots per region (8 regions, workgroup blk
                              // writes region blk mod 8): ceil(workgroups / 8) x TS
    uint32_t* live;           // optional, one word per shade workgroup: nonzero while a path of
                              // the workgroup goes on (set by ray generation, kept by shading)
};

// Ray queue record: {ox, oy, oz, excluded prim} {dx, dy, dz, pixel}; pixel = kNoRay: no ray.
constexpr uint32_t kNoRay = 0xFFFFFFFFu;
// shadow rays run along D = light point - origin; a hit at t >= kShadowTmax is the light itself
constexpr float kShadowTmax = 1.0f - 0x1p-10f;
constexpr int kTraceBlock = 64;    // one wave per workgroup
constexpr int kStackLds = 16;      // LDS stack entries per lane
constexpr bool kPreferWide = true; // traverse the four-wide nodes when the scene allows it
constexpr bool kLeafQueue = true;  // four-wide traversal queues its triangle tests per wave
constexpr bool kQuantized = true;  // and reads the quantized nodes
constexpr int kStackOvf = kMaxDepth - kStackLds + 16; // global overflow entries per lane
constexpr int kMaxTraceBlocks = 256 * 32;  // cap of the persistent grid (bounds the overflow area)
constexpr int kDefaultWavesPerCu = 24;     // persistent grid when the caller leaves it to the library
// A launch hands out its rays through kRayCounters counters kCounterStride words apart
// (kWorkWords words of work area per launch, zero at launch).
constexpr int kRayCounters = 8;
constexpr int kCounterStride = 64;
constexpr int kWorkWords = kRayCounters * kCounterStride;
// A compacted launch keeps region c's ray count kFillWord words after counter c: another
// 128-byte line, so the loads of the counts do not meet the claims' atomics on one line.
constexpr int kFillWord = 32;
constexpr int kDefaultLeafGate = 8;        // pt_group.leaf_gate when the caller leaves it to the library

struct TraceArgs {
    const float4* rays;
    uint32_t n;
    int32_t* out_prim;         // indexed by pixel (by_pixel) or by ray
    float* out_t;
    uint32_t* work;            // kWorkWords words: the ray counters, zero at launch
    uint32_t* partial;         // optional [grid] per-workgroup count of traced rays
    unsigned long long* stats; // optional [2]
    int32_t* ovf;              // [kStackOvf][grid threads]
    int by_pixel;
    int refill;                // a wave fetches new rays once this many lanes are idle (1..64)
    int waves_per_cu;          // persistent grid size, 0 = kDefaultWavesPerCu
    int leaf_gate;             // the inner-node phase ends when at most this many lanes lack a leaf
    int shadow;                // shadow rays: blocked iff a triangle lies at 0 < t < kShadowTmax (units of d)
    int skip_empty;            // rays whose pixel word is kNoRay are skipped (not traced, no output)
    int kind;                  // traversal kernel (kTraceChildPair...), -1 = trace_kind of the scene
    uint8_t* touched;          // optional (counting kernels): node flags, then triangle flags from touch_tri
    uint32_t touch_tri;
    uint32_t touch_bit;
    const uint32_t* fill;      // compacted launch: region c holds fill[c * kCounterStride] rays from
                               // slot c * region on (launch_shade's layout); the claims follow the
                               // regions and n is their sum.  null: n rays at [0, n)
    uint32_t region;
    const uint32_t* perm;      // with fill: ray i of the launch is rays[perm[i]], i < sum of fill
                               // (the sorted modes' order); null: ray i is rays[i]
    int max_blocks;            // > 0: the persistent grid has at most this many workgroups (the
                               // overflow area ovf holds that many); 0 = no cap beyond kMaxTraceBlocks
};

// One job of a merged launch (batched rendering): the shade, raygen and trace launches of a
// step cover every job in flight; a workgroup (shade, raygen) or a ray (trace) finds its job
// by binary search over block_start / ray_start (the table is sorted by both).
struct StepJob {
    DevScene sc;
    Frame f;
    int b, s;                  // bounce traced and shaded in this step, sample index
    int do_raygen;             // the step starts sample s (raygen writes q_out_raygen)
    int pad;
    float4* q_out_raygen;      // queue the primary rays go to (= q_in)
    const float4* q_in;        // rays traced this step (and read back by shade)
    float4* q_out;             // next rays
    float4* state;
    int32_t* hit_prim;         // [B+1][spp][h][w]
    float* hit_t;
    int32_t* trace_prim;       // hit_prim + plane of (b, s)
    float* trace_t;
    float* radiance;
    uint32_t block_start;      // first workgroup of the job in the merged raygen/shade grid
    uint32_t ray_start;        // first ray of the job in the merged trace index space
    uint32_t nrays;
    uint32_t pad2;
};

int trace_grid_blocks(int waves_per_cu = 0);   // persistent grid (workgroups): a multiple of 8, <= kMaxTraceBlocks
hipError_t launch_trace(const DevScene& sc, const TraceArgs& a, bool stats, hipStream_t st);
// merged launches over njobs jobs (table in device memory); total_rays = sum of nrays,
// total_blocks = sum of the jobs' workgroups; all jobs share f.TS and the grouping mode
// wide: every job's scene has four-wide nodes within the stack bound
// traversal kernel of a scene: child-pair nodes, four-wide nodes, or four-wide nodes with the
// per-wave queue of triangle tests (scenes of at most 2^26 triangles)
constexpr int kTraceChildPair = 0, kTraceWide = 1, kTraceWideQueue = 2, kTraceWideQueueQ = 3;
int trace_max_kind(const DevScene& sc);   // the widest kind the scene allows; every smaller kind works too
int trace_kind(const DevScene& sc);       // the kind used when the caller leaves it to the library
hipError_t launch_trace_multi(const StepJob* jobs, int njobs, const TraceArgs& a, int kind, hipStream_t st);
hipError_t launch_raygen_multi(const StepJob* jobs, int njobs, uint32_t total_blocks, int TS, hipStream_t st);
hipError_t launch_shade_multi(const StepJob* jobs, int njobs, uint32_t total_blocks, int TS, bool reuse,
                              hipStream_t st);
// memory-level probe (probe.hip)
hipError_t launch_probe_fill(uint32_t* buf, uint32_t nlines, hipStream_t st);
hipError_t launch_probe_read(const void* buf, size_t bytes, int passes, uint32_t* sink, hipStream_t st);
hipError_t launch_probe_chase(const uint32_t* buf, uint32_t nlines, int steps, uint32_t* sink, hipStream_t st);
hipError_t launch_zero(uint32_t* p, size_t n, hipStream_t st);
hipError_t launch_raygen(const Frame& f, int s, float4* q, float4* state, float4* rays_out, hipStream_t st);
// fill: null = the next rays at their slots (dead slots hold kNoRay records); else the live
// rays compacted into 8 regions of f.region slots, region r's count in fill[r * kCounterStride]
// (zero before the launch), dead rays not written
// keys_out: null, or (sorted modes, with fill) the reordering key of each next ray, written at
// the ray's queue slot (sort_key_slots)
// debug: null, or pt_outputs.debug (the record of hit b of every pixel with a path, b < B)
hipError_t launch_shade(const DevScene& sc, const Frame& f, int b, int s, const float4* q_in, float4* q_out,
                        float4* state, int32_t* hit_prim, float* hit_t, float* radiance, float4* rays_out,
                        float4* shadow_rays, float4* shadow_light, uint32_t* fill, uint32_t* keys_out, float4* debug,
                        hipStream_t st);

// flags of the per-ray record (the w word of pt_outputs.debug)
constexpr uint32_t kDbgActive = 1u << 0, kDbgRep = 1u << 5, kDbgReused = 1u << 6, kDbgValid = 1u << 7;
constexpr int kDbgClassShift = 1, kDbgCatShift = 3, kDbgSlotShift = 16;
// next-event estimation: adds shadow_light[p].rgb to the radiance of path p when its shadow
// ray exists (pixel word != kNoRay) and shadow_prim[p] == -1 (nothing in between)
hipError_t launch_nee_accumulate(const float4* shadow_rays, const float4* shadow_light, const int32_t* shadow_prim,
                                 uint32_t n, float4* state, hipStream_t st);
hipError_t launch_keys(const DevScene& sc, const float4* q, uint32_t n, uint32_t* keys, uint32_t* vals, int kind,
                       hipStream_t st);
// ray_count[i] = sum of partial[i * stride + j] for j < parts, i < launches
hipError_t launch_count_finalize(const uint32_t* partial, int stride, int parts, int launches, uint32_t* ray_count,
                                 hipStream_t st);
// sorted modes over a compacted queue (launch_shade's regions, counts in fill): the 30-bit keys
// that the shade kernel wrote at the live rays' queue slots (sort_key_slots: qslots = 8 x region
// words) gathered in region order with their slots, and the digit histograms
// (launch_keys_compacted), then a stable radix sort in 4 passes of 8-bit digits
// (launch_sort_compacted), whose *perm gives the queue slots in key order for the traversal
// (TraceArgs.perm); ws: sort_compacted_workspace_bytes
size_t sort_compacted_workspace_bytes(uint32_t nslots, uint32_t qslots);
uint32_t* sort_key_slots(void* ws, uint32_t nslots);
hipError_t launch_keys_compacted(const uint32_t* fill, uint32_t region, uint32_t nslots, void* ws, hipStream_t st);
hipError_t launch_sort_compacted(const uint32_t* fill, uint32_t nslots, void* ws, const uint32_t** perm,
                                 hipStream_t st);

// stable LSD radix sort of n (key, value) pairs by 32-bit keys (4 passes of 8-bit digits, one
// decoupled look-back pass each), in place
size_t sort_workspace_bytes(uint32_t n);
hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t n, void* ws, hipStream_t st);

}  // namespace pt
