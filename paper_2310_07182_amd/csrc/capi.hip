// C-ABI entry points of libpt: argument checks, scene build and upload, the
// frame loop (raygen -> [key -> sort -> gather] -> trace -> shade per bounce),
// workspace layout and HIP-event timing.  No entry point allocates device
// memory: the caller passes the scene arena, the workspace and the outputs.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"

using pt::DevScene;
using pt::Frame;

struct pt_scene_s {
    pt::HostBvh bvh;
    std::vector<float4> btris, otris;
    std::vector<uint32_t> tri_mat;
    std::vector<pt_material> mats;
    std::vector<uint32_t> emit;     // emissive triangles, original order (next-event estimation)
    uint32_t ntri = 0, nmat = 0;
    float env[3] = {0, 0, 0};
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    size_t off_nodes = 0, off_nodes4 = 0, off_nodes4q = 0, off_btris = 0, off_otris = 0, off_mat = 0, off_mats = 0, off_emit = 0,
           bytes = 0;
    bool uploaded = false;
    int device = -1;
    DevScene dev{};
};

struct BatchJob {
    bool used = false;
    bool finished = false;          // last step enqueued
    pt_job job{};
    pt::Frame f{};
    size_t off = 0, bytes = 0;      // arena range: q0, q1, state
    int s = 0, b = 0;               // next (sample, bounce) to trace
    hipEvent_t done_ev = nullptr;   // recorded after the job's last step
};

constexpr int kBatchRing = 4;       // launch tables in flight

struct pt_batch_s {
    int max_jobs = 0;
    pt_group group{};
    char* arena = nullptr;
    size_t bytes = 0;
    size_t table_off = 0, table_stride = 0, counter_off = 0, ovf_off = 0, pool_off = 0;
    std::vector<BatchJob> jobs;
    std::map<size_t, size_t> free_ranges;   // offset -> size, coalesced
    std::vector<std::vector<pt::StepJob>> host_tables;
    hipEvent_t ring_ev[kBatchRing] = {};
    bool ring_used[kBatchRing] = {};
    long long steps = 0;
    int device = -1;
    // static-run schedule and its captured graph
    size_t sched_off = 0, sched_bytes = 0;
    std::vector<uint32_t> graph_key;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t gstream = nullptr;      // capture / replay stream (the caller's may be the null stream)
    hipEvent_t gev_in = nullptr, gev_out = nullptr;
};

struct pt_timer_s {
    std::vector<hipEvent_t> ev;   // 2 per record
    std::vector<int32_t> kind, bounce;
    int cap = 0, n = 0;
};

namespace {

thread_local std::string g_err;

pt_status fail(pt_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

pt_status hip_fail(hipError_t e, const char* what) {
    return fail(PT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool is_reuse_mode(int mode) {
    return mode == PT_MODE_REUSE || mode == PT_MODE_REUSE_PLAIN || mode == PT_MODE_REUSE_WORLD;
}

bool is_sorted_mode(int mode) {
    return mode == PT_MODE_SORTED || mode == PT_MODE_SORTED_ORIGIN || mode == PT_MODE_SORTED_REIS ||
           mode == PT_MODE_SORTED_AILA;
}

constexpr int kDefaultRefill = 16;

bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// ---- host side of the arithmetic contract: camera basis
struct H3 {
    float x, y, z;
};
H3 h_sub(H3 a, H3 b) { return H3{a.x - b.x, a.y - b.y, a.z - b.z}; }
float h_dot(H3 a, H3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
H3 h_cross(H3 a, H3 b) { return H3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
H3 h_unit(H3 v) {
    float inv = 1.0f / sqrtf(h_dot(v, v));
    return H3{v.x * inv, v.y * inv, v.z * inv};
}

pt_status check_group(pt_group g, int bounces) {
    (void)bounces;
    if (!pow2(g.tile_w) || !pow2(g.tile_h) || !pow2(g.k))
        return fail(PT_EINVAL, "tile_w, tile_h and k must be powers of two (got %d, %d, %d)", g.tile_w, g.tile_h, g.k);
    const int wh = (int)g.tile_w * (int)g.tile_h;
    if (wh > 1024) return fail(PT_EINVAL, "tile_w * tile_h must be <= 1024 (got %d)", wh);
    if ((int)g.k > wh) return fail(PT_EINVAL, "k (%d) must divide tile_w * tile_h (%d)", g.k, wh);
    if (g.refill > 64) return fail(PT_EINVAL, "refill must be in [0, 64] (got %d)", g.refill);
    if (g.leaf_gate > 64) return fail(PT_EINVAL, "leaf_gate must be in [0, 64] (got %d)", g.leaf_gate);
    if (g.nee > 1) return fail(PT_EINVAL, "nee must be 0 or 1 (got %d)", g.nee);
    if (g.traversal > 4) return fail(PT_EINVAL, "traversal must be in [0, 4] (got %d)", g.traversal);
    if (g.frame_groups > 1) return fail(PT_EINVAL, "frame_groups must be 0 or 1 (got %d)", g.frame_groups);
    return PT_OK;
}

// super tile = one shade workgroup holding whole reuse tiles, >= 64 slots
void super_tile(int W, int H, int& SW, int& SH, int& cols) {
    const int WH = W * H;
    if (WH >= 64) {
        SW = W;
        SH = H;
        cols = 1;
        return;
    }
    const int nt = 64 / WH;
    cols = 8 / W;
    if (cols < 1) cols = 1;
    if (cols > nt) cols = nt;
    SW = cols * W;
    SH = (nt / cols) * H;
}

Frame make_frame(int w, int h, int spp, int B, pt_mode mode, pt_group g, uint64_t seed) {
    Frame f{};
    f.w = w;
    f.h = h;
    f.spp = spp;
    f.B = B;
    f.mode = (int)mode;
    f.W = g.tile_w;
    f.H = g.tile_h;
    f.K = g.k;
    f.WH = f.W * f.H;
    f.reuse_max = g.reuse_max_bounce ? g.reuse_max_bounce : 0xFFFF;   // 0: the library default, every bounce
    super_tile(f.W, f.H, f.SW, f.SH, f.cols);
    f.TS = f.SW * f.SH;
    f.nstx = (w + f.SW - 1) / f.SW;
    f.nsty = (h + f.SH - 1) / f.SH;
    f.ntx = (w + f.W - 1) / f.W;
    f.nslots = (uint32_t)f.nstx * (uint32_t)f.nsty * (uint32_t)f.TS;
    // compacted queues: 8 regions (shade workgroup blk writes region blk mod 8)
    f.region = (uint32_t)(((uint32_t)f.nstx * (uint32_t)f.nsty + 7u) / 8u) * (uint32_t)f.TS;
    f.seed = seed;
    f.nee = g.nee;
    f.frame_groups = g.frame_groups;
    return f;
}

// camera basis (host side of the arithmetic contract)
void set_camera(Frame& f, const pt_camera* cam, int w, int h) {
    H3 pos{cam->pos[0], cam->pos[1], cam->pos[2]};
    H3 at{cam->look_at[0], cam->look_at[1], cam->look_at[2]};
    H3 up{cam->up[0], cam->up[1], cam->up[2]};
    H3 fwd = h_unit(h_sub(at, pos));
    H3 right = h_unit(h_cross(fwd, up));
    H3 upv = h_cross(right, fwd);
    const float th = (float)tan((double)cam->vfov_deg * (3.14159265358979323846 / 360.0));
    const float vals[4][3] = {{pos.x, pos.y, pos.z}, {fwd.x, fwd.y, fwd.z}, {right.x, right.y, right.z}, {upv.x, upv.y, upv.z}};
    for (int a = 0; a < 3; ++a) {
        f.cpos[a] = vals[0][a];
        f.cfwd[a] = vals[1][a];
        f.cright[a] = vals[2][a];
        f.cup[a] = vals[3][a];
    }
    f.th = th;
    f.thx = th * ((float)w / (float)h);
}

struct Layout {
    size_t q0, q1, state, live, work, partial, sortws, ovf, total;
    size_t shray, shc, sprim, st, swork, spartial;   // next-event estimation
};

Layout layout(const Frame& f) {
    Layout L{};
    size_t o = 0;
    const size_t qb = (size_t)8 * f.region * 32;   // a ray queue: the slots, or the 8 regions of a compacted one
    const size_t launches = (size_t)(f.B + 1) * (size_t)f.spp;
    L.q0 = o;
    o = align256(o + qb);
    L.q1 = o;
    o = align256(o + qb);
    L.state = o;
    o = align256(o + qb);
    L.live = o;
    o = align256(o + (size_t)(f.nslots / (uint32_t)f.TS) * 4);
    L.work = o;
    o = align256(o + launches * pt::kWorkWords * 4);
    L.partial = o;
    o = align256(o + launches * pt::kMaxTraceBlocks * 4);
    if (is_sorted_mode(f.mode)) {
        L.sortws = o;
        o = align256(o + pt::sort_compacted_workspace_bytes(f.nslots, 8 * f.region));
    }
    if (f.nee) {
        L.shray = o;
        o = align256(o + qb);
        L.shc = o;
        o = align256(o + (size_t)f.nslots * 16);
        L.sprim = o;
        o = align256(o + (size_t)f.nslots * 4);
        L.st = o;
        o = align256(o + (size_t)f.nslots * 4);
        L.swork = o;
        o = align256(o + launches * pt::kWorkWords * 4);
        L.spartial = o;
        o = align256(o + launches * pt::kMaxTraceBlocks * 4);
    }
    L.ovf = o;
    o = align256(o + (size_t)pt::kMaxTraceBlocks * pt::kTraceBlock * pt::kStackOvf * 4);
    L.total = o;
    return L;
}

struct TimerScope {
    pt_timer t;
    hipStream_t st;
    int idx = -1;
    TimerScope(pt_timer t_, hipStream_t st_, int kind, int bounce) : t(t_), st(st_) {
        if (t && t->n < t->cap) {
            idx = t->n++;
            t->kind[idx] = kind;
            t->bounce[idx] = bounce;
            (void)hipEventRecord(t->ev[2 * idx], st);
        }
    }
    ~TimerScope() {
        if (idx >= 0) (void)hipEventRecord(t->ev[2 * idx + 1], st);
    }
};

}  // namespace

extern "C" {

pt_status pt_probe_memory(void* buf, size_t bytes, int passes, int chase_steps, float* read_gbps, float* chase_ns,
                          void* stream) {
    if (!buf || !read_gbps || !chase_ns) return fail(PT_EINVAL, "null argument");
    if (((uintptr_t)buf & 255) != 0) return fail(PT_EINVAL, "buffer must be 256-byte aligned");
    if (bytes < (64u << 10)) return fail(PT_EINVAL, "buffer must hold at least 64 KiB (got %zu)", bytes);
    if (passes < 1 || passes > (1 << 24) || chase_steps < 1 || chase_steps > (1 << 24))
        return fail(PT_EINVAL, "passes and chase_steps must be in [1, 2^24]");
    hipStream_t st = (hipStream_t)stream;
    size_t lines = bytes / 128;
    if (lines > (1ull << 31)) lines = 1ull << 31;
    uint32_t nlines = 1;
    while ((size_t)nlines * 2 <= lines) nlines *= 2;
    uint32_t* words = (uint32_t*)buf;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto& x : ev)
                if (x) (void)hipEventDestroy(x);
            return fail(PT_EDEVICE, "hipEventCreate failed");
        }
    hipError_t e = pt::launch_probe_fill(words, nlines, st);
    if (e == hipSuccess) e = pt::launch_probe_read(buf, bytes, 1, words + 1, st);   // warm the level
    if (e == hipSuccess) e = hipEventRecord(ev[0], st);
    if (e == hipSuccess) e = pt::launch_probe_read(buf, bytes, passes, words + 1, st);
    if (e == hipSuccess) e = hipEventRecord(ev[1], st);
    if (e == hipSuccess) e = pt::launch_probe_chase(words, nlines, chase_steps, words + 2, st);
    if (e == hipSuccess) e = hipEventRecord(ev[2], st);
    if (e == hipSuccess) e = hipEventSynchronize(ev[2]);
    float ms_read = 0.f, ms_chase = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms_read, ev[0], ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms_chase, ev[1], ev[2]);
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (e != hipSuccess) return hip_fail(e, "memory probe");
    *read_gbps = (float)((double)(bytes / 16) * 16.0 * passes / (ms_read * 1e-3) / 1e9);
    *chase_ns = (float)(ms_chase * 1e6 / chase_steps);
    return PT_OK;
}

const char* pt_last_error(void) { return g_err.c_str(); }

pt_status pt_device_info(int* compute_units, int* arch_major, int* arch_minor) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (compute_units) *compute_units = prop.multiProcessorCount;
    if (arch_major) *arch_major = prop.major;
    if (arch_minor) *arch_minor = prop.minor;
    return PT_OK;
}

pt_status pt_scene_create(const pt_scene_desc* d, pt_scene* out) {
    if (!d || !out) return fail(PT_EINVAL, "null argument");
    *out = nullptr;
    if (d->ntri > 0 && (!d->tris || !d->tri_mat)) return fail(PT_EINVAL, "null triangle arrays");
    if (d->nmat == 0 || !d->mats) return fail(PT_EINVAL, "at least one material is required");
    if (d->ntri > pt::kMaxTris) return fail(PT_EINVAL, "too many triangles (%u)", d->ntri);
    pt_scene s = new (std::nothrow) pt_scene_s();
    if (!s) return fail(PT_ENOMEM, "host allocation failed");
    try {
        const uint32_t n = d->ntri;
        for (uint32_t i = 0; i < n; ++i) {
            if (d->tri_mat[i] >= d->nmat) {
                delete s;
                return fail(PT_EINVAL, "triangle %u has material %u >= %u", i, d->tri_mat[i], d->nmat);
            }
        }
        for (int a = 0; a < 3; ++a) {
            s->lo[a] = INFINITY;
            s->hi[a] = -INFINITY;
        }
        for (size_t j = 0; j < 9 * (size_t)n; ++j) {
            const float v = d->tris[j];
            if (!std::isfinite(v)) {
                delete s;
                return fail(PT_EINVAL, "non-finite vertex coordinate at triangle %zu", j / 9);
            }
            const int a = (int)(j % 3);
            if (v < s->lo[a]) s->lo[a] = v;
            if (v > s->hi[a]) s->hi[a] = v;
        }
        if (n == 0)
            for (int a = 0; a < 3; ++a) s->lo[a] = s->hi[a] = 0.0f;
        std::string err;
        if (!pt::build_bvh(d->tris, n, s->bvh, err)) {
            delete s;
            return fail(PT_ENOMEM, "BVH build failed: %s", err.c_str());
        }
        s->ntri = n;
        s->nmat = d->nmat;
        s->btris.resize(3 * (size_t)n);
        s->otris.resize(3 * (size_t)n);
        for (uint32_t i = 0; i < n; ++i) {
            const float* v = d->tris + 9 * (size_t)i;
            for (int c = 0; c < 3; ++c)
                s->otris[3 * (size_t)i + c] = make_float4(v[3 * c], v[3 * c + 1], v[3 * c + 2], 0.0f);
        }
        for (uint32_t j = 0; j < n; ++j) {
            const uint32_t p = s->bvh.order[j];
            for (int c = 0; c < 3; ++c) s->btris[3 * (size_t)j + c] = s->otris[3 * (size_t)p + c];
            int32_t id = (int32_t)p;
            float fid;
            memcpy(&fid, &id, 4);
            s->btris[3 * (size_t)j].w = fid;
        }
        s->tri_mat.assign(d->tri_mat, d->tri_mat + n);
        s->mats.assign(d->mats, d->mats + d->nmat);
        for (uint32_t i = 0; i < n; ++i) {
            const float* em = s->mats[s->tri_mat[i]].emission;
            if (em[0] > 0.0f || em[1] > 0.0f || em[2] > 0.0f) s->emit.push_back(i);
        }
        for (int a = 0; a < 3; ++a) s->env[a] = d->env_radiance[a];
        size_t o = 0;
        s->off_nodes = o;
        o = align256(o + s->bvh.nodes.size() * sizeof(pt::BvhNode));
        s->off_nodes4 = o;
        o = align256(o + s->bvh.nodes4.size() * sizeof(pt::Bvh4Node));
        s->off_nodes4q = o;
        o = align256(o + s->bvh.nodes4q.size() * sizeof(pt::Bvh4QNode));
        s->off_btris = o;
        o = align256(o + s->btris.size() * sizeof(float4));
        s->off_otris = o;
        o = align256(o + s->otris.size() * sizeof(float4));
        s->off_mat = o;
        o = align256(o + s->tri_mat.size() * 4);
        s->off_mats = o;
        o = align256(o + s->mats.size() * sizeof(pt_material));
        s->off_emit = o;
        o = align256(o + s->emit.size() * 4);
        s->bytes = o;
    } catch (const std::bad_alloc&) {
        delete s;
        return fail(PT_ENOMEM, "host allocation failed");
    }
    *out = s;
    return PT_OK;
}

size_t pt_scene_device_bytes(pt_scene s) { return s ? s->bytes : 0; }

pt_status pt_scene_upload(pt_scene s, void* arena, size_t bytes, void* stream) {
    if (!s || !arena) return fail(PT_EINVAL, "null argument");
    if (((uintptr_t)arena & 255) != 0) return fail(PT_EINVAL, "arena must be 256-byte aligned");
    if (bytes < s->bytes) return fail(PT_ENOMEM, "arena too small: %zu < %zu", bytes, s->bytes);
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)arena;
    struct Part {
        size_t off;
        const void* src;
        size_t n;
    } parts[] = {
        {s->off_nodes, s->bvh.nodes.data(), s->bvh.nodes.size() * sizeof(pt::BvhNode)},
        {s->off_nodes4, s->bvh.nodes4.data(), s->bvh.nodes4.size() * sizeof(pt::Bvh4Node)},
        {s->off_nodes4q, s->bvh.nodes4q.data(), s->bvh.nodes4q.size() * sizeof(pt::Bvh4QNode)},
        {s->off_btris, s->btris.data(), s->btris.size() * sizeof(float4)},
        {s->off_otris, s->otris.data(), s->otris.size() * sizeof(float4)},
        {s->off_mat, s->tri_mat.data(), s->tri_mat.size() * 4},
        {s->off_mats, s->mats.data(), s->mats.size() * sizeof(pt_material)},
        {s->off_emit, s->emit.data(), s->emit.size() * 4},
    };
    for (const Part& p : parts) {
        if (p.n == 0) continue;
        hipError_t e = hipMemcpyAsync(base + p.off, p.src, p.n, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (scene upload)");
    }
    // host arrays must stay valid until the copies complete
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize (scene upload)");
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    DevScene& d = s->dev;
    d.nodes = (const float4*)(base + s->off_nodes);
    d.nodes4 = (const float4*)(base + s->off_nodes4);
    d.nodes4q = (const float4*)(base + s->off_nodes4q);
    d.quant = s->bvh.quant_ok ? 1u : 0u;
    // four-wide traversal pushes up to three siblings per level: use it when the stack bound holds
    d.wide = (pt::kPreferWide && 3u * s->bvh.max_depth4 + 4u <= (uint32_t)(pt::kStackLds + pt::kStackOvf)) ? 1u : 0u;
    d.btris = (const float4*)(base + s->off_btris);
    d.otris = (const float4*)(base + s->off_otris);
    d.tri_mat = (const uint32_t*)(base + s->off_mat);
    d.mats = (const pt_material*)(base + s->off_mats);
    d.emit = (const uint32_t*)(base + s->off_emit);
    d.ntri = s->ntri;
    d.nmat = s->nmat;
    d.nemit = (uint32_t)s->emit.size();
    for (int a = 0; a < 3; ++a) {
        d.env[a] = s->env[a];
        d.lo[a] = s->lo[a];
        d.hi[a] = s->hi[a];
    }
    s->uploaded = true;
    s->device = dev;
    return PT_OK;
}

pt_status pt_scene_get_info(pt_scene s, pt_scene_info* info) {
    if (!s || !info) return fail(PT_EINVAL, "null argument");
    info->ntri = s->ntri;
    info->nnodes = (uint32_t)s->bvh.nodes.size();
    info->max_depth = s->bvh.max_depth;
    info->max_leaf = s->bvh.max_leaf;
    for (int a = 0; a < 3; ++a) {
        info->lo[a] = s->lo[a];
        info->hi[a] = s->hi[a];
    }
    info->sah_cost = s->bvh.sah_cost;
    info->device_bytes = s->bytes;
    info->nemit = (uint32_t)s->emit.size();
    info->nnodes4 = (uint32_t)s->bvh.nodes4.size();
    info->max_depth4 = s->bvh.max_depth4;
    info->wide = (pt::kPreferWide && 3u * s->bvh.max_depth4 + 4u <= (uint32_t)(pt::kStackLds + pt::kStackOvf)) ? 1u : 0u;
    info->quant = s->bvh.quant_ok ? 1u : 0u;
    return PT_OK;
}

pt_status pt_scene_export_bvh(pt_scene s, void* nodes, uint32_t* order) {
    if (!s) return fail(PT_EINVAL, "null scene");
    if (nodes) memcpy(nodes, s->bvh.nodes.data(), s->bvh.nodes.size() * sizeof(pt::BvhNode));
    if (order && !s->bvh.order.empty()) memcpy(order, s->bvh.order.data(), s->bvh.order.size() * sizeof(uint32_t));
    return PT_OK;
}

pt_status pt_scene_export_bvh4(pt_scene s, void* nodes4) {
    if (!s || !nodes4) return fail(PT_EINVAL, "null argument");
    if (!s->bvh.nodes4.empty()) memcpy(nodes4, s->bvh.nodes4.data(), s->bvh.nodes4.size() * sizeof(pt::Bvh4Node));
    return PT_OK;
}

pt_status pt_scene_export_bvh4q(pt_scene s, void* nodes4q) {
    if (!s || !nodes4q) return fail(PT_EINVAL, "null argument");
    if (!s->bvh.nodes4q.empty())
        memcpy(nodes4q, s->bvh.nodes4q.data(), s->bvh.nodes4q.size() * sizeof(pt::Bvh4QNode));
    return PT_OK;
}

pt_status pt_scene_free(pt_scene s) {
    delete s;
    return PT_OK;
}

size_t pt_render_workspace_bytes(int w, int h, int spp, int bounces, pt_mode mode, pt_group g) {
    if (w <= 0 || h <= 0 || spp <= 0 || bounces < 0 || bounces > 64) return 0;
    if (check_group(g, bounces) != PT_OK) return 0;
    return layout(make_frame(w, h, spp, bounces, mode, g, 0)).total;
}

pt_status pt_render(pt_scene scene, const pt_camera* cam, int w, int h, int spp, int B, pt_mode mode, pt_group g,
                    uint64_t seed, void* workspace, size_t ws_bytes, const pt_outputs* out, void* stream) {
    if (!scene || !cam || !out) return fail(PT_EINVAL, "null argument");
    if (!scene->uploaded) return fail(PT_EINVAL, "scene not uploaded");
    if (w <= 0 || h <= 0 || spp <= 0) return fail(PT_EINVAL, "w, h, spp must be >= 1 (got %d, %d, %d)", w, h, spp);
    if (B < 0 || B > 64) return fail(PT_EINVAL, "bounces must be in [0, 64] (got %d)", B);
    if ((long long)w * (long long)h > (1ll << 30)) return fail(PT_EINVAL, "image too large");
    if (mode != PT_MODE_INCOHERENT && !is_reuse_mode(mode) && !is_sorted_mode(mode))
        return fail(PT_EINVAL, "unknown mode %d", (int)mode);
    pt_status cs = check_group(g, B);
    if (cs != PT_OK) return cs;
    if (g.nee && mode == PT_MODE_REUSE_WORLD)
        return fail(PT_EUNSUPPORTED, "next-event estimation is not combined with direct world-space reuse");
    if (!out->radiance || !out->hit_prim || !out->hit_t) return fail(PT_EINVAL, "radiance, hit_prim and hit_t are required");
    if (!workspace) return fail(PT_EINVAL, "null workspace");
    int dev = 0;
    hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess) return hip_fail(ge, "hipGetDevice");
    if (dev != scene->device) return fail(PT_EINVAL, "scene was uploaded on device %d, current device is %d", scene->device, dev);
    const int kind = (int)g.traversal - 1;   // -1: the scene's own choice
    if (kind > pt::trace_max_kind(scene->dev))
        return fail(PT_EINVAL, "traversal %d is not available for this scene (at most %d)", g.traversal,
                    pt::trace_max_kind(scene->dev) + 1);

    Frame f = make_frame(w, h, spp, B, mode, g, seed);
    if (is_sorted_mode(mode) && f.nslots > (1u << 27))
        return fail(PT_EINVAL, "sorted modes support at most 2^27 rays per bounce");
    const Layout L = layout(f);
    if (ws_bytes < L.total) return fail(PT_ENOMEM, "workspace too small: %zu < %zu", ws_bytes, L.total);
    set_camera(f, cam, w, h);
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)workspace;
    float4* q[2] = {(float4*)(ws + L.q0), (float4*)(ws + L.q1)};
    float4* state = (float4*)(ws + L.state);
    f.live = (uint32_t*)(ws + L.live);
    uint32_t* partial = (uint32_t*)(ws + L.partial);
    uint32_t* work = (uint32_t*)(ws + L.work);
    int32_t* ovf = (int32_t*)(ws + L.ovf);
    const size_t launches = (size_t)(B + 1) * (size_t)spp;
    hipError_t e;
    {
        TimerScope ts(out->timer, st, 6, -1);
        e = pt::launch_zero(work, launches * pt::kWorkWords, st);
        if (e == hipSuccess && out->stats) e = pt::launch_zero((uint32_t*)out->stats, (size_t)(B + 1) * 4, st);
        if (e == hipSuccess && f.nee) e = pt::launch_zero((uint32_t*)(ws + L.swork), launches * pt::kWorkWords, st);
        if (e == hipSuccess && out->shadow_count) e = pt::launch_zero(out->shadow_count, launches, st);
    }
    if (e != hipSuccess) return hip_fail(e, "launch (zero)");
    const int grid = pt::trace_grid_blocks(g.waves_per_cu);
    const size_t plane = (size_t)w * (size_t)h;
    for (int s = 0; s < spp; ++s) {
        {
            TimerScope ts(out->timer, st, 1, 0);
            e = pt::launch_raygen(f, s, q[0], state, (float4*)out->rays, st);
        }
        if (e != hipSuccess) return hip_fail(e, "launch (raygen)");
        for (int b = 0; b <= B; ++b) {
            const size_t li = (size_t)b * spp + s;
            const uint32_t n = f.nslots;
            // bounces after the first trace a compacted queue: the live rays the previous shade
            // wrote into 8 regions, counted in the fill words of this launch's work area
            const uint32_t* fill = b >= 1 ? work + li * pt::kWorkWords + pt::kFillWord : nullptr;
            const uint32_t* perm = nullptr;
            if (is_sorted_mode(mode) && b >= 1) {
                {
                    TimerScope ts(out->timer, st, 3, b);
                    e = pt::launch_keys_compacted(fill, f.region, f.nslots, ws + L.sortws, st);
                }
                if (e != hipSuccess) return hip_fail(e, "launch (keys)");
                {
                    TimerScope ts(out->timer, st, 4, b);
                    e = pt::launch_sort_compacted(fill, f.nslots, ws + L.sortws, &perm, st);
                }
                if (e != hipSuccess) return hip_fail(e, "launch (sort)");
            }
            pt::TraceArgs ta{};
            ta.rays = q[b & 1];
            ta.n = n;
            ta.fill = fill;
            ta.region = f.region;
            ta.perm = perm;   // sorted: the rays are read in key order
            ta.work = work + li * pt::kWorkWords;
            ta.out_prim = out->hit_prim + li * plane;
            ta.out_t = out->hit_t + li * plane;
            ta.partial = out->ray_count ? partial + li * pt::kMaxTraceBlocks : nullptr;
            ta.stats = out->stats ? (unsigned long long*)(out->stats + 2 * (size_t)b) : nullptr;
            if (out->stats && out->touched && b < 8 && s == 0) {
                ta.touched = out->touched;
                ta.touch_tri = (uint32_t)scene->bvh.nodes.size();
                ta.touch_bit = 1u << b;
            }
            ta.ovf = ovf;
            ta.by_pixel = 1;
            ta.refill = g.refill ? g.refill : kDefaultRefill;
            ta.waves_per_cu = g.waves_per_cu;
            ta.leaf_gate = (g.leaf_gate ? g.leaf_gate : pt::kDefaultLeafGate) - 1;
            ta.kind = kind;
            {
                TimerScope ts(out->timer, st, 0, b);
                e = pt::launch_trace(scene->dev, ta, out->stats != nullptr, st);
            }
            if (e != hipSuccess) return hip_fail(e, "launch (trace)");
            float4* shray = f.nee ? (float4*)(ws + L.shray) : nullptr;
            float4* shc = f.nee ? (float4*)(ws + L.shc) : nullptr;
            {
                TimerScope ts(out->timer, st, 2, b);
                // the next rays go compacted into the regions counted by the next launch's fill words
                uint32_t* fill_next = b < B ? work + ((size_t)(b + 1) * spp + s) * pt::kWorkWords + pt::kFillWord : nullptr;
                // sorted modes: the shade kernel writes each next ray's key beside it
                uint32_t* keys_next = is_sorted_mode(mode) && b < B ? pt::sort_key_slots(ws + L.sortws, f.nslots) : nullptr;
                e = pt::launch_shade(scene->dev, f, b, s, q[b & 1], q[(b + 1) & 1], state, out->hit_prim, out->hit_t,
                                     out->radiance, (float4*)out->rays, shray, shc, fill_next, keys_next,
                                     (float4*)out->debug, st);
            }
            if (e != hipSuccess) return hip_fail(e, "launch (shade)");
            if (f.nee && b < B) {
                // shadow rays of the Lambert points of this hit, then their light into the paths
                int32_t* sprim = (int32_t*)(ws + L.sprim);
                pt::TraceArgs sa{};
                sa.rays = shray;
                sa.n = n;
                sa.work = (uint32_t*)(ws + L.swork) + li * pt::kWorkWords;
                sa.out_prim = sprim;
                sa.out_t = (float*)(ws + L.st);
                sa.partial = out->shadow_count ? (uint32_t*)(ws + L.spartial) + li * pt::kMaxTraceBlocks : nullptr;
                sa.ovf = ovf;
                sa.by_pixel = 0;
                sa.shadow = 1;
                sa.skip_empty = 1;
                sa.refill = g.refill ? g.refill : kDefaultRefill;
                sa.waves_per_cu = g.waves_per_cu;
                sa.leaf_gate = (g.leaf_gate ? g.leaf_gate : pt::kDefaultLeafGate) - 1;
                sa.kind = kind;
                {
                    TimerScope ts(out->timer, st, 7, b);
                    e = pt::launch_trace(scene->dev, sa, false, st);
                }
                if (e != hipSuccess) return hip_fail(e, "launch (shadow trace)");
                {
                    TimerScope ts(out->timer, st, 8, b);
                    e = pt::launch_nee_accumulate(shray, shc, sprim, f.nslots, state, st);
                }
                if (e != hipSuccess) return hip_fail(e, "launch (shadow accumulate)");
            }
        }
    }
    if (out->ray_count) {
        TimerScope ts(out->timer, st, 6, -1);
        e = pt::launch_count_finalize(partial, pt::kMaxTraceBlocks, grid, (int)launches, out->ray_count, st);
        if (e != hipSuccess) return hip_fail(e, "launch (count)");
    }
    if (out->shadow_count && f.nee && B > 0) {
        // launches of bounces 0..B-1 hold shadow rays: the first B * spp entries
        TimerScope ts(out->timer, st, 6, -1);
        e = pt::launch_count_finalize((uint32_t*)(ws + L.spartial), pt::kMaxTraceBlocks, grid, B * spp,
                                      out->shadow_count, st);
        if (e != hipSuccess) return hip_fail(e, "launch (shadow count)");
    }
    return PT_OK;
}

size_t pt_trace_workspace_bytes(void) {
    return align256((size_t)pt::kWorkWords * 4) + align256((size_t)pt::kMaxTraceBlocks * pt::kTraceBlock * pt::kStackOvf * 4);
}

pt_status pt_trace(pt_scene scene, const float* rays, uint32_t n, int refill, int32_t* prim, float* t,
                   void* workspace, size_t ws_bytes, void* stream) {
    if (refill < 0 || refill > 64) return fail(PT_EINVAL, "refill must be in [0, 64] (got %d)", refill);
    if (!scene || (n > 0 && (!rays || !prim || !t)) || !workspace) return fail(PT_EINVAL, "null argument");
    if (!scene->uploaded) return fail(PT_EINVAL, "scene not uploaded");
    if (ws_bytes < pt_trace_workspace_bytes()) return fail(PT_ENOMEM, "workspace too small");
    if (n == 0) return PT_OK;
    hipStream_t st = (hipStream_t)stream;
    pt::TraceArgs ta{};
    ta.rays = (const float4*)rays;
    ta.n = n;
    ta.work = (uint32_t*)workspace;
    ta.out_prim = prim;
    ta.out_t = t;
    ta.ovf = (int32_t*)((char*)workspace + align256((size_t)pt::kWorkWords * 4));
    ta.by_pixel = 0;
    ta.refill = refill ? refill : kDefaultRefill;
    ta.leaf_gate = pt::kDefaultLeafGate - 1;
    ta.kind = -1;
    hipError_t e = pt::launch_zero(ta.work, pt::kWorkWords, st);
    if (e != hipSuccess) return hip_fail(e, "launch (zero)");
    e = pt::launch_trace(scene->dev, ta, false, st);
    if (e != hipSuccess) return hip_fail(e, "launch (trace)");
    return PT_OK;
}

}  // extern "C"

namespace {

// Scratch of pt_trace_static: the launch's ray counters, then the traversal stack overflow
// area of a persistent grid of at most kStaticTraceBlocks workgroups ([kStackOvf][grid lanes]
// int32).  File-scope device memory, one copy per device, held until the process ends.  In
// host code its name is not a device address: kernels get the address that
// hipGetSymbolAddress returns for the current device (static_scratch below).
constexpr int kStaticTraceBlocks = 2048;   // 8 waves per CU on 256 CUs
constexpr size_t kStaticWorkBytes = (size_t)pt::kWorkWords * 4;
constexpr size_t kStaticScratchBytes =
    kStaticWorkBytes + (size_t)kStaticTraceBlocks * pt::kTraceBlock * pt::kStackOvf * 4;
static_assert(kStaticWorkBytes % 256 == 0, "the overflow area stays 256-byte aligned");
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
pt_status static_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(PT_EUNSUPPORTED, "device %d is beyond the %d this library serves", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(PT_EDEVICE, "hipGetSymbolAddress(scratch) returned a null address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PT_OK;
}

}  // namespace

extern "C" {

size_t pt_trace_static_scratch_bytes(void) { return kStaticScratchBytes; }

pt_status pt_trace_static(pt_scene scene, const float* rays, uint32_t n, int refill, int waves_per_cu, int32_t* prim,
                          float* t, void* stream) {
    if (refill < 0 || refill > 64) return fail(PT_EINVAL, "refill must be in [0, 64] (got %d)", refill);
    if (waves_per_cu < 0 || waves_per_cu > 32) return fail(PT_EINVAL, "waves_per_cu must be in [0, 32] (got %d)", waves_per_cu);
    if (!scene || (n > 0 && (!rays || !prim || !t))) return fail(PT_EINVAL, "null argument");
    if (!scene->uploaded) return fail(PT_EINVAL, "scene not uploaded");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != scene->device) return fail(PT_EINVAL, "scene was uploaded on device %d, current device is %d", scene->device, dev);
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    // the scratch holds the overflow stacks of kStaticTraceBlocks workgroups: a larger grid is refused
    if (waves_per_cu > 0 && (long long)waves_per_cu * cus > kStaticTraceBlocks)
        return fail(PT_EINVAL, "waves_per_cu %d x %d compute units exceeds the %d workgroups the static scratch (%zu bytes) holds",
                    waves_per_cu, cus, kStaticTraceBlocks, kStaticScratchBytes);
    void* sp = nullptr;
    pt_status ps = static_scratch(&sp);
    if (ps != PT_OK) return ps;
    if (n == 0) return PT_OK;
    hipStream_t st = (hipStream_t)stream;
    pt::TraceArgs ta{};
    ta.rays = (const float4*)rays;
    ta.n = n;
    ta.work = (uint32_t*)sp;
    ta.out_prim = prim;
    ta.out_t = t;
    ta.ovf = (int32_t*)((char*)sp + kStaticWorkBytes);
    ta.by_pixel = 0;
    ta.refill = refill ? refill : kDefaultRefill;
    ta.waves_per_cu = waves_per_cu ? waves_per_cu : kStaticTraceBlocks / (cus > 0 ? cus : 1);
    ta.leaf_gate = pt::kDefaultLeafGate - 1;
    ta.kind = -1;
    ta.max_blocks = kStaticTraceBlocks;
    e = pt::launch_zero(ta.work, pt::kWorkWords, st);   // a fill kernel, not a memset node
    if (e != hipSuccess) return hip_fail(e, "launch (zero)");
    e = pt::launch_trace(scene->dev, ta, false, st);
    if (e != hipSuccess) return hip_fail(e, "launch (trace)");
    return PT_OK;
}

pt_status pt_ray_keys(pt_scene scene, const float* rays, uint32_t n, pt_mode mode, uint32_t* keys, void* stream) {
    if (!scene || (n > 0 && (!rays || !keys))) return fail(PT_EINVAL, "null argument");
    if (!scene->uploaded) return fail(PT_EINVAL, "scene not uploaded");
    if (!is_sorted_mode(mode)) return fail(PT_EINVAL, "mode %d is not a sorted mode", (int)mode);
    if (n == 0) return PT_OK;
    hipError_t e = pt::launch_keys(scene->dev, (const float4*)rays, n, keys, nullptr, (int)mode, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launch (keys)");
    return PT_OK;
}

size_t pt_sort_workspace_bytes(uint32_t n) { return pt::sort_workspace_bytes(n); }

pt_status pt_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t n, void* workspace, size_t ws_bytes, void* stream) {
    if (n > 0 && (!keys || !vals || !workspace)) return fail(PT_EINVAL, "null argument");
    if (n > (1u << 27)) return fail(PT_EINVAL, "at most 2^27 pairs (got %u)", n);
    if (ws_bytes < pt::sort_workspace_bytes(n)) return fail(PT_ENOMEM, "workspace too small");
    hipError_t e = pt::radix_sort_pairs(keys, vals, n, workspace, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launch (sort)");
    return PT_OK;
}

pt_status pt_timer_create(int capacity, pt_timer* out) {
    if (!out || capacity <= 0) return fail(PT_EINVAL, "bad argument");
    pt_timer t = new (std::nothrow) pt_timer_s();
    if (!t) return fail(PT_ENOMEM, "host allocation failed");
    t->cap = capacity;
    t->ev.resize(2 * (size_t)capacity);
    t->kind.resize(capacity);
    t->bounce.resize(capacity);
    for (auto& ev : t->ev) {
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            for (auto& x : t->ev)
                if (x) (void)hipEventDestroy(x);
            delete t;
            return hip_fail(e, "hipEventCreate");
        }
    }
    *out = t;
    return PT_OK;
}

pt_status pt_timer_reset(pt_timer t) {
    if (!t) return fail(PT_EINVAL, "null timer");
    t->n = 0;
    return PT_OK;
}

pt_status pt_timer_read(pt_timer t, float* ms, int32_t* kind, int32_t* bounce, int max, int* n) {
    if (!t || !n) return fail(PT_EINVAL, "null argument");
    const int m = t->n < max ? t->n : max;
    for (int i = 0; i < m; ++i) {
        hipError_t e = hipEventSynchronize(t->ev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float v = 0.0f;
        e = hipEventElapsedTime(&v, t->ev[2 * i], t->ev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        if (ms) ms[i] = v;
        if (kind) kind[i] = t->kind[i];
        if (bounce) bounce[i] = t->bounce[i];
    }
    *n = m;
    return PT_OK;
}

pt_status pt_timer_free(pt_timer t) {
    if (!t) return PT_OK;
    for (auto& e : t->ev)
        if (e) (void)hipEventDestroy(e);
    delete t;
    return PT_OK;
}


// ---------------------------------------------------------------------------- batches

// a job's arena: two ray queues and the path state (32 B per slot each), then one flag
// word per shade workgroup
static size_t job_bytes_of(const Frame& f) {
    return 3 * align256((size_t)f.nslots * 32) + align256((size_t)(f.nslots / (uint32_t)f.TS) * 4);
}

size_t pt_batch_job_bytes(const pt_job* job, pt_group group) {
    if (!job || job->w <= 0 || job->h <= 0 || job->spp <= 0 || job->bounces < 0 || job->bounces > 64) return 0;
    if (check_group(group, job->bounces) != PT_OK) return 0;
    return job_bytes_of(make_frame(job->w, job->h, job->spp, job->bounces, (pt_mode)job->mode, group, 0));
}

static size_t batch_table_stride(int max_jobs) { return align256((size_t)max_jobs * sizeof(pt::StepJob)); }

size_t pt_batch_base_bytes(int max_jobs) {
    if (max_jobs <= 0 || max_jobs > 65536) return 0;
    return kBatchRing * batch_table_stride(max_jobs) + align256((size_t)kBatchRing * pt::kWorkWords * 4) +
           align256((size_t)pt::kMaxTraceBlocks * pt::kTraceBlock * pt::kStackOvf * 4);
}

static bool pool_alloc(pt_batch bt, size_t n, size_t* off) {
    for (auto it = bt->free_ranges.begin(); it != bt->free_ranges.end(); ++it) {
        if (it->second >= n) {
            *off = it->first;
            const size_t rest = it->second - n;
            const size_t at = it->first + n;
            bt->free_ranges.erase(it);
            if (rest) bt->free_ranges[at] = rest;
            return true;
        }
    }
    return false;
}

static void pool_free(pt_batch bt, size_t off, size_t n) {
    auto it = bt->free_ranges.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != bt->free_ranges.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        bt->free_ranges.erase(nx);
    }
    if (it != bt->free_ranges.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            bt->free_ranges.erase(it);
        }
    }
}

static void batch_drop_graph(pt_batch bt) {
    if (bt->gexec) (void)hipGraphExecDestroy(bt->gexec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    bt->gexec = nullptr;
    bt->graph = nullptr;
    bt->graph_key.clear();
    if (bt->sched_bytes) pool_free(bt, bt->sched_off, bt->sched_bytes);
    bt->sched_bytes = 0;
}

pt_status pt_batch_create(int max_jobs, pt_group group, void* arena, size_t bytes, pt_batch* out) {
    if (!out || !arena) return fail(PT_EINVAL, "null argument");
    *out = nullptr;
    if (max_jobs <= 0 || max_jobs > 65536) return fail(PT_EINVAL, "max_jobs must be in [1, 65536]");
    pt_status cs = check_group(group, 0);
    if (cs != PT_OK) return cs;
    if (group.nee) return fail(PT_EUNSUPPORTED, "batches do not run next-event estimation");
    if (((uintptr_t)arena & 255) != 0) return fail(PT_EINVAL, "arena must be 256-byte aligned");
    const size_t base = pt_batch_base_bytes(max_jobs);
    if (bytes < base) return fail(PT_ENOMEM, "arena too small: %zu < %zu", bytes, base);
    pt_batch bt = new (std::nothrow) pt_batch_s();
    if (!bt) return fail(PT_ENOMEM, "host allocation failed");
    bt->max_jobs = max_jobs;
    bt->group = group;
    bt->arena = (char*)arena;
    bt->bytes = bytes;
    bt->table_stride = batch_table_stride(max_jobs);
    bt->table_off = 0;
    bt->counter_off = kBatchRing * bt->table_stride;
    bt->ovf_off = bt->counter_off + align256((size_t)kBatchRing * pt::kWorkWords * 4);
    bt->pool_off = base;
    try {
        bt->jobs.resize(max_jobs);
        bt->host_tables.resize(kBatchRing);
        for (auto& t : bt->host_tables) t.reserve(max_jobs);
    } catch (...) {
        delete bt;
        return fail(PT_ENOMEM, "host allocation failed");
    }
    if (bytes > base) bt->free_ranges[base] = bytes - base;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        delete bt;
        return hip_fail(e, "hipGetDevice");
    }
    bt->device = dev;
    for (int i = 0; i < kBatchRing; ++i) {
        e = hipEventCreateWithFlags(&bt->ring_ev[i], hipEventDisableTiming);
        if (e != hipSuccess) {
            pt_batch_free(bt);
            return hip_fail(e, "hipEventCreate");
        }
    }
    for (auto& j : bt->jobs) {
        e = hipEventCreateWithFlags(&j.done_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            pt_batch_free(bt);
            return hip_fail(e, "hipEventCreate");
        }
    }
    e = hipStreamCreateWithFlags(&bt->gstream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->gev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->gev_out, hipEventDisableTiming);
    if (e != hipSuccess) {
        pt_batch_free(bt);
        return hip_fail(e, "stream/event creation");
    }
    *out = bt;
    return PT_OK;
}

pt_status pt_batch_submit(pt_batch bt, const pt_job* job, uint32_t* job_id) {
    if (!bt || !job || !job_id) return fail(PT_EINVAL, "null argument");
    if (!job->scene || !job->scene->uploaded) return fail(PT_EINVAL, "job scene is not uploaded");
    if (job->scene->device != bt->device) return fail(PT_EINVAL, "job scene lives on another device");
    if ((int)bt->group.traversal - 1 > pt::trace_max_kind(job->scene->dev))
        return fail(PT_EINVAL, "traversal %d is not available for this job's scene", bt->group.traversal);
    if (job->mode != PT_MODE_INCOHERENT && job->mode != PT_MODE_REUSE)
        return fail(PT_EUNSUPPORTED, "batches support the incoherent and reuse modes");
    if (job->w <= 0 || job->h <= 0 || job->spp <= 0 || job->bounces < 0 || job->bounces > 64)
        return fail(PT_EINVAL, "bad job size (w %d, h %d, spp %d, bounces %d)", job->w, job->h, job->spp, job->bounces);
    if ((long long)job->w * job->h > (1ll << 30)) return fail(PT_EINVAL, "image too large");
    if (!job->radiance || !job->hit_prim || !job->hit_t) return fail(PT_EINVAL, "job outputs are required");
    int slot = -1;
    for (int i = 0; i < bt->max_jobs; ++i)
        if (!bt->jobs[i].used) {
            slot = i;
            break;
        }
    if (slot < 0) return fail(PT_EBUSY, "no free job slot");
    const size_t need = pt_batch_job_bytes(job, bt->group);
    size_t off = 0;
    if (!pool_alloc(bt, need, &off)) return fail(PT_EBUSY, "arena has no free range of %zu bytes", need);
    BatchJob& J = bt->jobs[slot];
    J.used = true;
    J.finished = false;
    J.job = *job;
    J.f = make_frame(job->w, job->h, job->spp, job->bounces, (pt_mode)job->mode, bt->group, job->seed);
    set_camera(J.f, &job->camera, job->w, job->h);
    J.off = off;
    J.bytes = need;
    J.s = 0;
    J.b = 0;
    *job_id = (uint32_t)slot;
    batch_drop_graph(bt);
    return PT_OK;
}

// fill the launch-table entries of the jobs' current steps; returns jobs, blocks, rays
static int batch_fill_table(pt_batch bt, const std::vector<int>& ids, std::vector<pt::StepJob>& tab,
                            const std::vector<int>& bs, const std::vector<int>& ss, uint32_t* blocks,
                            uint32_t* rays, bool* any_reuse) {
    tab.clear();
    uint32_t blk = 0, ray = 0;
    *any_reuse = false;
    for (size_t k = 0; k < ids.size(); ++k) {
        BatchJob& J = bt->jobs[ids[k]];
        const int b = bs[k], sm = ss[k];
        char* base = bt->arena + J.off;
        const size_t qb = align256((size_t)J.f.nslots * 32);
        float4* q[2] = {(float4*)base, (float4*)(base + qb)};
        pt::StepJob t{};
        t.sc = J.job.scene->dev;
        t.f = J.f;
        t.b = b;
        t.s = sm;
        t.do_raygen = b == 0;
        t.q_out_raygen = q[0];
        t.q_in = q[b & 1];
        t.q_out = q[(b + 1) & 1];
        t.state = (float4*)(base + 2 * qb);
        t.f.live = (uint32_t*)(base + 3 * qb);
        t.hit_prim = J.job.hit_prim;
        t.hit_t = J.job.hit_t;
        const size_t plane = (size_t)J.f.w * J.f.h;
        t.trace_prim = J.job.hit_prim + ((size_t)b * J.f.spp + sm) * plane;
        t.trace_t = J.job.hit_t + ((size_t)b * J.f.spp + sm) * plane;
        t.radiance = J.job.radiance;
        t.block_start = blk;
        t.ray_start = ray;
        t.nrays = J.f.nslots;
        blk += J.f.nslots / (uint32_t)J.f.TS;
        ray += J.f.nslots;
        if (J.f.mode == PT_MODE_REUSE) *any_reuse = true;
        tab.push_back(t);
    }
    *blocks = blk;
    *rays = ray;
    return (int)tab.size();
}

static hipError_t batch_launch_step(pt_batch bt, const pt::StepJob* dtab, int njobs, uint32_t blocks, uint32_t rays,
                                    bool reuse, uint32_t* counter, pt_timer timer, hipStream_t st) {
    int ts = 0;
    for (auto& J : bt->jobs)
        if (J.used) {
            ts = J.f.TS;
            break;
        }
    hipError_t e;
    {
        TimerScope tsc(timer, st, 1, -1);
        e = pt::launch_zero(counter, pt::kWorkWords, st);
        if (e == hipSuccess) e = pt::launch_raygen_multi(dtab, njobs, blocks, ts, st);
    }
    if (e != hipSuccess) return e;
    pt::TraceArgs ta{};
    ta.n = rays;
    ta.work = counter;
    ta.ovf = (int32_t*)(bt->arena + bt->ovf_off);
    ta.by_pixel = 1;
    ta.refill = bt->group.refill ? bt->group.refill : kDefaultRefill;
    ta.waves_per_cu = bt->group.waves_per_cu;
    ta.leaf_gate = (bt->group.leaf_gate ? bt->group.leaf_gate : pt::kDefaultLeafGate) - 1;
    // one kernel for every job: the one asked for, else the narrowest kind any of their scenes needs
    int kind = pt::kTraceWideQueueQ;
    for (auto& J : bt->jobs)
        if (J.used) kind = std::min(kind, pt::trace_kind(J.job.scene->dev));
    if (bt->group.traversal) kind = bt->group.traversal - 1;   // every job's scene allows it (checked at submit)
    ta.kind = kind;
    {
        TimerScope tsc(timer, st, 0, -1);
        e = pt::launch_trace_multi(dtab, njobs, ta, kind, st);
    }
    if (e != hipSuccess) return e;
    TimerScope tsc(timer, st, 2, -1);
    return pt::launch_shade_multi(dtab, njobs, blocks, ts, reuse, st);
}

pt_status pt_batch_step(pt_batch bt, void* stream, int* active) {
    if (!bt) return fail(PT_EINVAL, "null batch");
    hipStream_t st = (hipStream_t)stream;
    std::vector<int> ids, bs, ss;
    for (int i = 0; i < bt->max_jobs; ++i) {
        BatchJob& J = bt->jobs[i];
        if (J.used && !J.finished) {
            ids.push_back(i);
            bs.push_back(J.b);
            ss.push_back(J.s);
        }
    }
    if (active) *active = (int)ids.size();
    if (ids.empty()) return PT_OK;
    const int slot = (int)(bt->steps % kBatchRing);
    if (bt->ring_used[slot]) {
        hipError_t e = hipEventSynchronize(bt->ring_ev[slot]);   // the table slot is free again
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    }
    std::vector<pt::StepJob>& tab = bt->host_tables[slot];
    uint32_t blocks = 0, rays = 0;
    bool reuse = false;
    const int n = batch_fill_table(bt, ids, tab, bs, ss, &blocks, &rays, &reuse);
    pt::StepJob* dtab = (pt::StepJob*)(bt->arena + bt->table_off + (size_t)slot * bt->table_stride);
    hipError_t e = hipMemcpyAsync(dtab, tab.data(), (size_t)n * sizeof(pt::StepJob), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (launch table)");
    uint32_t* counter = (uint32_t*)(bt->arena + bt->counter_off) + (size_t)slot * pt::kWorkWords;
    e = batch_launch_step(bt, dtab, n, blocks, rays, reuse, counter, nullptr, st);
    if (e != hipSuccess) return hip_fail(e, "launch (batch step)");
    e = hipEventRecord(bt->ring_ev[slot], st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    bt->ring_used[slot] = true;
    ++bt->steps;
    for (int id : ids) {
        BatchJob& J = bt->jobs[id];
        if (++J.b > J.f.B) {
            J.b = 0;
            if (++J.s == J.f.spp) {
                J.finished = true;
                e = hipEventRecord(J.done_ev, st);
                if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
            }
        }
    }
    return PT_OK;
}

pt_status pt_batch_poll(pt_batch bt, uint32_t id, int* done) {
    if (!bt || !done || id >= (uint32_t)bt->max_jobs || !bt->jobs[id].used) return fail(PT_EINVAL, "bad job id");
    BatchJob& J = bt->jobs[id];
    *done = 0;
    if (!J.finished) return PT_OK;
    hipError_t e = hipEventQuery(J.done_ev);
    if (e == hipSuccess) *done = 1;
    else if (e != hipErrorNotReady) return hip_fail(e, "hipEventQuery");
    return PT_OK;
}

pt_status pt_batch_release(pt_batch bt, uint32_t id) {
    if (!bt || id >= (uint32_t)bt->max_jobs || !bt->jobs[id].used) return fail(PT_EINVAL, "bad job id");
    int done = 0;
    pt_status st = pt_batch_poll(bt, id, &done);
    if (st != PT_OK) return st;
    if (!done) return fail(PT_EBUSY, "job %u has not finished", id);
    BatchJob& J = bt->jobs[id];
    pool_free(bt, J.off, J.bytes);
    J.used = false;
    J.finished = false;
    batch_drop_graph(bt);
    return PT_OK;
}

pt_status pt_batch_run(pt_batch bt, int use_graph, pt_timer timer, void* stream) {
    if (!bt) return fail(PT_EINVAL, "null batch");
    hipStream_t st = (hipStream_t)stream;
    std::vector<int> ids;
    for (int i = 0; i < bt->max_jobs; ++i)
        if (bt->jobs[i].used) ids.push_back(i);
    if (ids.empty()) return PT_OK;
    // wait for steps still in flight that use the launch-table ring
    for (int i = 0; i < kBatchRing; ++i)
        if (bt->ring_used[i]) {
            hipError_t e = hipEventSynchronize(bt->ring_ev[i]);
            if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        }
    // the static schedule: step k traces bounce (k mod (B+1)) of sample k / (B+1) of each job
    // that has that many steps
    std::vector<uint32_t> key;
    for (int id : ids) {
        key.push_back((uint32_t)id);
        key.push_back((uint32_t)(bt->jobs[id].off >> 8));
    }
    int nsteps = 0;
    for (int id : ids) nsteps = std::max(nsteps, bt->jobs[id].f.spp * (bt->jobs[id].f.B + 1));
    const bool rebuild = key != bt->graph_key || !bt->sched_bytes;
    std::vector<std::vector<pt::StepJob>> tabs(nsteps);
    std::vector<uint32_t> tblocks(nsteps), trays(nsteps);
    std::vector<char> treuse(nsteps);
    for (int k = 0; k < nsteps; ++k) {
        std::vector<int> sid, bs, ss;
        for (int id : ids) {
            const BatchJob& J = bt->jobs[id];
            if (k < J.f.spp * (J.f.B + 1)) {
                sid.push_back(id);
                bs.push_back(k % (J.f.B + 1));
                ss.push_back(k / (J.f.B + 1));
            }
        }
        bool r = false;
        batch_fill_table(bt, sid, tabs[k], bs, ss, &tblocks[k], &trays[k], &r);
        treuse[k] = r;
    }
    if (rebuild) {
        batch_drop_graph(bt);
        size_t need = 0;
        for (int k = 0; k < nsteps; ++k) need += align256(tabs[k].size() * sizeof(pt::StepJob));
        need += align256((size_t)nsteps * pt::kWorkWords * 4);
        size_t off = 0;
        if (!pool_alloc(bt, need, &off)) return fail(PT_ENOMEM, "arena has no room for the schedule (%zu bytes)", need);
        bt->sched_off = off;
        bt->sched_bytes = need;
        size_t o = off;
        for (int k = 0; k < nsteps; ++k) {
            hipError_t e = hipMemcpyAsync(bt->arena + o, tabs[k].data(), tabs[k].size() * sizeof(pt::StepJob),
                                          hipMemcpyHostToDevice, st);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (schedule)");
            o += align256(tabs[k].size() * sizeof(pt::StepJob));
        }
        hipError_t e = hipStreamSynchronize(st);   // host tables go out of scope
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        bt->graph_key = key;
    }
    auto enqueue = [&](pt_timer tm) -> hipError_t {
        size_t o = bt->sched_off;
        uint32_t* counters =
            (uint32_t*)(bt->arena + bt->sched_off + bt->sched_bytes - align256((size_t)nsteps * pt::kWorkWords * 4));
        for (int k = 0; k < nsteps; ++k) {
            const pt::StepJob* dtab = (const pt::StepJob*)(bt->arena + o);
            hipError_t e = batch_launch_step(bt, dtab, (int)tabs[k].size(), tblocks[k], trays[k], treuse[k] != 0,
                                             counters + (size_t)k * pt::kWorkWords, tm, st);
            if (e != hipSuccess) return e;
            o += align256(tabs[k].size() * sizeof(pt::StepJob));
        }
        return hipSuccess;
    };
    hipError_t e;
    if (use_graph) {
        if (!bt->gexec) {
            // capture on the batch's own stream: the caller's stream may be the null stream
            hipStream_t user = st;
            st = bt->gstream;
            e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
            hipError_t le = enqueue(nullptr);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(st, &g);
            st = user;
            if (le != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return hip_fail(le, "launch (batch capture)");
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            bt->graph = g;
            e = hipGraphInstantiate(&bt->gexec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                bt->graph = nullptr;
                bt->gexec = nullptr;
                return hip_fail(e, "hipGraphInstantiate");
            }
        }
        // order the replay after the caller's earlier work and the caller's later work after it
        e = hipEventRecord(bt->gev_in, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(bt->gstream, bt->gev_in, 0);
        if (e == hipSuccess) e = hipGraphLaunch(bt->gexec, bt->gstream);
        if (e == hipSuccess) e = hipEventRecord(bt->gev_out, bt->gstream);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, bt->gev_out, 0);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    } else {
        e = enqueue(timer);
        if (e != hipSuccess) return hip_fail(e, "launch (batch run)");
    }
    for (int id : ids) {
        BatchJob& J = bt->jobs[id];
        J.finished = true;
        J.s = J.f.spp;
        J.b = 0;
        e = hipEventRecord(J.done_ev, st);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    return PT_OK;
}

pt_status pt_batch_free(pt_batch bt) {
    if (!bt) return PT_OK;
    for (int i = 0; i < kBatchRing; ++i)
        if (bt->ring_ev[i]) {
            if (bt->ring_used[i]) (void)hipEventSynchronize(bt->ring_ev[i]);
            (void)hipEventDestroy(bt->ring_ev[i]);
        }
    for (auto& j : bt->jobs)
        if (j.done_ev) {
            if (j.finished) (void)hipEventSynchronize(j.done_ev);
            (void)hipEventDestroy(j.done_ev);
        }
    if (bt->gexec) (void)hipGraphExecDestroy(bt->gexec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    if (bt->gstream) {
        (void)hipStreamSynchronize(bt->gstream);
        (void)hipStreamDestroy(bt->gstream);
    }
    if (bt->gev_in) (void)hipEventDestroy(bt->gev_in);
    if (bt->gev_out) (void)hipEventDestroy(bt->gev_out);
    delete bt;
    return PT_OK;
}

}  // extern "C"
