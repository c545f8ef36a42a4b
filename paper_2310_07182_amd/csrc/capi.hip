// C-ABI entry points of libpt: argument checks, scene build and upload, the
// frame loop (raygen -> [key -> sort -> gather] -> trace -> shade per bounce),
// workspace layout and HIP-event timing.  No entry point allocates device
// memory: the caller passes the scene arena, the workspace and the outputs.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
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
    uint32_t ntri = 0, nmat = 0;
    float env[3] = {0, 0, 0};
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    size_t off_nodes = 0, off_btris = 0, off_otris = 0, off_mat = 0, off_mats = 0, bytes = 0;
    bool uploaded = false;
    int device = -1;
    DevScene dev{};
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

constexpr int kDefaultRefill = 32;

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
    f.reuse_max = g.reuse_max_bounce;
    super_tile(f.W, f.H, f.SW, f.SH, f.cols);
    f.TS = f.SW * f.SH;
    f.nstx = (w + f.SW - 1) / f.SW;
    f.nsty = (h + f.SH - 1) / f.SH;
    f.ntx = (w + f.W - 1) / f.W;
    f.nslots = (uint32_t)f.nstx * (uint32_t)f.nsty * (uint32_t)f.TS;
    f.seed = seed;
    return f;
}

struct Layout {
    size_t q0, q1, state, work, partial, keys, vals, qs, sortws, ovf, total;
};

Layout layout(const Frame& f) {
    Layout L{};
    size_t o = 0;
    const size_t qb = (size_t)f.nslots * 32;
    const size_t launches = (size_t)(f.B + 1) * (size_t)f.spp;
    L.q0 = o;
    o = align256(o + qb);
    L.q1 = o;
    o = align256(o + qb);
    L.state = o;
    o = align256(o + qb);
    L.work = o;
    o = align256(o + launches * 4);
    L.partial = o;
    o = align256(o + launches * pt::kMaxTraceBlocks * 4);
    if (f.mode == PT_MODE_SORTED) {
        L.keys = o;
        o = align256(o + (size_t)f.nslots * 4);
        L.vals = o;
        o = align256(o + (size_t)f.nslots * 4);
        L.qs = o;
        o = align256(o + qb);
        L.sortws = o;
        o = align256(o + pt::sort_workspace_bytes(f.nslots));
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
        for (int a = 0; a < 3; ++a) s->env[a] = d->env_radiance[a];
        size_t o = 0;
        s->off_nodes = o;
        o = align256(o + s->bvh.nodes.size() * sizeof(pt::BvhNode));
        s->off_btris = o;
        o = align256(o + s->btris.size() * sizeof(float4));
        s->off_otris = o;
        o = align256(o + s->otris.size() * sizeof(float4));
        s->off_mat = o;
        o = align256(o + s->tri_mat.size() * 4);
        s->off_mats = o;
        o = align256(o + s->mats.size() * sizeof(pt_material));
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
        {s->off_btris, s->btris.data(), s->btris.size() * sizeof(float4)},
        {s->off_otris, s->otris.data(), s->otris.size() * sizeof(float4)},
        {s->off_mat, s->tri_mat.data(), s->tri_mat.size() * 4},
        {s->off_mats, s->mats.data(), s->mats.size() * sizeof(pt_material)},
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
    d.btris = (const float4*)(base + s->off_btris);
    d.otris = (const float4*)(base + s->off_otris);
    d.tri_mat = (const uint32_t*)(base + s->off_mat);
    d.mats = (const pt_material*)(base + s->off_mats);
    d.ntri = s->ntri;
    d.nmat = s->nmat;
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
    return PT_OK;
}

pt_status pt_scene_export_bvh(pt_scene s, void* nodes, uint32_t* order) {
    if (!s) return fail(PT_EINVAL, "null scene");
    if (nodes) memcpy(nodes, s->bvh.nodes.data(), s->bvh.nodes.size() * sizeof(pt::BvhNode));
    if (order && !s->bvh.order.empty()) memcpy(order, s->bvh.order.data(), s->bvh.order.size() * sizeof(uint32_t));
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
    if (mode != PT_MODE_INCOHERENT && mode != PT_MODE_SORTED && mode != PT_MODE_REUSE)
        return fail(PT_EINVAL, "unknown mode %d", (int)mode);
    pt_status cs = check_group(g, B);
    if (cs != PT_OK) return cs;
    if (!out->radiance || !out->hit_prim || !out->hit_t) return fail(PT_EINVAL, "radiance, hit_prim and hit_t are required");
    if (!workspace) return fail(PT_EINVAL, "null workspace");
    int dev = 0;
    hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess) return hip_fail(ge, "hipGetDevice");
    if (dev != scene->device) return fail(PT_EINVAL, "scene was uploaded on device %d, current device is %d", scene->device, dev);

    Frame f = make_frame(w, h, spp, B, mode, g, seed);
    if (mode == PT_MODE_SORTED && f.nslots > (1u << 27)) return fail(PT_EINVAL, "sorted mode supports at most 2^27 rays per bounce");
    const Layout L = layout(f);
    if (ws_bytes < L.total) return fail(PT_ENOMEM, "workspace too small: %zu < %zu", ws_bytes, L.total);
    {
        // camera basis (host side of the arithmetic contract)
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
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)workspace;
    float4* q[2] = {(float4*)(ws + L.q0), (float4*)(ws + L.q1)};
    float4* state = (float4*)(ws + L.state);
    uint32_t* partial = (uint32_t*)(ws + L.partial);
    uint32_t* work = (uint32_t*)(ws + L.work);
    int32_t* ovf = (int32_t*)(ws + L.ovf);
    const size_t launches = (size_t)(B + 1) * (size_t)spp;
    hipError_t e;
    {
        TimerScope ts(out->timer, st, 6, -1);
        e = pt::launch_zero(work, launches, st);
        if (e == hipSuccess && out->stats) e = pt::launch_zero((uint32_t*)out->stats, (size_t)(B + 1) * 4, st);
    }
    if (e != hipSuccess) return hip_fail(e, "launch (zero)");
    const int grid = pt::trace_grid_blocks();
    const size_t plane = (size_t)w * (size_t)h;
    for (int s = 0; s < spp; ++s) {
        {
            TimerScope ts(out->timer, st, 1, 0);
            e = pt::launch_raygen(f, s, q[0], state, (float4*)out->rays, st);
        }
        if (e != hipSuccess) return hip_fail(e, "launch (raygen)");
        for (int b = 0; b <= B; ++b) {
            const size_t li = (size_t)b * spp + s;
            const float4* tq = q[b & 1];
            const uint32_t n = f.nslots;
            if (mode == PT_MODE_SORTED && b >= 1) {
                uint32_t* keys = (uint32_t*)(ws + L.keys);
                uint32_t* vals = (uint32_t*)(ws + L.vals);
                float4* qs = (float4*)(ws + L.qs);
                {
                    TimerScope ts(out->timer, st, 3, b);
                    e = pt::launch_keys(scene->dev, q[b & 1], f.nslots, keys, vals, st);
                }
                if (e != hipSuccess) return hip_fail(e, "launch (keys)");
                {
                    TimerScope ts(out->timer, st, 4, b);
                    e = pt::radix_sort_pairs(keys, vals, f.nslots, ws + L.sortws, st);
                }
                if (e != hipSuccess) return hip_fail(e, "launch (sort)");
                {
                    TimerScope ts(out->timer, st, 5, b);
                    e = pt::launch_gather(q[b & 1], vals, f.nslots, qs, st);
                }
                if (e != hipSuccess) return hip_fail(e, "launch (gather)");
                tq = qs;   // dead rays (key 0xFFFFFFFF) sort last and are skipped by the trace
            }
            pt::TraceArgs ta{};
            ta.rays = tq;
            ta.n = n;
            ta.work = work + li;
            ta.out_prim = out->hit_prim + li * plane;
            ta.out_t = out->hit_t + li * plane;
            ta.partial = out->ray_count ? partial + li * pt::kMaxTraceBlocks : nullptr;
            ta.stats = out->stats ? (unsigned long long*)(out->stats + 2 * (size_t)b) : nullptr;
            ta.ovf = ovf;
            ta.by_pixel = 1;
            ta.refill = g.refill ? g.refill : kDefaultRefill;
            {
                TimerScope ts(out->timer, st, 0, b);
                e = pt::launch_trace(scene->dev, ta, out->stats != nullptr, st);
            }
            if (e != hipSuccess) return hip_fail(e, "launch (trace)");
            {
                TimerScope ts(out->timer, st, 2, b);
                e = pt::launch_shade(scene->dev, f, b, s, q[b & 1], q[(b + 1) & 1], state, out->hit_prim, out->hit_t,
                                     out->radiance, (float4*)out->rays, st);
            }
            if (e != hipSuccess) return hip_fail(e, "launch (shade)");
        }
    }
    if (out->ray_count) {
        TimerScope ts(out->timer, st, 6, -1);
        e = pt::launch_count_finalize(partial, pt::kMaxTraceBlocks, grid, (int)launches, out->ray_count, st);
        if (e != hipSuccess) return hip_fail(e, "launch (count)");
    }
    return PT_OK;
}

size_t pt_trace_workspace_bytes(void) {
    return 256 + align256((size_t)pt::kMaxTraceBlocks * pt::kTraceBlock * pt::kStackOvf * 4);
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
    ta.ovf = (int32_t*)((char*)workspace + 256);
    ta.by_pixel = 0;
    ta.refill = refill ? refill : kDefaultRefill;
    hipError_t e = pt::launch_zero(ta.work, 1, st);
    if (e != hipSuccess) return hip_fail(e, "launch (zero)");
    e = pt::launch_trace(scene->dev, ta, false, st);
    if (e != hipSuccess) return hip_fail(e, "launch (trace)");
    return PT_OK;
}

pt_status pt_ray_keys(pt_scene scene, const float* rays, uint32_t n, uint32_t* keys, void* stream) {
    if (!scene || (n > 0 && (!rays || !keys))) return fail(PT_EINVAL, "null argument");
    if (!scene->uploaded) return fail(PT_EINVAL, "scene not uploaded");
    if (n == 0) return PT_OK;
    hipError_t e = pt::launch_keys(scene->dev, (const float4*)rays, n, keys, nullptr, (hipStream_t)stream);
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

}  // extern "C"
