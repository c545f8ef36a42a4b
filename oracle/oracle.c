/*
 * CPU oracle for "Generate Coherent Rays Directly" (Liu et al., EG 2024).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the GPU library.  It shares no code,
 * header, table or constant with the GPU library; both are written from the
 * same arithmetic contract (IEEE binary32, round to nearest even, no fused
 * multiply-add, correctly rounded division and square root, explicit operation
 * order in every expression below).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared.
 *
 * What is pinned and how is listed per function; a function with no external
 * pin would say "parity unpinned" here (none does).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#if defined(__FAST_MATH__)
#error "the oracle must be built without fast-math"
#endif

typedef struct { float x, y, z; } v3;

static v3 mk(float x, float y, float z) { v3 r; r.x = x; r.y = y; r.z = z; return r; }
static v3 vadd(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 vsub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 vscale(v3 a, float s) { return mk(a.x * s, a.y * s, a.z * s); }
static v3 vneg(v3 a) { return mk(-a.x, -a.y, -a.z); }
static float vdot(v3 a, v3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
static v3 vcross(v3 a, v3 b)
{
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static v3 vnormalize(v3 v)
{
    float inv = 1.0f / sqrtf(vdot(v, v));
    return vscale(v, inv);
}
static float comp(v3 v, int i) { return i == 0 ? v.x : (i == 1 ? v.y : v.z); }
static v3 load3(const float* p) { return mk(p[0], p[1], p[2]); }
static void store3(float* p, v3 v) { p[0] = v.x; p[1] = v.y; p[2] = v.z; }

static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* ------------------------------------------------------------------------
 * Counter-based RNG: Philox4x64-10 (Salmon et al., SC'11).
 * Pin: numpy.random.Philox (the same generator) in the test suite.
 * ---------------------------------------------------------------------- */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        unsigned __int128 p0 = (unsigned __int128)M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ x1 ^ k0, n1 = lo1, n2 = hi0 ^ x3 ^ k1, n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* draw for (index, sample, bounce, stream); stream 0 = pixel, 1 = tile */
static void draw(uint64_t seed, uint64_t index, int sample, int bounce, int stream, uint64_t out[4])
{
    uint64_t ctr[4] = {index, (uint64_t)sample, (uint64_t)bounce, (uint64_t)stream};
    uint64_t key[2] = {seed, 0};
    orc_philox4x64_10(ctr, key, out);
}

/* top 24 bits -> [0, 1 - 2^-24], exact in binary32 */
static float u01(uint64_t x) { return (float)(uint32_t)(x >> 40) * 0x1p-24f; }

/* ------------------------------------------------------------------------
 * sin and cos of 2*pi*u, u in [0,1): exact octant reduction of 8u, then the
 * Taylor series of sin (degree 9) and cos (degree 10) on [0, pi/4].
 * Pin: exhaustive comparison with float64 sin/cos over all 2^24 grid inputs.
 * ---------------------------------------------------------------------- */
static void sincos2pi(float u, float* sn, float* cs)
{
    const float PI_4 = (float)(3.14159265358979323846 / 4.0);
    const float S3 = (float)(-1.0 / 6.0), S5 = (float)(1.0 / 120.0);
    const float S7 = (float)(-1.0 / 5040.0), S9 = (float)(1.0 / 362880.0);
    const float C2 = -0.5f, C4 = (float)(1.0 / 24.0), C6 = (float)(-1.0 / 720.0);
    const float C8 = (float)(1.0 / 40320.0), C10 = (float)(-1.0 / 3628800.0);
    float v = u * 8.0f;
    int o = (int)v;
    float f = v - (float)o;
    float g = (o & 1) ? 1.0f - f : f;
    float th = g * PI_4;
    float t2 = th * th;
    float s = th + (th * t2) * (S3 + t2 * (S5 + t2 * (S7 + t2 * S9)));
    float c = 1.0f + t2 * (C2 + t2 * (C4 + t2 * (C6 + t2 * (C8 + t2 * C10))));
    switch (o & 7) {
    case 0: *sn = s;  *cs = c;  break;
    case 1: *sn = c;  *cs = s;  break;
    case 2: *sn = c;  *cs = -s; break;
    case 3: *sn = s;  *cs = -c; break;
    case 4: *sn = -s; *cs = -c; break;
    case 5: *sn = -c; *cs = -s; break;
    case 6: *sn = -c; *cs = s;  break;
    default: *sn = -s; *cs = c; break;
    }
}

void orc_sincos2pi(const float* u, uint32_t n, float* s, float* c)
{
    for (uint32_t i = 0; i < n; ++i) sincos2pi(u[i], &s[i], &c[i]);
}

/* ------------------------------------------------------------------------
 * Pinhole camera (a path starts at a pixel, Section 3.1).
 * Pin: rays hit the pixel's own screen position (test), furnace closed form.
 * ---------------------------------------------------------------------- */
typedef struct { v3 pos, fwd, right, up; float th, thx; } cam_basis;

static cam_basis camera_basis(const orc_camera* c, int w, int h)
{
    cam_basis b;
    b.pos = load3(c->pos);
    b.fwd = vnormalize(vsub(load3(c->look_at), b.pos));
    b.right = vnormalize(vcross(b.fwd, load3(c->up)));
    b.up = vcross(b.right, b.fwd);
    b.th = (float)tan((double)c->vfov_deg * (3.14159265358979323846 / 360.0));
    b.thx = b.th * ((float)w / (float)h);
    return b;
}

static void camera_ray(const cam_basis* cb, int w, int h, int x, int y, float u0, float u1, v3* o, v3* d)
{
    float px = ((float)x + u0) / (float)w;
    float py = ((float)y + u1) / (float)h;
    float fx = (2.0f * px - 1.0f) * cb->thx;
    float fy = (1.0f - 2.0f * py) * cb->th;
    v3 dir = mk((fx * cb->right.x + fy * cb->up.x) + cb->fwd.x,
                (fx * cb->right.y + fy * cb->up.y) + cb->fwd.y,
                (fx * cb->right.z + fy * cb->up.z) + cb->fwd.z);
    *o = cb->pos;
    *d = vnormalize(dir);
}

void orc_camera_ray(const orc_camera* cam, int w, int h, int x, int y, float u0, float u1,
                    float o[3], float d[3])
{
    cam_basis cb = camera_basis(cam, w, h);
    v3 oo, dd;
    camera_ray(&cb, w, h, x, y, u0, u1, &oo, &dd);
    store3(o, oo);
    store3(d, dd);
}

/* ------------------------------------------------------------------------
 * Watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013), two-sided.
 * Pin: float64 brute force (numpy), interior rays of closed meshes never miss,
 * exact t on axis-aligned quads.
 * ---------------------------------------------------------------------- */
typedef struct { v3 o; int kx, ky, kz; float Sx, Sy, Sz; } ray_pre;

static ray_pre ray_prepare(v3 o, v3 d)
{
    ray_pre r;
    r.o = o;
    float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    int kz = 0;
    float m = ax;
    if (ay > m) { kz = 1; m = ay; }
    if (az > m) { kz = 2; }
    int kx = kz + 1; if (kx == 3) kx = 0;
    int ky = kx + 1; if (ky == 3) ky = 0;
    if (comp(d, kz) < 0.0f) { int tmp = kx; kx = ky; ky = tmp; }
    r.kx = kx; r.ky = ky; r.kz = kz;
    r.Sx = comp(d, kx) / comp(d, kz);
    r.Sy = comp(d, ky) / comp(d, kz);
    r.Sz = 1.0f / comp(d, kz);
    return r;
}

/* returns 1 and *t on a hit with 0 < t < +inf */
static int tri_hit(const ray_pre* r, const float* v, float* t_out)
{
    v3 A = vsub(load3(v), r->o), B = vsub(load3(v + 3), r->o), C = vsub(load3(v + 6), r->o);
    float Ax = comp(A, r->kx) - r->Sx * comp(A, r->kz);
    float Ay = comp(A, r->ky) - r->Sy * comp(A, r->kz);
    float Bx = comp(B, r->kx) - r->Sx * comp(B, r->kz);
    float By = comp(B, r->ky) - r->Sy * comp(B, r->kz);
    float Cx = comp(C, r->kx) - r->Sx * comp(C, r->kz);
    float Cy = comp(C, r->ky) - r->Sy * comp(C, r->kz);
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return 0;
    float det = (U + V) + W;
    if (det == 0.0f) return 0;
    float Az = r->Sz * comp(A, r->kz);
    float Bz = r->Sz * comp(B, r->kz);
    float Cz = r->Sz * comp(C, r->kz);
    float T = (U * Az + V * Bz) + W * Cz;
    float t = T / det;
    if (!(t > 0.0f) || !(t < INFINITY)) return 0;
    *t_out = t;
    return 1;
}

/* (t, prim) lexicographic order */
static int better(float t, int32_t p, float bt, int32_t bp) { return t < bt || (t == bt && p < bp); }

/* ------------------------------------------------------------------------
 * Scene and the oracle's own BVH (binned surface-area heuristic over 16
 * centroid bins, leaves of at most 4 triangles, object-median fallback when
 * all centroids coincide).  The BVH only prunes: the closest hit is the
 * (t, prim) minimum over all triangles.  Boxes are padded by 1e-5 of the scene
 * extent and tested in float64, so pruning never drops a hit of the float32
 * test.  Pin: brute force over all triangles (orc_trace_brute) and float64
 * brute force in numpy.
 * ---------------------------------------------------------------------- */
typedef struct { float lo[3], hi[3]; int32_t a; int32_t count; } onode; /* leaf: count>0, a=first */

struct orc_scene {
    float* tris;          /* [ntri][9] original order */
    uint32_t ntri;
    uint32_t* tri_mat;
    orc_material* mats;
    uint32_t nmat;
    float env[3];
    float lo[3], hi[3];
    onode* nodes;
    uint32_t nnodes;
    uint32_t* order;      /* leaf slots -> original prim */
    double pad;
    uint32_t* emit;       /* emissive triangles (any emission channel > 0), original order */
    uint32_t nemit;
};

static float* g_cent;  /* build scratch: centroids (the oracle is single-threaded) */
static float* g_tlo;   /* per-triangle bounds */
static float* g_thi;

static void swap_u32(uint32_t* a, uint32_t* b) { uint32_t t = *a; *a = *b; *b = t; }

/* quickselect on centroid axis, ties ordered by prim id: k-th smallest at k */
static void select_kth(uint32_t* idx, int64_t lo, int64_t hi, int64_t k, int axis)
{
    while (hi > lo) {
        int64_t mid = lo + (hi - lo) / 2;
        float pv = g_cent[(size_t)idx[mid] * 3 + axis];
        uint32_t pid = idx[mid];
        int64_t i = lo, j = hi;
        while (i <= j) {
            for (;;) {
                float c = g_cent[(size_t)idx[i] * 3 + axis];
                if (c < pv || (c == pv && idx[i] < pid)) ++i; else break;
            }
            for (;;) {
                float c = g_cent[(size_t)idx[j] * 3 + axis];
                if (c > pv || (c == pv && idx[j] > pid)) --j; else break;
            }
            if (i <= j) { swap_u32(&idx[i], &idx[j]); ++i; --j; }
        }
        if (k <= j) hi = j;
        else if (k >= i) lo = i;
        else return;
    }
}

static double half_area(const float lo[3], const float hi[3])
{
    double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
    if (dx < 0 || dy < 0 || dz < 0) return 0.0;
    return dx * dy + dy * dz + dz * dx;
}

static void grow(float lo[3], float hi[3], const float* plo, const float* phi)
{
    for (int a = 0; a < 3; ++a) {
        if (plo[a] < lo[a]) lo[a] = plo[a];
        if (phi[a] > hi[a]) hi[a] = phi[a];
    }
}

#define NBINS 16
static void build_rec(orc_scene* s, uint32_t node, int64_t first, int64_t n)
{
    onode* nd = &s->nodes[node];
    uint32_t* idx = s->order + first;
    for (int a = 0; a < 3; ++a) { nd->lo[a] = INFINITY; nd->hi[a] = -INFINITY; }
    float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; ++i) {
        grow(nd->lo, nd->hi, g_tlo + (size_t)idx[i] * 3, g_thi + (size_t)idx[i] * 3);
        const float* c = g_cent + (size_t)idx[i] * 3;
        grow(clo, chi, c, c);
    }
    if (n <= 4) { nd->a = (int32_t)first; nd->count = (int32_t)n; return; }
    int best_axis = -1, best_split = 0;
    double best_cost = INFINITY;
    for (int a = 0; a < 3; ++a) {
        double ext = (double)chi[a] - clo[a];
        if (!(ext > 0.0)) continue;
        float blo[NBINS][3], bhi[NBINS][3];
        int64_t cnt[NBINS];
        for (int b = 0; b < NBINS; ++b) {
            cnt[b] = 0;
            for (int k = 0; k < 3; ++k) { blo[b][k] = INFINITY; bhi[b][k] = -INFINITY; }
        }
        double scale = NBINS / ext;
        for (int64_t i = 0; i < n; ++i) {
            int b = (int)(((double)g_cent[(size_t)idx[i] * 3 + a] - clo[a]) * scale);
            if (b >= NBINS) b = NBINS - 1;
            if (b < 0) b = 0;
            ++cnt[b];
            grow(blo[b], bhi[b], g_tlo + (size_t)idx[i] * 3, g_thi + (size_t)idx[i] * 3);
        }
        double rarea[NBINS];
        int64_t rcnt[NBINS];
        float rlo[3] = {INFINITY, INFINITY, INFINITY}, rhi[3] = {-INFINITY, -INFINITY, -INFINITY};
        int64_t rc = 0;
        for (int b = NBINS - 1; b > 0; --b) {
            grow(rlo, rhi, blo[b], bhi[b]);
            rc += cnt[b];
            rarea[b] = half_area(rlo, rhi);
            rcnt[b] = rc;
        }
        float llo[3] = {INFINITY, INFINITY, INFINITY}, lhi[3] = {-INFINITY, -INFINITY, -INFINITY};
        int64_t lc = 0;
        for (int b = 0; b < NBINS - 1; ++b) {
            grow(llo, lhi, blo[b], bhi[b]);
            lc += cnt[b];
            if (lc == 0 || rcnt[b + 1] == 0) continue;
            double cost = half_area(llo, lhi) * (double)lc + rarea[b + 1] * (double)rcnt[b + 1];
            if (cost < best_cost) { best_cost = cost; best_axis = a; best_split = b + 1; }
        }
    }
    int64_t half;
    if (best_axis < 0) {
        half = n / 2;   /* all centroids coincide: object median by prim id */
        select_kth(idx, 0, n - 1, half, 0);
    } else {
        double ext = (double)chi[best_axis] - clo[best_axis];
        double scale = NBINS / ext;
        int64_t i = 0, j = n - 1;
        while (i <= j) {
            int b = (int)(((double)g_cent[(size_t)idx[i] * 3 + best_axis] - clo[best_axis]) * scale);
            if (b >= NBINS) b = NBINS - 1;
            if (b < best_split) ++i;
            else { swap_u32(&idx[i], &idx[j]); --j; }
        }
        half = i;
        if (half == 0 || half == n) { half = n / 2; select_kth(idx, 0, n - 1, half, best_axis); }
    }
    uint32_t left = s->nnodes;
    s->nnodes += 2;
    nd = &s->nodes[node];
    nd->a = (int32_t)left;
    nd->count = 0;
    build_rec(s, left, first, half);
    build_rec(s, left + 1, first + half, n - half);
}

orc_scene* orc_scene_create(const float* tris, uint32_t ntri, const uint32_t* tri_mat,
                            const orc_material* mats, uint32_t nmat, const float env[3])
{
    orc_scene* s = (orc_scene*)calloc(1, sizeof(orc_scene));
    if (!s) return NULL;
    s->ntri = ntri;
    s->nmat = nmat;
    s->tris = (float*)malloc((size_t)ntri * 9 * sizeof(float) + 4);
    s->tri_mat = (uint32_t*)malloc((size_t)ntri * sizeof(uint32_t) + 4);
    s->mats = (orc_material*)malloc((size_t)nmat * sizeof(orc_material) + 4);
    s->order = (uint32_t*)malloc((size_t)ntri * sizeof(uint32_t) + 4);
    s->nodes = (onode*)malloc((size_t)(2 * ntri + 1) * sizeof(onode));
    g_cent = (float*)malloc((size_t)ntri * 3 * sizeof(float) + 4);
    g_tlo = (float*)malloc((size_t)ntri * 3 * sizeof(float) + 4);
    g_thi = (float*)malloc((size_t)ntri * 3 * sizeof(float) + 4);
    if (!s->tris || !s->tri_mat || !s->mats || !s->order || !s->nodes || !g_cent || !g_tlo || !g_thi) {
        orc_scene_free(s);
        free(g_cent); free(g_tlo); free(g_thi);
        g_cent = g_tlo = g_thi = NULL;
        return NULL;
    }
    memcpy(s->tris, tris, (size_t)ntri * 9 * sizeof(float));
    memcpy(s->tri_mat, tri_mat, (size_t)ntri * sizeof(uint32_t));
    memcpy(s->mats, mats, (size_t)nmat * sizeof(orc_material));
    s->emit = (uint32_t*)malloc((size_t)ntri * sizeof(uint32_t) + 4);
    if (!s->emit) { orc_scene_free(s); free(g_cent); free(g_tlo); free(g_thi); g_cent = g_tlo = g_thi = NULL; return NULL; }
    for (uint32_t i = 0; i < ntri; ++i) {
        const float* e = mats[tri_mat[i]].emission;
        if (e[0] > 0.0f || e[1] > 0.0f || e[2] > 0.0f) s->emit[s->nemit++] = i;
    }
    for (int a = 0; a < 3; ++a) { s->env[a] = env[a]; s->lo[a] = INFINITY; s->hi[a] = -INFINITY; }
    for (uint32_t i = 0; i < ntri; ++i) {
        s->order[i] = i;
        for (int a = 0; a < 3; ++a) {
            float v0 = tris[(size_t)i * 9 + a], v1 = tris[(size_t)i * 9 + 3 + a], v2 = tris[(size_t)i * 9 + 6 + a];
            g_cent[(size_t)i * 3 + a] = (float)(((double)v0 + (double)v1 + (double)v2) / 3.0);
            float mn = v0 < v1 ? v0 : v1; mn = mn < v2 ? mn : v2;
            float mx = v0 > v1 ? v0 : v1; mx = mx > v2 ? mx : v2;
            g_tlo[(size_t)i * 3 + a] = mn;
            g_thi[(size_t)i * 3 + a] = mx;
            if (mn < s->lo[a]) s->lo[a] = mn;
            if (mx > s->hi[a]) s->hi[a] = mx;
        }
    }
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) {
        double e = (double)s->hi[a] - (double)s->lo[a];
        if (e > ext) ext = e;
    }
    s->pad = 1e-5 * (ext > 0.0 ? ext : 1.0);
    s->nnodes = 1;
    if (ntri > 0) build_rec(s, 0, 0, ntri);
    else { s->nodes[0].count = 0; s->nodes[0].a = 0; }
    free(g_cent); free(g_tlo); free(g_thi);
    g_cent = g_tlo = g_thi = NULL;
    return s;
}

void orc_scene_free(orc_scene* s)
{
    if (!s) return;
    free(s->tris); free(s->tri_mat); free(s->mats); free(s->order); free(s->nodes); free(s->emit);
    free(s);
}

void orc_scene_bounds(const orc_scene* s, float lo[3], float hi[3])
{
    for (int a = 0; a < 3; ++a) { lo[a] = s->lo[a]; hi[a] = s->hi[a]; }
}

/* padded slab test in float64; returns 1 and the entry distance if the ray
 * segment [0, tcull] meets the padded box */
static int box_test(const orc_scene* s, const onode* nd, const double o[3], const double d[3],
                    double tcull, double* tnear_out)
{
    double tn = 0.0, tf = INFINITY;
    for (int a = 0; a < 3; ++a) {
        double lo = (double)nd->lo[a] - s->pad, hi = (double)nd->hi[a] + s->pad;
        if (d[a] == 0.0) {
            if (o[a] < lo || o[a] > hi) return 0;
            continue;
        }
        double t0 = (lo - o[a]) / d[a], t1 = (hi - o[a]) / d[a];
        if (t0 > t1) { double tmp = t0; t0 = t1; t1 = tmp; }
        if (t0 > tn) tn = t0;
        if (t1 < tf) tf = t1;
    }
    if (tn > tf || tn > tcull) return 0;
    *tnear_out = tn;
    return 1;
}

typedef struct { float t1; int32_t p1; float t2; int32_t p2; } hit2;

static void consider(hit2* h, float t, int32_t p)
{
    if (better(t, p, h->t1, h->p1)) {
        h->t2 = h->t1; h->p2 = h->p1;
        h->t1 = t; h->p1 = p;
    } else if (better(t, p, h->t2, h->p2)) {
        h->t2 = t; h->p2 = p;
    }
}

/* closest and second-closest distinct-prim hit; exclude = origin prim */
static hit2 trace_one(const orc_scene* s, v3 o, v3 d, int32_t exclude, uint64_t* nv, uint64_t* nt)
{
    hit2 h;
    h.t1 = INFINITY; h.p1 = INT32_MAX; h.t2 = INFINITY; h.p2 = INT32_MAX;
    if (s->ntri == 0) return h;
    ray_pre rp = ray_prepare(o, d);
    double od[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
    uint32_t stack[256];
    int sp = 0;
    double tn;
    if (!box_test(s, &s->nodes[0], od, dd, INFINITY, &tn)) return h;
    stack[sp++] = 0;
    while (sp > 0) {
        const onode* nd = &s->nodes[stack[--sp]];
        if (nv) ++*nv;
        if (nd->count > 0) {
            for (int i = 0; i < nd->count; ++i) {
                uint32_t prim = s->order[nd->a + i];
                if ((int32_t)prim == exclude) continue;
                if (nt) ++*nt;
                float t;
                if (tri_hit(&rp, s->tris + (size_t)prim * 9, &t)) consider(&h, t, (int32_t)prim);
            }
            continue;
        }
        double cull = (double)h.t2;
        double t0, t1;
        int h0 = box_test(s, &s->nodes[nd->a], od, dd, cull, &t0);
        int h1 = box_test(s, &s->nodes[nd->a + 1], od, dd, cull, &t1);
        if (h0 && h1) {
            if (t1 < t0) { stack[sp++] = (uint32_t)nd->a; stack[sp++] = (uint32_t)nd->a + 1; }
            else { stack[sp++] = (uint32_t)nd->a + 1; stack[sp++] = (uint32_t)nd->a; }
        } else if (h0) stack[sp++] = (uint32_t)nd->a;
        else if (h1) stack[sp++] = (uint32_t)nd->a + 1;
    }
    return h;
}

static void ray_unpack(const float* r, v3* o, v3* d, int32_t* excl)
{
    *o = mk(r[0], r[1], r[2]);
    int32_t e; memcpy(&e, &r[3], 4);
    *excl = e;
    *d = mk(r[4], r[5], r[6]);
}

void orc_trace(const orc_scene* s, const float* rays, uint32_t n, int32_t* prim, float* t,
               float* t2, uint64_t* node_visits, uint64_t* tri_tests)
{
    for (uint32_t i = 0; i < n; ++i) {
        v3 o, d; int32_t ex;
        ray_unpack(rays + (size_t)i * 8, &o, &d, &ex);
        hit2 h = trace_one(s, o, d, ex, node_visits, tri_tests);
        int miss = h.p1 == INT32_MAX;
        if (prim) prim[i] = miss ? -1 : h.p1;
        if (t) t[i] = miss ? INFINITY : h.t1;
        if (t2) t2[i] = h.p2 == INT32_MAX ? INFINITY : h.t2;
    }
}

void orc_trace_brute(const orc_scene* s, const float* rays, uint32_t n, int32_t* prim, float* t)
{
    for (uint32_t i = 0; i < n; ++i) {
        v3 o, d; int32_t ex;
        ray_unpack(rays + (size_t)i * 8, &o, &d, &ex);
        ray_pre rp = ray_prepare(o, d);
        float bt = INFINITY; int32_t bp = INT32_MAX;
        for (uint32_t j = 0; j < s->ntri; ++j) {
            if ((int32_t)j == ex) continue;
            float tt;
            if (tri_hit(&rp, s->tris + (size_t)j * 9, &tt) && better(tt, (int32_t)j, bt, bp)) { bt = tt; bp = (int32_t)j; }
        }
        prim[i] = bp == INT32_MAX ? -1 : bp;
        t[i] = bp == INT32_MAX ? INFINITY : bt;
    }
}

/* ------------------------------------------------------------------------
 * Shading-point frame.
 * Offset: Waechter & Binder, "A Fast and Robust Method for Avoiding
 * Self-Intersection" (Ray Tracing Gems, 2019).  Pin: the offset point lies on
 * the normal side of the plane and within a few ulp (test).
 * ONB: Duff et al., "Building an Orthonormal Basis, Revisited" (JCGT 2017),
 * applied to the face-forward geometric normal (tangent space of Section 3.2).
 * Pin: orthonormality and handedness (test).
 * ---------------------------------------------------------------------- */
static v3 offset_origin(v3 p, v3 n)
{
    const float origin = 1.0f / 32.0f, float_scale = 1.0f / 65536.0f, int_scale = 256.0f;
    int32_t ofx = (int32_t)(int_scale * n.x), ofy = (int32_t)(int_scale * n.y), ofz = (int32_t)(int_scale * n.z);
    float pix = u2f((uint32_t)((int32_t)f2u(p.x) + (p.x < 0.0f ? -ofx : ofx)));
    float piy = u2f((uint32_t)((int32_t)f2u(p.y) + (p.y < 0.0f ? -ofy : ofy)));
    float piz = u2f((uint32_t)((int32_t)f2u(p.z) + (p.z < 0.0f ? -ofz : ofz)));
    return mk(fabsf(p.x) < origin ? p.x + float_scale * n.x : pix,
              fabsf(p.y) < origin ? p.y + float_scale * n.y : piy,
              fabsf(p.z) < origin ? p.z + float_scale * n.z : piz);
}

void orc_offset_origin(const float p[3], const float n[3], float out[3])
{
    store3(out, offset_origin(load3(p), load3(n)));
}

static void onb(v3 n, v3* T, v3* B)
{
    float s = copysignf(1.0f, n.z);
    float a = -1.0f / (s + n.z);
    float b = (n.x * n.y) * a;
    *T = mk(1.0f + ((s * n.x) * n.x) * a, s * b, -(s * n.x));
    *B = mk(b, s + (n.y * n.y) * a, -n.y);
}

void orc_onb(const float n[3], float t[3], float b[3])
{
    v3 T, B;
    onb(load3(n), &T, &B);
    store3(t, T);
    store3(b, B);
}

static v3 to_world(v3 q, v3 T, v3 B, v3 n)
{
    return mk((q.x * T.x + q.y * B.x) + q.z * n.x,
              (q.x * T.y + q.y * B.y) + q.z * n.y,
              (q.x * T.z + q.y * B.z) + q.z * n.z);
}

/* ------------------------------------------------------------------------
 * BSDF sampling in tangent space (z = normal).
 * Lambert: cosine-weighted hemisphere (Malley); weight = albedo.
 *   Pin: E[z] = 2/3, E[z^2] = 1/2 and a histogram test (test suite).
 * GGX: Walter et al. 2007 normal sampling, Smith G, Schlick F.
 *   Pin: mean weight equals the quadrature of the reflectance integral.
 * Mirror: reflection about the normal; weight = albedo.
 *   Pin: the next ray of every mirror hit of a frame equals d - 2 (d.n) n in
 *   float64 world space; an open mirror floor returns albedo * L_env exactly.
 * ---------------------------------------------------------------------- */
static v3 sample_lambert(float u2, float u3)
{
    float r = sqrtf(u2);
    float sn, cs;
    sincos2pi(u3, &sn, &cs);
    float z2 = 1.0f - u2;
    return mk(r * cs, r * sn, sqrtf(z2 > 0.0f ? z2 : 0.0f));
}

void orc_sample_lambert(float u2, float u3, float q[3]) { store3(q, sample_lambert(u2, u3)); }

static float smith_g1(v3 v, float a2)
{
    float z2 = v.z * v.z;
    float num = 1.0f - z2;
    float tan2 = (num > 0.0f ? num : 0.0f) / z2;
    return 2.0f / (1.0f + sqrtf(1.0f + a2 * tan2));
}

static int sample_ggx(v3 wi, float alpha, const float f0[3], float u2, float u3, v3* wo, float w[3])
{
    if (!(wi.z > 0.0f)) return 0;
    float a2 = alpha * alpha;
    float tan2m = (a2 * u2) / (1.0f - u2);
    float cm = 1.0f / sqrtf(1.0f + tan2m);
    float sm2 = 1.0f - cm * cm;
    float sm = sqrtf(sm2 > 0.0f ? sm2 : 0.0f);
    float sn, cs;
    sincos2pi(u3, &sn, &cs);
    v3 m = mk(sm * cs, sm * sn, cm);
    float wim = vdot(wi, m);
    if (!(wim > 0.0f)) return 0;
    float k = 2.0f * wim;
    v3 o = mk(k * m.x - wi.x, k * m.y - wi.y, k * m.z - wi.z);
    if (!(o.z > 0.0f)) return 0;
    float g = ((smith_g1(wi, a2) * smith_g1(o, a2)) * wim) / (wi.z * cm);
    float c = 1.0f - wim;
    float c5 = ((c * c) * (c * c)) * c;
    for (int i = 0; i < 3; ++i) {
        float F = f0[i] + (1.0f - f0[i]) * c5;
        w[i] = F * g;
    }
    *wo = o;
    return 1;
}

int orc_sample_ggx(const float wi[3], float alpha, const float f0[3], float u2, float u3,
                   float wo[3], float weight[3])
{
    v3 o;
    int ok = sample_ggx(load3(wi), alpha, f0, u2, u3, &o, weight);
    if (ok) store3(wo, o);
    return ok;
}

/* ------------------------------------------------------------------------
 * Interleaved grouping (Section 3.3): pixels of a W x H tile are numbered in
 * screen order, the numbers are shuffled by the affine congruence
 * s(i) = (a*i + c) mod WH (a odd, so a bijection because WH is a power of
 * two), and pixels whose shuffled numbers share the quotient by K form a group.
 * Pin: bijection, exactly K members per full-tile group, every pixel's slot
 * equal to the shuffle recomputed from the tile draw in the test.
 * ---------------------------------------------------------------------- */
static void shuffle_params(int wh, uint64_t x0, uint64_t x1, uint32_t* a, uint32_t* c)
{
    if (wh <= 1) { *a = 1; *c = 0; return; }
    *a = 2u * (uint32_t)(x0 % (uint64_t)(wh / 2)) + 1u;
    *c = (uint32_t)(x1 % (uint64_t)wh);
}

void orc_shuffle(int wh, uint64_t x0, uint64_t x1, uint32_t* slot)
{
    uint32_t a, c;
    shuffle_params(wh, x0, x1, &a, &c);
    for (int i = 0; i < wh; ++i) slot[i] = (uint32_t)(((uint64_t)a * (uint64_t)i + c) % (uint64_t)wh);
}

/* ------------------------------------------------------------------------
 * Keys of the reordering baselines (Section 4 names the methods; Section 2.1
 * says what each encodes).  A coordinate x in [lo, lo + ext] is quantized to
 * nb bits as floor(((x - lo) / ext) * 2^nb), clamped to [0, 2^nb - 1] (NaN and
 * values below lo give 0); a direction component d in [-1, 1] is quantized the
 * same way with lo = -1, ext = 2.  Bits are interleaved most significant first.
 *   TwoPoint: origin and the point at a fixed length of 0.25 times the largest
 *     scene extent, 5 bits per coordinate, order ox oy oz ex ey ez (30 bits).
 *   Origin: origin only, 10 bits per coordinate, order ox oy oz (30 bits).
 *   Reis: origin in the high bits (6 bits per coordinate, interleaved), then the
 *     direction (4 bits per component, interleaved): 18 + 12 bits.
 *   Aila: origin and direction bits interleaved, 5 bits per value, order
 *     ox oy oz dx dy dz (30 bits).
 * Pin: bit-by-bit rebuild of every kind in the test suite.
 * ---------------------------------------------------------------------- */
static uint32_t quant(float x, float lo, float ext, int nb)
{
    if (!(ext > 0.0f)) return 0;
    const float top = (float)(1u << nb);
    float f = ((x - lo) / ext) * top;
    if (!(f > 0.0f)) return 0;    /* also maps NaN to 0 */
    if (f >= top - 1.0f) return (1u << nb) - 1u;
    return (uint32_t)f;
}

/* interleave the low nb bits of n values, most significant bit first */
static uint32_t interleave(const uint32_t* q, int n, int nb)
{
    uint32_t key = 0;
    for (int bit = nb - 1; bit >= 0; --bit)
        for (int c = 0; c < n; ++c) key = (key << 1) | ((q[c] >> bit) & 1u);
    return key;
}

uint32_t orc_ray_key_kind(int kind, const float lo[3], const float hi[3], const float o[3], const float d[3])
{
    float ext[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
    uint32_t q[6];
    switch (kind) {
    case ORC_MODE_SORTED_ORIGIN:
        for (int a = 0; a < 3; ++a) q[a] = quant(o[a], lo[a], ext[a], 10);
        return interleave(q, 3, 10);
    case ORC_MODE_SORTED_REIS: {
        uint32_t qd[3];
        for (int a = 0; a < 3; ++a) { q[a] = quant(o[a], lo[a], ext[a], 6); qd[a] = quant(d[a], -1.0f, 2.0f, 4); }
        return (interleave(q, 3, 6) << 12) | interleave(qd, 3, 4);
    }
    case ORC_MODE_SORTED_AILA:
        for (int a = 0; a < 3; ++a) { q[a] = quant(o[a], lo[a], ext[a], 5); q[3 + a] = quant(d[a], -1.0f, 2.0f, 5); }
        return interleave(q, 6, 5);
    default: {   /* TwoPoint */
        float mx = ext[0];
        if (ext[1] > mx) mx = ext[1];
        if (ext[2] > mx) mx = ext[2];
        float L = 0.25f * mx;
        float e[3] = {o[0] + L * d[0], o[1] + L * d[1], o[2] + L * d[2]};
        for (int a = 0; a < 3; ++a) { q[a] = quant(o[a], lo[a], ext[a], 5); q[3 + a] = quant(e[a], lo[a], ext[a], 5); }
        return interleave(q, 6, 5);
    }
    }
}

uint32_t orc_ray_key(const float lo[3], const float hi[3], const float o[3], const float d[3])
{
    return orc_ray_key_kind(ORC_MODE_SORTED, lo, hi, o, d);
}

static int is_reuse_mode(int mode)
{
    return mode == ORC_MODE_REUSE || mode == ORC_MODE_REUSE_PLAIN || mode == ORC_MODE_REUSE_WORLD;
}

static int is_sorted_mode(int mode)
{
    return mode == ORC_MODE_SORTED || mode == ORC_MODE_SORTED_ORIGIN || mode == ORC_MODE_SORTED_REIS ||
           mode == ORC_MODE_SORTED_AILA;
}

/* ------------------------------------------------------------------------
 * The path tracer.
 * ---------------------------------------------------------------------- */
typedef struct {
    v3 o, d;            /* current ray */
    int32_t excl;       /* prim the ray leaves from */
    int alive;          /* a ray is pending for the current bounce */
    float T[3], L[3];
    /* filled by the shading phase */
    int32_t prim; float t, t2;
    int active;         /* scatters at this hit */
    uint32_t kind;
    v3 origin, n, Tt, Bt, wi;
    v3 own_q; float own_w[3]; int own_ok;
    v3 use_q; float use_w[3]; int use_ok;
    int use_world; v3 use_dw;   /* direct world-space reuse: the shared world direction */
    int nee_prev;       /* the current ray left a Lambert point where NEE counted direct light */
    int32_t flags;
} opath;

typedef struct { uint32_t key; uint32_t idx; } keyidx;

static int cmp_keyidx(const void* a, const void* b)
{
    const keyidx* x = (const keyidx*)a;
    const keyidx* y = (const keyidx*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

static int absorbing(const orc_material* m)
{
    return m->albedo[0] == 0.0f && m->albedo[1] == 0.0f && m->albedo[2] == 0.0f;
}

/* own (independent) exit direction of path p at its hit; kind-specific */
static void own_sample(const orc_material* m, opath* p, float u2, float u3)
{
    if (m->kind == 0) {
        p->own_q = sample_lambert(u2, u3);
        for (int i = 0; i < 3; ++i) p->own_w[i] = m->albedo[i];
        p->own_ok = 1;
    } else if (m->kind == 1) {
        p->own_ok = sample_ggx(p->wi, m->alpha, m->albedo, u2, u3, &p->own_q, p->own_w);
    } else {
        p->own_q = mk(-p->wi.x, -p->wi.y, p->wi.z);
        for (int i = 0; i < 3; ++i) p->own_w[i] = m->albedo[i];
        p->own_ok = p->own_q.z > 0.0f;
    }
}

/* ------------------------------------------------------------------------
 * Next-event estimation at a Lambert scattering point (the paper's future-work
 * extension, Section 6): one emissive triangle chosen uniformly from the
 * pixel draw of stream 2 (x0 mod nemit), a uniform point on it from x1, x2
 * (b0 = 1 - sqrt(u1), b1 = u2 sqrt(u1), b2 = (1 - b0) - b1), and a shadow ray
 * from the scattering point's offset origin along D = point - origin, blocked by
 * any triangle other than the scattering one at 0 < t < 1 - 2^-10 (t in units of
 * D).  Unblocked and with D in the upper hemisphere, it adds
 * (T * albedo) * (Le * ((cos_s * cos_l) / (|D|^2 |D|^2)) * (nemit / (2 pi))),
 * cos_s = D.n and cos_l = |D.(e1 x e2)| unnormalized: the area-sampling
 * estimator f Le cos cos / (r^2 pdf_A) with f = albedo / pi, pdf_A = 1/(nemit A).
 * Emission that a ray sampled at a Lambert point then hits is not added again.
 * ---------------------------------------------------------------------- */
#define ORC_SHADOW_TMAX (1.0f - 0x1p-10f)

static void nee_sample(const orc_scene* s, const opath* p, const orc_material* m, uint64_t seed,
                       size_t pixel, int smp, int b, float C[3], v3* D, int* ok)
{
    *ok = 0;
    if (s->nemit == 0) return;
    uint64_t r[4];
    draw(seed, pixel, smp, b, 2, r);
    uint32_t e = s->emit[(uint32_t)(r[0] % (uint64_t)s->nemit)];
    float u1 = u01(r[1]), u2 = u01(r[2]);
    const float* v = s->tris + (size_t)e * 9;
    v3 v0 = load3(v), v1 = load3(v + 3), v2 = load3(v + 6);
    float su = sqrtf(u1);
    float b0 = 1.0f - su, b1 = u2 * su;
    float b2 = (1.0f - b0) - b1;
    v3 q = mk((b0 * v0.x + b1 * v1.x) + b2 * v2.x, (b0 * v0.y + b1 * v1.y) + b2 * v2.y,
              (b0 * v0.z + b1 * v1.z) + b2 * v2.z);
    v3 d = vsub(q, p->origin);
    float cs = vdot(d, p->n);
    if (!(cs > 0.0f)) return;
    v3 nl = vcross(vsub(v1, v0), vsub(v2, v0));
    float cl = fabsf(vdot(d, nl));
    float d2 = vdot(d, d);
    float g = (cs * cl) / (d2 * d2);
    float k = g * ((float)s->nemit * (float)(1.0 / (2.0 * 3.14159265358979323846)));
    const float* Le = s->mats[s->tri_mat[e]].emission;
    for (int c = 0; c < 3; ++c) C[c] = (p->T[c] * m->albedo[c]) * (Le[c] * k);
    *D = d;
    *ok = 1;
}

int orc_render(const orc_scene* s, const orc_camera* cam, int w, int h, int spp, int B,
               int mode, int W, int H, int K, int reuse_max_bounce, int frame_groups, uint64_t seed,
               const uint8_t* tile_mask, int nee, orc_outputs* out)
{
    if (w <= 0 || h <= 0 || spp <= 0 || B < 0 || W <= 0 || H <= 0 || K <= 0) return -1;
    if ((W & (W - 1)) || (H & (H - 1)) || (K & (K - 1)) || K > W * H || W * H > 65536) return -1;
    if (mode < 0 || mode > 7) return -1;
    if (nee && mode == ORC_MODE_REUSE_WORLD) return -1;   /* a member that dies after NEE is not covered */
    const int WH = W * H;
    const int ntx = (w + W - 1) / W, nty = (h + H - 1) / H;
    const size_t npix = (size_t)w * (size_t)h;
    cam_basis cb = camera_basis(cam, w, h);

    opath* P = (opath*)calloc(npix, sizeof(opath));
    uint8_t* rendered = (uint8_t*)calloc(npix, 1);
    uint32_t* list = (uint32_t*)malloc(npix * sizeof(uint32_t) + 4);
    keyidx* ki = (keyidx*)malloc(npix * sizeof(keyidx) + 4);
    float* acc = (float*)calloc(npix * 3, sizeof(float));
    if (!P || !rendered || !list || !ki || !acc) {
        free(P); free(rendered); free(list); free(ki); free(acc);
        return -2;
    }
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int tile = (y / H) * ntx + (x / W);
            rendered[(size_t)y * w + x] = tile_mask ? (tile_mask[tile] != 0) : 1;
        }
    const size_t plane = npix;
    for (int b = 0; b <= B; ++b) {
        if (out->rays_per_bounce) out->rays_per_bounce[b] = 0;
        for (int smp = 0; smp < spp; ++smp)
            for (size_t i = 0; i < npix; ++i) {
                if (!rendered[i]) continue;
                size_t at = ((size_t)b * spp + smp) * plane + i;
                if (out->hit_prim) out->hit_prim[at] = -2;
                if (out->hit_t) out->hit_t[at] = INFINITY;
                if (out->hit_t2) out->hit_t2[at] = INFINITY;
                if (out->rays) memset(out->rays + at * 8, 0, 8 * sizeof(float));
                if (b < B) {
                    if (out->dbg_flags) out->dbg_flags[at] = 0;
                    if (out->dbg_keys) out->dbg_keys[at] = 0xFFFFFFFFu;
                    if (out->dbg_q) { out->dbg_q[at * 3] = 0.0f; out->dbg_q[at * 3 + 1] = 0.0f; out->dbg_q[at * 3 + 2] = 0.0f; }
                }
            }
    }

    uint32_t* member = (uint32_t*)malloc((size_t)WH * sizeof(uint32_t) + 4); /* slot -> pixel+1 */
    v3* tree = (v3*)malloc((size_t)WH * sizeof(v3) + 4);
    if (!member || !tree) {
        free(P); free(rendered); free(list); free(ki); free(acc); free(member); free(tree);
        return -2;
    }

    for (int smp = 0; smp < spp; ++smp) {
        /* primary rays */
        for (int y = 0; y < h; ++y)
            for (int x = 0; x < w; ++x) {
                size_t i = (size_t)y * w + x;
                opath* p = &P[i];
                memset(p, 0, sizeof(*p));
                if (!rendered[i]) continue;
                uint64_t r[4];
                draw(seed, i, smp, 0, 0, r);
                camera_ray(&cb, w, h, x, y, u01(r[0]), u01(r[1]), &p->o, &p->d);
                p->excl = -1;
                p->alive = 1;
                p->nee_prev = 0;
                p->T[0] = p->T[1] = p->T[2] = 1.0f;
            }
        for (int b = 0; b <= B; ++b) {
            /* ---- intersect ---- */
            size_t nl = 0;
            for (size_t i = 0; i < npix; ++i)
                if (P[i].alive) list[nl++] = (uint32_t)i;
            if (is_sorted_mode(mode) && b >= 1) {
                for (size_t j = 0; j < nl; ++j) {
                    opath* p = &P[list[j]];
                    float o[3] = {p->o.x, p->o.y, p->o.z}, d[3] = {p->d.x, p->d.y, p->d.z};
                    ki[j].key = orc_ray_key_kind(mode, s->lo, s->hi, o, d);
                    ki[j].idx = list[j];
                }
                qsort(ki, nl, sizeof(keyidx), cmp_keyidx);
                for (size_t j = 0; j < nl; ++j) list[j] = ki[j].idx;
            }
            for (size_t j = 0; j < nl; ++j) {
                opath* p = &P[list[j]];
                if (out->rays) {
                    float* rr = out->rays + (((size_t)b * spp + smp) * plane + list[j]) * 8;
                    uint32_t pxi = list[j];
                    rr[0] = p->o.x; rr[1] = p->o.y; rr[2] = p->o.z; memcpy(&rr[3], &p->excl, 4);
                    rr[4] = p->d.x; rr[5] = p->d.y; rr[6] = p->d.z; memcpy(&rr[7], &pxi, 4);
                }
                hit2 hh = trace_one(s, p->o, p->d, p->excl, NULL, NULL);
                p->prim = hh.p1 == INT32_MAX ? -1 : hh.p1;
                p->t = hh.p1 == INT32_MAX ? INFINITY : hh.t1;
                p->t2 = hh.p2 == INT32_MAX ? INFINITY : hh.t2;
                size_t at = ((size_t)b * spp + smp) * plane + list[j];
                if (out->hit_prim) out->hit_prim[at] = p->prim;
                if (out->hit_t) out->hit_t[at] = p->t;
                if (out->hit_t2) out->hit_t2[at] = p->t2;
            }
            if (out->rays_per_bounce) out->rays_per_bounce[b] += nl;

            /* ---- shade: emission, termination, frame, own sample ---- */
            for (size_t i = 0; i < npix; ++i) {
                opath* p = &P[i];
                p->active = 0;
                p->flags = 0;
                if (!p->alive) continue;
                if (p->prim < 0) {
                    for (int c = 0; c < 3; ++c) p->L[c] = p->L[c] + p->T[c] * s->env[c];
                    p->alive = 0;
                    continue;
                }
                const orc_material* m = &s->mats[s->tri_mat[p->prim]];
                if (!(nee && p->nee_prev))
                    for (int c = 0; c < 3; ++c) p->L[c] = p->L[c] + p->T[c] * m->emission[c];
                if (b == B || absorbing(m)) { p->alive = 0; continue; }
                const float* v = s->tris + (size_t)p->prim * 9;
                v3 v0 = load3(v), v1 = load3(v + 3), v2 = load3(v + 6);
                v3 n = vnormalize(vcross(vsub(v1, v0), vsub(v2, v0)));
                if (vdot(n, p->d) > 0.0f) n = vneg(n);
                v3 hp = mk(p->o.x + p->t * p->d.x, p->o.y + p->t * p->d.y, p->o.z + p->t * p->d.z);
                p->origin = offset_origin(hp, n);
                p->n = n;
                onb(n, &p->Tt, &p->Bt);
                v3 md = vneg(p->d);
                p->wi = mk(vdot(md, p->Tt), vdot(md, p->Bt), vdot(md, n));
                p->kind = m->kind;
                p->active = 1;
                uint64_t r[4];
                draw(seed, i, smp, b, 0, r);
                own_sample(m, p, u01(r[2]), u01(r[3]));
                p->use_q = p->own_q;
                p->use_ok = p->own_ok;
                p->use_world = 0;
                for (int c = 0; c < 3; ++c) p->use_w[c] = p->own_w[c];
                p->flags = ORC_F_ACTIVE | ((int32_t)m->kind << ORC_F_CLASS_SH);
                if (nee && m->kind == 0) {
                    float C[3];
                    v3 D;
                    int ok;
                    nee_sample(s, p, m, seed, i, smp, b, C, &D, &ok);
                    if (ok) {
                        hit2 sh = trace_one(s, p->origin, D, p->prim, NULL, NULL);
                        int blocked = sh.p1 != INT32_MAX && sh.t1 < ORC_SHADOW_TMAX;
                        if (out->shadow_rays) out->shadow_rays[b] += 1;
                        if (!blocked)
                            for (int c = 0; c < 3; ++c) p->L[c] = p->L[c] + C[c];
                    }
                }
            }

            /* ---- generate: direction reuse inside interleaved groups ----
             * A reused direction is weighted by the receiving pixel's own material
             * (its own albedo for Lambert).  Pin: closed box of per-face albedos,
             * L = E (1 + rho_own) exactly; open floor, L = rho_own * L_env exactly.
             * REUSE: tangent-space rules of Section 3.2 in groups interleaved by the
             * per-tile shuffle of Section 3.3.  REUSE_PLAIN: the same rules in groups of
             * K consecutive screen-order pixels (no shuffle: the ablation of Section 3.3).
             * REUSE_WORLD: direct reuse of Section 3.1 -- the active member with the
             * smallest slot samples its own direction and every other Lambert member
             * takes it unchanged in world space, weighted by its own albedo; the path of
             * a member below whose surface that direction points ends; glossy and
             * specular members sample their own. */
            if (b < B && is_reuse_mode(mode) && b + 1 <= reuse_max_bounce) {
                for (int ty = 0; ty < nty; ++ty)
                    for (int tx = 0; tx < ntx; ++tx) {
                        int tile = ty * ntx + tx;
                        if (tile_mask && !tile_mask[tile]) continue;
                        /* Section 3.3: the group composition varies per tile and per frame.
                         * frame_groups = 0 draws a new shuffle at every bounce (b); 1 keeps
                         * the frame's first draw (bounce index 0) at every bounce, so the
                         * members that shared a direction at one hit group again at the next. */
                        uint64_t r[4];
                        draw(seed, (uint64_t)tile, smp, frame_groups ? 0 : b, 1, r);
                        uint32_t a = 1, c = 0;
                        if (mode != ORC_MODE_REUSE_PLAIN) shuffle_params(WH, r[0], r[1], &a, &c);
                        for (int sl = 0; sl < WH; ++sl) member[sl] = 0;
                        for (int iy = 0; iy < H; ++iy)
                            for (int ix = 0; ix < W; ++ix) {
                                int x = tx * W + ix, y = ty * H + iy;
                                if (x >= w || y >= h) continue;
                                uint32_t i = (uint32_t)(iy * W + ix);
                                uint32_t sl = (uint32_t)(((uint64_t)a * i + c) % (uint64_t)WH);
                                member[sl] = (uint32_t)((size_t)y * w + x) + 1u;
                                P[(size_t)y * w + x].flags |= (int32_t)(sl << ORC_F_SLOT_SH);
                            }
                        for (int g = 0; g < WH / K && mode == ORC_MODE_REUSE_WORLD; ++g) {
                            int rep = -1;
                            for (int j = 0; j < K && rep < 0; ++j) {
                                uint32_t mm = member[g * K + j];
                                if (mm && P[mm - 1].active) rep = (int)(mm - 1);
                            }
                            if (rep < 0) continue;
                            opath* pr = &P[rep];
                            pr->flags |= ORC_F_REP;
                            if (!pr->own_ok) continue;
                            v3 wdir = to_world(pr->own_q, pr->Tt, pr->Bt, pr->n);
                            for (int j = 0; j < K; ++j) {
                                uint32_t mm = member[g * K + j];
                                if (!mm || (int)(mm - 1) == rep) continue;
                                opath* p = &P[mm - 1];
                                if (!p->active || p->kind != 0) continue;
                                p->use_world = 1;
                                p->use_dw = wdir;
                                p->use_ok = vdot(wdir, p->n) > 0.0f;
                                const orc_material* m = &s->mats[s->tri_mat[p->prim]];
                                for (int cc = 0; cc < 3; ++cc) p->use_w[cc] = m->albedo[cc];
                                p->flags |= ORC_F_REUSED;
                            }
                        }
                        for (int g = 0; g < WH / K && mode != ORC_MODE_REUSE_WORLD; ++g) {
                            int nd = 0, ng = 0;
                            int rep = -1;
                            for (int j = 0; j < K; ++j) {
                                uint32_t mm = member[g * K + j];
                                if (!mm || !P[mm - 1].active) continue;
                                if (P[mm - 1].kind == 0) { ++nd; if (rep < 0) rep = (int)(mm - 1); }
                                else ++ng;
                            }
                            if (nd + ng == 0) continue;
                            int cat = ng == 0 ? 1 : (nd == 0 ? 2 : 3);
                            v3 q = mk(0, 0, 0);
                            int have = 0;
                            if (cat == 1) {
                                q = P[rep].own_q;
                                have = 1;
                                P[rep].flags |= ORC_F_REP;
                            } else if (cat == 3) {
                                int nvalid = 0;
                                for (int j = 0; j < K; ++j) {
                                    uint32_t mm = member[g * K + j];
                                    tree[j] = mk(0.0f, 0.0f, 0.0f);
                                    if (mm && P[mm - 1].active && P[mm - 1].kind != 0 && P[mm - 1].own_ok) {
                                        tree[j] = P[mm - 1].own_q;
                                        ++nvalid;
                                    }
                                }
                                for (int n = K; n > 1; n /= 2)
                                    for (int j = 0; j < n / 2; ++j) tree[j] = vadd(tree[2 * j], tree[2 * j + 1]);
                                if (nvalid > 0) {
                                    q = vnormalize(tree[0]);
                                    have = 1;
                                }
                            }
                            for (int j = 0; j < K; ++j) {
                                uint32_t mm = member[g * K + j];
                                if (!mm) continue;
                                opath* p = &P[mm - 1];
                                if (!p->active) continue;
                                p->flags |= cat << ORC_F_CAT_SH;
                                if (p->kind == 0 && have) {
                                    p->use_q = q;
                                    p->use_ok = 1;
                                    const orc_material* m = &s->mats[s->tri_mat[p->prim]];
                                    for (int cc = 0; cc < 3; ++cc) p->use_w[cc] = m->albedo[cc];
                                    if (!(cat == 1 && (int)(mm - 1) == rep)) p->flags |= ORC_F_REUSED;
                                }
                            }
                        }
                    }
            }

            /* ---- next rays ---- */
            for (size_t i = 0; i < npix; ++i) {
                opath* p = &P[i];
                if (!p->active) continue;
                if (p->use_ok) p->flags |= ORC_F_VALID;
                size_t at = ((size_t)b * spp + smp) * plane + i;
                if (out->dbg_flags) out->dbg_flags[at] = p->flags;
                v3 dq = p->use_world ? p->use_dw : p->use_q;   /* world direction for direct reuse */
                if (out->dbg_q) { out->dbg_q[at * 3] = dq.x; out->dbg_q[at * 3 + 1] = dq.y; out->dbg_q[at * 3 + 2] = dq.z; }
                if (!p->use_ok) { p->alive = 0; continue; }
                v3 nd = p->use_world ? p->use_dw : to_world(p->use_q, p->Tt, p->Bt, p->n);
                for (int c = 0; c < 3; ++c) p->T[c] = p->T[c] * p->use_w[c];
                p->nee_prev = nee && p->kind == 0;
                p->o = p->origin;
                p->d = nd;
                p->excl = p->prim;
                if (out->dbg_keys) {
                    float o[3] = {p->o.x, p->o.y, p->o.z}, d[3] = {nd.x, nd.y, nd.z};
                    out->dbg_keys[at] = orc_ray_key_kind(is_sorted_mode(mode) ? mode : ORC_MODE_SORTED, s->lo, s->hi, o, d);
                }
            }
        }
        for (size_t i = 0; i < npix; ++i) {
            if (!rendered[i]) continue;
            for (int c = 0; c < 3; ++c) acc[i * 3 + c] = smp == 0 ? P[i].L[c] : acc[i * 3 + c] + P[i].L[c];
        }
    }
    if (out->radiance)
        for (size_t i = 0; i < npix; ++i) {
            if (!rendered[i]) continue;
            for (int c = 0; c < 3; ++c) out->radiance[i * 3 + c] = acc[i * 3 + c] / (float)spp;
        }
    free(P); free(rendered); free(list); free(ki); free(acc); free(member); free(tree);
    return 0;
}
