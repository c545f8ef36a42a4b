// HIP kernels of libpt for gfx950 (MI355X).
//
// Wavefront path tracer: raygen -> [key -> sort -> gather] -> trace -> shade, per
// bounce.  Arithmetic on the ray chain is binary32 without FMA contraction (the
// library is compiled with -ffp-contract=off), correctly rounded division and
// square root, in the operation order fixed by the arithmetic contract, so that
// hit ids are reproducible bit for bit.  Box tests only prune and use explicit
// conservative margins.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "kernels.h"

namespace pt {
namespace {

// ------------------------------------------------------------------ vector helpers
struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 mk3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 sub3(V3 a, V3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 add3(V3 a, V3 b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 scl3(V3 a, float s) { return mk3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ float dot3(V3 a, V3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ __forceinline__ V3 cross3(V3 a, V3 b) {
    return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ V3 unit3(V3 v) {
    float inv = 1.0f / sqrtf(dot3(v, v));
    return scl3(v, inv);
}
__device__ __forceinline__ V3 xyz(float4 v) { return mk3(v.x, v.y, v.z); }
// component-wise select: a select of whole structs can be lowered to a select of their
// addresses, which puts the candidates in scratch memory
__device__ __forceinline__ V3 sel3(bool c, V3 a, V3 b) { return mk3(c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z); }

// ------------------------------------------------------------------ Philox4x64-10
struct U64x4 {
    uint64_t v[4];
};
__device__ __forceinline__ U64x4 philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t k1 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
        uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    return U64x4{{c0, c1, c2, c3}};
}
__device__ __forceinline__ float unit01(uint64_t x) { return (float)(uint32_t)(x >> 40) * 0x1p-24f; }

// sin and cos of 2*pi*u: exact octant reduction, Taylor polynomials on [0, pi/4]
__device__ __forceinline__ void sincos_turn(float u, float& sn, float& cs) {
    const float kQuarterPi = (float)(3.14159265358979323846 / 4.0);
    const float s3 = (float)(-1.0 / 6.0), s5 = (float)(1.0 / 120.0);
    const float s7 = (float)(-1.0 / 5040.0), s9 = (float)(1.0 / 362880.0);
    const float c2 = -0.5f, c4 = (float)(1.0 / 24.0), c6 = (float)(-1.0 / 720.0);
    const float c8 = (float)(1.0 / 40320.0), c10 = (float)(-1.0 / 3628800.0);
    float v = u * 8.0f;
    int oct = (int)v;
    float f = v - (float)oct;
    float g = (oct & 1) ? 1.0f - f : f;
    float a = g * kQuarterPi;
    float a2 = a * a;
    float s = a + (a * a2) * (s3 + a2 * (s5 + a2 * (s7 + a2 * s9)));
    float c = 1.0f + a2 * (c2 + a2 * (c4 + a2 * (c6 + a2 * (c8 + a2 * c10))));
    // (sin, cos) by octant: (s,c) (c,s) (c,-s) (s,-c) (-s,-c) (-c,-s) (-c,s) (-s,c)
    oct &= 7;
    bool swap = ((oct + 1) & 2) != 0;       // octants 1,2,5,6
    float p = swap ? c : s, q = swap ? s : c;
    sn = (oct >= 4) ? -p : p;
    cs = (oct >= 2 && oct <= 5) ? -q : q;
}

// ------------------------------------------------------------------ frame
__device__ __forceinline__ V3 push_off(V3 p, V3 n) {
    // Waechter & Binder integer-ulp offset along n
    const float kOrigin = 1.0f / 32.0f, kFloatScale = 1.0f / 65536.0f, kIntScale = 256.0f;
    int ox = (int)(kIntScale * n.x), oy = (int)(kIntScale * n.y), oz = (int)(kIntScale * n.z);
    float px = __int_as_float(__float_as_int(p.x) + (p.x < 0.0f ? -ox : ox));
    float py = __int_as_float(__float_as_int(p.y) + (p.y < 0.0f ? -oy : oy));
    float pz = __int_as_float(__float_as_int(p.z) + (p.z < 0.0f ? -oz : oz));
    return mk3(fabsf(p.x) < kOrigin ? p.x + kFloatScale * n.x : px,
               fabsf(p.y) < kOrigin ? p.y + kFloatScale * n.y : py,
               fabsf(p.z) < kOrigin ? p.z + kFloatScale * n.z : pz);
}

__device__ __forceinline__ void frame_of(V3 n, V3& t, V3& bt) {
    float s = copysignf(1.0f, n.z);
    float a = -1.0f / (s + n.z);
    float b = (n.x * n.y) * a;
    t = mk3(1.0f + ((s * n.x) * n.x) * a, s * b, -(s * n.x));
    bt = mk3(b, s + (n.y * n.y) * a, -n.y);
}

__device__ __forceinline__ V3 tangent_to_world(V3 q, V3 t, V3 bt, V3 n) {
    return mk3((q.x * t.x + q.y * bt.x) + q.z * n.x, (q.x * t.y + q.y * bt.y) + q.z * n.y,
               (q.x * t.z + q.y * bt.z) + q.z * n.z);
}

// ------------------------------------------------------------------ BSDF sampling (tangent space)
__device__ __forceinline__ V3 cosine_dir(float u2, float u3) {
    float r = sqrtf(u2);
    float sn, cs;
    sincos_turn(u3, sn, cs);
    float z2 = 1.0f - u2;
    return mk3(r * cs, r * sn, sqrtf(z2 > 0.0f ? z2 : 0.0f));
}

__device__ __forceinline__ float g1_smith(float z, float a2) {
    float z2 = z * z;
    float num = 1.0f - z2;
    float tan2 = (num > 0.0f ? num : 0.0f) / z2;
    return 2.0f / (1.0f + sqrtf(1.0f + a2 * tan2));
}

// GGX exit (Walter et al. 2007 sampling of the normal, Smith G, Schlick F), written
// without early returns: the caller selects by the returned validity.
__device__ __forceinline__ bool ggx_dir(V3 wi, float alpha, const float* f0, float u2, float u3, V3& wo, float* w) {
    const float a2 = alpha * alpha;
    const float tan2m = (a2 * u2) / (1.0f - u2);
    const float cm = 1.0f / sqrtf(1.0f + tan2m);
    const float sm2 = 1.0f - cm * cm;
    const float sm = sqrtf(sm2 > 0.0f ? sm2 : 0.0f);
    float sn, cs;
    sincos_turn(u3, sn, cs);
    const V3 m = mk3(sm * cs, sm * sn, cm);
    const float wim = dot3(wi, m);
    const float k = 2.0f * wim;
    const V3 o = mk3(k * m.x - wi.x, k * m.y - wi.y, k * m.z - wi.z);
    const float g = ((g1_smith(wi.z, a2) * g1_smith(o.z, a2)) * wim) / (wi.z * cm);
    const float c = 1.0f - wim;
    const float c5 = ((c * c) * (c * c)) * c;
#pragma unroll
    for (int i = 0; i < 3; ++i) w[i] = (f0[i] + (1.0f - f0[i]) * c5) * g;
    wo = o;
    return wi.z > 0.0f && wim > 0.0f && o.z > 0.0f;
}

// ------------------------------------------------------------------ watertight ray/triangle
struct RayPre {
    float ox, oy, oz;   // origin, permuted to (kx, ky, kz)
    float sx, sy, sz;
    int kx, ky, kz;
};

__device__ __forceinline__ float pick(float a, float b, float c, int k) { return k == 0 ? a : (k == 1 ? b : c); }

__device__ __forceinline__ RayPre prepare(V3 o, V3 d) {
    RayPre r;
    float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    int kz = 0;
    float m = ax;
    if (ay > m) {
        kz = 1;
        m = ay;
    }
    if (az > m) kz = 2;
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    float dkz = pick(d.x, d.y, d.z, kz);
    if (dkz < 0.0f) {
        int t = kx;
        kx = ky;
        ky = t;
    }
    r.kx = kx;
    r.ky = ky;
    r.kz = kz;
    r.sx = pick(d.x, d.y, d.z, kx) / dkz;
    r.sy = pick(d.x, d.y, d.z, ky) / dkz;
    r.sz = 1.0f / dkz;
    r.ox = pick(o.x, o.y, o.z, kx);
    r.oy = pick(o.x, o.y, o.z, ky);
    r.oz = pick(o.x, o.y, o.z, kz);
    return r;
}

__device__ __forceinline__ float dprod_diff(float a, float b, float c, float d) {
    return (float)((double)a * (double)b - (double)c * (double)d);
}

// hit with 0 < t < inf: returns true and t
__device__ __forceinline__ bool tri_test(const RayPre& r, float4 p0, float4 p1, float4 p2, float& t_out) {
    float Ax = pick(p0.x, p0.y, p0.z, r.kx) - r.ox, Ay = pick(p0.x, p0.y, p0.z, r.ky) - r.oy;
    float Az0 = pick(p0.x, p0.y, p0.z, r.kz) - r.oz;
    float Bx = pick(p1.x, p1.y, p1.z, r.kx) - r.ox, By = pick(p1.x, p1.y, p1.z, r.ky) - r.oy;
    float Bz0 = pick(p1.x, p1.y, p1.z, r.kz) - r.oz;
    float Cx = pick(p2.x, p2.y, p2.z, r.kx) - r.ox, Cy = pick(p2.x, p2.y, p2.z, r.ky) - r.oy;
    float Cz0 = pick(p2.x, p2.y, p2.z, r.kz) - r.oz;
    Ax = Ax - r.sx * Az0;
    Ay = Ay - r.sy * Az0;
    Bx = Bx - r.sx * Bz0;
    By = By - r.sy * Bz0;
    Cx = Cx - r.sx * Cz0;
    Cy = Cy - r.sy * Cz0;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = dprod_diff(Cx, By, Cy, Bx);
        V = dprod_diff(Ax, Cy, Ay, Cx);
        W = dprod_diff(Bx, Ay, By, Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    float det = (U + V) + W;
    if (det == 0.0f) return false;
    float Az = r.sz * Az0, Bz = r.sz * Bz0, Cz = r.sz * Cz0;
    float T = (U * Az + V * Bz) + W * Cz;
    float t = T / det;
    if (!(t > 0.0f) || !(t < INFINITY)) return false;
    t_out = t;
    return true;
}

// ------------------------------------------------------------------ traversal
// Slab test of one child box; conservative: the far distance is widened by
// (1 + 2*gamma_3) (Ize, "Robust BVH Ray Traversal", JCGT 2013) and the caller
// culls against the best distance widened by 2^-18.
constexpr float kFarScale = 1.0f + 2.0f * (3.0f * 0x1p-24f) / (1.0f - 3.0f * 0x1p-24f);
constexpr float kCullScale = 1.0f + 0x1p-18f;

__device__ __forceinline__ float slab(float lx, float hx, float ly, float hy, float lz, float hz, V3 o, V3 inv,
                                      float tcull, bool& hit) {
    float x0 = (lx - o.x) * inv.x, x1 = (hx - o.x) * inv.x;
    float y0 = (ly - o.y) * inv.y, y1 = (hy - o.y) * inv.y;
    float z0 = (lz - o.z) * inv.z, z1 = (hz - o.z) * inv.z;
    float tn = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), 0.0f));
    float tf = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fmaxf(z0, z1)) * kFarScale;
    hit = tn <= tf && tn <= tcull;
    return tn;
}

constexpr int32_t kDone = INT32_MIN;   // = kEmpty: never a node or leaf code

// Closest-hit traversal, one ray per lane, after Aila & Laine ("Understanding the
// efficiency of ray traversal on GPUs", HPG 2009), shaped for 64-wide waves:
//  * inner-node phase: lanes walk inner nodes; a lane that reaches a leaf postpones
//    it and keeps walking (speculative traversal) until it reaches a second one.
//    The phase ends once at most `leaf_gate` lanes are still without a leaf: waiting
//    for all 64 lanes leaves most of them parked.
//  * leaf phase, wave-wide: the triangles of every held leaf are listed as (lane,
//    triangle) pairs and spread over all 64 lanes, idle ones included; each result
//    returns to the lane that owns the ray by cross-lane shuffles, where the (t,
//    prim id) minimum is kept.  A lane tests its pairs with the owner's ray.
//  * persistent lanes with refill: a lane whose ray is finished takes a new ray from
//    the queue once `refill` lanes are idle, so a wave is not held by its slowest ray.
// Culling only ever prunes (conservative box test), and every leaf that is reached
// is tested, so the result is the exact (t, prim id) minimum.  All loops below are
// wave-uniform: every lane reaches every shuffle and barrier.
constexpr int32_t kNoLeaf = 0;   // never a leaf code (leaf codes are negative)
constexpr int kLeafCountBits = kMaxLeaf < 2 ? 1 : (kMaxLeaf < 4 ? 2 : (kMaxLeaf < 8 ? 3 : 4));
static_assert(kMaxLeaf >= 1 && kMaxLeaf <= 8, "leaf codes hold counts 1..8");
static_assert(kTraceBlock == 64, "the pair list stores a lane in 6 bits");
using PairT = std::conditional_t<(kMaxLeaf <= 4), uint8_t, uint16_t>;   // lane + triangle-in-leaf

__device__ __forceinline__ void cswap(float& ta, int32_t& ka, float& tb, int32_t& kb) {
    const bool sw = tb < ta;
    const float t = sw ? tb : ta;
    const int32_t k = sw ? kb : ka;
    tb = sw ? ta : tb;
    kb = sw ? ka : kb;
    ta = t;
    ka = k;
}

// Rays are handed out by kRayCounters counters, one per XCD (workgroups are dispatched to
// the XCDs round robin), counter c owning the chunks of 64 rays whose chunk number is c
// modulo kRayCounters.  The counters advance at about the same pace, so the rays in flight
// stay in one compact stretch of the queue while the atomics spread over kRayCounters
// addresses instead of queueing on one.  A wave whose counter has run out moves on to the
// next; after all of them the wave is done.
__device__ __forceinline__ uint64_t claimed_ray(uint32_t v, uint32_t c) {
    return ((((uint64_t)(v >> 6)) * kRayCounters + c) << 6) | (v & 63u);
}

// The v-th ray counter c hands out, as an index into the launch's rays, or kNoClaim.  Plain
// and permuted launches: the 64-ray chunks of [0, n) numbered c mod 8.  Compacted launches
// (fill, no permutation): the first nc = fill[c] slots of region c.  The index is monotone
// in v, so the first v without a ray ends the counter.
constexpr uint64_t kNoClaim = ~0ull;
constexpr uint32_t kSpread = 64;   // stripes of the spread claim order of launches with fewer rays than lanes
__device__ __forceinline__ uint64_t claim_index(bool regions, uint32_t region, uint32_t v, uint32_t c, uint32_t n,
                                                uint32_t nc) {
    if (regions) return v < nc ? (uint64_t)c * region + v : kNoClaim;
    const uint64_t i = claimed_ray(v, c);
    return i < n ? i : kNoClaim;
}

// rays of the launch: a.n, or the sum of the region counts of a compacted launch
__device__ __forceinline__ uint32_t launch_rays(const TraceArgs& a) {
    if (!a.fill) return a.n;
    uint32_t n = 0;
#pragma unroll
    for (int c = 0; c < kRayCounters; ++c) n += a.fill[c * kCounterStride];
    return n;
}

template <bool STATS, bool MULTI, bool WIDE>
__global__ __launch_bounds__(kTraceBlock) void k_trace(DevScene sc, TraceArgs a, uint32_t gthreads,
                                                       const StepJob* jobs, int njobs) {
    __shared__ int32_t stk[kStackLds][kTraceBlock];
    __shared__ PairT pairs[kTraceBlock * kMaxLeaf];   // lane | (triangle in leaf) << 6
    const int lane = threadIdx.x;
    const uint32_t gtid = blockIdx.x * kTraceBlock + lane;
    // merged launches (MULTI) never use compacted or permuted queues
    const uint32_t* const fillp = MULTI ? nullptr : a.fill;
    const uint32_t* const permp = MULTI ? nullptr : a.perm;
    const bool regions = fillp && !permp;
    const uint32_t n = MULTI ? a.n : launch_rays(a);
    uint32_t ncq = fillp ? fillp[(blockIdx.x % kRayCounters) * kCounterStride] : 0u;   // rays of counter cq
    const unsigned long long lt = (1ull << lane) - 1ull;
    unsigned long long nv = 0, nt = 0;
    uint32_t traced = 0;
    bool have = false;
    bool exhausted = false;   // wave-uniform: the queue is used up
    uint32_t cq = blockIdx.x % kRayCounters;   // wave-uniform: the counter claimed from
    int tries = 0;
    uint32_t oi = 0;
    V3 o = mk3(0.f, 0.f, 0.f), inv = o;
    RayPre rp{};
    int32_t excl = -1, best_p = INT32_MAX, node = kDone, leaf = kNoLeaf;
    float best_t = INFINITY, tcull = INFINITY;
    int sp = 0, novf = 0;
    // scene and output of the lane's ray: kernel arguments for one job, per lane for a merged launch
    const float4* nodes = sc.nodes;
    const float4* nodes4 = sc.nodes4;
    const float4* btris = sc.btris;
    int32_t* oprim = a.out_prim;
    float* ot = a.out_t;
    for (;;) {
        // ---- refill idle lanes with the next rays of the queue
        const unsigned long long idle = __ballot(!have);
        if (!exhausted && idle != 0 && (__popcll(idle) >= a.refill || idle == ~0ull)) {
            // a launch with few rays spreads them over every wave (latency hiding) instead of
            // filling the first waves' 64 lanes and leaving the others without work
            const uint32_t share = n / gridDim.x + 1u;
            const uint32_t nidle = (uint32_t)__popcll(idle);
            const uint32_t need = nidle < share ? nidle : share;
            const uint32_t c = cq;
            const uint32_t nc = ncq;
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(a.work + c * kCounterStride, need);
            base = __shfl(base, 0);
            if (claim_index(regions, a.region, base + need, c, n, nc) == kNoClaim) {   // this counter has no rays left
                if (++tries == kRayCounters) exhausted = true;
                cq = (cq + 1u) % kRayCounters;
                ncq = fillp ? fillp[cq * kCounterStride] : 0u;
            }
            const uint32_t rank = (uint32_t)__popcll(idle & lt);
            if (!have && rank < need) {
                const uint64_t i64 = claim_index(regions, a.region, base + rank, c, n, nc);
                const uint32_t i = (uint32_t)i64;
                if (i64 != kNoClaim) {
                    const float4* rays = a.rays;
                    uint32_t li = permp ? permp[i] : i;   // sorted launches read the rays through the sort's permutation
                    if constexpr (MULTI) {
                        int lo = 0, hi = njobs - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (jobs[mid].ray_start <= i) lo = mid; else hi = mid - 1;
                        }
                        const StepJob& J = jobs[lo];
                        li = i - J.ray_start;
                        rays = J.q_in;
                        nodes = J.sc.nodes;
                        nodes4 = J.sc.nodes4;
                        btris = J.sc.btris;
                        oprim = J.trace_prim;
                        ot = J.trace_t;
                    }
                    // set up without a branch on the pixel word, so that the three loads of
                    // the ray are issued together (one wait, not two in a row)
                    const float4 r0 = rays[2 * (size_t)li], r1 = rays[2 * (size_t)li + 1];
                    const uint32_t pix = __float_as_uint(r1.w);
                    o = xyz(r0);
                    const V3 d = xyz(r1);
                    excl = __float_as_int(r0.w);
                    inv = mk3(1.0f / d.x, 1.0f / d.y, 1.0f / d.z);
                    rp = prepare(o, d);
                    // a shadow ray only asks whether anything lies before the light point:
                    // hits are kept from t < kShadowTmax on, and INT32_MIN never loses a tie
                    best_t = a.shadow ? kShadowTmax : INFINITY;
                    tcull = a.shadow ? kShadowTmax * kCullScale : INFINITY;
                    best_p = a.shadow ? INT32_MIN : INT32_MAX;
                    sp = 0;
                    novf = 0;
                    node = 0;
                    leaf = kNoLeaf;
                    oi = a.by_pixel ? pix : li;
                    have = !(a.by_pixel || a.skip_empty) || pix != kNoRay;   // else the lane stays idle
                }
            }
        }
        if (__ballot(have) == 0) {
            if (exhausted) break;
            continue;
        }
        // ---- inner nodes; a leaf that is reached is postponed while the slot is free
        for (;;) {
            if (have && node >= 0) {
                if constexpr (WIDE) {
                    // four children: nearest hit next, the other hits pushed far to near
                    const float4* nd = nodes4 + 8 * (size_t)node;
                    const float4 lx = nd[0], hx = nd[1], ly = nd[2], hy = nd[3], lz = nd[4], hz = nd[5], cc = nd[6];
                    if (STATS) {
                    ++nv;
                    if (a.touched) a.touched[node] |= (uint8_t)a.touch_bit;
                }
                    bool h0, h1, h2, h3;
                    float a0 = slab(lx.x, hx.x, ly.x, hy.x, lz.x, hz.x, o, inv, tcull, h0);
                    float a1 = slab(lx.y, hx.y, ly.y, hy.y, lz.y, hz.y, o, inv, tcull, h1);
                    float a2 = slab(lx.z, hx.z, ly.z, hy.z, lz.z, hz.z, o, inv, tcull, h2);
                    float a3 = slab(lx.w, hx.w, ly.w, hy.w, lz.w, hz.w, o, inv, tcull, h3);
                    int32_t k0 = __float_as_int(cc.x), k1 = __float_as_int(cc.y), k2 = __float_as_int(cc.z),
                            k3 = __float_as_int(cc.w);
                    h0 = h0 && k0 != kEmpty;
                    h1 = h1 && k1 != kEmpty;
                    h2 = h2 && k2 != kEmpty;
                    h3 = h3 && k3 != kEmpty;
                    const int nh = (int)h0 + (int)h1 + (int)h2 + (int)h3;
                    a0 = h0 ? a0 : INFINITY;
                    a1 = h1 ? a1 : INFINITY;
                    a2 = h2 ? a2 : INFINITY;
                    a3 = h3 ? a3 : INFINITY;
                    // sorting network on (distance, code): misses (+inf) end up last
                    cswap(a0, k0, a1, k1);
                    cswap(a2, k2, a3, k3);
                    cswap(a0, k0, a2, k2);
                    cswap(a1, k1, a3, k3);
                    cswap(a1, k1, a2, k2);
                    if (nh == 0) {
                        node = kDone;   // pop below
                    } else {
                        node = k0;
                        if (sp + nh - 1 > kStackLds) {
                            if (novf + kStackLds / 2 > kStackOvf) {
                                node = kDone;   // unreachable within the depth bound of wide trees
                                leaf = kNoLeaf;
                                sp = 0;
                                novf = 0;
                            } else {
                                for (int e = 0; e < kStackLds / 2; ++e)
                                    a.ovf[(size_t)(novf + e) * gthreads + gtid] = stk[e][lane];
                                for (int e = 0; e < kStackLds / 2; ++e) stk[e][lane] = stk[e + kStackLds / 2][lane];
                                novf += kStackLds / 2;
                                sp -= kStackLds / 2;
                            }
                        }
                        if (node != kDone) {
                            if (nh == 4) stk[sp++][lane] = k3;
                            if (nh >= 3) stk[sp++][lane] = k2;
                            if (nh >= 2) stk[sp++][lane] = k1;
                        }
                    }
                } else {
                    const float4* nd = nodes + 4 * (size_t)node;
                    const float4 n0 = nd[0], n1 = nd[1], n2 = nd[2], n3 = nd[3];
                    if (STATS) {
                    ++nv;
                    if (a.touched) a.touched[node] |= (uint8_t)a.touch_bit;
                }
                    const int32_t c0 = __float_as_int(n3.x), c1 = __float_as_int(n3.y);
                    bool h0, h1;
                    const float t0 = slab(n0.x, n0.y, n0.z, n0.w, n2.x, n2.y, o, inv, tcull, h0);
                    const float t1 = slab(n1.x, n1.y, n1.z, n1.w, n2.z, n2.w, o, inv, tcull, h1);
                    h0 = h0 && c0 != kEmpty;
                    h1 = h1 && c1 != kEmpty;
                    if (h0 && h1) {
                        const bool swp = t1 < t0;
                        const int32_t far = swp ? c0 : c1;
                        node = swp ? c1 : c0;
                        if (sp == kStackLds) {
                            // the BVH depth bound keeps the stack within kStackLds + kStackOvf
                            // entries; the check keeps every access in bounds regardless
                            if (novf + kStackLds / 2 > kStackOvf) {
                                node = kDone;   // give the ray up (the pop below finds the stack empty)
                                leaf = kNoLeaf;
                                sp = 0;
                                novf = 0;
                            } else {
                                // spill the lower half of the LDS stack to this lane's overflow column
                                for (int e = 0; e < kStackLds / 2; ++e)
                                    a.ovf[(size_t)(novf + e) * gthreads + gtid] = stk[e][lane];
                                for (int e = 0; e < kStackLds / 2; ++e) stk[e][lane] = stk[e + kStackLds / 2][lane];
                                novf += kStackLds / 2;
                                sp = kStackLds / 2;
                            }
                        }
                        if (node != kDone) stk[sp++][lane] = far;
                    } else if (h0) {
                        node = c0;
                    } else if (h1) {
                        node = c1;
                    } else {
                        node = kDone;   // pop below
                    }
                }
                if (node == kDone || (node < 0 && leaf == kNoLeaf)) {
                    if (node != kDone) leaf = node;
                    // pop
                    if (sp == 0 && novf > 0) {
                        const int m = novf < kStackLds / 2 ? novf : kStackLds / 2;
                        for (int e = 0; e < m; ++e) stk[e][lane] = a.ovf[(size_t)(novf - m + e) * gthreads + gtid];
                        novf -= m;
                        sp = m;
                    }
                    node = sp > 0 ? stk[--sp][lane] : kDone;
                }
            }
            // few lanes are still looking for their first leaf: test the leaves now
            if ((int)__popcll(__ballot(have && node >= 0 && leaf == kNoLeaf)) <= a.leaf_gate) break;
        }
        // ---- leaves, wave-wide: the postponed one, then the next node while it is a leaf
        for (;;) {
            if (have && leaf == kNoLeaf && node < 0 && node != kDone) {
                leaf = node;
                if (sp == 0 && novf > 0) {
                    const int m = novf < kStackLds / 2 ? novf : kStackLds / 2;
                    for (int e = 0; e < m; ++e) stk[e][lane] = a.ovf[(size_t)(novf - m + e) * gthreads + gtid];
                    novf -= m;
                    sp = m;
                }
                node = sp > 0 ? stk[--sp][lane] : kDone;
            }
            const bool hold = have && leaf != kNoLeaf;
            if (__ballot(hold) == 0) break;
            const uint32_t code = ~(uint32_t)leaf;
            const uint32_t first = code >> 3;
            const uint32_t cnt = hold ? (code & 7u) + 1u : 0u;
            // exclusive prefix sum of the triangle counts over the wave, one ballot per bit
            uint32_t off = 0, total = 0;
#pragma unroll
            for (int bit = 0; bit < kLeafCountBits; ++bit) {
                const unsigned long long qb = __ballot((cnt >> bit) & 1u);
                off += (uint32_t)__popcll(qb & lt) << bit;
                total += (uint32_t)__popcll(qb) << bit;
            }
            for (uint32_t j = 0; j < cnt; ++j) pairs[off + j] = (PairT)((uint32_t)lane | (j << 6));
            __syncthreads();
            const int perm = rp.kx | (rp.ky << 2) | (rp.kz << 4);
            for (uint32_t base = 0; base < total; base += kTraceBlock) {
                const uint32_t p = base + (uint32_t)lane;
                const bool valid = p < total;
                const uint32_t e = valid ? (uint32_t)pairs[p] : 0u;
                const int src = (int)(e & 63u);
                // the owner's ray, leaf and triangle array
                RayPre q;
                q.ox = __shfl(rp.ox, src);
                q.oy = __shfl(rp.oy, src);
                q.oz = __shfl(rp.oz, src);
                q.sx = __shfl(rp.sx, src);
                q.sy = __shfl(rp.sy, src);
                q.sz = __shfl(rp.sz, src);
                const int qperm = __shfl(perm, src);
                q.kx = qperm & 3;
                q.ky = (qperm >> 2) & 3;
                q.kz = (qperm >> 4) & 3;
                const int32_t qexcl = __shfl(excl, src);
                const uint32_t qtri = __shfl(first, src) + (e >> 6);
                const float4* qtris = btris;
                if constexpr (MULTI) {
                    const uint64_t bp = (uint64_t)(uintptr_t)btris;
                    const uint32_t lo = __shfl((uint32_t)bp, src), hi = __shfl((uint32_t)(bp >> 32), src);
                    qtris = (const float4*)(uintptr_t)(((uint64_t)hi << 32) | lo);
                }
                float t = INFINITY;
                int32_t pid = INT32_MAX;
                if (valid) {
                    const float4* tp = qtris + 3 * (size_t)qtri;
                    const float4 p0 = tp[0], p1 = tp[1], p2 = tp[2];
                    const int32_t id = __float_as_int(p0.w);
                    if (STATS) {
                        ++nt;
                        if (a.touched) a.touched[a.touch_tri + qtri] |= (uint8_t)a.touch_bit;
                    }
                    float th;
                    if (tri_test(q, p0, p1, p2, th) && id != qexcl) {
                        t = th;
                        pid = id;
                    }
                }
                // each owner takes the results of its pairs that fell into this block of 64
#pragma unroll
                for (int jj = 0; jj < kMaxLeaf; ++jj) {
                    const int s = (int)off + jj - (int)base;
                    const int sl = s < 0 ? 0 : (s > kTraceBlock - 1 ? kTraceBlock - 1 : s);
                    const float tt = __shfl(t, sl);
                    const int32_t pp = __shfl(pid, sl);
                    if (jj < (int)cnt && s >= 0 && s < kTraceBlock && (tt < best_t || (tt == best_t && pp < best_p))) {
                        best_t = tt;
                        best_p = pp;
                        tcull = tt * kCullScale;
                        if (a.shadow) node = kDone;   // blocked: the shadow ray is answered
                    }
                }
            }
            __syncthreads();   // the pair list is rewritten by the next round
            leaf = kNoLeaf;
        }
        if (have && node == kDone) {
            oprim[oi] = (best_p == INT32_MAX || best_p == INT32_MIN) ? -1 : best_p;
            ot[oi] = best_t;
            ++traced;
            have = false;
        }
    }
    // per-workgroup count of traced rays (no atomics on a shared counter)
    unsigned int tsum = traced;
    for (int off = 32; off > 0; off >>= 1) tsum += __shfl_down(tsum, off);
    if (a.partial && lane == 0) a.partial[blockIdx.x] = tsum;
    if (STATS) {
        for (int off = 32; off > 0; off >>= 1) {
            nv += __shfl_down(nv, off);
            nt += __shfl_down(nt, off);
        }
        if (lane == 0) {
            atomicAdd(a.stats, nv);
            atomicAdd(a.stats + 1, nt);
        }
    }
}

// Closest-hit traversal over the four-wide nodes with a per-wave queue of triangle tests.
// A lane that reaches a leaf appends (lane, triangle) entries for its triangles to a ring
// in LDS and walks on at once; never holding a leaf, it never waits for one.  The wave
// tests the queue 64 entries at a time, one entry per lane with the owner's ray (taken
// by cross-lane shuffles), and folds each hit into the owner's (t, prim id) minimum,
// kept in LDS as one 64-bit key (t's bits above the prim id: both are non-negative, so
// the integer order is the lexicographic one) by an LDS atomic minimum.  A partial block
// is tested when `leaf_gate` + 1 lanes have finished walking and wait on queued tests,
// when the queue holds kFlushPerWalker entries per walking lane, or when no lane can walk
// on.  Owners re-read their key after every block to cull against it.  Culling prunes
// only, and every queued triangle is tested, so the result is the exact (t, prim id)
// minimum, as in k_trace.  Rays are claimed from the spread counters as in k_trace, each
// claim at most the launch's even share per wave.  Once the counters are used up (the
// drain, where most lanes would idle while a few rays finish), a walking lane with pending
// stack entries gives its top entry to a free lane, which walks that subtree with a copy of
// the ray; its triangle tests fold into the owner's key, and the owner writes the hit once no
// lane walks any part of its ray.  Which lane visits a subtree changes only the visiting
// order, so the result stays the exact (t, prim id) minimum.

// Slab tests of the four children of a quantized node (g = {p, step x}; child planes in
// q0 = {lo x, hi x, lo y, hi y}, q1 = {lo z, hi z, step y, step z}, one byte per child).
// Along an axis, the distance to plane p + q * 2^e is t = q * a + b with a = 2^e * inv
// (exact) and b = (p - o) * inv (two roundings).  b is moved by 2^-21 |b| (more than the
// 2.01 ulp its roundings can be off, plus the rounding of the move, one fused operation)
// toward the near side for near planes and the far side for far planes, so that the single
// rounding of the fused q * a + b is the only error left, relative to t, which the
// far-distance widening of the child-pair test covers.  Near and far planes are chosen by the sign of inv.  A direction component
// of zero gives infinities or NaN along that axis, which drop the axis from the min and
// max below (never a wrong cull).  The fused multiply-add is used on purpose: this test
// only prunes, and every result stays the exact (t, prim id) minimum.
constexpr float kQSlack = 0x1p-21f;
// Rays with |1/d| above this along some axis (a direction component of zero or below 2^-64)
// take the float boxes of the four-wide node of the same index instead: there the
// quantized form would drop the axis instead of culling by it, and 2^e / d could overflow.
// The node's steps are at most 2^60 (scenes that need more do not get quantized nodes), so
// 2^e * inv stays finite below this bound.
constexpr float kQMaxInv = 0x1p64f;

__device__ __forceinline__ float qplane(uint32_t q, int j, float a, float b) {
    return fmaf((float)((q >> (8 * j)) & 0xFFu), a, b);
}

__device__ __forceinline__ void qslab4(float4 g, float4 q0, float4 q1, V3 o, V3 inv, float tcull, float& t0,
                                       float& t1, float& t2, float& t3, bool& h0, bool& h1, bool& h2, bool& h3) {
    const float ax = g.w * inv.x, ay = q1.z * inv.y, az = q1.w * inv.z;
    const float bx = (g.x - o.x) * inv.x, by = (g.y - o.y) * inv.y, bz = (g.z - o.z) * inv.z;
    const float nbx = fmaf(fabsf(bx), -kQSlack, bx), fbx = fmaf(fabsf(bx), kQSlack, bx);
    const float nby = fmaf(fabsf(by), -kQSlack, by), fby = fmaf(fabsf(by), kQSlack, by);
    const float nbz = fmaf(fabsf(bz), -kQSlack, bz), fbz = fmaf(fabsf(bz), kQSlack, bz);
    const bool px = inv.x >= 0.0f, py = inv.y >= 0.0f, pz = inv.z >= 0.0f;
    const uint32_t nqx = __float_as_uint(px ? q0.x : q0.y), fqx = __float_as_uint(px ? q0.y : q0.x);
    const uint32_t nqy = __float_as_uint(py ? q0.z : q0.w), fqy = __float_as_uint(py ? q0.w : q0.z);
    const uint32_t nqz = __float_as_uint(pz ? q1.x : q1.y), fqz = __float_as_uint(pz ? q1.y : q1.x);
    float tn[4];
    bool hh[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float n = fmaxf(fmaxf(qplane(nqx, j, ax, nbx), qplane(nqy, j, ay, nby)),
                              fmaxf(qplane(nqz, j, az, nbz), 0.0f));
        const float f = fminf(fminf(qplane(fqx, j, ax, fbx), qplane(fqy, j, ay, fby)), qplane(fqz, j, az, fbz)) *
                        kFarScale;
        tn[j] = n;
        hh[j] = n <= fminf(f, tcull);   // f is never NaN here (flat directions take the float boxes)
    }
    t0 = tn[0];
    t1 = tn[1];
    t2 = tn[2];
    t3 = tn[3];
    h0 = hh[0];
    h1 = hh[1];
    h2 = hh[2];
    h3 = hh[3];
}

constexpr int kLeafQ = 512;                    // ring entries per wave
constexpr uint32_t kFlushPerWalker = 4;        // queued tests per walking lane that trigger a partial block
constexpr uint32_t kQTriBits = 26;             // triangle index bits of an entry; the lane sits above
constexpr uint32_t kQTriMask = (1u << kQTriBits) - 1u;
static_assert(kLeafQ >= 2 * kTraceBlock + kTraceBlock * kMaxLeaf, "one step appends at most 64 leaves");
static_assert((kLeafQ & (kLeafQ - 1)) == 0, "the ring wraps by masking");

// Position of the r-th set bit (r counted from 0) of m, which has more than r set bits.
__device__ __forceinline__ int nth_set_bit(unsigned long long m, uint32_t r) {
    int base = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const uint32_t c = (uint32_t)__popcll(m & ((1ull << w) - 1ull));
        const bool up = r >= c;
        r = up ? r - c : r;
        m = up ? m >> w : m;
        base += up ? w : 0;
    }
    return base;
}

__device__ __forceinline__ unsigned long long hit_key(float t, uint32_t p) {
    return ((unsigned long long)__float_as_uint(t) << 32) | p;
}

template <bool STATS, bool MULTI, bool QN>
__global__ __launch_bounds__(kTraceBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_trace_q(DevScene sc, TraceArgs a, uint32_t gthreads,
                                                         const StepJob* jobs, int njobs) {
    __shared__ int32_t stk[kStackLds][kTraceBlock];
    __shared__ uint32_t queue[kLeafQ];
    __shared__ unsigned long long bestk[kTraceBlock];
    const int lane = threadIdx.x;
    const uint32_t gtid = blockIdx.x * kTraceBlock + lane;
    // merged launches (MULTI) never use compacted or permuted queues
    const uint32_t* const fillp = MULTI ? nullptr : a.fill;
    const uint32_t* const permp = MULTI ? nullptr : a.perm;
    const bool regions = fillp && !permp;
    const uint32_t n = MULTI ? a.n : launch_rays(a);
    uint32_t ncq = fillp ? fillp[(blockIdx.x % kRayCounters) * kCounterStride] : 0u;   // rays of counter cq
    const unsigned long long lt = (1ull << lane) - 1ull;
    // a shadow ray keeps hits at t < kShadowTmax; prim ids are below INT32_MAX
    const unsigned long long key0 = a.shadow ? hit_key(kShadowTmax, 0u) : hit_key(INFINITY, (uint32_t)INT32_MAX);
    unsigned long long nv = 0, nt = 0;
    uint32_t traced = 0;
    bool have = false;               // the lane walks a ray (its own, or part of another lane's)
    bool own = false;                // the lane holds a claimed ray whose hit it writes
    int owner = lane;                // the lane whose ray this lane walks
    bool exhausted = false;          // wave-uniform: the queue of rays is used up
    uint32_t cq = blockIdx.x % kRayCounters;   // wave-uniform: the counter claimed from
    int tries = 0;
    uint32_t qhead = 0, qtail = 0;   // wave-uniform ring positions: tested up to qhead, filled up to qtail
    uint32_t last = 0;               // position of the lane's last entry; pending while qhead <= last
    uint32_t oi = 0;
    V3 o = mk3(0.f, 0.f, 0.f), inv = o;
    RayPre rp{};
    int32_t excl = -1, node = kDone;
    float tcull = INFINITY;
    int sp = 0, novf = 0;
    const float4* nodes4 = QN ? sc.nodes4q : sc.nodes4;
    const float4* nodesf = sc.nodes4;   // float boxes: rays with a direction component below 2^-64
    bool flat = false;
    const float4* btris = sc.btris;
    int32_t* oprim = a.out_prim;
    float* ot = a.out_t;
    // One step of the wave.  Main phase (DRAIN false, while the queue lasts): idle lanes take
    // new rays, every lane walks its own ray.  Drain (DRAIN true, the queue used up): free
    // lanes take pending subtrees of the others (below).  Returns false when the drain ends.
    auto step = [&](auto drain_tag) -> bool {
        constexpr bool DRAIN = decltype(drain_tag)::value;
        // ---- refill idle lanes with the next rays of the queue
        const unsigned long long idle = __ballot(!have);
        // (merged launches run only this instantiation: no claims once the counters are used up)
        if (!DRAIN && !exhausted && idle != 0 && (__popcll(idle) >= a.refill || idle == ~0ull)) {
            // a launch with few rays spreads them over every wave (latency hiding) instead of
            // filling the first waves' 64 lanes and leaving the others without work
            const uint32_t share = n / gridDim.x + 1u;
            const uint32_t nidle = (uint32_t)__popcll(idle);
            const uint32_t need = nidle < share ? nidle : share;
            const uint32_t c = cq;
            const uint32_t nc = ncq;
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(a.work + c * kCounterStride, need);
            base = __shfl(base, 0);
            if (claim_index(regions, a.region, base + need, c, n, nc) == kNoClaim) {   // this counter has no rays left
                if (++tries == kRayCounters) exhausted = true;
                cq = (cq + 1u) % kRayCounters;
                ncq = fillp ? fillp[cq * kCounterStride] : 0u;
            }
            const uint32_t rank = (uint32_t)__popcll(idle & lt);
            if (!have && rank < need) {
                // a launch with fewer rays than lanes is latency-bound: each wave's rays are
                // spread over the queue (a stripe transpose, a bijection on the rays of the
                // counter, or of the launch), so that neighbouring rays, alike in a reuse group
                // or in key order, do not all land in one wave and leave it last to finish
                uint32_t v = base + rank;
                const bool spread = !MULTI && n < gthreads;
                if (spread && regions && v < nc) {
                    const uint32_t sq = nc / kSpread, sr = nc % kSpread, st = v % kSpread, sp = v / kSpread;
                    v = st * sq + (st < sr ? st : sr) + sp;
                }
                uint64_t i64 = claim_index(regions, a.region, v, c, n, nc);
                if (spread && !regions && i64 != kNoClaim) {
                    const uint32_t w = (uint32_t)i64;
                    const uint32_t sq = n / kSpread, sr = n % kSpread, st = w % kSpread, sp = w / kSpread;
                    i64 = st * sq + (st < sr ? st : sr) + sp;
                }
                const uint32_t i = (uint32_t)i64;
                if (i64 != kNoClaim) {
                    const float4* rays = a.rays;
                    uint32_t li = permp ? permp[i] : i;   // sorted launches read the rays through the sort's permutation
                    if constexpr (MULTI) {
                        int lo = 0, hi = njobs - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (jobs[mid].ray_start <= i) lo = mid; else hi = mid - 1;
                        }
                        const StepJob& J = jobs[lo];
                        li = i - J.ray_start;
                        rays = J.q_in;
                        nodes4 = QN ? J.sc.nodes4q : J.sc.nodes4;
                        nodesf = J.sc.nodes4;
                        btris = J.sc.btris;
                        oprim = J.trace_prim;
                        ot = J.trace_t;
                    }
                    // set up without a branch on the pixel word, so that the three loads of
                    // the ray are issued together (one wait, not two in a row)
                    const float4 r0 = rays[2 * (size_t)li], r1 = rays[2 * (size_t)li + 1];
                    const uint32_t pix = __float_as_uint(r1.w);
                    o = xyz(r0);
                    const V3 d = xyz(r1);
                    excl = __float_as_int(r0.w);
                    inv = mk3(1.0f / d.x, 1.0f / d.y, 1.0f / d.z);
                    rp = prepare(o, d);
                    flat = !(fabsf(inv.x) <= kQMaxInv && fabsf(inv.y) <= kQMaxInv && fabsf(inv.z) <= kQMaxInv);
                    bestk[lane] = key0;
                    tcull = a.shadow ? kShadowTmax * kCullScale : INFINITY;
                    sp = 0;
                    novf = 0;
                    node = 0;
                    last = qhead - 1u;
                    oi = a.by_pixel ? pix : li;
                    have = !(a.by_pixel || a.skip_empty) || pix != kNoRay;   // else the lane stays idle
                }
            }
        }
        // ---- once the queue is used up, free lanes take pending subtrees of the wave's other
        // rays (the drain): a walking lane gives the top entry of its stack to a free lane,
        // which walks that subtree with a copy of the ray and folds its hits into the owner's
        // key; the owner writes the hit once no lane walks any part of its ray
        if constexpr (DRAIN) {
            const unsigned long long fm = idle;
            const unsigned long long dm = __ballot(have && node != kDone && sp > 0);
            if (fm != 0 && dm != 0) {
                const uint32_t nf = (uint32_t)__popcll(fm), nd = (uint32_t)__popcll(dm);
                const uint32_t np = nf < nd ? nf : nd;
                const uint32_t rf = (uint32_t)__popcll(fm & lt), rd = (uint32_t)__popcll(dm & lt);
                const bool helper = !have && rf < np;
                const bool donor = ((dm >> lane) & 1ull) && rd < np;
                const int d = nth_set_bit(dm, helper ? rf : 0u);
                const int32_t give = donor ? stk[sp - 1][lane] : 0;
                if (donor) --sp;
                // the helper copies the donor's ray, field by field
                float v;
                v = __shfl(o.x, d); o.x = helper ? v : o.x;
                v = __shfl(o.y, d); o.y = helper ? v : o.y;
                v = __shfl(o.z, d); o.z = helper ? v : o.z;
                v = __shfl(inv.x, d); inv.x = helper ? v : inv.x;
                v = __shfl(inv.y, d); inv.y = helper ? v : inv.y;
                v = __shfl(inv.z, d); inv.z = helper ? v : inv.z;
                v = __shfl(rp.ox, d); rp.ox = helper ? v : rp.ox;
                v = __shfl(rp.oy, d); rp.oy = helper ? v : rp.oy;
                v = __shfl(rp.oz, d); rp.oz = helper ? v : rp.oz;
                v = __shfl(rp.sx, d); rp.sx = helper ? v : rp.sx;
                v = __shfl(rp.sy, d); rp.sy = helper ? v : rp.sy;
                v = __shfl(rp.sz, d); rp.sz = helper ? v : rp.sz;
                v = __shfl(tcull, d); tcull = helper ? v : tcull;
                int u;
                u = __shfl(rp.kx | (rp.ky << 2) | (rp.kz << 4) | ((int)flat << 6), d);
                if (helper) {
                    rp.kx = u & 3;
                    rp.ky = (u >> 2) & 3;
                    rp.kz = (u >> 4) & 3;
                    flat = (u >> 6) != 0;
                }
                u = __shfl(excl, d); excl = helper ? u : excl;
                u = __shfl(owner, d); owner = helper ? u : owner;
                u = __shfl(give, d); node = helper ? u : node;
                if constexpr (MULTI) {
                    const float4* pp[3] = {nodes4, nodesf, btris};
                    for (int j = 0; j < 3; ++j) {
                        const uint64_t w = (uint64_t)(uintptr_t)pp[j];
                        const uint32_t lo = (uint32_t)__shfl((uint32_t)w, d), hi = (uint32_t)__shfl((uint32_t)(w >> 32), d);
                        pp[j] = helper ? (const float4*)(uintptr_t)(((uint64_t)hi << 32) | lo) : pp[j];
                    }
                    nodes4 = pp[0];
                    nodesf = pp[1];
                    btris = pp[2];
                }
                if (helper) {
                    sp = 0;
                    novf = 0;
                    last = qhead - 1u;
                    have = true;
                }
            }
        }
        if (__ballot(have) == 0) {
            if constexpr (DRAIN) {
                // nothing walks: every owner's result is complete
                if (own) {
                    const unsigned long long k = bestk[lane];
                    oprim[oi] = k == key0 ? -1 : (int32_t)(uint32_t)k;
                    ot[oi] = __uint_as_float((uint32_t)(k >> 32));
                    ++traced;
                    own = false;
                }
                return false;
            }
            return !exhausted;
        }
        // ---- a lane on a leaf queues its triangles and takes the next node
        const bool on_leaf = have && node < 0 && node != kDone;
        const uint32_t code = ~(uint32_t)node;
        const uint32_t cnt = on_leaf ? (code & 7u) + 1u : 0u;
        uint32_t off = 0, total = 0;
#pragma unroll
        for (int bit = 0; bit < kLeafCountBits; ++bit) {
            const unsigned long long qb = __ballot((cnt >> bit) & 1u);
            off += (uint32_t)__popcll(qb & lt) << bit;
            total += (uint32_t)__popcll(qb) << bit;
        }
        if (on_leaf) {
            // a leaf holds at most kMaxLeaf triangles: one predicated store each
            const uint32_t tag = ((uint32_t)lane << kQTriBits) | (code >> 3);
            const uint32_t pos = qtail + off;
#pragma unroll
            for (uint32_t j = 0; j < (uint32_t)kMaxLeaf; ++j)
                if (j < cnt) queue[(pos + j) & (uint32_t)(kLeafQ - 1)] = tag + j;
            last = qtail + off + cnt - 1u;
            if (sp == 0 && novf > 0) {
                const int m = novf < kStackLds / 2 ? novf : kStackLds / 2;
                for (int e = 0; e < m; ++e) stk[e][lane] = a.ovf[(size_t)(novf - m + e) * gthreads + gtid];
                novf -= m;
                sp = m;
            }
            node = sp > 0 ? stk[--sp][lane] : kDone;
        }
        qtail += total;
        // ---- one inner node: the nearest hit child next, the other hits pushed far to near
        if (have && node >= 0) {
            bool h0, h1, h2, h3;
            float a0, a1, a2, a3;
            // the codes are the same in both node arrays: read them from the array the lane
            // walks before any branch (one 16-byte load, not one per path)
            const float4 cc = QN ? nodes4[4 * (size_t)node + 1] : nodes4[8 * (size_t)node + 6];
            if (QN && !flat) {
                const float4* nd = nodes4 + 4 * (size_t)node;
                const float4 g = nd[0], q0 = nd[2], q1 = nd[3];
                qslab4(g, q0, q1, o, inv, tcull, a0, a1, a2, a3, h0, h1, h2, h3);
            } else {
                const float4* nd = (QN ? nodesf : nodes4) + 8 * (size_t)node;
                const float4 lx = nd[0], hx = nd[1], ly = nd[2], hy = nd[3], lz = nd[4], hz = nd[5];
                a0 = slab(lx.x, hx.x, ly.x, hy.x, lz.x, hz.x, o, inv, tcull, h0);
                a1 = slab(lx.y, hx.y, ly.y, hy.y, lz.y, hz.y, o, inv, tcull, h1);
                a2 = slab(lx.z, hx.z, ly.z, hy.z, lz.z, hz.z, o, inv, tcull, h2);
                a3 = slab(lx.w, hx.w, ly.w, hy.w, lz.w, hz.w, o, inv, tcull, h3);
            }
            if (STATS) {
                    ++nv;
                    if (a.touched) a.touched[node] |= (uint8_t)a.touch_bit;
                }
            int32_t k0 = __float_as_int(cc.x), k1 = __float_as_int(cc.y), k2 = __float_as_int(cc.z),
                    k3 = __float_as_int(cc.w);
            h0 = h0 && k0 != kEmpty;
            h1 = h1 && k1 != kEmpty;
            h2 = h2 && k2 != kEmpty;
            h3 = h3 && k3 != kEmpty;
            const int nh = (int)h0 + (int)h1 + (int)h2 + (int)h3;
            a0 = h0 ? a0 : INFINITY;
            a1 = h1 ? a1 : INFINITY;
            a2 = h2 ? a2 : INFINITY;
            a3 = h3 ? a3 : INFINITY;
            cswap(a0, k0, a1, k1);
            cswap(a2, k2, a3, k3);
            cswap(a0, k0, a2, k2);
            cswap(a1, k1, a3, k3);
            cswap(a1, k1, a2, k2);
            if (nh == 0) {
                if (sp == 0 && novf > 0) {
                    const int m = novf < kStackLds / 2 ? novf : kStackLds / 2;
                    for (int e = 0; e < m; ++e) stk[e][lane] = a.ovf[(size_t)(novf - m + e) * gthreads + gtid];
                    novf -= m;
                    sp = m;
                }
                node = sp > 0 ? stk[--sp][lane] : kDone;
            } else {
                node = k0;
                if (sp + nh - 1 > kStackLds) {
                    if (novf + kStackLds / 2 > kStackOvf) {
                        node = kDone;   // unreachable within the depth bound of wide trees
                        sp = 0;
                        novf = 0;
                    } else {
                        for (int e = 0; e < kStackLds / 2; ++e)
                            a.ovf[(size_t)(novf + e) * gthreads + gtid] = stk[e][lane];
                        for (int e = 0; e < kStackLds / 2; ++e) stk[e][lane] = stk[e + kStackLds / 2][lane];
                        novf += kStackLds / 2;
                        sp -= kStackLds / 2;
                    }
                }
                if (node != kDone) {
                    if (nh == 4) stk[sp++][lane] = k3;
                    if (nh >= 3) stk[sp++][lane] = k2;
                    if (nh >= 2) stk[sp++][lane] = k1;
                }
            }
        }
        // ---- queued triangle tests: every whole block of 64, and a partial one when lanes wait on it
        const bool waiting = have && node == kDone && (int32_t)(last - qhead) >= 0;
        const int walking = __popcll(__ballot(have && node != kDone));
        // a partial block is tested when lanes wait on it, and when the queue holds kFlushPerWalker
        // entries per walking lane: a wave with few walking rays would otherwise fill it slowly
        // and walk on without culling against the hits it has queued
        bool partial = qtail != qhead && (walking == 0 || __popcll(__ballot(waiting)) > a.leaf_gate ||
                                          qtail - qhead >= kFlushPerWalker * (uint32_t)walking);
        if (qtail - qhead >= (uint32_t)kTraceBlock || partial) {
            const int perm = rp.kx | (rp.ky << 2) | (rp.kz << 4);
            __syncthreads();   // the entries written above are visible to every lane
            do {
                const uint32_t p = qhead + (uint32_t)lane;
                const bool valid = (int32_t)(qtail - p) > 0;
                const uint32_t e = valid ? queue[p & (uint32_t)(kLeafQ - 1)] : 0u;
                const int src = (int)(e >> kQTriBits);
                RayPre r;
                r.ox = __shfl(rp.ox, src);
                r.oy = __shfl(rp.oy, src);
                r.oz = __shfl(rp.oz, src);
                r.sx = __shfl(rp.sx, src);
                r.sy = __shfl(rp.sy, src);
                r.sz = __shfl(rp.sz, src);
                const int qperm = __shfl(perm, src);
                r.kx = qperm & 3;
                r.ky = (qperm >> 2) & 3;
                r.kz = (qperm >> 4) & 3;
                const int32_t qexcl = __shfl(excl, src);
                int qown = src;   // the key the hit folds into: the owner of the walking lane's ray
                if constexpr (DRAIN) qown = __shfl(owner, src);
                const float4* qtris = btris;
                if constexpr (MULTI) {
                    const uint64_t bp = (uint64_t)(uintptr_t)btris;
                    const uint32_t lo = __shfl((uint32_t)bp, src), hi = __shfl((uint32_t)(bp >> 32), src);
                    qtris = (const float4*)(uintptr_t)(((uint64_t)hi << 32) | lo);
                }
                if (valid) {
                    const float4* tp = qtris + 3 * (size_t)(e & kQTriMask);
                    const float4 p0 = tp[0], p1 = tp[1], p2 = tp[2];
                    const int32_t id = __float_as_int(p0.w);
                    if (STATS) {
                        ++nt;
                        if (a.touched) a.touched[a.touch_tri + (e & kQTriMask)] |= (uint8_t)a.touch_bit;
                    }
                    float th;
                    if (tri_test(r, p0, p1, p2, th) && id != qexcl) atomicMin(&bestk[qown], hit_key(th, (uint32_t)id));
                }
                const uint32_t left = qtail - qhead;
                qhead += left < (uint32_t)kTraceBlock ? left : (uint32_t)kTraceBlock;
                partial = false;
            } while (qtail - qhead >= (uint32_t)kTraceBlock);
            __syncthreads();   // the minima are complete; the ring slots are free again
            if (have) {
                const unsigned long long k = bestk[DRAIN ? owner : lane];
                tcull = __uint_as_float((uint32_t)(k >> 32)) * kCullScale;
                if (a.shadow && k != key0) {   // blocked: the shadow ray is answered
                    node = kDone;
                    sp = 0;
                    novf = 0;
                }
            }
        }
        // ---- walks that are finished and whose tests are all done; then the hits of owners
        // whose ray no lane walks any more
        if constexpr (!DRAIN) {
            if (have && node == kDone && (int32_t)(last - qhead) < 0) {
                const unsigned long long k = bestk[lane];
                const uint32_t kp = (uint32_t)k;
                oprim[oi] = k == key0 ? -1 : (int32_t)kp;
                ot[oi] = __uint_as_float((uint32_t)(k >> 32));
                ++traced;
                have = false;
            }
        } else {
            if (have && node == kDone && (int32_t)(last - qhead) < 0) have = false;
            // owners some lane still walks for (wave-uniform)
            unsigned long long walked = __ballot(have && owner == lane);
            if (__ballot(own && !have) != 0) {
                unsigned long long hl = __ballot(have && owner != lane);
                while (hl != 0) {
                    const int h = __ffsll((long long)hl) - 1;
                    hl &= hl - 1ull;
                    walked |= 1ull << __builtin_amdgcn_readlane(owner, h);
                }
            }
            if (own && !have && ((walked >> lane) & 1ull) == 0) {
                const unsigned long long k = bestk[lane];
                const uint32_t kp = (uint32_t)k;
                oprim[oi] = k == key0 ? -1 : (int32_t)kp;
                ot[oi] = __uint_as_float((uint32_t)(k >> 32));
                ++traced;
                own = false;
            }
        }
        return true;
    };
    if constexpr (MULTI) {
        // merged launches of a batch: their many small jobs leave little drain, and the
        // copies of the per-lane job pointers a donation needs cost registers: no donation
        while (step(std::false_type{})) {
        }
    } else {
        while (!exhausted) step(std::false_type{});
        // the drain: every lane that walks owns its ray
        own = have;
        owner = lane;
        while (step(std::true_type{})) {
        }
    }
    unsigned int tsum = traced;
    for (int off = 32; off > 0; off >>= 1) tsum += __shfl_down(tsum, off);
    if (a.partial && lane == 0) a.partial[blockIdx.x] = tsum;
    if (STATS) {
        for (int off = 32; off > 0; off >>= 1) {
            nv += __shfl_down(nv, off);
            nt += __shfl_down(nt, off);
        }
        if (lane == 0) {
            atomicAdd(a.stats, nv);
            atomicAdd(a.stats + 1, nt);
        }
    }
}

// ------------------------------------------------------------------ slot <-> pixel mapping
struct SlotPix {
    int x, y, tin, i;
    bool inside;
};
__device__ __forceinline__ SlotPix slot_pixel(const Frame& f, uint32_t block, int l) {
    SlotPix r;
    const int stx = (int)(block % (uint32_t)f.nstx), sty = (int)(block / (uint32_t)f.nstx);
    r.tin = l / f.WH;
    r.i = l - r.tin * f.WH;
    const int tcol = r.tin % f.cols, trow = r.tin / f.cols;
    r.x = stx * f.SW + tcol * f.W + (r.i % f.W);
    r.y = sty * f.SH + trow * f.H + (r.i / f.W);
    r.inside = r.x < f.w && r.y < f.h;
    return r;
}

__device__ __forceinline__ void raygen_body(const Frame& f, int s, uint32_t blk, float4* q, float4* state,
                                            float4* rays_out) {
    const int l = threadIdx.x;
    const uint32_t p = blk * (uint32_t)f.TS + (uint32_t)l;
    const SlotPix sp = slot_pixel(f, blk, l);
    float4 r0 = make_float4(0.f, 0.f, 0.f, __int_as_float(-1)), r1 = make_float4(0.f, 0.f, 0.f, __uint_as_float(kNoRay));
    float4 s0 = make_float4(1.f, 1.f, 1.f, __uint_as_float(0u)), s1 = make_float4(0.f, 0.f, 0.f, __uint_as_float(p));
    if (sp.inside) {
        const uint32_t pix = (uint32_t)sp.y * (uint32_t)f.w + (uint32_t)sp.x;
        const U64x4 rnd = philox(pix, (uint64_t)s, 0, 0, f.seed);
        const float u0 = unit01(rnd.v[0]), u1 = unit01(rnd.v[1]);
        const float px = ((float)sp.x + u0) / (float)f.w;
        const float py = ((float)sp.y + u1) / (float)f.h;
        const float fx = (2.0f * px - 1.0f) * f.thx;
        const float fy = (1.0f - 2.0f * py) * f.th;
        V3 d = mk3((fx * f.cright[0] + fy * f.cup[0]) + f.cfwd[0], (fx * f.cright[1] + fy * f.cup[1]) + f.cfwd[1],
                   (fx * f.cright[2] + fy * f.cup[2]) + f.cfwd[2]);
        d = unit3(d);
        r0 = make_float4(f.cpos[0], f.cpos[1], f.cpos[2], __int_as_float(-1));
        r1 = make_float4(d.x, d.y, d.z, __uint_as_float(pix));
        s0.w = __uint_as_float(1u);
        if (rays_out) {
            const size_t at = 2 * ((size_t)s * f.w * f.h + pix);
            rays_out[at] = r0;
            rays_out[at + 1] = r1;
        }
    }
    q[2 * (size_t)p] = r0;
    q[2 * (size_t)p + 1] = r1;
    state[2 * (size_t)p] = s0;
    state[2 * (size_t)p + 1] = s1;
    if (f.live && l == 0) f.live[blk] = 1u;
}

__global__ __launch_bounds__(1024) void k_raygen(Frame f, int s, float4* q, float4* state, float4* rays_out) {
    raygen_body(f, s, blockIdx.x, q, state, rays_out);
}

// workgroup -> job of a merged launch (the table is sorted by block_start)
__device__ __forceinline__ int job_of_block(const StepJob* jobs, int njobs, uint32_t blk) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].block_start <= blk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(1024) void k_raygen_multi(const StepJob* jobs, int njobs) {
    const int j = job_of_block(jobs, njobs, blockIdx.x);
    const StepJob& J = jobs[j];
    if (!J.do_raygen) return;
    raygen_body(J.f, J.s, blockIdx.x - J.block_start, J.q_out_raygen, J.state, nullptr);
}

// ------------------------------------------------------------------ reordering keys (sorted modes)
// nb-bit quantization of x over [lo, lo + ext]: floor(((x - lo) / ext) * 2^nb), clamped
__device__ __forceinline__ uint32_t qbits(float x, float lo, float ext, int nb) {
    if (!(ext > 0.0f)) return 0u;
    const float top = (float)(1u << nb);
    const float f = ((x - lo) / ext) * top;
    if (!(f > 0.0f)) return 0u;
    if (f >= top - 1.0f) return (1u << nb) - 1u;
    return (uint32_t)f;
}

// 30-bit reordering key of a live ray for a sorted mode (bits interleaved most significant first)
__device__ __forceinline__ uint32_t ray_key(const DevScene& sc, float4 r0, float4 r1, int kind) {
    const float ex = sc.hi[0] - sc.lo[0], ey = sc.hi[1] - sc.lo[1], ez = sc.hi[2] - sc.lo[2];
    uint32_t key = 0;
    if (kind == PT_MODE_SORTED_ORIGIN) {
        const uint32_t qc[3] = {qbits(r0.x, sc.lo[0], ex, 10), qbits(r0.y, sc.lo[1], ey, 10),
                                qbits(r0.z, sc.lo[2], ez, 10)};
#pragma unroll
        for (int bit = 9; bit >= 0; --bit)
#pragma unroll
            for (int c = 0; c < 3; ++c) key = (key << 1) | ((qc[c] >> bit) & 1u);
    } else if (kind == PT_MODE_SORTED_REIS) {
        const uint32_t qo[3] = {qbits(r0.x, sc.lo[0], ex, 6), qbits(r0.y, sc.lo[1], ey, 6),
                                qbits(r0.z, sc.lo[2], ez, 6)};
        const uint32_t qd[3] = {qbits(r1.x, -1.0f, 2.0f, 4), qbits(r1.y, -1.0f, 2.0f, 4),
                                qbits(r1.z, -1.0f, 2.0f, 4)};
#pragma unroll
        for (int bit = 5; bit >= 0; --bit)
#pragma unroll
            for (int c = 0; c < 3; ++c) key = (key << 1) | ((qo[c] >> bit) & 1u);
#pragma unroll
        for (int bit = 3; bit >= 0; --bit)
#pragma unroll
            for (int c = 0; c < 3; ++c) key = (key << 1) | ((qd[c] >> bit) & 1u);
    } else {
        uint32_t qc[6];
        if (kind == PT_MODE_SORTED_AILA) {
            qc[3] = qbits(r1.x, -1.0f, 2.0f, 5);
            qc[4] = qbits(r1.y, -1.0f, 2.0f, 5);
            qc[5] = qbits(r1.z, -1.0f, 2.0f, 5);
        } else {   // TwoPoint: the point at a fixed length of 0.25 x the largest extent
            float mx = ex;
            if (ey > mx) mx = ey;
            if (ez > mx) mx = ez;
            const float len = 0.25f * mx;
            qc[3] = qbits(r0.x + len * r1.x, sc.lo[0], ex, 5);
            qc[4] = qbits(r0.y + len * r1.y, sc.lo[1], ey, 5);
            qc[5] = qbits(r0.z + len * r1.z, sc.lo[2], ez, 5);
        }
        qc[0] = qbits(r0.x, sc.lo[0], ex, 5);
        qc[1] = qbits(r0.y, sc.lo[1], ey, 5);
        qc[2] = qbits(r0.z, sc.lo[2], ez, 5);
#pragma unroll
        for (int bit = 4; bit >= 0; --bit)
#pragma unroll
            for (int c = 0; c < 6; ++c) key = (key << 1) | ((qc[c] >> bit) & 1u);
    }
    return key;
}

// ------------------------------------------------------------------ shade + next direction
// One workgroup = one super tile (whole reuse tiles), one thread per slot.
__device__ __forceinline__ void shade_body(const DevScene& sc, const Frame& f, int b, int s, uint32_t blk,
                                           const float4* __restrict__ q_in, float4* __restrict__ q_out,
                                           float4* state, int32_t* hit_prim, float* hit_t, float* radiance,
                                           float4* rays_out, float4* shadow_rays, float4* shadow_light, float* lds,
                                           uint32_t* fill, uint32_t* keys_out, float4* debug) {
    // group exchange in LDS, TS entries each: own tangent exit, tree sums, info bits, min active slot
    const int TS = f.TS;
    float* sq0 = lds;
    float* sq1 = lds + TS;
    float* sq2 = lds + 2 * TS;
    float* ss0 = lds + 3 * TS;
    float* ss1 = lds + 4 * TS;
    float* ss2 = lds + 5 * TS;
    int* sinfo = (int*)(lds + 6 * TS);
    int* srep = (int*)(lds + 7 * TS);
    const int l = threadIdx.x;
    const uint32_t p = blk * (uint32_t)f.TS + (uint32_t)l;
    const SlotPix spx = slot_pixel(f, blk, l);
    const uint32_t pix = spx.inside ? (uint32_t)spx.y * (uint32_t)f.w + (uint32_t)spx.x : 0u;
    float4 s0 = state[2 * (size_t)p], s1 = state[2 * (size_t)p + 1];
    float T[3] = {s0.x, s0.y, s0.z}, L[3] = {s1.x, s1.y, s1.z};
    const bool alive_in = (__float_as_uint(s0.w) & 1u) != 0;
    const bool nee_prev = (__float_as_uint(s0.w) & 2u) != 0;   // the ray left a Lambert point with NEE
    bool alive = alive_in;
    const uint32_t qpos = __float_as_uint(s1.w);
    const size_t plane = (size_t)f.w * (size_t)f.h;
    const size_t hb = ((size_t)b * f.spp + s) * plane;
    if (f.live && f.live[blk] == 0u) {
        // every path of the workgroup is over (its flag, from the last bounce, is uniform):
        // only the outputs that every slot gets are written (the empty shadow rays, the
        // debug record, and the dead entries of a plain queue, at the slots themselves: the
        // group shuffle permutes the workgroup's slots)
        if (shadow_rays) {
            shadow_rays[2 * (size_t)p] = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
            shadow_rays[2 * (size_t)p + 1] = make_float4(0.f, 0.f, 0.f, __uint_as_float(kNoRay));
            shadow_light[p] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        if (debug && b < f.B && spx.inside)
            debug[((size_t)b * f.spp + s) * plane + pix] = make_float4(0.f, 0.f, 0.f, __uint_as_float(0u));
        if (!fill && b < f.B) {
            q_out[2 * (size_t)p] = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
            q_out[2 * (size_t)p + 1] = make_float4(0.f, 0.f, 0.f, __uint_as_float(kNoRay));
        }
        return;
    }
    // The shading below is straight-line code: every lane evaluates every candidate
    // exit and the results are selected by material kind.  (A divergent three-way
    // branch here was miscompiled: registers live into the last branch were reused
    // by the others.)  The arithmetic of each candidate is unchanged.
    int32_t prim = -1;
    float t = 0.0f;
    if (alive_in) {
        prim = hit_prim[hb + pix];
        t = hit_t[hb + pix];
    }
    // a path that is already over reads no ray and keeps its state as it is: later bounces
    // read only its cleared alive bit, and the next sample's ray generation rewrites it
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0;
    if (alive_in) {
        r0 = q_in[2 * (size_t)qpos];
        r1 = q_in[2 * (size_t)qpos + 1];
    }
    const V3 o = xyz(r0), d = xyz(r1);
    const bool hit = alive_in && prim >= 0;
    pt_material m;
    m.kind = 0;
    for (int c = 0; c < 3; ++c) {
        m.albedo[c] = 0.0f;
        m.emission[c] = 0.0f;
    }
    m.alpha = 0.0f;
    float4 tv0 = make_float4(0.f, 0.f, 0.f, 0.f), tv1 = tv0, tv2 = tv0;
    if (hit) {
        m = sc.mats[sc.tri_mat[prim]];
        const float4* tp = sc.otris + 3 * (size_t)prim;
        tv0 = tp[0];
        tv1 = tp[1];
        tv2 = tp[2];
    }
    // emission that next-event estimation already counted at the previous Lambert point is skipped
    const bool add_le = alive_in && !(hit && nee_prev);
    for (int c = 0; c < 3; ++c) {
        const float le = hit ? m.emission[c] : sc.env[c];
        L[c] = add_le ? L[c] + T[c] * le : L[c];
    }
    const bool absorb = m.albedo[0] == 0.0f && m.albedo[1] == 0.0f && m.albedo[2] == 0.0f;
    const bool active = hit && b < f.B && !absorb;
    bool died = alive_in && !active;
    const uint32_t kind = m.kind;
    V3 n = unit3(cross3(sub3(xyz(tv1), xyz(tv0)), sub3(xyz(tv2), xyz(tv0))));
    if (dot3(n, d) > 0.0f) n = mk3(-n.x, -n.y, -n.z);
    const V3 hp = mk3(o.x + t * d.x, o.y + t * d.y, o.z + t * d.z);
    const V3 origin = push_off(hp, n);
    V3 tt, bt;
    frame_of(n, tt, bt);
    const V3 md = mk3(-d.x, -d.y, -d.z);
    const V3 wi = mk3(dot3(md, tt), dot3(md, bt), dot3(md, n));
    const U64x4 rnd = philox(pix, (uint64_t)s, (uint64_t)b, 0, f.seed);
    const float u2 = unit01(rnd.v[2]), u3 = unit01(rnd.v[3]);
    const V3 lam = cosine_dir(u2, u3);
    V3 gg;
    float gw[3];
    const bool g_ok = ggx_dir(wi, m.alpha, m.albedo, u2, u3, gg, gw);
    const V3 mir = mk3(-wi.x, -wi.y, wi.z);
    const V3 own = sel3(kind == 0, lam, sel3(kind == 1, gg, mir));
    const bool own_ok = active && (kind == 0 ? true : (kind == 1 ? g_ok : mir.z > 0.0f));
    float w3[3];
    for (int c = 0; c < 3; ++c) w3[c] = kind == 1 ? gw[c] : m.albedo[c];
    // next-event estimation: one emissive triangle and a point on it, a shadow ray from the
    // offset origin along D = point - origin; the light is added once the ray is unblocked
    float4 sh0 = make_float4(0.f, 0.f, 0.f, __int_as_float(-1)), sh1 = make_float4(0.f, 0.f, 0.f, __uint_as_float(kNoRay));
    float4 shl = make_float4(0.f, 0.f, 0.f, 0.f);
    if (shadow_rays && f.nee && active && kind == 0 && sc.nemit > 0) {
        const U64x4 rl = philox(pix, (uint64_t)s, (uint64_t)b, 2, f.seed);
        const uint32_t e = sc.emit[(uint32_t)(rl.v[0] % (uint64_t)sc.nemit)];
        const float u1 = unit01(rl.v[1]), uu2 = unit01(rl.v[2]);
        const float4* lp = sc.otris + 3 * (size_t)e;
        const V3 l0 = xyz(lp[0]), l1 = xyz(lp[1]), l2 = xyz(lp[2]);
        const float su = sqrtf(u1);
        const float b0 = 1.0f - su, b1 = uu2 * su;
        const float b2 = (1.0f - b0) - b1;
        const V3 lq = mk3((b0 * l0.x + b1 * l1.x) + b2 * l2.x, (b0 * l0.y + b1 * l1.y) + b2 * l2.y,
                          (b0 * l0.z + b1 * l1.z) + b2 * l2.z);
        const V3 D = sub3(lq, origin);
        const float cs = dot3(D, n);
        if (cs > 0.0f) {
            const V3 nl = cross3(sub3(l1, l0), sub3(l2, l0));
            const float cl = fabsf(dot3(D, nl));
            const float d2 = dot3(D, D);
            const float g = (cs * cl) / (d2 * d2);
            const float k = g * ((float)sc.nemit * (float)(1.0 / (2.0 * 3.14159265358979323846)));
            const pt_material& ml = sc.mats[sc.tri_mat[e]];
            shl = make_float4((T[0] * m.albedo[0]) * (ml.emission[0] * k), (T[1] * m.albedo[1]) * (ml.emission[1] * k),
                              (T[2] * m.albedo[2]) * (ml.emission[2] * k), 0.0f);
            sh0 = make_float4(origin.x, origin.y, origin.z, __int_as_float(prim));
            sh1 = make_float4(D.x, D.y, D.z, __uint_as_float(pix));
        }
    }
    if (shadow_rays) {
        shadow_rays[2 * (size_t)p] = sh0;
        shadow_rays[2 * (size_t)p + 1] = sh1;
        shadow_light[p] = shl;
    }
    V3 use = own;
    bool use_ok = own_ok;
    // per-ray record of the rules applied (pt_outputs.debug): active, material class, group
    // category, representative, reused, ray exists, shuffled slot
    uint32_t dfl = active ? (kDbgActive | ((uint32_t)kind << kDbgClassShift)) : 0u;
    bool use_world = false;   // direct reuse: the next direction is given in world space
    V3 wdir = mk3(0.f, 0.f, 0.f);
    uint32_t newpos = p;
    const bool world = f.mode == PT_MODE_REUSE_WORLD;
    const bool reuse = (f.mode == PT_MODE_REUSE || f.mode == PT_MODE_REUSE_PLAIN || world) && b < f.B &&
                       b + 1 <= f.reuse_max;
    if (reuse) {
        // interleaved grouping: shuffle screen-order numbers inside the tile (not in the
        // plain ablation, whose groups are consecutive screen-order pixels)
        uint32_t slot = 0;
        {
            const uint32_t tile = (uint32_t)(spx.y / f.H) * (uint32_t)f.ntx + (uint32_t)(spx.x / f.W);
            const U64x4 rnd = philox(tile, (uint64_t)s, f.frame_groups ? 0u : (uint64_t)b, 1, f.seed);
            uint32_t ma = 1, mc = 0;
            if (f.WH > 1 && f.mode != PT_MODE_REUSE_PLAIN) {
                ma = 2u * (uint32_t)(rnd.v[0] & (uint64_t)(f.WH / 2 - 1)) + 1u;
                mc = (uint32_t)(rnd.v[1] & (uint64_t)(f.WH - 1));
            }
            slot = (ma * (uint32_t)spx.i + mc) & (uint32_t)(f.WH - 1);
        }
        const int e = spx.tin * f.WH + (int)slot;
        const bool gl_exit = active && kind != 0 && own_ok;
        // direct reuse shares the own exit in world space; x = 2 marks a sample that died
        const V3 ow = tangent_to_world(own, tt, bt, n);
        const V3 shared = sel3(world, sel3(own_ok, ow, mk3(2.0f, 0.0f, 0.0f)), own);
        sq0[e] = shared.x;
        sq1[e] = shared.y;
        sq2[e] = shared.z;
        ss0[e] = gl_exit ? own.x : 0.0f;
        ss1[e] = gl_exit ? own.y : 0.0f;
        ss2[e] = gl_exit ? own.z : 0.0f;
        sinfo[e] = (active ? (kind == 0 ? 1 : 2) : 0) | (gl_exit ? 4 : 0);
        srep[e] = active ? (int)slot : 0x7FFFFFFF;
        __syncthreads();
        // pairwise tree over each group's K consecutive entries (in place, stride doubling)
        for (int stride = 1; stride < f.K; stride <<= 1) {
            if ((l & (2 * stride - 1)) == 0) {
                ss0[l] = ss0[l] + ss0[l + stride];
                ss1[l] = ss1[l] + ss1[l + stride];
                ss2[l] = ss2[l] + ss2[l + stride];
                sinfo[l] |= sinfo[l + stride];
                srep[l] = min(srep[l], srep[l + stride]);
            }
            __syncthreads();
        }
        const int root = spx.tin * f.WH + ((int)slot / f.K) * f.K;
        const int info = sinfo[root];
        const int rslot = srep[root] < f.WH ? srep[root] : 0;
        const int r = spx.tin * f.WH + rslot;
        // diffuse group: every member takes the representative's tangent direction
        const bool take_rep = !world && active && kind == 0 && !(info & 2);
        // hybrid group: diffuse members take the normalized sum of the glossy/specular exits
        const bool take_avg = !world && active && kind == 0 && (info & 2) && (info & 4);
        const V3 repq = mk3(sq0[r], sq1[r], sq2[r]);
        const V3 avgq = unit3(mk3(ss0[root], ss1[root], ss2[root]));
        use = sel3(take_rep, repq, sel3(take_avg, avgq, use));
        use_ok = (take_rep || take_avg) ? true : use_ok;
        // direct reuse: Lambert members other than the representative take its world
        // direction; a member below whose surface it points ends its path
        use_world = world && active && kind == 0 && srep[root] < f.WH && (int)slot != rslot && repq.x <= 1.5f;
        wdir = repq;
        use_ok = use_world ? dot3(repq, n) > 0.0f : use_ok;
        if (active) {
            dfl |= slot << kDbgSlotShift;
            if (!world) {
                const uint32_t cat = (info & 1) ? ((info & 2) ? 3u : 1u) : ((info & 2) ? 2u : 0u);
                dfl |= cat << kDbgCatShift;
                if (cat == 1u && (int)slot == rslot) dfl |= kDbgRep;
                if ((take_rep && (int)slot != rslot) || take_avg) dfl |= kDbgReused;
            } else {
                if (srep[root] < f.WH && (int)slot == rslot) dfl |= kDbgRep;
                if (use_world) dfl |= kDbgReused;
            }
        }
        newpos = blk * (uint32_t)TS + (uint32_t)e;
    }
    if (debug && b < f.B && spx.inside) {
        const V3 dq = sel3(use_world, wdir, use);
        debug[((size_t)b * f.spp + s) * plane + pix] =
            active ? make_float4(dq.x, dq.y, dq.z, __uint_as_float(dfl | (use_ok ? kDbgValid : 0u)))
                   : make_float4(0.f, 0.f, 0.f, __uint_as_float(0u));
    }
    if (fill && b < f.B) {
        // the compacted queue: the live rays of workgroup blk go, in their queue order (group by
        // group in reuse modes), to the next free places of region blk mod 8 (one counter per
        // region, one atomic per workgroup); the traversal's counter c hands out region c
        int* cf = (int*)(lds + (f.mode == PT_MODE_REUSE || f.mode == PT_MODE_REUSE_PLAIN || world ? 8 * TS : 0));
        int* cw = cf + TS;
        const bool live = active && use_ok;
        const int epos = (int)(newpos - blk * (uint32_t)TS);
        __syncthreads();
        cf[epos] = live ? 1 : 0;
        __syncthreads();
        const bool fl = cf[l] != 0;
        const unsigned long long bm = __ballot(fl);
        const int wv = l >> 6, ln = l & 63;
        const int pre = __popcll(bm & ((1ull << ln) - 1ull));
        if (ln == 0) cw[wv] = __popcll(bm);
        __syncthreads();
        if (l == 0) {
            int tot = 0;
            for (int w = 0; w < (TS + 63) / 64; ++w) {
                const int c = cw[w];
                cw[16 + w] = tot;
                tot += c;
            }
            cw[32] = tot > 0 ? (int)atomicAdd(fill + (blk & 7u) * (uint32_t)kCounterStride, (uint32_t)tot) : 0;
        }
        __syncthreads();
        cf[l] = cw[32] + cw[16 + wv] + pre;   // place of queue position l among the region's rays
        __syncthreads();
        newpos = live ? (blk & 7u) * f.region + (uint32_t)cf[epos] : p;
    }
    if (b < f.B) {
        float4 o0 = make_float4(0.f, 0.f, 0.f, __int_as_float(-1)), o1 = make_float4(0.f, 0.f, 0.f, __uint_as_float(kNoRay));
        if (active && use_ok) {
            const V3 nd = sel3(use_world, wdir, tangent_to_world(use, tt, bt, n));
            for (int c = 0; c < 3; ++c) T[c] = T[c] * w3[c];
            o0 = make_float4(origin.x, origin.y, origin.z, __int_as_float(prim));
            o1 = make_float4(nd.x, nd.y, nd.z, __uint_as_float(pix));
            if (rays_out) {
                const size_t at = 2 * (((size_t)(b + 1) * f.spp + s) * plane + pix);
                rays_out[at] = o0;
                rays_out[at + 1] = o1;
            }
        } else if (active) {
            died = true;
        }
        if (!fill || (active && use_ok)) {   // a compacted queue holds live rays only
            q_out[2 * (size_t)newpos] = o0;
            q_out[2 * (size_t)newpos + 1] = o1;
            // sorted modes: the ray's reordering key beside it (read by the sort, not the ray)
            if (keys_out && fill && active && use_ok) keys_out[newpos] = ray_key(sc, o0, o1, f.mode);
        }
    }
    if (died) {
        alive = false;
        float* rp = radiance + 3 * (size_t)pix;
        for (int c = 0; c < 3; ++c) {
            float v = s == 0 ? L[c] : rp[c] + L[c];
            if (s == f.spp - 1) v = v / (float)f.spp;
            rp[c] = v;
        }
        for (int bb = b + 1; bb <= f.B; ++bb) {
            const size_t at = ((size_t)bb * f.spp + s) * plane + pix;
            hit_prim[at] = -2;
            hit_t[at] = INFINITY;
        }
    }
    // the next hit's emission is skipped when this point estimated its direct light
    const bool nee_next = alive && f.nee && kind == 0;
    if (alive_in) {
        state[2 * (size_t)p] = make_float4(T[0], T[1], T[2], __uint_as_float((alive ? 1u : 0u) | (nee_next ? 2u : 0u)));
        state[2 * (size_t)p + 1] = make_float4(L[0], L[1], L[2], __uint_as_float(newpos));
    }
    if (f.live) {   // every thread has read the flag before this barrier
        const int any = __syncthreads_or(alive ? 1 : 0);
        if (l == 0) f.live[blk] = any ? 1u : 0u;
    }
}

__global__ __launch_bounds__(1024) void k_shade(DevScene sc, Frame f, int b, int s, const float4* __restrict__ q_in,
                                                float4* __restrict__ q_out, float4* state, int32_t* hit_prim,
                                                float* hit_t, float* radiance, float4* rays_out, float4* shadow_rays,
                                                float4* shadow_light, uint32_t* fill, uint32_t* keys_out, float4* debug) {
    extern __shared__ float lds[];
    shade_body(sc, f, b, s, blockIdx.x, q_in, q_out, state, hit_prim, hit_t, radiance, rays_out, shadow_rays,
               shadow_light, lds, fill, keys_out, debug);
}

// adds the light of unblocked shadow rays to their paths (one thread per path slot)
__global__ __launch_bounds__(256) void k_nee_accumulate(const float4* shadow_rays, const float4* shadow_light,
                                                        const int32_t* shadow_prim, uint32_t n, float4* state) {
    const uint32_t p = blockIdx.x * 256u + threadIdx.x;
    if (p >= n) return;
    if (__float_as_uint(shadow_rays[2 * (size_t)p + 1].w) == kNoRay || shadow_prim[p] != -1) return;
    const float4 c = shadow_light[p];
    float4 s1 = state[2 * (size_t)p + 1];
    s1.x = s1.x + c.x;
    s1.y = s1.y + c.y;
    s1.z = s1.z + c.z;
    state[2 * (size_t)p + 1] = s1;
}

__global__ __launch_bounds__(1024) void k_shade_multi(const StepJob* jobs, int njobs) {
    extern __shared__ float lds[];
    const int j = job_of_block(jobs, njobs, blockIdx.x);
    const StepJob& J = jobs[j];
    shade_body(J.sc, J.f, J.b, J.s, blockIdx.x - J.block_start, J.q_in, J.q_out, J.state, J.hit_prim, J.hit_t,
               J.radiance, nullptr, nullptr, nullptr, lds, nullptr, nullptr, nullptr);
}

// ------------------------------------------------------------------ reordering keys
// keys of n rays in a plain queue (dead rays, pixel word kNoRay, get 0xFFFFFFFF)
__global__ __launch_bounds__(256) void k_keys(DevScene sc, const float4* q, uint32_t n, uint32_t* keys,
                                              uint32_t* vals, int kind) {
    const uint32_t j = blockIdx.x * 256u + threadIdx.x;
    if (j < n) {
        const float4 r0 = q[2 * (size_t)j], r1 = q[2 * (size_t)j + 1];
        const bool live = __float_as_uint(r1.w) != kNoRay;
        keys[j] = live ? ray_key(sc, r0, r1, kind) : 0xFFFFFFFFu;
        if (vals) vals[j] = j;
    }
}

// ------------------------------------------------------------------ stable radix sort, one pass per digit
// Each pass is a single kernel (in the manner of single-pass "onesweep" radix sorts, with
// a two-level look-back in place of Merrill and Garland's walk over every lower tile): a
// workgroup takes the next tile id from a counter (ids follow the order workgroups start in,
// so every lower tile belongs to a workgroup that is already running), counts the tile's
// digits and publishes the counts, ranks its keys stably, and adds the counts of the lower
// tiles from per-block sums.  Keys are staged in LDS in digit order and written out in runs.
// The global start of each digit comes from histograms of all passes taken before the first
// pass.
constexpr int kOsThreads = 256;
constexpr uint32_t kHistCopies = 8;   // copies of the digit histograms (workgroup mod 8)
constexpr int kOsItems = 16;
constexpr uint32_t kOsTile = (uint32_t)kOsThreads * kOsItems;
constexpr uint32_t kLbAgg = 1u << 30, kLbInc = 2u << 30, kLbCount = (1u << 30) - 1u;

// exclusive scan over the 256 threads of a workgroup; *total = sum
__device__ __forceinline__ uint32_t scan256(uint32_t v, uint32_t* wsum, uint32_t* total) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kOsThreads / 64; ++w) {
        before += w < wave ? wsum[w] : 0u;
        all += wsum[w];
    }
    __syncthreads();
    if (total) *total = all;
    return before + x - v;
}

// rays of a compacted launch (the region counts of fill), or n when fill is null
__device__ __forceinline__ uint32_t fill_total(const uint32_t* fill, uint32_t n) {
    if (!fill) return n;
    uint32_t t = 0;
#pragma unroll
    for (int c = 0; c < kRayCounters; ++c) t += fill[c * kCounterStride];
    return t;
}

// Keys of the live rays of a compacted queue (sorted modes): ray i (i < the launch's rays, in
// region order) gets the key the shade kernel wrote at its queue slot (kslot) and the slot
// itself; the digit histograms of all `passes` passes of d bits each are added to
// hist[copy][pass][2^d], copy = workgroup mod kHistCopies (one copy per XCD: fewer
// device-wide atomics on each word; a pass adds the copies up).  Also clears the look-back
// words of the passes.  1024 threads x kKeysPerThread rays per workgroup, the loads issued
// together.
constexpr int kKeysPerThread = 8;
template <int D>
__global__ __launch_bounds__(1024) void k_keys_compacted(const uint32_t* kslot, const uint32_t* fill,
                                                         uint32_t region, uint32_t* keys, uint32_t* vals,
                                                         int passes, uint32_t* hist, uint32_t* lookback,
                                                         uint32_t lookback_words) {
    constexpr uint32_t R = 1u << D;
    __shared__ uint32_t h[4 * R];   // passes <= 4
    for (uint32_t d = threadIdx.x; d < 4 * R; d += 1024) h[d] = 0;
    for (size_t w = (size_t)blockIdx.x * 1024 + threadIdx.x; w < lookback_words; w += (size_t)gridDim.x * 1024)
        lookback[w] = 0;
    __syncthreads();
    uint32_t cnt[kRayCounters], total = 0;
#pragma unroll
    for (int c = 0; c < kRayCounters; ++c) {
        cnt[c] = fill[c * kCounterStride];
        total += cnt[c];
    }
    uint32_t pos[kKeysPerThread], key[kKeysPerThread];
#pragma unroll
    for (int e = 0; e < kKeysPerThread; ++e) {
        const uint32_t i = (blockIdx.x * kKeysPerThread + (uint32_t)e) * 1024u + threadIdx.x;
        uint32_t c = 0, v = i;
        while (c + 1 < (uint32_t)kRayCounters && v >= cnt[c]) {
            v -= cnt[c];
            ++c;
        }
        pos[e] = c * region + v;
        key[e] = i < total ? kslot[pos[e]] : 0u;
    }
#pragma unroll
    for (int e = 0; e < kKeysPerThread; ++e) {
        const uint32_t i = (blockIdx.x * kKeysPerThread + (uint32_t)e) * 1024u + threadIdx.x;
        if (i < total) {
            keys[i] = key[e];
            vals[i] = pos[e];
            for (int ps = 0; ps < passes; ++ps) atomicAdd(&h[ps * R + ((key[e] >> (D * ps)) & (R - 1u))], 1u);
        }
    }
    __syncthreads();
    uint32_t* const hc = hist + (blockIdx.x % kHistCopies) * (uint32_t)passes * R;
    for (uint32_t d = threadIdx.x; d < (uint32_t)passes * R; d += 1024)
        if (h[d]) atomicAdd(&hc[d], h[d]);
}

// digit histograms of all passes of d-bit digits over n keys (a plain sort), in kHistCopies
// copies as above
template <int D>
__global__ __launch_bounds__(256) void k_digit_hist(const uint32_t* keys, uint32_t n, int passes, uint32_t* hist) {
    constexpr uint32_t R = 1u << D;
    __shared__ uint32_t h[4 * R];
    for (uint32_t d = threadIdx.x; d < 4 * R; d += 256) h[d] = 0;
    __syncthreads();
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
        const uint32_t key = keys[i];
        for (int ps = 0; ps < passes; ++ps) atomicAdd(&h[ps * R + ((key >> (D * ps)) & (R - 1u))], 1u);
    }
    __syncthreads();
    uint32_t* const hc = hist + (blockIdx.x % kHistCopies) * (uint32_t)passes * R;
    for (uint32_t d = threadIdx.x; d < (uint32_t)passes * R; d += 256)
        if (h[d]) atomicAdd(&hc[d], h[d]);
}

// One stable pass over digit (key >> shift) & (2^d - 1) of n keys (n = the rays of fill when
// fill is given), 2^d a multiple of the workgroup's 256 threads (DPT digits per thread).
// ghist: the pass's digit histogram over all keys, in kHistCopies copies gstride words
// apart; lookback: lb_words(tiles, d) words, zero on entry (tile counts, then block
// counts, then block counters); tile_ctr: zero on entry.
//
// Tile t (ids in start order) holds keys [t * kOsTile, ...), wave w of it the kOsItems x 64
// consecutive keys from w * kOsItems * 64 on.  The pass: count the tile's digits and publish
// the counts; the last tile of each block of kLbBlock tiles to publish adds up the block's
// counts and publishes them; rank the keys stably (each wave ranks its own keys round by
// round with per-wave digit counters, no barrier between rounds) and stage the tile in LDS
// in digit order; add the counts of the lower blocks and of the lower tiles of its own block
// (two rounds of loads instead of a walk over every lower tile); write the runs out.  Every
// lower tile belongs to a workgroup that started earlier and publishes without waiting on
// anything, so every wait below ends.
constexpr int kLbBlock = 16;
static_assert(kOsThreads == 256, "scan256 spans the workgroup");

__device__ __forceinline__ uint32_t lb_wait(const uint32_t* w) {
    uint32_t v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while ((v & ~kLbCount) == 0) v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return v & kLbCount;
}

// sum of the published words w[i * stride], i < m (m <= kLbBlock), loads issued together
__device__ __forceinline__ uint32_t lb_sum(const uint32_t* w, size_t stride, uint32_t m) {
    uint32_t v[kLbBlock];
#pragma unroll
    for (int i = 0; i < kLbBlock; ++i)
        v[i] = (uint32_t)i < m ? __hip_atomic_load(w + (size_t)i * stride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                               : kLbAgg;
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kLbBlock; ++i) {
        if ((v[i] & ~kLbCount) == 0) v[i] = kLbAgg | lb_wait(w + (size_t)i * stride);   // not published yet
        sum += (uint32_t)i < m ? (v[i] & kLbCount) : 0u;
    }
    return sum;
}

template <int D>
__global__ __launch_bounds__(kOsThreads) void k_onesweep(const uint32_t* kin, const uint32_t* vin, uint32_t* kout,
                                                         uint32_t* vout, const uint32_t* fill, uint32_t n_plain,
                                                         int shift, const uint32_t* ghist, uint32_t gstride,
                                                         uint32_t* lookback, uint32_t* tile_ctr) {
    constexpr uint32_t R = 1u << D;
    static_assert(R % (uint32_t)kOsThreads == 0, "whole digits per thread");
    constexpr int DPT = (int)(R / kOsThreads);           // digits per thread
    constexpr int W = kOsThreads / 64;
    constexpr uint32_t WK = (uint32_t)kOsItems * 64u;   // keys per wave
    __shared__ uint32_t s_cnt[R];      // the tile's digit counts
    __shared__ uint32_t s_gbase[R];    // destination of the tile's first key of each digit
    __shared__ uint32_t s_lbase[R];    // tile-local start of each digit
    __shared__ uint32_t s_wcnt[W][R];  // per-wave running digit counts, then per-wave offsets
    __shared__ uint32_t s_k[kOsTile], s_v[kOsTile];   // the tile in digit order
    __shared__ uint32_t s_wsum[8];
    __shared__ uint32_t s_tile, s_last;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const uint32_t n = fill_total(fill, n_plain);
    const uint32_t tiles = gridDim.x;
    const uint32_t nblk = (tiles + kLbBlock - 1) / kLbBlock;
    uint32_t* const bagg = lookback + (size_t)tiles * R;   // [nblk][R] block counts
    uint32_t* const bctr = bagg + (size_t)nblk * R;        // [nblk] tiles of the block published
    if (tid == 0) s_tile = atomicAdd(tile_ctr, 1u);
#pragma unroll
    for (int e = 0; e < DPT; ++e) {
        const uint32_t d = (uint32_t)tid + (uint32_t)e * kOsThreads;
        s_cnt[d] = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) s_wcnt[w][d] = 0;
    }
    __syncthreads();
    const uint32_t t = s_tile;
    const uint32_t first = t * kOsTile;
    if (first >= n) return;   // the whole workgroup: no tile left
    const uint32_t valid_n = n - first < kOsTile ? n - first : kOsTile;
    const uint32_t wfirst = (uint32_t)wave * WK + (uint32_t)lane;
    uint32_t k[kOsItems], v[kOsItems];
#pragma unroll
    for (int r = 0; r < kOsItems; ++r) {
        const uint32_t j = wfirst + (uint32_t)r * 64u;
        k[r] = j < valid_n ? kin[first + j] : 0u;
        v[r] = j < valid_n ? vin[first + j] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kOsItems; ++r)
        if (wfirst + (uint32_t)r * 64u < valid_n) atomicAdd(&s_cnt[(k[r] >> shift) & (R - 1u)], 1u);
    __syncthreads();
    // publish the tile's counts; the block's last tile to do so publishes the block's counts
    // (digits tid + e * 256: neighbouring threads, neighbouring words)
    const uint32_t blk = t / kLbBlock, b0 = blk * kLbBlock;
    const uint32_t bsize = tiles - b0 < (uint32_t)kLbBlock ? tiles - b0 : (uint32_t)kLbBlock;
#pragma unroll
    for (int e = 0; e < DPT; ++e) {
        const uint32_t d = (uint32_t)tid + (uint32_t)e * kOsThreads;
        __hip_atomic_store(&lookback[(size_t)t * R + d], kLbAgg | s_cnt[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (tid == 0) s_last = atomicAdd(&bctr[blk], 1u) == bsize - 1u ? 1u : 0u;
    __syncthreads();
    if (s_last) {
#pragma unroll
        for (int e = 0; e < DPT; ++e) {
            const uint32_t d = (uint32_t)tid + (uint32_t)e * kOsThreads;
            const uint32_t sum = lb_sum(lookback + (size_t)b0 * R + d, R, bsize);
            __hip_atomic_store(&bagg[(size_t)blk * R + d], kLbInc | sum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // exclusive prefixes over the digits, of the global histogram and of the tile's counts
    // (here each thread takes DPT consecutive digits)
    {
        uint32_t gv[DPT], lv[DPT], gsum = 0, lsum = 0;
#pragma unroll
        for (int e = 0; e < DPT; ++e) {
            const uint32_t d = (uint32_t)tid * DPT + (uint32_t)e;
            uint32_t g = 0;
#pragma unroll
            for (uint32_t c = 0; c < kHistCopies; ++c) g += ghist[c * gstride + d];
            gv[e] = g;
            lv[e] = s_cnt[d];
            gsum += g;
            lsum += lv[e];
        }
        uint32_t gpre = scan256(gsum, s_wsum, nullptr);
        uint32_t lpre = scan256(lsum, s_wsum, nullptr);
#pragma unroll
        for (int e = 0; e < DPT; ++e) {
            const uint32_t d = (uint32_t)tid * DPT + (uint32_t)e;
            s_gbase[d] = gpre;
            s_lbase[d] = lpre;
            gpre += gv[e];
            lpre += lv[e];
        }
    }
    // stable ranking in index order (wave, round, lane): per-wave running counts, the
    // lowest lane of each digit in a round adding the round's keys of that digit
    uint32_t rk[kOsItems];
#pragma unroll
    for (int r = 0; r < kOsItems; ++r) {
        const bool ok = wfirst + (uint32_t)r * 64u < valid_n;
        const uint32_t dg = (k[r] >> shift) & (R - 1u);
        unsigned long long same = __ballot(ok);
#pragma unroll
        for (int bit = 0; bit < D; ++bit) {
            const unsigned long long bb = __ballot((dg >> bit) & 1u);
            same &= ((dg >> bit) & 1u) ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(same & lt);
        const uint32_t before = ok ? s_wcnt[wave][dg] : 0u;
        rk[r] = before + rank;
        if (ok && rank == 0) s_wcnt[wave][dg] = before + (uint32_t)__popcll(same);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < DPT; ++e) {   // per-wave counts -> offsets of each wave's keys in its digit's run
        const uint32_t d = (uint32_t)tid + (uint32_t)e * kOsThreads;
        uint32_t acc = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint32_t c = s_wcnt[w][d];
            s_wcnt[w][d] = acc;
            acc += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kOsItems; ++r) {
        if (wfirst + (uint32_t)r * 64u < valid_n) {
            const uint32_t dg = (k[r] >> shift) & (R - 1u);
            const uint32_t lpos = s_lbase[dg] + s_wcnt[wave][dg] + rk[r];
            s_k[lpos] = k[r];
            s_v[lpos] = v[r];
        }
    }
    // keys of each digit in the lower tiles: the lower blocks, then the block's lower tiles
#pragma unroll
    for (int e = 0; e < DPT; ++e) {
        const uint32_t d = (uint32_t)tid + (uint32_t)e * kOsThreads;
        uint32_t below = 0;
        for (uint32_t bb = 0; bb < blk; bb += kLbBlock) {
            const uint32_t m = blk - bb < (uint32_t)kLbBlock ? blk - bb : (uint32_t)kLbBlock;
            below += lb_sum(bagg + (size_t)bb * R + d, R, m);
        }
        below += lb_sum(lookback + (size_t)b0 * R + d, R, t - b0);
        s_gbase[d] += below;
    }
    __syncthreads();
    // runs of equal digits go to consecutive places, written by consecutive threads
    for (uint32_t i = tid; i < valid_n; i += kOsThreads) {
        const uint32_t key = s_k[i];
        const uint32_t dg = (key >> shift) & (R - 1u);
        const uint32_t dst = s_gbase[dg] + (i - s_lbase[dg]);
        if (dst < n) {   // always, when the histograms describe the keys
            kout[dst] = key;
            vout[dst] = s_v[i];
        }
    }
}

__global__ __launch_bounds__(256) void k_count_finalize(const uint32_t* partial, int stride, int parts,
                                                        uint32_t* ray_count) {
    __shared__ uint32_t red[256];
    uint32_t sum = 0;
    const uint32_t* p = partial + (size_t)blockIdx.x * (size_t)stride;
    for (int j = threadIdx.x; j < parts; j += 256) sum += p[j];
    red[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) ray_count[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_zero(uint32_t* p, size_t n) {
    const size_t j = (size_t)blockIdx.x * 256u + threadIdx.x;
    if (j < n) p[j] = 0u;
}

int g_trace_blocks[64] = {0};
int g_cus[64] = {0};

}  // namespace

// ------------------------------------------------------------------ launchers
int trace_grid_blocks(int waves_per_cu) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (g_trace_blocks[dev] == 0) {
        int cus = 0, per = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_trace<false, false, false>, kTraceBlock, 0) != hipSuccess ||
            per <= 0)
            per = 8;
        int g = cus * per;
        if (g > kMaxTraceBlocks) g = kMaxTraceBlocks;
        g &= ~7;   // a multiple of the 8 XCDs
        if (g < 8) g = 8;
        g_trace_blocks[dev] = g;
        g_cus[dev] = cus;
    }
    int g = g_trace_blocks[dev];
    const int want = (g_cus[dev] * (waves_per_cu > 0 ? waves_per_cu : kDefaultWavesPerCu)) & ~7;
    if (want >= 8 && want < g) g = want;
    return g;
}

int trace_max_kind(const DevScene& sc) {
    if (!sc.wide) return kTraceChildPair;
    if (sc.ntri > kQTriMask + 1u) return kTraceWide;
    return sc.quant ? kTraceWideQueueQ : kTraceWideQueue;
}

int trace_kind(const DevScene& sc) {
    if (!(kPreferWide && sc.wide)) return kTraceChildPair;
    if (!(kLeafQueue && sc.ntri <= kQTriMask + 1u)) return kTraceWide;
    return (kQuantized && sc.quant) ? kTraceWideQueueQ : kTraceWideQueue;
}

hipError_t launch_trace(const DevScene& sc, const TraceArgs& a, bool stats, hipStream_t st) {
    int g = trace_grid_blocks(a.waves_per_cu);
    if (a.max_blocks > 0 && g > a.max_blocks) g = a.max_blocks & ~7;   // still a multiple of the 8 XCDs
    if (g < 8) return hipErrorInvalidValue;
    const uint32_t gthreads = (uint32_t)g * kTraceBlock;
    if (a.refill < 1 || a.refill > 64) return hipErrorInvalidValue;
    const StepJob* none = nullptr;
    if (a.kind > trace_max_kind(sc)) return hipErrorInvalidValue;
    switch (a.kind >= 0 ? a.kind : trace_kind(sc)) {
    case kTraceWideQueueQ:
        if (stats)
            hipLaunchKernelGGL((k_trace_q<true, false, true>), dim3(g), dim3(kTraceBlock), 0, st, sc, a, gthreads, none, 0);
        else
            hipLaunchKernelGGL((k_trace_q<false, false, true>), dim3(g), dim3(kTraceBlock), 0, st, sc, a, gthreads, none, 0);
        break;
    case kTraceWideQueue:
        if (stats)
            hipLaunchKernelGGL((k_trace_q<true, false, false>), dim3(g), dim3(kTraceBlock), 0, st, sc, a, gthreads, none, 0);
        else
            hipLaunchKernelGGL((k_trace_q<false, false, false>), dim3(g), dim3(kTraceBlock), 0, st, sc, a, gthreads, none, 0);
        break;
    case kTraceWide:
        if (stats)
            hipLaunchKernelGGL((k_trace<true, false, true>), dim3(g), dim3(kTraceBlock), 0, st, sc, a, gthreads, none, 0);
        else
            hipLaunchKernelGGL((k_trace<false, false, true>), dim3(g), dim3(kTraceBlock), 0, st, sc, a, gthreads, none, 0);
        break;
    default:
        if (stats)
            hipLaunchKernelGGL((k_trace<true, false, false>), dim3(g), dim3(kTraceBlock), 0, st, sc, a, gthreads, none, 0);
        else
            hipLaunchKernelGGL((k_trace<false, false, false>), dim3(g), dim3(kTraceBlock), 0, st, sc, a, gthreads, none, 0);
    }
    return hipGetLastError();
}

hipError_t launch_trace_multi(const StepJob* jobs, int njobs, const TraceArgs& a, int kind, hipStream_t st) {
    const int g = trace_grid_blocks(a.waves_per_cu);
    const uint32_t gthreads = (uint32_t)g * kTraceBlock;
    if (a.refill < 1 || a.refill > 64 || njobs < 1) return hipErrorInvalidValue;
    DevScene none{};
    if (kind == kTraceWideQueueQ)
        hipLaunchKernelGGL((k_trace_q<false, true, true>), dim3(g), dim3(kTraceBlock), 0, st, none, a, gthreads, jobs, njobs);
    else if (kind == kTraceWideQueue)
        hipLaunchKernelGGL((k_trace_q<false, true, false>), dim3(g), dim3(kTraceBlock), 0, st, none, a, gthreads, jobs, njobs);
    else if (kind == kTraceWide)
        hipLaunchKernelGGL((k_trace<false, true, true>), dim3(g), dim3(kTraceBlock), 0, st, none, a, gthreads, jobs, njobs);
    else
        hipLaunchKernelGGL((k_trace<false, true, false>), dim3(g), dim3(kTraceBlock), 0, st, none, a, gthreads, jobs,
                           njobs);
    return hipGetLastError();
}

hipError_t launch_raygen_multi(const StepJob* jobs, int njobs, uint32_t total_blocks, int TS, hipStream_t st) {
    if (total_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_raygen_multi, dim3(total_blocks), dim3(TS), 0, st, jobs, njobs);
    return hipGetLastError();
}

hipError_t launch_shade_multi(const StepJob* jobs, int njobs, uint32_t total_blocks, int TS, bool reuse,
                              hipStream_t st) {
    if (total_blocks == 0) return hipSuccess;
    const size_t lds = reuse ? (size_t)TS * 8 * sizeof(float) : 0;
    hipLaunchKernelGGL(k_shade_multi, dim3(total_blocks), dim3(TS), lds, st, jobs, njobs);
    return hipGetLastError();
}

hipError_t launch_zero(uint32_t* p, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_raygen(const Frame& f, int s, float4* q, float4* state, float4* rays_out, hipStream_t st) {
    const unsigned blocks = (unsigned)(f.nslots / (uint32_t)f.TS);
    hipLaunchKernelGGL(k_raygen, dim3(blocks), dim3(f.TS), 0, st, f, s, q, state, rays_out);
    return hipGetLastError();
}

hipError_t launch_shade(const DevScene& sc, const Frame& f, int b, int s, const float4* q_in, float4* q_out,
                        float4* state, int32_t* hit_prim, float* hit_t, float* radiance, float4* rays_out,
                        float4* shadow_rays, float4* shadow_light, uint32_t* fill, uint32_t* keys_out, float4* debug,
                        hipStream_t st) {
    const unsigned blocks = (unsigned)(f.nslots / (uint32_t)f.TS);
    const bool reuse = f.mode == PT_MODE_REUSE || f.mode == PT_MODE_REUSE_PLAIN || f.mode == PT_MODE_REUSE_WORLD;
    // reuse exchange (8 words per slot), then the compaction's ranks (1 per slot) and wave sums (40)
    const size_t lds = ((reuse ? (size_t)f.TS * 8 : 0) + (fill ? (size_t)f.TS + 40 : 0)) * sizeof(float);
    hipLaunchKernelGGL(k_shade, dim3(blocks), dim3(f.TS), lds, st, sc, f, b, s, q_in, q_out, state, hit_prim, hit_t,
                       radiance, rays_out, shadow_rays, shadow_light, fill, keys_out, debug);
    return hipGetLastError();
}

hipError_t launch_nee_accumulate(const float4* shadow_rays, const float4* shadow_light, const int32_t* shadow_prim,
                                 uint32_t n, float4* state, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_nee_accumulate, dim3((n + 255) / 256), dim3(256), 0, st, shadow_rays, shadow_light,
                       shadow_prim, n, state);
    return hipGetLastError();
}

hipError_t launch_keys(const DevScene& sc, const float4* q, uint32_t n, uint32_t* keys, uint32_t* vals, int kind,
                       hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_keys, dim3((n + 255) / 256), dim3(256), 0, st, sc, q, n, keys, vals, kind);
    return hipGetLastError();
}

hipError_t launch_count_finalize(const uint32_t* partial, int stride, int parts, int launches, uint32_t* ray_count,
                                 hipStream_t st) {
    if (launches <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_finalize, dim3(launches), dim3(256), 0, st, partial, stride, parts, ray_count);
    return hipGetLastError();
}

// ---- sorted modes and the plain sort
// 30-bit keys: 4 passes of 8-bit digits.  3 passes of 10-bit digits (the same kernel, 4 digits
// per thread) measured slower: 40 against 26 us per pass over the ~2M live rays of a 1080p
// bounce on MI355X.  A workgroup's LDS grows from 39 to 60 KB (2 workgroups per CU instead of
// 4), its count words fourfold, and at ~4 keys per digit and tile the writes are short runs.
constexpr int kRenderDigit = 8;
constexpr int kRenderPasses = 4;
static_assert(kRenderDigit * kRenderPasses >= 30 && kRenderPasses <= 4, "the keys' 30 bits, at most 4 passes");
constexpr int kPlainDigit = 8;                 // 32-bit keys: 4 passes of 8-bit digits
constexpr int kPlainPasses = 4;

static uint32_t sort_tiles(uint32_t n) { return (n + kOsTile - 1) / kOsTile; }
// look-back words of one pass of d-bit digits over this many tiles: tile counts, block
// counts (2^d words each), block counters
static size_t lb_words(uint32_t tiles, int d) {
    const size_t nb = (tiles + kLbBlock - 1) / kLbBlock;
    return ((size_t)tiles + nb) * ((size_t)1 << d) + nb;
}
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// render workspace: keys, vals, their alternates (n each), the histograms and tile counters
// (zeroed per bounce), the look-back words of every pass
size_t sort_compacted_workspace_bytes(uint32_t n, uint32_t qslots) {
    const size_t R = (size_t)1 << kRenderDigit;
    return 4 * al256((size_t)n * 4) + al256((kHistCopies * kRenderPasses * R + kRenderPasses) * 4) +
           al256((size_t)kRenderPasses * lb_words(sort_tiles(n), kRenderDigit) * 4) + al256((size_t)qslots * 4);
}

struct SortWs {
    uint32_t *keys, *vals, *kalt, *valt, *hist, *ctr, *lookback, *kslot;
};

static SortWs sort_ws(void* ws, uint32_t n) {
    const size_t R = (size_t)1 << kRenderDigit;
    char* p = (char*)ws;
    SortWs w;
    w.keys = (uint32_t*)p;
    p += al256((size_t)n * 4);
    w.vals = (uint32_t*)p;
    p += al256((size_t)n * 4);
    w.kalt = (uint32_t*)p;
    p += al256((size_t)n * 4);
    w.valt = (uint32_t*)p;
    p += al256((size_t)n * 4);
    w.hist = (uint32_t*)p;
    w.ctr = w.hist + kHistCopies * kRenderPasses * R;
    p += al256((kHistCopies * kRenderPasses * R + kRenderPasses) * 4);
    w.lookback = (uint32_t*)p;
    p += al256((size_t)kRenderPasses * lb_words(sort_tiles(n), kRenderDigit) * 4);
    w.kslot = (uint32_t*)p;
    return w;
}

uint32_t* sort_key_slots(void* ws, uint32_t nslots) { return sort_ws(ws, nslots).kslot; }

hipError_t launch_keys_compacted(const uint32_t* fill, uint32_t region, uint32_t nslots, void* ws, hipStream_t st) {
    const uint32_t R = 1u << kRenderDigit;
    const SortWs w = sort_ws(ws, nslots);
    hipError_t e = launch_zero(w.hist, (size_t)kHistCopies * kRenderPasses * R + kRenderPasses, st);
    if (e != hipSuccess) return e;
    const uint32_t kb = (nslots + kKeysPerThread * 1024 - 1) / (kKeysPerThread * 1024);
    hipLaunchKernelGGL(k_keys_compacted<kRenderDigit>, dim3(kb), dim3(1024), 0, st, w.kslot, fill, region, w.keys,
                       w.vals, kRenderPasses, w.hist, w.lookback,
                       (uint32_t)((size_t)kRenderPasses * lb_words(sort_tiles(nslots), kRenderDigit)));
    return hipGetLastError();
}

hipError_t launch_sort_compacted(const uint32_t* fill, uint32_t nslots, void* ws, const uint32_t** perm,
                                 hipStream_t st) {
    const uint32_t R = 1u << kRenderDigit;
    const SortWs w = sort_ws(ws, nslots);
    const uint32_t tiles = sort_tiles(nslots);
    uint32_t *kin = w.keys, *vin = w.vals, *kout = w.kalt, *vout = w.valt;
    for (int ps = 0; ps < kRenderPasses; ++ps) {
        hipLaunchKernelGGL(k_onesweep<kRenderDigit>, dim3(tiles), dim3(kOsThreads), 0, st, kin, vin, kout, vout, fill,
                           0u, kRenderDigit * ps, w.hist + (size_t)ps * R, (uint32_t)(kRenderPasses * R),
                           w.lookback + (size_t)ps * lb_words(tiles, kRenderDigit), w.ctr + ps);
        uint32_t* tk = kin;
        kin = kout;
        kout = tk;
        uint32_t* tv = vin;
        vin = vout;
        vout = tv;
    }
    *perm = vin;   // after the last pass: the queue slots in key order
    return hipGetLastError();
}

size_t sort_workspace_bytes(uint32_t n) {
    const size_t R = (size_t)1 << kPlainDigit;
    return 2 * al256((size_t)n * 4) + al256((kHistCopies * kPlainPasses * R + kPlainPasses) * 4) +
           al256((size_t)kPlainPasses * lb_words(sort_tiles(n), kPlainDigit) * 4);
}

hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t n, void* ws, hipStream_t st) {
    if (n <= 1) return hipSuccess;
    const uint32_t R = 1u << kPlainDigit;
    const uint32_t tiles = sort_tiles(n);
    char* p = (char*)ws;
    uint32_t* kalt = (uint32_t*)p;
    p += al256((size_t)n * 4);
    uint32_t* valt = (uint32_t*)p;
    p += al256((size_t)n * 4);
    uint32_t* hist = (uint32_t*)p;
    uint32_t* ctr = hist + kHistCopies * kPlainPasses * R;
    hipError_t e = launch_zero(hist, sort_workspace_bytes(n) / 4 - 2 * al256((size_t)n * 4) / 4, st);
    if (e != hipSuccess) return e;
    uint32_t* lookback = (uint32_t*)(p + al256((kHistCopies * kPlainPasses * R + kPlainPasses) * 4));
    const uint32_t hblocks = (n + 255) / 256 < 128u ? (n + 255) / 256 : 128u;
    hipLaunchKernelGGL(k_digit_hist<kPlainDigit>, dim3(hblocks), dim3(256), 0, st, keys, n, kPlainPasses, hist);
    uint32_t *kin = keys, *vin = vals, *kout = kalt, *vout = valt;
    for (int ps = 0; ps < kPlainPasses; ++ps) {
        hipLaunchKernelGGL(k_onesweep<kPlainDigit>, dim3(tiles), dim3(kOsThreads), 0, st, kin, vin, kout, vout,
                           (const uint32_t*)nullptr, n, kPlainDigit * ps, hist + (size_t)ps * R,
                           (uint32_t)(kPlainPasses * R), lookback + (size_t)ps * lb_words(tiles, kPlainDigit), ctr + ps);
        uint32_t* tk = kin;
        kin = kout;
        kout = tk;
        uint32_t* tv = vin;
        vin = vout;
        vout = tv;
    }
    return hipGetLastError();   // an even number of passes: the result is back in keys/vals
}

}  // namespace pt
