/*
 * CPU oracle for "Generate Coherent Rays Directly" (Liu et al., EG 2024).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package's smoke check
 * and the benchmark's CPU-baseline leg may load this library.  The GPU
 * library never includes, links or calls it, and this code includes nothing
 * from the GPU library.
 *
 * A plain single-threaded path tracer that follows the paper step by step:
 * intersect, shade, generate the next ray (Section 1), with the next ray's
 * direction either sampled independently ("NoOpt", Table 1), reordered by a
 * two-point Morton key (the sorted baseline, Section 2.1 / Section 4), or
 * reused inside interleaved groups by the per-category rules of Sections
 * 3.2-3.3.  Arithmetic is IEEE binary32, round to nearest even, no fused
 * multiply-add, correctly rounded division and square root, in the operation
 * order that the arithmetic contract fixes.
 */
#ifndef CRD_ORACLE_H
#define CRD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* material record, 32 bytes (kind 0 Lambert, 1 GGX, 2 mirror) */
typedef struct {
    uint32_t kind;
    float albedo[3];
    float alpha;
    float emission[3];
} orc_material;

typedef struct {
    float pos[3], look_at[3], up[3];
    float vfov_deg;
} orc_camera;

typedef struct orc_scene orc_scene;

/* render outputs; every pointer may be NULL */
typedef struct {
    float* radiance;          /* [h][w][3] */
    int32_t* hit_prim;        /* [B+1][spp][h][w]: -1 miss, -2 no ray traced */
    float* hit_t;             /* same shape, +inf for miss / no ray */
    float* hit_t2;            /* same shape: second-nearest distinct-prim t (+inf if none) */
    float* dbg_q;             /* [B][spp][h][w][3] tangent-space direction used for ray b+1 */
    int32_t* dbg_flags;       /* [B][spp][h][w] see ORC_F_* */
    uint32_t* dbg_keys;       /* [B][spp][h][w] two-point key of ray b+1 (sorted mode) */
    float* rays;              /* [B+1][spp][h][w][8] ray traced at bounce b {o, excluded, d, pixel} */
    uint64_t* rays_per_bounce;/* [B+1] */
    uint64_t* shadow_rays;    /* [B+1] shadow rays traced at hit b (next-event estimation) */
} orc_outputs;

enum { ORC_MODE_INCOHERENT = 0, ORC_MODE_SORTED = 1, ORC_MODE_REUSE = 2, ORC_MODE_SORTED_ORIGIN = 3,
       ORC_MODE_SORTED_REIS = 4, ORC_MODE_SORTED_AILA = 5, ORC_MODE_REUSE_PLAIN = 6, ORC_MODE_REUSE_WORLD = 7 };

/* debug flag bits for the ray generated at hit b (ray index b+1) */
#define ORC_F_ACTIVE   (1 << 0)     /* the path scatters at this hit */
#define ORC_F_CLASS_SH 1            /* 2 bits: material kind */
#define ORC_F_CAT_SH   3            /* 2 bits: 0 none, 1 diffuse, 2 glossy, 3 hybrid */
#define ORC_F_REP      (1 << 5)     /* representative of a diffuse group */
#define ORC_F_REUSED   (1 << 6)     /* direction taken from the group rule */
#define ORC_F_VALID    (1 << 7)     /* the path survives scattering (a ray b+1 exists) */
#define ORC_F_SLOT_SH  16           /* 16 bits: shuffled slot s(i) */

/* scene: triangles [ntri][3][3], per-triangle material id, material table */
orc_scene* orc_scene_create(const float* tris, uint32_t ntri, const uint32_t* tri_mat,
                            const orc_material* mats, uint32_t nmat, const float env[3]);
void orc_scene_free(orc_scene* s);
void orc_scene_bounds(const orc_scene* s, float lo[3], float hi[3]);

/* closest hit of n rays; ray = {ox,oy,oz, exclude(int bits), dx,dy,dz, unused} */
void orc_trace(const orc_scene* s, const float* rays, uint32_t n, int32_t* prim, float* t,
               float* t2, uint64_t* node_visits, uint64_t* tri_tests);
void orc_trace_brute(const orc_scene* s, const float* rays, uint32_t n, int32_t* prim, float* t);

/* nee: next-event estimation toward the emissive triangles at Lambert scattering points
 * (not with ORC_MODE_REUSE_WORLD) */
int orc_render(const orc_scene* s, const orc_camera* cam, int w, int h, int spp, int bounces,
               int mode, int tile_w, int tile_h, int k, int reuse_max_bounce, int frame_groups, uint64_t seed,
               const uint8_t* tile_mask, int nee, orc_outputs* out);

/* individual steps, exported for the pins */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
void orc_sincos2pi(const float* u, uint32_t n, float* s, float* c);
void orc_onb(const float n[3], float t[3], float b[3]);
void orc_sample_lambert(float u2, float u3, float q[3]);
int orc_sample_ggx(const float wi[3], float alpha, const float f0[3], float u2, float u3,
                   float wo[3], float weight[3]);
void orc_offset_origin(const float p[3], const float n[3], float out[3]);
void orc_shuffle(int wh, uint64_t x0, uint64_t x1, uint32_t* slot);
uint32_t orc_ray_key(const float lo[3], const float hi[3], const float o[3], const float d[3]);
/* key of one of the sorted modes (ORC_MODE_SORTED = TwoPoint, _ORIGIN, _REIS, _AILA) */
uint32_t orc_ray_key_kind(int kind, const float lo[3], const float hi[3], const float o[3], const float d[3]);
void orc_camera_ray(const orc_camera* cam, int w, int h, int x, int y, float u0, float u1,
                    float o[3], float d[3]);

#ifdef __cplusplus
}
#endif
#endif
