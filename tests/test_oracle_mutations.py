"""Mutation check of the oracle's pins.

Each case plants one plausible mistake in a copy of oracle/oracle.c (a dropped
term, a wrong sign, index or constant, a rule applied to the wrong pixel),
builds the copy on the CPU and runs the pins that cover that step against it
through PT_ORACLE_LIB: the pins must fail.  A case whose original text no
longer occurs exactly once in the oracle fails too, so the list follows the
source.  Nothing here runs on a GPU.
"""
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")
ORACLE_H = os.path.join(ROOT, "oracle", "oracle.h")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")

# (name, original text, planted mistake, pins expected to catch it)
MUTATIONS = [
    ("mirror_exit_sign",
     "p->own_q = mk(-p->wi.x, -p->wi.y, p->wi.z);",
     "p->own_q = mk(-p->wi.x, p->wi.y, p->wi.z);",
     "mirror"),
    ("mirror_weight_untinted",
     "        for (int i = 0; i < 3; ++i) p->own_w[i] = m->albedo[i];\n        p->own_ok = p->own_q.z > 0.0f;",
     "        for (int i = 0; i < 3; ++i) p->own_w[i] = 1.0f;\n        p->own_ok = p->own_q.z > 0.0f;",
     "open_floor"),
    ("reused_weight_from_representative",
     "                                    const orc_material* m = &s->mats[s->tri_mat[p->prim]];\n"
     "                                    for (int cc = 0; cc < 3; ++cc) p->use_w[cc] = m->albedo[cc];\n"
     "                                    if (!(cat == 1",
     "                                    const orc_material* m = &s->mats[s->tri_mat[P[rep >= 0 ? rep : (int)(mm - 1)].prim]];\n"
     "                                    for (int cc = 0; cc < 3; ++cc) p->use_w[cc] = m->albedo[cc];\n"
     "                                    if (!(cat == 1",
     "own_albedo or open_floor"),
    ("world_reuse_weight_from_representative",
     "                                const orc_material* m = &s->mats[s->tri_mat[p->prim]];\n"
     "                                for (int cc = 0; cc < 3; ++cc) p->use_w[cc] = m->albedo[cc];\n"
     "                                p->flags |= ORC_F_REUSED;",
     "                                const orc_material* m = &s->mats[s->tri_mat[pr->prim]];\n"
     "                                for (int cc = 0; cc < 3; ++cc) p->use_w[cc] = m->albedo[cc];\n"
     "                                p->flags |= ORC_F_REUSED;",
     "own_albedo or open_floor"),
    ("env_without_throughput",
     "p->L[c] = p->L[c] + p->T[c] * s->env[c];",
     "p->L[c] = p->L[c] + s->env[c];",
     "open_floor"),
    ("emission_without_throughput",
     "p->L[c] = p->L[c] + p->T[c] * m->emission[c];",
     "p->L[c] = p->L[c] + m->emission[c];",
     "furnace"),
    ("radiance_not_averaged",
     "out->radiance[i * 3 + c] = acc[i * 3 + c] / (float)spp;",
     "out->radiance[i * 3 + c] = acc[i * 3 + c];",
     "furnace"),
    ("lambert_radius_linear",
     "    float r = sqrtf(u2);\n    float sn, cs;",
     "    float r = u2;\n    float sn, cs;",
     "lambert"),
    ("ggx_fresnel_cubic",
     "float c5 = ((c * c) * (c * c)) * c;",
     "float c5 = (c * c) * c;",
     "ggx"),
    ("ggx_no_masking",
     "float g = ((smith_g1(wi, a2) * smith_g1(o, a2)) * wim) / (wi.z * cm);",
     "float g = wim / (wi.z * cm);",
     "ggx"),
    ("onb_bitangent_sign",
     "*B = mk(b, s + (n.y * n.y) * a, -n.y);",
     "*B = mk(b, s + (n.y * n.y) * a, n.y);",
     "onb"),
    ("offset_int_scale",
     "int_scale = 256.0f;",
     "int_scale = 128.0f;",
     "offset"),
    ("shuffle_multiplier",
     "*a = 2u * (uint32_t)(x0 % (uint64_t)(wh / 2)) + 1u;",
     "*a = 2u * (uint32_t)(x0 % (uint64_t)(wh / 2)) + 3u;",
     "rules_per_category or world_reuse_rules"),
    ("shuffle_offset_word",
     "*c = (uint32_t)(x1 % (uint64_t)wh);",
     "*c = (uint32_t)(x0 % (uint64_t)wh);",
     "rules_per_category or world_reuse_rules"),
    ("representative_largest_slot",
     "if (P[mm - 1].kind == 0) { ++nd; if (rep < 0) rep = (int)(mm - 1); }",
     "if (P[mm - 1].kind == 0) { ++nd; rep = (int)(mm - 1); }",
     "rules_per_category"),
    ("hybrid_sum_not_normalized",
     "q = vnormalize(tree[0]);",
     "q = tree[0];",
     "rules_per_category"),
    ("hybrid_sum_includes_diffuse",
     "if (mm && P[mm - 1].active && P[mm - 1].kind != 0 && P[mm - 1].own_ok) {",
     "if (mm && P[mm - 1].active && P[mm - 1].own_ok) {",
     "rules_per_category"),
    ("glossy_members_reuse_too",
     "if (p->kind == 0 && have) {",
     "if (have) {",
     "rules_per_category or glossy_only"),
    ("edge_sign_test_two_edges",
     "if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return 0;",
     "if ((U < 0.0f || V < 0.0f) && (U > 0.0f || V > 0.0f)) return 0;",
     "float64 or interior or shared_edge"),
    ("camera_vertical_aspect",
     "float fy = (1.0f - 2.0f * py) * cb->th;",
     "float fy = (1.0f - 2.0f * py) * cb->thx;",
     "camera"),
    ("twopoint_length",
     "float L = 0.25f * mx;",
     "float L = 0.5f * mx;",
     "ray_key"),
    ("sincos_octant_swap",
     "case 1: *sn = c;  *cs = s;  break;",
     "case 1: *sn = s;  *cs = c;  break;",
     "sincos"),
    ("philox_weyl_constant",
     "W1 = 0xBB67AE8584CAA73Bull;",
     "W1 = 0xBB67AE8584CAA73Dull;",
     "philox"),
    ("frame_groups_ignored",
     "draw(seed, (uint64_t)tile, smp, frame_groups ? 0 : b, 1, r);",
     "draw(seed, (uint64_t)tile, smp, b, 1, r);",
     "composition"),
    ("groups_never_redrawn",
     "draw(seed, (uint64_t)tile, smp, frame_groups ? 0 : b, 1, r);",
     "draw(seed, (uint64_t)tile, smp, 0, 1, r);",
     "composition"),
    ("nee_light_count_dropped",
     "float k = g * ((float)s->nemit * (float)(1.0 / (2.0 * 3.14159265358979323846)));",
     "float k = g * (float)(1.0 / (2.0 * 3.14159265358979323846));",
     "nee"),
]


def _run(case, tmp):
    name, orig, mut, pins = case
    src = open(ORACLE_C).read()
    count = src.count(orig)
    if count != 1:
        return name, f"original text occurs {count} times"
    d = os.path.join(tmp, name)
    os.makedirs(d)
    shutil.copy(ORACLE_H, d)
    with open(os.path.join(d, "oracle.c"), "w") as f:
        f.write(src.replace(orig, mut))
    lib = os.path.join(d, "liboracle.so")
    b = subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-o", lib,
                        os.path.join(d, "oracle.c"), "-lm"], capture_output=True, text=True)
    if b.returncode != 0:
        return name, "mutant does not compile: " + b.stderr[-400:]
    env = dict(os.environ, PT_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", PINS, "-k", pins],
                       capture_output=True, text=True, cwd=ROOT, env=env, timeout=600)
    if r.returncode == 1:
        return name, None   # at least one pin failed: the mistake is caught
    return name, f"pins '{pins}' gave exit code {r.returncode}: " + r.stdout[-600:]


def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp, ThreadPoolExecutor(4) as ex:
        results = list(ex.map(lambda c: _run(c, tmp), MUTATIONS))
    missed = [(n, why) for n, why in results if why]
    assert not missed, missed


def test_unmutated_oracle_passes_the_same_selections():
    # the selections above select pins that pass on the oracle as it is
    sel = " or ".join(sorted({m[3] for m in MUTATIONS}))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", PINS, "-k", sel],
                       capture_output=True, text=True, cwd=ROOT, timeout=900)
    assert r.returncode == 0, r.stdout[-2000:]
