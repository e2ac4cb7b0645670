"""Mutation check of the oracle's pins: each plausible mistake below is
planted in a copy of oracle.c (built to a temporary library), the fast CPU
pins are run against it, and at least one pin must fail.  A mutant that no
pin catches would mean that part of the oracle is parity unpinned."""
import importlib
import os
import subprocess

import pytest

import oracle
from oracle import build as obuild
from oracle import oracle as omod

HERE = os.path.dirname(os.path.abspath(__file__))

# (name, text in oracle.c, replacement)
MUTANTS = [
    ("sign of dL/dd", "dA * (-bt[q].A / sc->delta)", "dA * (bt[q].A / sc->delta)"),
    ("camera Jacobian transposed",
     "for (int j = 0; j < 3; ++j) gw[j] = vw[0 * 4 + j] * gc[0] + vw[1 * 4 + j] * gc[1] + vw[2 * 4 + j] * gc[2];",
     "for (int j = 0; j < 3; ++j) gw[j] = vw[j * 4 + 0] * gc[0] + vw[j * 4 + 1] * gc[1] + vw[j * 4 + 2] * gc[2];"),
    ("perspective term dropped", "-c[i] / (c[2] * c[2] * t)", "0.0 * c[i]"),
    ("barycentric adjoint sign", "double gx = -w[i] * gxs, gy = -w[i] * gys;", "double gx = w[i] * gxs, gy = w[i] * gys;"),
    ("edge-change term dropped", "orc_add_kf(cx, g, ev->f, b, s + X, gex, gey);", ";"),
    ("keyframe X always the segment start", "*X = (2 * rem <= (long)(K - 1)) ? 0 : 1;", "*X = 0;"),
    ("depth tie to the highest face index", "(ev[j].depth == ev[best].depth && ev[j].f < ev[best].f)",
     "(ev[j].depth == ev[best].depth && ev[j].f > ev[best].f)"),
    ("image y not flipped", "double v = (double)(H - 2 * r - 1) / (double)H;",
     "double v = (double)(2 * r + 1 - H) / (double)H;"),
    ("App. B coefficient sign", "A1[0] = -(x20 - x21) * (y10 - y11) + (x10 - x11) * (y20 - y21);",
     "A1[0] = (x20 - x21) * (y10 - y11) + (x10 - x11) * (y20 - y21);"),
    ("no guard band on the closest point", "#define ORC_GUARD_ULPS 8.0", "#define ORC_GUARD_ULPS 0.0"),
    ("bbox pairs not counted", "t->cnt[CNT_BBOX] += 1;", ";"),
    ("background product includes its own factor", "double dA = gI[sc->C] * t->pre[q] * t->suf[q + 1];",
     "double dA = gI[sc->C] * t->pre[q + 1] * t->suf[q + 1];"),
]

# fast pins (module, function, kwargs)
PINS = [
    ("test_oracle_render", "test_full_field_of_view_square_covers_expected_columns", {}),
    ("test_oracle_render", "test_translating_square_box_filter_count", {"K": 16, "S": 1}),
    ("test_oracle_render", "test_translating_square_box_filter_count", {"K": 23, "S": 3}),
    ("test_oracle_render", "test_fast_solver_equals_naive_solve", {}),
    ("test_oracle_render", "test_keyframe_distance_exact_for_translation_and_at_keyframes", {}),
    ("test_oracle_render", "test_single_static_triangle_closed_forms", {}),
    ("test_oracle_render", "test_two_triangles_background_product_and_depth_order", {}),
    ("test_oracle_solver", "test_schedule_matches_global_uniform_times", {}),
    ("test_oracle_grad", "test_attribute_gradient_is_exact_for_a_linear_functional", {}),
    ("test_oracle_grad", "test_vertex_gradient_matches_frozen_decision_fd", {"seed": 5}),
    ("test_oracle_grad", "test_closest_point_weights_carry_gradient", {}),
    ("test_oracle_guard", "test_counters_match_brute_force_single_triangle", {}),
    ("test_oracle_guard", "test_guard_band_pins_clamp_decision_of_closest_point", {}),
]


def _fails(mod, fn, kw):
    try:
        getattr(importlib.import_module(mod), fn)(**kw)
    except Exception:
        return True
    return False


@pytest.fixture
def mutant_lib(tmp_path):
    src = open(obuild.SRC).read()
    saved = (obuild.SRC, obuild.LIB, omod._lib)

    def load(old, new):
        assert src.count(old) == 1, old
        path = tmp_path / "mut.c"
        path.write_text(src.replace(old, new))
        lib = tmp_path / f"libmut{abs(hash(old)) % 10**8}.so"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-shared",
                        "-fPIC", str(path), "-o", str(lib), "-lm"], check=True)
        obuild.SRC, obuild.LIB = str(path), str(lib)
        omod._lib = None

    yield load
    obuild.SRC, obuild.LIB, omod._lib = saved


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_every_mutant_is_caught(mutant_lib, name, old, new):
    mutant_lib(old, new)
    caught = [f"{fn}{kw or ''}" for mod, fn, kw in PINS if _fails(mod, fn, kw)]
    assert caught, f"mutant '{name}' passes every pin"


def test_unmutated_oracle_passes_the_pins():
    assert not [fn for mod, fn, kw in PINS if _fails(mod, fn, kw)]
