"""Planted mistakes in the oracle fail its pins (no GPU).

Each case copies the oracle's C sources, plants one plausible mistake (a
dropped or extra term, a wrong sign, an inverted order, a check switched
off), builds the variant into a temporary library and runs the pins named
for it against that library in a child process: they must fail.  The same
pins pass against the unmodified oracle in the rest of the suite.
"""
import os
import shutil
import subprocess
import sys

import pytest

import oracle.oracle as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

PINS_COST = "tests/test_oracle_cost_pins.py"
PINS_MESH = "tests/test_oracle_mesh_pins.py"
PINS_PRED = "tests/test_oracle_predicates.py"

# name: (file, original text, planted text, pins that must fail)
MUTANTS = {
    "skinny_counts_vanishing_faces": (
        "oracle_mesh.c",
        "            if (face_has(m, f, s) && face_has(m, f, r)) continue;\n            S = S + skinny_term(",
        "            S = S + skinny_term(",
        [f"{PINS_COST}::test_skinny_sum_restated", f"{PINS_COST}::test_flat_patch_closed_form"]),
    "skinny_at_old_positions": (
        "oracle_mesh.c",
        "            S = S + skinny_term(corner_after(m, f, 0, s, r, vbar), corner_after(m, f, 1, s, r, vbar),\n"
        "                                corner_after(m, f, 2, s, r, vbar));",
        "            S = S + skinny_term(m->V + 3 * (int64_t)m->F[3 * (int64_t)f], "
        "m->V + 3 * (int64_t)m->F[3 * (int64_t)f + 1],\n"
        "                                m->V + 3 * (int64_t)m->F[3 * (int64_t)f + 2]);",
        [f"{PINS_COST}::test_skinny_sum_restated", f"{PINS_COST}::test_flat_patch_closed_form"]),
    "skinny_one_end_only": (
        "oracle_mesh.c",
        "    for (int side = 0; side < 2; side++) {\n        int32_t v = side ? r : s;",
        "    for (int side = 0; side < 1; side++) {\n        int32_t v = side ? r : s;",
        [f"{PINS_COST}::test_skinny_sum_restated", f"{PINS_COST}::test_flat_patch_closed_form"]),
    "cap_keeps_largest_keys": (
        "oracle_mesh.c",
        "        for (int64_t i = need; i < npass; i++) reason[pass[i]] = 4;",
        "        for (int64_t i = 0; i < npass - need; i++) reason[pass[i]] = 4;",
        [f"{PINS_COST}::test_cap_keeps_smallest_keys"]),
    "quadric_offset_sign": (
        "oracle_mesh.c",
        "    double d = -(nx * p0[0] + ny * p0[1] + nz * p0[2]);",
        "    double d = (nx * p0[0] + ny * p0[1] + nz * p0[2]);",
        [f"{PINS_MESH}::test_quadric_is_sum_of_squared_plane_distances"]),
    "selection_ignores_one_ring": (
        "oracle_mesh.c",
        "        int all = 1;\n        for (int i = 0; i < n; i++)\n            if (Ct[ring[i]] != k) { all = 0; break; }",
        "        int all = 1;\n        for (int i = 0; i < n / 2; i++)\n            if (Ct[ring[i]] != k) { all = 0; break; }",
        [f"{PINS_MESH}::test_selection_pairwise_definition"]),
    "key_order_inverted": (
        "oracle_mesh.c",
        "    uint32_t o = (u >> 31) ? ~u : (u | 0x80000000u);",
        "    uint32_t o = (u >> 31) ? (u | 0x80000000u) : ~u;",
        [f"{PINS_MESH}::test_key_order_matches_float32_order"]),
    "link_condition_off": (
        "oracle_mesh.c",
        "    if (!link_ok(m, a, b)) return 1;",
        "    (void)link_ok;",
        [f"{PINS_MESH}::test_link_condition_fixtures"]),
    "flip_check_off": (
        "oracle_mesh.c",
        "        if (!(dot > 0.0)) return 2;",
        "        (void)dot;",
        [f"{PINS_MESH}::test_flip_rejections_match_exact_normal_test"]),
    "shared_edge_opposite_side": (
        "oracle_tri.c",
        "    return sc * sd > 0;",
        "    return sc * sd < 0;",
        [f"{PINS_PRED}::test_coplanar_figure_cases", f"{PINS_PRED}::test_tri_pair_matches_exact_lp"]),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_its_pins(name, tmp_path):
    fname, old, new, pins = MUTANTS[name]
    for src in orc.SOURCES + ("oracle_internal.h",):
        shutil.copy(os.path.join(ORACLE, src), tmp_path / src)
    text = (tmp_path / fname).read_text()
    assert text.count(old) == 1, f"{name}: the planted site is not unique or has moved"
    (tmp_path / fname).write_text(text.replace(old, new))
    lib = orc.build(src_dir=str(tmp_path), out=str(tmp_path / "liboracle_mutant.so"))
    env = dict(os.environ, PAMO_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] + pins,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    # 1: tests ran and some failed (a crash of the variant counts as failing too)
    assert r.returncode == 1 or r.returncode < 0, f"{name}: pins did not fail\n{r.stdout[-2000:]}{r.stderr[-2000:]}"
    assert "failed" in r.stdout or r.returncode < 0


def test_unplanted_copy_passes(tmp_path):
    """The harness itself: an unmodified copy built the same way passes the
    pins the mutants are run against."""
    for src in orc.SOURCES + ("oracle_internal.h",):
        shutil.copy(os.path.join(ORACLE, src), tmp_path / src)
    lib = orc.build(src_dir=str(tmp_path), out=str(tmp_path / "liboracle_copy.so"))
    pins = sorted({p for m in MUTANTS.values() for p in m[3]})
    env = dict(os.environ, PAMO_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] + pins,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
