"""The C-ABI library: it loads, exports every function include/igamg.h
declares, and its host-only entry points and argument checks work without a
GPU (no compute call is made here)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "igamg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(igamg_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def ig():
    from paper_1902_01818_amd import igamg
    return igamg


def test_exports_every_declared_symbol(ig):
    names = _declared()
    assert len(names) >= 16
    for n in names:
        assert hasattr(ig._lib, n), n
    assert sorted(ig.EXPORTED) == names


def test_options_layout(ig):
    # the ctypes mirror of igamg_options must have the C size
    o = ig.make_options()
    assert o.precision == 0 and o.outer == 0 and o.max_rhs == 0
    assert o.damping_tau == 0.25 and o.scaling_delta == 0.1 and o.mu == 1 and o.nu == 1


def test_strerror(ig):
    for code in (0, -1, -2, -3, -4, 1):
        assert ig._lib.igamg_strerror(code)
    assert ig._lib.igamg_strerror(0) == b"success"


def test_footprint_scales_with_batch_and_precision(ig):
    import workloads
    cfg = workloads.config("c2")
    b1 = ig.footprint(cfg["corners"], cfg["elems"], cfg["p"])
    b64 = ig.footprint(cfg["corners"], cfg["elems"], cfg["p"], max_rhs=64)
    b32 = ig.footprint(cfg["corners"], cfg["elems"], cfg["p"], precision="fp32")
    # float32 holds half the bytes per stored value but assembles its
    # stencils in float64 first, so only the batch ordering is fixed
    assert b64 > b1 > 0 and b32 > 0


def _setup_code(ig, corners, elems, degree, sigma=5.0, **opts):
    P, keep, degree = ig._patches(corners, elems, degree)
    o = ig.make_options(**opts)
    h = ctypes.c_void_p()
    return ig._lib.igamg_setup(ctypes.byref(P), degree, sigma, ctypes.byref(o), None,
                               ctypes.byref(h))


def test_setup_rejects_invalid_input_before_gpu_work(ig):
    sq = np.array([[[0, 0], [1, 0], [0, 1], [1, 1]]], dtype=np.float64)
    el = np.array([[4, 4]], dtype=np.int32)
    assert _setup_code(ig, sq, el, 0) == ig.EINVAL                         # degree
    assert _setup_code(ig, sq, el, 9) == ig.EINVAL
    assert _setup_code(ig, sq, el, 2, sigma=0.0) == ig.EINVAL              # SIPG penalty
    assert _setup_code(ig, sq, el, 2, max_rhs=-1) == ig.EINVAL
    assert _setup_code(ig, sq, el, 2, gs_tile=10) == ig.EUNSUPPORTED      # tile != 2(p+1)
    # a degree per patch: SIPG only, 2D and 3D (any smoother); degrees 1..8
    two = np.array([[[0, 0], [1, 0], [0, 1], [1, 1]], [[1, 0], [2, 0], [1, 1], [2, 1]]],
                   dtype=np.float64)
    el2 = np.array([[4, 4], [2, 2]], dtype=np.int32)
    assert _setup_code(ig, two, el2, [2, 3], smoother="scms", conforming=True) == ig.EUNSUPPORTED
    assert _setup_code(ig, two, el2, [2, 9], smoother="scms") == ig.EINVAL
    cubes = np.array([[[x + a, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)]
                      for a in (0, 1)], dtype=np.float64)
    assert _setup_code(ig, cubes, np.full((2, 3), 2, dtype=np.int32), [2, 3],
                       smoother="scms", conforming=True) == ig.EUNSUPPORTED
    assert _setup_code(ig, cubes, np.full((2, 3), 2, dtype=np.int32), [2, 5],
                       smoother="scms") == ig.EUNSUPPORTED   # 3D degrees 1..4
    # stored operator rows exist only with a Gauss-Seidel smoother in the SIPG space
    assert _setup_code(ig, sq, el, 2, smoother="scms", operator_apply="rows") == ig.EUNSUPPORTED
    assert _setup_code(ig, sq, el, 2, conforming=True, smoother="scms",
                       operator_apply="rows") == ig.EUNSUPPORTED
    cube = np.array([[[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)]], dtype=np.float64)
    e4 = np.array([[4, 4, 4]], dtype=np.int32)
    # 3D: degree 1..4; the smoother / operator-form rules of 2D
    assert _setup_code(ig, cube, e4, 5, smoother="gs") == ig.EUNSUPPORTED
    assert _setup_code(ig, cube, e4, 2, smoother="scms", operator_apply="rows") == ig.EUNSUPPORTED


def test_problem_size_matches_oracle_numbering(ig):
    import oracle
    import workloads
    from oracle.hierarchy import level_elements
    for name, scale, n_expected in (("c1", 1, 1089), ("c2", 8, None), ("c2", 1, 115652)):
        cfg = workloads.config(name, scale)
        n, lv = ig.problem_size(cfg["corners"], cfg["elems"], cfg["p"], conforming=cfg["conforming"],
                                smoother=cfg["smoother"])
        if n_expected is None:
            n_expected = oracle.setup(cfg["corners"], cfg["elems"], cfg["p"],
                                      conforming=cfg["conforming"]).N
        assert n == n_expected
        assert lv == len(level_elements(cfg["elems"]))


def test_problem_size_3d_matches_oracle_numbering(ig):
    """3D SIPG (trilinear 2x2x2 patches, checkerboard 48/64 at p = 3 and the
    same layout divided by 8): unknown count after Dirichlet elimination and
    level count equal the oracle's."""
    import numpy as np
    import workloads
    from oracle.discretize import Topology, Level
    from oracle.hierarchy import level_elements
    for scale in (1, 8):
        cfg = workloads.config("c3", scale)
        n, lv = ig.problem_size(cfg["corners"], cfg["elems"], cfg["p"], smoother="gs")
        lev = Level(Topology(cfg["corners"]), np.asarray(cfg["elems"]), cfg["p"], False, None)
        assert n == lev.N
        assert lv == len(level_elements(cfg["elems"]))
    assert n == 6048


def test_binding_constants_match_header(ig):
    """The binding's option and status values are the header's #defines."""
    import re
    text = open(os.path.join(ROOT, "include", "igamg.h")).read()
    defs = {m.group(1): int(m.group(2))
            for m in re.finditer(r"#define (IGAMG_\w+) \(?(-?\d+)\)?", text)}
    assert (ig.OK, ig.EINVAL, ig.EUNSUPPORTED, ig.ENOMEM, ig.EHIP, ig.ENOCONV) == tuple(
        defs["IGAMG_" + k] for k in ("OK", "EINVAL", "EUNSUPPORTED", "ENOMEM", "EHIP", "ENOCONV"))
    assert (ig.SIPG, ig.CONFORMING) == (defs["IGAMG_SIPG"], defs["IGAMG_CONFORMING"])
    assert ig.SMOOTHERS == {"hybrid": defs["IGAMG_SMOOTHER_HYBRID"],
                            "scms": defs["IGAMG_SMOOTHER_SCMS"], "gs": defs["IGAMG_SMOOTHER_GS"]}
    assert ig.PRECISIONS == {"fp64": defs["IGAMG_FP64"], "fp32": defs["IGAMG_FP32"],
                             "bf16": defs["IGAMG_BF16_SCMS"]}
    assert ig.OUTERS == {"pcg": defs["IGAMG_OUTER_PCG"], "mg": defs["IGAMG_OUTER_MG"],
                         "fcg": defs["IGAMG_OUTER_FCG"], "ir": defs["IGAMG_OUTER_IR"]}
    assert ig.APPLIES == {"auto": defs["IGAMG_APPLY_AUTO"], "sumfact": defs["IGAMG_APPLY_SUMFACT"],
                          "rows": defs["IGAMG_APPLY_ROWS"]}
    assert ig.MANUFACTURED_SINE == defs["IGAMG_MANUFACTURED_SINE"]


def test_entry_point_arity_matches_header(ig):
    """Every binding argtypes list has as many entries as the header's
    prototype has parameters (a stale binding would pass garbage)."""
    import re
    text = open(os.path.join(ROOT, "include", "igamg.h")).read()
    protos = {m.group(1): m.group(2) for m in
              re.finditer(r"\b(igamg_\w+)\(([^;{]*?)\);", text, flags=re.S)}
    for name in ig.EXPORTED:
        args = protos[name].strip()
        n = 0 if args in ("", "void") else args.count(",") + 1
        fn = getattr(ig._lib, name)
        if fn.argtypes is not None:
            assert len(fn.argtypes) == n, (name, len(fn.argtypes), n)


def test_options_struct_layout_matches_header(ig):
    """The ctypes mirror of igamg_options lists the header's fields in order."""
    import re
    text = open(os.path.join(ROOT, "include", "igamg.h")).read()
    body = text[text.index("typedef struct {\n  int discretization;"):]
    body = body[:body.index("} igamg_options;")]
    fields = re.findall(r"^\s+(?:int|double) (\w+);", body, re.M)
    assert fields == [f for f, _ in ig.Options._fields_]
