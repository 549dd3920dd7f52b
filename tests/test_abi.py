"""CPU-side checks of the C-ABI library: it loads, exports every symbol that
include/af.h declares, validates arguments on the host, and its host
quadtree logic (balance check, side relations, regrid) agrees with the
oracle's.  No kernel is launched here."""
import os
import re

import numpy as np
import pytest

import afsynth
import oracle
import paper_2205_07572_amd as af
from paper_2205_07572_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "af.h")


def _declared(path=HEADER):
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(af_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = _lib.load()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(_lib.EXPORTS) == names


def test_measurement_probes_stay_out_of_the_public_header():
    """Benchmark helpers are declared in the library's internal probe header,
    exported, and not part of include/af.h."""
    L = _lib.load()
    probe_h = os.path.join(os.path.dirname(HEADER), "..", "paper_2205_07572_amd", "csrc", "af_probe.h")
    names = _declared(probe_h)
    assert names == sorted(_lib.PROBES)
    for n in names:
        assert hasattr(L, n), n
        assert n not in _declared()


@pytest.mark.parametrize("field,value,status", [("m", 12, _lib.AF_ERR_ARG), ("eq", 5, _lib.AF_ERR_ARG),
                                                ("prec", 3, _lib.AF_ERR_ARG), ("lmax", 40, _lib.AF_ERR_ARG),
                                                ("lx", -1.0, _lib.AF_ERR_ARG), ("c", 0.0, _lib.AF_ERR_ARG)])
def test_ctx_rejects_bad_problems(field, value, status):
    p = af.Problem(eq=1, prec=0, m=16)
    setattr(p, field, value)
    with pytest.raises(af.AFError) as e:
        af.Context(p)
    assert e.value.status == status


@pytest.mark.parametrize("qmax", [0.0, -1.0, float("inf")])
def test_burgers_needs_a_bound_on_q(qmax):
    with pytest.raises(af.AFError) as e:
        af.Context(af.Problem(eq=af.BURGERS, prec=0, m=16, qmax=qmax))
    assert e.value.status == _lib.AF_ERR_ARG


@pytest.mark.parametrize("prec,nblocks,iters", [(7, 1, 1), (0, 0, 1), (1, 1, 0)])
def test_fma_probe_validates_arguments(prec, nblocks, iters):
    """Rejected on the host before any launch (no GPU needed)."""
    import ctypes
    buf = ctypes.create_string_buffer(8)
    st = _lib.load().af_fma_probe(prec, ctypes.cast(buf, ctypes.c_void_p), nblocks, iters, None)
    assert st == _lib.AF_ERR_ARG


def test_tile_heights_validated():
    ctx = af.Context(af.Problem(eq=0, prec=1, m=32))
    assert ctx.tile in (4, 8)
    ctx.tile = 4
    assert ctx.tile == 4
    with pytest.raises(af.AFError):
        ctx.tile = 3


def test_default_advance_shape_follows_the_velocity_signs():
    """Advection lists the shapes that only the upwind one-pass kernel runs
    (its source pattern needs both velocity components positive); the default
    shape is one of them only for such a velocity."""
    up = af.Context(af.Problem(eq=0, prec=1, m=32, a=1.0, b=0.5))
    mixed = af.Context(af.Problem(eq=0, prec=1, m=32, a=0.8, b=-0.45))
    assert up.advance_shapes() == mixed.advance_shapes()
    k_up, _ = up.advance_shape
    k_mixed, _ = mixed.advance_shape
    assert k_up == max(k for k, _ in up.advance_shapes())
    assert 0 < k_mixed < k_up


@pytest.mark.parametrize("leaves,msg", [
    ([(0, 0, 0), (0, 1, 0), (0, 0, 1)], "cover"),                       # hole
    ([(0, 0, 0), (0, 1, 0), (0, 0, 1), (0, 1, 1), (1, 0, 0)], "overlap"),  # overlap
    ([(1, 0, 0), (0, 1, 0), (0, 0, 1), (0, 1, 1), (1, 1, 0), (1, 0, 1), (1, 1, 1)], "sorted"),
])
def test_hierarchy_rejects_bad_leaf_sets(leaves, msg):
    ctx = af.Context(af.Problem(eq=0, prec=0, m=8, n0x=2, n0y=2, lmax=3))
    with pytest.raises(af.AFError) as e:
        af.Hierarchy(ctx, leaves)
    assert msg in str(e.value)


def test_hierarchy_rejects_unbalanced():
    ctx = af.Context(af.Problem(eq=0, prec=0, m=8, n0x=4, n0y=4, lmax=3))
    leaves = [(0, ix, iy) for iy in range(4) for ix in range(4) if (ix, iy) != (1, 1)]
    leaves += [(1, 2 + (q & 1), 2 + (q >> 1)) for q in range(4) if q != 3]
    leaves += [(2, 6 + (q & 1), 6 + (q >> 1)) for q in range(4)]
    with pytest.raises(af.AFError) as e:
        af.Hierarchy(ctx, afsynth.sort_leaves(leaves))
    assert e.value.status == _lib.AF_ERR_BALANCE


@pytest.mark.parametrize("seed", range(10))
def test_regrid_and_side_relations_match_oracle(seed):
    rng = np.random.default_rng(seed)
    n0x, n0y = 2 + seed % 2, 2 + (seed // 2) % 3
    ctx = af.Context(af.Problem(eq=1, prec=0, m=8, n0x=n0x, n0y=n0y, lmax=4))
    o = oracle.Hier(1, 8, n0x, n0y, 4)
    leaves = afsynth.uniform_leaves(n0x, n0y, 1)
    o.set_leaves(leaves)
    h = af.Hierarchy(ctx, leaves)
    for _ in range(6):
        tags = rng.integers(-1, 2, len(leaves)).astype(np.int8)
        o.regrid(tags)
        h = h.regrid(tags)
        assert h.leaves() == o.leaves()
        np.testing.assert_array_equal(h.side_relations(), o.side_relations())
        leaves = h.leaves()
    assert len(set(l for l, _, _ in leaves)) >= 2


def test_level_ranges_cover_sorted_leaves():
    ctx = af.Context(af.Problem(eq=0, prec=0, m=8, n0x=2, n0y=2, lmax=2))
    h = af.Hierarchy(ctx, afsynth.diagonal_leaves(2, 1))
    total = 0
    for l in range(3):
        f, c = h.level_range(l)
        assert all(lv == l for lv, _, _ in h.leaves()[f:f + c])
        total += c
    assert total == len(h) and h.finest() == 2


def test_missing_library_fails_loudly(tmp_path):
    """No CPU fallback: with libaf.so absent, the first call into the
    package raises instead of computing anything."""
    import subprocess
    import sys
    code = (
        "import paper_2205_07572_amd as af, paper_2205_07572_amd._lib as L\n"
        f"L.LIB_PATH = {str(tmp_path / 'absent.so')!r}\n"
        "L._lib = None\n"
        "try:\n"
        "    af.Context(af.Problem())\n"
        "except RuntimeError as e:\n"
        "    print('raised:', e)\n"
        "else:\n"
        "    raise SystemExit('no error')\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert "raised:" in r.stdout and "is not built" in r.stdout


def _fake_pair(ctx, npatch):
    """Two states with aligned non-null pointers: enough for the host-side
    validation, which rejects the calls below before anything is launched."""
    import ctypes
    pair = (_lib.af_state * 2)()
    for k in range(2):
        for q in range(4):
            pair[k].dof[q] = ctypes.c_void_p(4096 * (1 + 4 * k + q))
        pair[k].npatch = npatch
        pair[k].pitch = ctx.prob.m + 5
    return pair


def test_noalloc_sum_rejects_too_many_leaves_and_undeployed_hierarchies():
    """af_reduce_sum_noalloc: more partial sums than its static scratch holds
    is AF_ERR_ARG; a hierarchy whose tables are not on the device yet is
    AF_ERR_STATE (uploading them would allocate)."""
    import ctypes
    L = _lib.load()
    out = ctypes.c_void_p(4096)
    big = af.Context(af.Problem(eq=1, prec=1, m=8, n0x=257, n0y=256, lmax=0))   # 65792 leaves x 3 > 196608
    hb = af.Hierarchy(big, afsynth.uniform_leaves(257, 256, 0))
    st = L.af_reduce_sum_noalloc(big.h, hb.h, _fake_pair(big, len(hb)), 0, out, None)
    assert st == _lib.AF_ERR_ARG and b"exceeds the static scratch" in L.af_last_error()
    ok = af.Context(af.Problem(eq=1, prec=1, m=8, n0x=256, n0y=256, lmax=0))    # exactly 196608: admitted
    ho = af.Hierarchy(ok, afsynth.uniform_leaves(256, 256, 0))
    st = L.af_reduce_sum_noalloc(ok.h, ho.h, _fake_pair(ok, len(ho)), 0, out, None)
    assert st == _lib.AF_ERR_STATE and b"not uploaded" in L.af_last_error()


@pytest.mark.parametrize("nsteps,flags", [(0, 0), (-3, 0), (2, 1), (2, 4)])
def test_coarse_steps_validates_count_and_flags(nsteps, flags):
    """af_amr_coarse_steps rejects a non-positive step count and any flag but
    AF_STEP_GLOBAL (graph replay included) before it touches the device."""
    import ctypes
    ctx = af.Context(af.Problem(eq=1, prec=0, m=8, n0x=2, n0y=2, lmax=1))
    h = af.Hierarchy(ctx, afsynth.uniform_leaves(2, 2, 0))
    mk = ctypes.c_uint32(0)
    st = _lib.load().af_amr_coarse_steps(ctx.h, h.h, None, ctypes.byref(mk), 0.0, 1e-3, nsteps,
                                         ctypes.c_void_p(16), flags, None)
    assert st == _lib.AF_ERR_ARG
