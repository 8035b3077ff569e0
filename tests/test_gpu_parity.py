"""GPU parity: the HIP library against the FP64 oracle on the same seeded inputs.

Tolerances: FP64 storage |dphi|_inf <= 1e-10 (rounding order only); FP32 storage
|dphi|_inf <= 1e-5 against the FP64 oracle; contact angle within 0.5 degrees.
"""
import math
import os

import numpy as np
import pytest

import workloads
from tests.helpers import maxdiff, oracle_for, oracle_theta

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
# FP32 storage against the FP64 oracle: relative mass difference after 5000 steps
FP32_MASS_TOL = 3e-9


def _zeta(case):
    return (case.classes() & 1).astype(bool)


def _compare(gf, of, zeta, tol_phi, tol_other):
    assert maxdiff(gf["phi"], of["phi"], zeta) <= tol_phi, maxdiff(gf["phi"], of["phi"], zeta)
    assert maxdiff(gf["mu"], of["mu"], zeta) <= tol_other
    assert maxdiff(gf["p"], of["p"], zeta) <= tol_other
    for d in range(gf["u"].shape[0]):
        assert maxdiff(gf["u"][d], of["u"][d], zeta) <= tol_other


def test_init_fields_fp64(P):
    c = workloads.flat_128x64_fp64()
    g = P.Case.from_case(c, "f64")
    o = oracle_for(c)
    zeta = _zeta(g)
    assert np.array_equal(zeta, o.domain(o.zeta))
    _compare(g.fields(), o.fields(), zeta, 1e-13, 1e-13)
    # ghost values (phi on ghost nodes is reported too)
    ghost = (g.classes() & 4).astype(bool)
    assert maxdiff(g.fields()["phi"], o.fields()["phi"], ghost) <= 1e-13


@pytest.mark.parametrize("shape,periodic", [((128, 64), (True, False)), ((67, 37), (True, False)),
                                            ((61, 45), (False, False)), ((5, 33), (True, False))])
def test_parity_fp64_short(P, shape, periodic):
    """200 steps on several shapes, including ragged tiles and a 5-wide periodic domain."""
    nx, ny = shape
    c = workloads.flat_droplet_case(nx, ny, min(20.0, 0.3 * ny), 60.0, 4.0)
    c["periodic"] = periodic
    g = P.Case.from_case(c, "f64")
    o = oracle_for(c)
    zeta = _zeta(g)
    for k in range(4):
        g.step(50)
        o.step(50)
        _compare(g.fields(), o.fields(), zeta, 1e-12, 1e-12)
        assert abs(g.diagnostics()["mass"] - o.mass()) <= 1e-11 * o.mass()


def test_parity_fp64_flat_128x64_golden(P):
    """128x64 FP64 flat-wall droplet, 5000 steps; fields and mass trajectory against the
    stored oracle run (tests/golden/make_golden.py)."""
    gold = np.load(os.path.join(GOLDEN, "flat_128x64_fp64.npz"), allow_pickle=False)
    c = workloads.flat_128x64_fp64()
    g = P.Case.from_case(c, "f64")
    zeta = _zeta(g)
    every = int(gold["mass_every"])
    masses = []
    for k in range(len(gold["mass"])):
        masses.append(g.diagnostics()["mass"])
        if k + 1 < len(gold["mass"]):
            g.step(every)
    assert g.steps == int(gold["steps"])
    rel = np.abs(np.array(masses) - gold["mass"]) / gold["mass"]
    assert rel.max() <= 1e-10, rel.max()
    f = g.fields()
    assert maxdiff(f["phi"], gold["phi"], zeta) <= 1e-10
    assert maxdiff(f["p"], gold["p"], zeta) <= 1e-10
    d = g.diagnostics()
    assert abs(d["theta_deg"] - float(gold["theta"])) <= 0.5


def test_parity_fp32_flat_128x64_golden(P):
    gold = np.load(os.path.join(GOLDEN, "flat_128x64_fp64.npz"), allow_pickle=False)
    c = workloads.flat_128x64_fp64()
    g = P.Case.from_case(c, "f32")
    zeta = _zeta(g)
    g.step(int(gold["steps"]))
    f = g.fields()
    err = maxdiff(f["phi"], gold["phi"], zeta)
    print(f"FP32 |dphi|_inf after {int(gold['steps'])} steps: {err:.3e}")
    assert err <= 1e-5
    d = g.diagnostics()
    assert abs(d["theta_deg"] - float(gold["theta"])) <= 0.5
    rel_mass = abs(d["mass"] - float(gold["mass"][-1])) / float(gold["mass"][-1])
    print(f"FP32 relative mass difference: {rel_mass:.3e}")
    assert rel_mass <= FP32_MASS_TOL, rel_mass


def test_theta_parity_fp64_on_a_moving_drop(P):
    """Contact angle of the GPU diagnostics (moment reduction + host circle fit)
    against the oracle's estimator on the oracle's fields, FP64, on a drop that
    spreads from 90 deg towards the prescribed 60 deg: equal within 1e-6 deg
    after the angle has moved by more than 5 deg (and at the start).""" 
    import math
    from oracle import diagnostics as odiag
    W, sigma = 4.0, 1e-2
    c = workloads.flat_droplet_case(96, 48, 15.0, 60.0, W, sigma)
    g = P.Case.from_case(c, "f64", mobility=0.2)
    o = oracle_for(c, mobility=0.2)
    th0 = g.diagnostics()["theta_deg"]
    o0 = odiag.contact_angle(o.fields()["phi"], o.domain(o.zeta), c["wall"], W)[0]
    assert abs(th0 - o0) <= 1e-6, (th0, o0)
    g.step(5000)
    o.step(5000)
    th = g.diagnostics()["theta_deg"]
    ot = odiag.contact_angle(o.fields()["phi"], o.domain(o.zeta), c["wall"], W)[0]
    print(f"theta: start {th0:.6f}, after 5000 steps GPU {th:.9f} oracle {ot:.9f}")
    assert abs(th - th0) >= 5.0, (th0, th)
    assert abs(th - ot) <= 1e-6, (th, ot)
    assert math.isfinite(th)


def test_parity_d3q19_fp64(P):
    """D3Q19 for both sets, staircase inclined wall, all faces walls: 40 steps."""
    c = workloads.inclined_droplet_case_3d(n=24, radius=7.0, theta=45.0, width=4.0)
    g = P.Case.from_case(c, "f64")
    o = oracle_for(c)
    zeta = _zeta(g)
    assert np.array_equal(zeta, o.domain(o.zeta))
    _compare(g.fields(), o.fields(), zeta, 1e-13, 1e-13)
    for k in range(2):
        g.step(20)
        o.step(20)
        _compare(g.fields(), o.fields(), zeta, 1e-12, 1e-12)


def test_parity_d3q19_d3q7_fp64(P):
    """D3Q19 for f and the stencils, D3Q7 for g (Sec. 2.1.3), staircase inclined
    wall: 40 steps against the FP64 oracle with the same lattices."""
    c = workloads.inclined_droplet_case_3d(n=24, radius=7.0, theta=45.0, width=4.0)
    c["phase_lattice"] = "D3Q7"
    g = P.Case.from_case(c, "f64")
    o = oracle_for(c)
    assert o.g.shape[0] == 7
    zeta = _zeta(g)
    assert np.array_equal(zeta, o.domain(o.zeta))
    _compare(g.fields(), o.fields(), zeta, 1e-13, 1e-13)
    for k in range(2):
        g.step(20)
        o.step(20)
        _compare(g.fields(), o.fields(), zeta, 1e-12, 1e-12)


def test_mass_budget_identity_d3q7(P):
    """The mass budget with D3Q7 for g, FP64 on the GPU."""
    c = workloads.inclined_droplet_case_3d(n=20, radius=6.0, theta=60.0, width=4.0)
    c["phase_lattice"] = "D3Q7"
    g = P.Case.from_case(c, "f64")
    g.step(50)
    d0 = g.diagnostics()
    g.step(1)
    d1 = g.diagnostics()
    resid = d1["mass"] - d0["mass"] + 1.5 * d1["s_sum"] - 0.5 * d0["s_sum"]
    assert abs(resid) <= 1e-12 * d0["mass"], resid


def test_parity_d3q19_periodic_fp32(P):
    c = workloads.inclined_droplet_case_3d(n=20, radius=6.0, theta=120.0, width=4.0)
    c["periodic"] = (False, True, False)
    g = P.Case.from_case(c, "f32")
    o = oracle_for(c)
    zeta = _zeta(g)
    g.step(30)
    o.step(30)
    _compare(g.fields(), o.fields(), zeta, 1e-5, 1e-5)


def test_mass_budget_identity(P):
    """M(t+1) - M(t) = -(1.5 S(t) - 0.5 S(t-1)) with S the sum of s over zeta = 1."""
    c = workloads.flat_128x64_fp64()
    g = P.Case.from_case(c, "f64")
    g.step(100)
    d0 = g.diagnostics()
    g.step(1)
    d1 = g.diagnostics()
    resid = d1["mass"] - d0["mass"] + 1.5 * d1["s_sum"] - 0.5 * d0["s_sum"]
    assert abs(resid) <= 1e-12 * d0["mass"], resid


def test_graph_equals_eager_bitwise(P):
    c = workloads.flat_droplet_case(96, 48, 14.0, 120.0, 4.0)
    a = P.Case.from_case(c, "f32")
    b = P.Case.from_case(c, "f32")
    a.set_graph_chunk(0)
    b.set_graph_chunk(16)
    a.step(101)
    b.step(101)
    fa, fb = a.fields(), b.fields()
    assert np.array_equal(fa["phi"], fb["phi"]) and np.array_equal(fa["u"], fb["u"])


def test_tile_shape_invariance_bitwise(P):
    c = workloads.flat_droplet_case(150, 70, 20.0, 45.0, 4.0)
    ref = None
    for tile in [(64, 4, 1), (128, 2, 1), (64, 1, 1), (256, 4, 1)]:
        g = P.Case.from_case(c, "f32")
        g.set_tile(*tile)
        g.step(60)
        f = g.fields()
        if ref is None:
            ref = f
        else:
            assert np.array_equal(ref["phi"], f["phi"]) and np.array_equal(ref["p"], f["p"])


def test_translation_bitwise(P):
    """Shifting the initial field along the periodic axis shifts the result exactly."""
    c = workloads.flat_droplet_case(128, 48, 14.0, 70.0, 4.0)
    c2 = dict(c)
    c2["phi0"] = np.roll(c["phi0"], 37, axis=1)
    a = P.Case.from_case(c, "f32")
    b = P.Case.from_case(c2, "f32")
    a.step(80)
    b.step(80)
    assert np.array_equal(np.roll(a.fields()["phi"], 37, axis=1), b.fields()["phi"])


def test_checkpoint_resume_bitwise(P):
    c = workloads.flat_droplet_case(96, 48, 14.0, 60.0, 4.0)
    a = P.Case.from_case(c, "f32")
    a.step(30)
    blob = a.get_state()
    a.step(40)
    b = P.Case.from_case(c, "f32")
    b.set_state(blob)
    assert b.steps == 30
    b.step(40)
    assert np.array_equal(a.fields()["phi"], b.fields()["phi"])


def test_checkpoint_keeps_fp16_scales(P):
    """FP16-deviation checkpoints carry the scales the populations are stored
    with: a blob taken after the scales moved resumes bit for bit in a fresh
    case (initial scales), in the same case after a diagnostics call moved its
    scales again, and in a group member."""
    c = workloads.flat_droplet_case(96, 48, 14.0, 60.0, 4.0)
    a = P.Case.from_case(c, "f16dev")
    a.step(30)
    sf, sg = a.fp16_scales()
    a.set_fp16_scales(sf / 64, sg / 32)          # out of the band: the upkeep will move them
    blob = a.get_state()
    a.step(40)
    ref = a.fields()["phi"]
    b = P.Case.from_case(c, "f16dev")
    b.set_state(blob)
    assert b.fp16_scales() == (sf / 64, sg / 32)
    b.step(40)
    assert np.array_equal(b.fields()["phi"], ref)
    a.diagnostics()                              # moves the scales back into the band
    assert a.fp16_scales() != (sf / 64, sg / 32)
    a.set_state(blob)
    assert a.fp16_scales() == (sf / 64, sg / 32)
    a.step(40)
    assert np.array_equal(a.fields()["phi"], ref)
    m = P.Case.from_case(c, "f16dev")
    g = P.Group()
    g.add(m)
    g.step(6)
    m.set_state(blob)
    g.step(40)
    assert m.steps == 70
    assert np.array_equal(m.fields()["phi"], ref)
    g.remove(m)
    g.close()


def test_workspace_create_matches(P):
    c = workloads.flat_droplet_case(96, 48, 14.0, 60.0, 4.0)
    a = P.Case.from_case(c, "f32")
    b = P.Case.from_case(c, "f32", workspace=True)
    a.step(25)
    b.step(25)
    assert np.array_equal(a.fields()["phi"], b.fields()["phi"])


def test_uniform_phase_is_fixed_point(P):
    """phi = 1 everywhere with walls: mu = 0, F = 0, u = 0; populations do not move."""
    c = workloads.flat_droplet_case(64, 32, 10.0, 60.0, 4.0)
    c["phi0"] = np.ones_like(c["phi0"])
    c["theta_deg"] = 90.0   # cos(theta) = 0: no wall term at phi = 1 either way
    g = P.Case.from_case(c, "f64")
    f0 = g.fields()
    g.step(50)
    f1 = g.fields()
    assert np.array_equal(f0["phi"], f1["phi"])
    assert np.abs(f1["u"]).max() == 0.0


def _geom(lattice):
    if lattice == "D2Q9":
        c = workloads.cylinder_case(97, 45, 0.3, 110.0)
    else:
        c = workloads.inclined_droplet_case_3d(n=22, radius=6.0, theta=50.0, width=4.0)
        c["periodic"] = (False, True, False)
        if lattice == "D3Q19/D3Q7":
            c["phase_lattice"] = "D3Q7"
    return c


@pytest.mark.parametrize("lattice,storage", [("D2Q9", "f64"), ("D2Q9", "f32"), ("D2Q9", "f16dev"),
                                             ("D3Q19", "f64"), ("D3Q19", "f32"),
                                             ("D3Q19", "f16dev"), ("D3Q19/D3Q7", "f64"),
                                             ("D3Q19/D3Q7", "f32"), ("D3Q19/D3Q7", "f16dev")])
def test_fused_step_equals_three_kernel_path_bitwise(P, lattice, storage):
    """The one-kernel step (every tile variant) and the phi / mu / collide kernels
    give bit-identical fields; the geometry has ghost nodes inside the domain."""
    c = _geom(lattice)
    ref = P.Case.from_case(c, storage)
    ref.set_step_kernel(-1)
    ref.set_graph_chunk(0)
    ref.step(24)
    fr = ref.fields()
    for v in range(len(P.step_variants(lattice))):
        g = P.Case.from_case(c, storage)
        g.set_step_kernel(v)
        g.step(24)
        f = g.fields()
        for k in ("phi", "p", "u", "mu"):
            assert np.array_equal(f[k], fr[k]), (v, k)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev"])
def test_march_columns_bitwise(P, storage):
    """The fused z-marching step (variants 11, 12: 64 x 4 or 64 x 8 columns of 32
    planes) against the phi / mu / collide kernels, on domains taller than
    one column segment: closed z with a staircase wall crossing segment
    boundaries, periodic z, and periodic x with a ragged x edge."""
    cases = []
    c = workloads.inclined_droplet_case_3d(n=24, radius=6.0, theta=50.0, width=4.0)
    # stretch the 24^3 case along z: 24 x 20 x 75, closed in x and z, periodic in y
    nz = 75
    mask = workloads.inclined_plane((24, 20, nz), (12.0, 30.0), 30.0)
    phi0 = workloads.droplet((24, 20, nz), (12.0, 10.0, 30.0), 7.0, 4.0)
    cases.append(dict(c, shape=(24, 20, nz), periodic=(False, True, False), mask=mask, phi0=phi0))
    cases.append(dict(cases[0], periodic=(False, True, True)))
    m2 = np.zeros((70, 11, 70), np.uint8)
    m2[:3] = 1
    cases.append(dict(c, shape=(70, 11, 70), periodic=(True, False, True), mask=m2,
                      phi0=workloads.droplet((70, 11, 70), (35.0, 5.0, 8.0), 6.0, 4.0)))
    for c in cases:
        ref = P.Case.from_case(c, storage)
        ref.set_step_kernel(-1)
        ref.set_graph_chunk(0)
        ref.step(12)
        fr = ref.fields()
        sr = ref.get_state()
        for v in (11, 12):
            g = P.Case.from_case(c, storage)
            g.set_step_kernel(v)
            g.set_graph_chunk(0)
            g.step(12)
            f = g.fields()
            for k in ("phi", "p", "u", "mu"):
                assert np.array_equal(f[k], fr[k]), (c["shape"], c["periodic"], v, k)
            assert np.array_equal(g.get_state(), sr), (c["shape"], c["periodic"], v)


@pytest.mark.parametrize("lattice,variants", [("D2Q9", (1, 6)), ("D3Q19", (7, 8, 12))])
def test_xcd_orders_bitwise(P, lattice, variants):
    """The three XCD dispatch orders (round-robin, contiguous runs, chunks of
    tile rows; the chunked grid is padded with idle workgroups) only move work
    between XCDs: the fields stay bit-identical."""
    c = _geom(lattice)
    for v in variants:
        out = []
        for xo in (0, 1, 2):
            g = P.Case.from_case(c, "f32")
            g.set_step_kernel(v)
            g.set_step_options(xo, False)
            g.step(16)
            out.append(g.get_state())
        assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2]), v


@pytest.mark.parametrize("variant", [1, 3, 6])
def test_fused_narrow_periodic_and_ragged(P, variant):
    """Tiles wider than a 3- or 5-node periodic domain, ragged tile edges and a
    domain closed in x (fused 64 x 8 (1) and 64 x 16 (3) tiles, split step (6))."""
    for shape, per_x in (((5, 40), True), ((3, 24), True), ((70, 13), True), ((70, 13), False),
                         ((133, 21), False)):
        c = workloads.flat_droplet_case(shape[0], shape[1], 4.0, 70.0, 4.0)
        c["periodic"] = (per_x, False)
        a = P.Case.from_case(c, "f64")
        a.set_step_kernel(-1)
        b = P.Case.from_case(c, "f64")
        b.set_step_kernel(variant)
        a.step(20)
        b.step(20)
        assert np.array_equal(a.fields()["phi"], b.fields()["phi"]), (shape, per_x)
        assert np.array_equal(a.get_state(), b.get_state()), (shape, per_x)


@pytest.mark.parametrize("phase", ["", "D3Q7"])
def test_parity_d3q19_fp32_and_fp16dev_vs_oracle(P, phase):
    """D3Q19 inclined staircase, 300 steps (g on D3Q19, or on D3Q7): FP32 within
    1e-5 of the FP64 oracle; FP16-deviation storage (FP16 moving populations,
    FP32 compute) within 2e-4, with its error printed."""
    c = workloads.inclined_droplet_case_3d(n=24, radius=7.0, theta=60.0, width=4.0)
    if phase:
        c["phase_lattice"] = phase
    o = oracle_for(c)
    o.step(300)
    of = o.fields()
    errs = {}
    for st in ("f32", "f16dev"):
        g = P.Case.from_case(c, st)
        g.step(300)
        zeta = _zeta(g)
        errs[st] = maxdiff(g.fields()["phi"], of["phi"], zeta)
    print(f"D3Q19{'/' + phase if phase else ''} 300 steps |dphi|_inf vs FP64 oracle: "
          f"FP32 {errs['f32']:.2e}, "
          f"FP16-dev {errs['f16dev']:.2e}")
    assert errs["f32"] <= 1e-5
    assert errs["f16dev"] <= 2e-4


def test_fp16dev_flat_128x64_error_statement(P):
    """The 128x64 flat-wall geometry in FP16-deviation storage, 5000 steps, against the
    stored FP64 oracle run: error stated and bounded."""
    gold = np.load(os.path.join(GOLDEN, "flat_128x64_fp64.npz"), allow_pickle=False)
    c = workloads.flat_128x64_fp64()
    g = P.Case.from_case(c, "f16dev")
    zeta = _zeta(g)
    g.step(int(gold["steps"]))
    err = maxdiff(g.fields()["phi"], gold["phi"], zeta)
    d = g.diagnostics()
    print(f"FP16-dev |dphi|_inf after 5000 steps: {err:.3e}; theta {d['theta_deg']:.4f} "
          f"vs {float(gold['theta']):.4f}")
    assert err <= 1e-4
    assert abs(d["theta_deg"] - float(gold["theta"])) <= 0.5


def test_fp16_scale_rescale_and_upkeep(P):
    """FP16-deviation scales (powers of two per set): raising a scale rescales the
    stored state exactly; scales pushed out of band are moved back into it by
    diagnostics without changing the fields; the run then continues within the
    FP16 error of an untouched run.  Bad scales and other storage are refused."""
    c = workloads.inclined_droplet_case_3d(n=20, radius=6.0, theta=60.0, width=4.0)
    a = P.Case.from_case(c, "f16dev")
    b = P.Case.from_case(c, "f16dev")
    a.step(40)
    b.step(40)
    sf, sg = a.fp16_scales()
    f0 = a.fields()
    a.set_fp16_scales(2 * sf, 2 * sg)               # exact
    assert a.fp16_scales() == (2 * sf, 2 * sg)
    assert np.array_equal(a.fields()["phi"], f0["phi"])
    a.set_fp16_scales(sf / 64, sg / 64)              # largest stored magnitude far below band
    f1 = a.fields()
    assert maxdiff(f1["phi"], f0["phi"]) < 1e-5
    a.diagnostics()                                   # moves both scales up by a power of two
    sf2, sg2 = a.fp16_scales()
    assert sf2 > sf / 64 and sg2 > sg / 64
    assert math.log2(sf2).is_integer() and math.log2(sg2).is_integer()
    assert np.array_equal(a.fields()["phi"], f1["phi"])
    a.step(100)
    b.step(100)
    zeta = _zeta(a)
    err = maxdiff(a.fields()["phi"], b.fields()["phi"], zeta)
    print(f"FP16 rescaled run vs untouched run after 100 steps: |dphi|_inf {err:.2e}")
    assert err < 1e-4
    with pytest.raises(P.PflbmError):
        a.set_fp16_scales(3.0, sg2)
    with pytest.raises(P.PflbmError):
        P.Case.from_case(c, "f32").set_fp16_scales(1.0, 1.0)


@pytest.mark.parametrize("chi_case", [1, 3])
def test_parity_chi_cases_fp64(P, chi_case):
    """Appendix A cases 1 and 3: the ghost rule of Eq. (cubicc) and the wall term
    of Eq. (chemical_potencial112) scaled by 0 or 2, against the oracle in FP64
    (ragged 67 x 37 tiles; ghost values compared too)."""
    c = workloads.flat_droplet_case(67, 37, 11.0, 60.0, 4.0)
    c["chi_case"] = chi_case
    g = P.Case.from_case(c, "f64")
    o = oracle_for(c)
    zeta = _zeta(g)
    ghost = (g.classes() & 4).astype(bool)
    for k in range(4):
        g.step(50)
        o.step(50)
        gf, of = g.fields(), o.fields()
        _compare(gf, of, zeta, 1e-12, 1e-12)
        assert maxdiff(gf["phi"], of["phi"], ghost) <= 1e-12


def _flat_3d(chi_case, n=(24, 20, 18)):
    shape = n
    mask = workloads.flat_walls(shape)
    phi0 = workloads.droplet(shape, (n[0] / 2, n[1] / 2, -0.5), 6.0, 4.0)
    wall = dict(kind="plane", point=(0.0, 0.0, -0.5), normal=(0.0, 0.0, 1.0))
    c = workloads._case("D3Q19", shape, (True, True, False), mask, phi0, 120.0, 1e-3, 4.0, wall)
    c["chi_case"] = chi_case
    return c


@pytest.mark.parametrize("lattice,chi_case", [("D2Q9", 1), ("D2Q9", 3), ("D3Q19", 1),
                                              ("D3Q19", 3)])
def test_chi_cases_every_step_variant_bitwise(P, lattice, chi_case):
    """Every step kernel applies the same ghost rule: FP32 fields bit-identical
    to the three-kernel path for cases 1 and 3, in 2D and 3D; the 3D case is
    also checked against the oracle (FP32 storage, 1e-5)."""
    if lattice == "D2Q9":
        c = workloads.flat_droplet_case(70, 21, 6.0, 120.0, 4.0)
        c["chi_case"] = chi_case
    else:
        c = _flat_3d(chi_case)
    ref = P.Case.from_case(c, "f32")
    ref.set_step_kernel(-1)
    ref.step(30)
    fr = ref.fields()
    for v in range(len(P.step_variants(lattice))):
        g = P.Case.from_case(c, "f32")
        g.set_step_kernel(v)
        g.step(30)
        f = g.fields()
        for k in ("phi", "p", "u", "mu"):
            assert np.array_equal(f[k], fr[k]), (v, k)
    if lattice == "D3Q19":
        o = oracle_for(c)
        o.step(30)
        assert maxdiff(fr["phi"], o.fields()["phi"], _zeta(ref)) < 1e-5


def test_chi_cases_refuse_curved_walls(P):
    """Cases 1 and 3 need axis-aligned walls: a cylinder is refused at creation."""
    c = workloads.cylinder_case(64, 32, 0.3, 100.0)
    c["chi_case"] = 1
    with pytest.raises(P.PflbmError):
        P.Case.from_case(c, "f32")
    c["chi_case"] = 2
    P.Case.from_case(c, "f32").close()


def test_parity_body_force_and_variable_viscosity_fp64(P):
    """Gravity (F_b) and nu_l != nu_g (tau_f per node from nu(phi)) against the
    oracle in FP64, on the flat-wall drop, 200 steps."""
    c = workloads.flat_droplet_case(67, 37, 11.0, 60.0, 4.0)
    over = dict(body_force=(0.0, -2e-6, 0.0), nu_l=0.12, nu_g=0.04)
    g = P.Case.from_case(c, "f64", **over)
    o = oracle_for(c, **over)
    zeta = _zeta(g)
    for k in range(4):
        g.step(50)
        o.step(50)
        _compare(g.fields(), o.fields(), zeta, 1e-12, 1e-12)


def _patchy_2d():
    c = workloads.flat_droplet_case(67, 37, 11.0, 120.0, 4.0)
    tm = np.full((37, 67), 120.0)
    tm[0, :30] = 60.0            # bottom row: 60 deg on the left, 120 on the right
    tm[-1, :] = 95.0             # top row
    c["theta_map"] = tm
    return c


def _patchy_3d():
    c = workloads.inclined_droplet_case_3d(n=22, radius=6.0, theta=100.0, width=4.0)
    tm = np.full(c["mask"].shape, 100.0)
    tm[:, :, :11] = 50.0          # x < 11: 50 deg
    c["theta_map"] = tm
    return c


@pytest.mark.parametrize("make", [_patchy_2d, _patchy_3d], ids=["2d", "3d"])
def test_parity_theta_map_fp64(P, make):
    """Heterogeneous wetting (a contact angle per solid node) against the
    oracle in FP64, 200 steps; the per-node wall coefficients travel as table
    entries in the node words."""
    c = make()
    g = P.Case.from_case(c, "f64")
    o = oracle_for(c)
    zeta = _zeta(g)
    for k in range(4):
        g.step(50)
        o.step(50)
        _compare(g.fields(), o.fields(), zeta, 1e-12, 1e-12)


@pytest.mark.parametrize("make,lattice", [(_patchy_2d, "D2Q9"), (_patchy_3d, "D3Q19")],
                         ids=["2d", "3d"])
def test_theta_map_every_variant_and_group_bitwise(P, make, lattice):
    """Every step kernel reads the per-node coefficients: FP32 fields
    bit-identical to the three-kernel path; inside a group beside a uniform case
    the patchy case matches its run alone."""
    c = make()
    ref = P.Case.from_case(c, "f32")
    ref.set_step_kernel(-1)
    ref.step(20)
    fr = ref.fields()
    for v in range(len(P.step_variants(lattice))):
        g = P.Case.from_case(c, "f32")
        g.set_step_kernel(v)
        g.step(20)
        assert np.array_equal(g.fields()["phi"], fr["phi"]), v
        assert np.array_equal(g.fields()["mu"], fr["mu"]), v
    other = dict(c)
    other.pop("theta_map")
    grp = P.Group()
    ms = [P.Case.from_case(x, "f32") for x in (c, other)]
    for m in ms:
        grp.add(m)
    grp.step(20)
    for x, m in zip((c, other), ms):
        a = P.Case.from_case(x, "f32")
        a.step(20)
        assert np.array_equal(m.fields()["phi"], a.fields()["phi"])


def test_theta_map_refusals(P):
    """Angles outside (0, 180) on solid nodes, and more than 1023 distinct wall
    coefficients (a random angle per solid node of a 30^3 staircase), are
    refused at creation."""
    c = _patchy_2d()
    c["theta_map"] = c["theta_map"].copy()
    c["theta_map"][0, 5] = 180.0
    with pytest.raises(P.PflbmError):
        P.Case.from_case(c, "f32")
    c = workloads.inclined_droplet_case_3d(n=30, radius=6.0, theta=100.0, width=4.0)
    c["theta_map"] = np.random.default_rng(1).uniform(20.0, 160.0, c["mask"].shape)
    with pytest.raises(P.PflbmError):
        P.Case.from_case(c, "f32")


@pytest.mark.parametrize("variant", [1, 6, -1])
def test_degenerate_one_wide_and_all_solid(P, variant):
    """Degenerate inputs: a periodic domain one node wide (every x neighbour is
    the node itself) against the oracle in FP64, for the fused, split and
    three-kernel paths; and an all-solid domain (no zeta = 1 node), which steps
    and reports zero mass without a non-finite flag."""
    ny = 24
    y = np.arange(ny)[:, None]
    phi0 = (0.5 + 0.5 * np.tanh(2.0 * (8.0 - y) / 4.0)) * np.ones((ny, 1))
    c = dict(lattice="D2Q9", shape=(1, ny), periodic=(True, False),
             mask=workloads.flat_walls((1, ny)), phi0=phi0, theta_deg=60.0, sigma=1e-3,
             width=4.0, tau=0.8, mobility=0.1, rho_l=10.0, rho_g=1.0, wall=None)
    g = P.Case.from_case(c, "f64")
    g.set_step_kernel(variant)
    o = oracle_for(c)
    g.step(50)
    o.step(50)
    _compare(g.fields(), o.fields(), _zeta(g), 1e-12, 1e-12)
    g.close()
    s = dict(c, shape=(40, 12), periodic=(True, True), mask=np.ones((12, 40), np.uint8),
             phi0=np.zeros((12, 40)))
    h = P.Case.from_case(s, "f32")
    h.set_step_kernel(variant)
    h.step(10)
    d = h.diagnostics()
    assert d["mass"] == 0.0 and not d["nonfinite"] and d["n_points"] == 0
    h.close()


@pytest.mark.parametrize("D", [2, 3])
def test_laplace_law_on_the_gpu(P, D):
    """Laplace's law at the paper's surface tension (sigma = 0.005, W = 4) for
    free droplets stepped by the default kernels in FP32: p_in - p_out =
    sigma / R in 2D and 2 sigma / R in 3D, within 3 % (2D) and 5 % (3D).  The
    pressure difference is averaged over the tail of the run (acoustic ringing)
    and R is the fitted phi = 1/2 radius."""
    from oracle import diagnostics as odiag
    sigma, W = 0.005, 4.0
    n = 96 if D == 2 else 48
    radii_in = (16.0, 24.0, 32.0) if D == 2 else (10.0, 13.0, 16.0)
    shape = (n,) * D
    X = np.indices(shape[::-1]).astype(float)
    r = np.sqrt(sum((X[d] - n / 2) ** 2 for d in range(D)))
    for R in radii_in:
        phi0 = workloads.droplet(shape, (n / 2,) * D, R, W)
        c = dict(lattice="D2Q9" if D == 2 else "D3Q19", shape=shape, periodic=(True,) * D,
                 mask=np.zeros(shape[::-1], np.uint8), phi0=phi0, sigma=sigma, width=W,
                 theta_deg=90.0, tau=0.8, mobility=0.1, rho_l=10.0, rho_g=1.0, wall=None)
        g = P.Case.from_case(c, "f32")
        g.set_graph_chunk(50)
        g.step(6000)
        dps, rs = [], []
        for k in range(40):
            g.step(50)
            f = g.fields()
            dps.append(f["p"][r < R - 2 * W].mean() - f["p"][r > R + 2 * W].mean())
            pts = odiag.interface_points(f["phi"], np.ones(shape[::-1], bool))
            rs.append(odiag.kasa_fit(pts)[1])
        g.close()
        ratio = np.mean(dps) * np.mean(rs) / ((D - 1) * sigma)
        print(f"D={D} R0={R}: (p_in - p_out) R / ((D-1) sigma) = {ratio:.4f}")
        assert abs(ratio - 1.0) < (0.03 if D == 2 else 0.05), (R, ratio)


def test_flat_interface_relaxes_to_the_tanh_profile(P):
    """The equilibrium profile of the double-well free energy across a flat
    interface is 0.5 + 0.5 tanh(2x / W) with W = sqrt(8 kappa / beta): a liquid
    slab in a periodic box, started from a sharp step, relaxes to it (FP32,
    default kernels) within 0.02 at every node, with the interface positions
    where the slab's mass puts them."""
    ny, W = 128, 4.0
    y = np.arange(ny, dtype=float)
    step = ((y >= 32) & (y < 96)).astype(float)
    phi0 = np.tile(step[:, None], (1, 8))
    c = dict(lattice="D2Q9", shape=(8, ny), periodic=(True, True),
             mask=np.zeros((ny, 8), np.uint8), phi0=phi0, sigma=0.005, width=W,
             theta_deg=90.0, tau=0.8, mobility=0.1, rho_l=10.0, rho_g=1.0, wall=None)
    g = P.Case.from_case(c, "f32")
    g.set_graph_chunk(100)
    g.step(20000)
    phi = g.fields()["phi"][:, 3]
    # interfaces at y = 31.5 and 95.5 (mass 64 rows, symmetric), sampled at nodes
    want = 0.5 * (np.tanh(2.0 * (y - 31.5) / W) - np.tanh(2.0 * (y - 95.5) / W))
    err = np.abs(phi - want).max()
    print(f"flat interface: max |phi - tanh profile| = {err:.3e}")
    assert err < 0.02
