"""CPU tests of the C interface: the library loads, exports every declared
symbol, and its host-side pieces (lattice tables, node classification,
parameter checks, footprint) agree with the oracle and the paper.  No device
work is started here."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import workloads
from oracle import lattice as olat
from tests.helpers import oracle_for

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pflbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pflbm_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(P):
    lib = ct.CDLL(P.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    # and the binding wraps every one of them under the same name
    assert set(names) <= set(P.EXPORTED), set(names) - set(P.EXPORTED)


@pytest.mark.parametrize("name,L", [("D2Q9", olat.D2Q9), ("D3Q19", olat.D3Q19),
                                    ("D3Q19/D3Q7", olat.D3Q19), ("D3Q7", olat.D3Q7)])
def test_library_lattice_tables(P, name, L):
    t = P.lattice_table(name)
    D = L.D
    assert len(t["w"]) == L.Q
    c = t["c"][:, :D].astype(float)
    w = t["w"]
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(np.einsum("q,qa,qb->ab", w, c, c) - np.eye(D) * L.cs2).max() < 1e-15
    assert np.array_equal(t["c"][t["opp"]], -t["c"])
    # same velocity set and weights as the oracle (built from the paper's formulas)
    lib_set = {tuple(v[:D]): (wi, ki) for v, wi, ki in zip(t["c"], w, t["k"])}
    for v, wi, ki in zip(L.c, L.w, L.k):
        wl, kl = lib_set[tuple(int(a) for a in v)]
        assert abs(wl - wi) < 1e-16 and abs(kl - ki) < 1e-15
    if D == 2:
        assert np.all(t["c"][:, 2] == 0)


def _classes_from_oracle(c):
    o = oracle_for(c)
    z = o.domain(o.zeta)
    e = o.domain(o.eps) > 0
    g = o.domain(o.ghost)
    return z.astype(np.uint8) | (e.astype(np.uint8) << 1) | (g.astype(np.uint8) << 2)


CASES = {
    "flat": lambda: workloads.flat_droplet_case(37, 21, 6.0, 60.0),
    "flat_closed": lambda: dict(workloads.flat_droplet_case(37, 21, 6.0, 60.0),
                                periodic=(False, False)),
    "cylinder": lambda: workloads.cylinder_case(64, 32, 0.3, 100.0),
    "incline2d": lambda: dict(workloads.flat_droplet_case(40, 30, 6.0, 60.0),
                              mask=workloads.inclined_plane((40, 30), (20.0, 10.0), 26.0)),
    "incline3d": lambda: workloads.inclined_droplet_case_3d(n=14, radius=4.0, width=3.0),
    "sphere3d": lambda: dict(workloads.inclined_droplet_case_3d(n=12, radius=3.0, width=3.0),
                             mask=workloads.ball((12, 12, 12), (6.0, 6.0, 3.0), 3.5),
                             periodic=(True, False, True)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_host_classification_matches_oracle(P, name):
    """Node marks of Sec. 2.2.2 from the library's host code equal the oracle's
    (written separately); ghost nodes inside the domain included."""
    c = CASES[name]()
    prm = P.params_from_case(c, "f32")
    got = P.classify(prm, c["mask"])
    want = _classes_from_oracle(c)
    assert np.array_equal(got, want)


def _params(P, **kw):
    c = workloads.flat_droplet_case(32, 16, 5.0, 60.0)
    return P.params_from_case(c, "f32", **kw)


@pytest.mark.parametrize("field,value,code", [
    ("tau", 0.5, -1), ("mobility", 0.0, -1), ("theta_deg", 0.0, -1),
    ("theta_deg", 180.0, -1), ("beta", -1.0, -1), ("rho_g", 0.0, -1),
    ("lattice", 7, -6), ("storage", 9, -6), ("nx", 0, -1), ("nz", 3, -1),
    ("struct_size", 8, -1), ("tau_phi", 0.4, -1), ("wall_kind", 5, -1), ("chi_case", 4, -1),
    ("chi_case", -1, -1)])
def test_parameter_validation(P, field, value, code):
    prm = _params(P)
    setattr(prm, field, value)
    n = ct.c_size_t(0)
    rc = P.lib.pflbm_footprint(ct.byref(prm), ct.byref(n))
    assert rc == code
    assert len(P.lib.pflbm_last_error()) > 0


def test_null_arguments(P):
    prm = _params(P)
    assert P.lib.pflbm_footprint(None, None) == -1
    assert P.lib.pflbm_footprint(ct.byref(prm), None) == -1
    out = ct.c_void_p()
    assert P.lib.pflbm_create(ct.byref(prm), None, None, None, ct.byref(out)) == -1
    assert P.lib.pflbm_step(None, 1) == -1
    assert P.lib.pflbm_fields(None, None, None, None, None) == -1
    assert P.lib.pflbm_group_step(None, 1) == -1
    assert P.lib.pflbm_step_count(None) == -1
    P.lib.pflbm_destroy(None)            # no-op
    P.lib.pflbm_group_destroy(None)      # no-op
    assert P.lib.pflbm_strerror(-4) == b"non-finite values"


def test_footprint_scales_with_storage(P):
    """Bytes per node: FP64 > FP32 > FP16-deviation, and linear in the node count."""
    c = workloads.flat_droplet_case(256, 128, 20.0, 60.0)
    b = {s: P.footprint(P.params_from_case(c, s)) / (256 * 130) for s in ("f64", "f32", "f16dev")}
    assert b["f64"] > b["f32"] > b["f16dev"]
    # D2Q9 FP32: f 9x4 B and g 8x4 + 8 B per buffer, two buffers each, plus 5 fields
    assert 2 * (36 + 40) + 4 * 4 + 4 < b["f32"] < 2 * (36 + 40) + 4 * 4 + 4 + 8
    c2 = workloads.flat_droplet_case(512, 256, 20.0, 60.0)
    r = P.footprint(P.params_from_case(c2, "f32")) / P.footprint(P.params_from_case(c, "f32"))
    assert 3.9 < r < 4.1


def test_d3q7_phase_lattice_params_and_footprint(P):
    """D3Q7 for g (Sec. 2.1.3) shrinks each g buffer from 19 to 7 populations per
    node slot: 12 x 4 B fewer per buffer in FP32, two buffers."""
    c = workloads.inclined_droplet_case_3d(n=24, radius=6.0, width=4.0)
    a = P.params_from_case(c, "f32")
    c7 = dict(c, phase_lattice="D3Q7")
    b = P.params_from_case(c7, "f32")
    assert a.lattice == P.D3Q19 and b.lattice == P.D3Q19_D3Q7
    fa, fb = P.footprint(a), P.footprint(b)
    slots = fa - fb
    assert slots > 0 and slots % (2 * 12 * 4) == 0
    nslots = slots // (2 * 12 * 4)
    assert 26 ** 3 <= nslots <= 64 * 26 * 26 + 256
    # classes do not depend on the phase lattice
    assert np.array_equal(P.classify(a, c["mask"]), P.classify(b, c["mask"]))
    with pytest.raises(ValueError):
        P.params_from_case(dict(workloads.flat_droplet_case(32, 16, 5.0, 60.0),
                                phase_lattice="D3Q7"), "f32")


def test_table1_case_geometry():
    """The Sec. 3.1 flat-plate input: a plate 0.25 Ny thick, 0.05 Ny above the
    lower edge, periodic everywhere, a semicircular droplet centred on the wall
    plane (half a node below the plate's top row) with R = 50, 40 at 20 deg and
    30 at 10 deg."""
    import json
    c = workloads.table1_case(60.0)
    rows = np.where(c["mask"].any(axis=1))[0]
    assert rows.min() == 6 and rows.max() == 37 and c["mask"][6:38].all()
    assert c["periodic"] == (True, True) and c["wall"]["point"][1] == 36.5
    assert c["mobility"] == 0.01 and c["sigma"] == 0.005 and c["width"] == 4.0
    assert [workloads.table1_case(t)["radius"] for t in (10.0, 20.0, 30.0)] == [30.0, 40.0, 50.0]
    # a semicircle: nothing below the plate's top row (its underside boundary
    # nodes and the gas under the plate start dry); the top row and above hold
    # the circle's upper half
    phi0 = c["phi0"]
    assert phi0[:37].max() == 0.0
    assert phi0[37, 128] > 0.99 and phi0[37 + 49, 128] > 0.5 > phi0[37 + 52, 128]
    paper = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                        "table1_2d_paper.json")))
    assert paper["prescribed_deg"] == [int(t) for t in workloads.TABLE1_ANGLES]


def test_sec3_incline_and_cylinder_geometry(P):
    """The Sec. 3.2 and 3.3 inputs as the paper describes them: solid below
    y = slope x with the drop centred on that line at x = Nx/2; a cylinder of
    R_s = 60 centred at (Nx/2, Ny/2 - 50) with the drop centred at (Nx/2, Ny/2);
    both classify, and the wall the angle is measured against is the line moved
    one node into the solid / the circle of radius R_s - 1."""
    import math
    for slope in workloads.SEC32_SLOPES:
        c = workloads.sec32_incline_case(60.0, slope)
        m = c["mask"]
        assert m.shape == (256, 256)
        y, x = 100, 150
        assert m[y, x] == (1 if y < slope * x else 0)
        assert c["phi0"][int(round(slope * 128)) + 10, 128] > 0.99        # inside the drop
        n = c["wall"]["normal"]
        assert abs(math.hypot(*n) - 1) < 1e-12 and abs(n[1] / -n[0] - 1 / slope) < 1e-9
        d = c["wall"]["point"][1] - slope * c["wall"]["point"][0]      # line offset of the plane
        assert abs(abs(d) * math.cos(math.atan(slope)) - 1.0) < 1e-9 and d < 0
        cls = P.classify(P.params_from_case(c, "f32"), m)
        assert (cls & 1).sum() > 0 and ((cls & 2) > 0).sum() == (m == 0).sum()
    c = workloads.sec33_cylinder_case(90.0)
    m = c["mask"]
    assert m[78, 128] == 1 and m[78 + 59, 128] == 1 and m[78 + 61, 128] == 0
    assert c["wall"]["radius"] == 59.0 and c["width"] == 6.0 and c["mobility"] == 0.01
    assert c["phi0"][160, 128] > 0.99 and c["phi0"][185, 128] < 0.01
    assert P.classify(P.params_from_case(c, "f32"), m).any()


def test_table1_case_3d_geometry(P):
    """The 3D plate of Sec. 3.1 (scaled): plate 0.25 Nz thick from 0.05 Nz, drop
    centred at (Nx/2, Ny/2, 0.25 Nz) as printed, dry below the plate's top row;
    classifies; the golden file carries the paper's 3D column."""
    import json
    c = workloads.table1_case_3d(90.0, (32, 32, 64))
    m = c["mask"]
    layers = np.where(m.any(axis=(1, 2)))[0]
    assert layers.min() == 3 and layers.max() == 18 and m[3:19].all()
    assert c["wall"]["point"][2] == 17.5 and c["radius"] == 25.0
    assert c["phi0"][:18].max() == 0.0 and c["phi0"][18 + 5, 16, 16] > 0.99
    assert P.classify(P.params_from_case(c, "f32"), m).any()
    paper = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                        "table1_2d_paper.json")))
    assert len(paper["paper_3d_deg"]) == len(paper["prescribed_deg"]) == 11


def test_header_is_plain_c_and_links(P, tmp_path):
    """include/pflbm.h compiles as C99 with warnings as errors, and a C program
    using it links against libpflbm.so and runs the host-only calls (footprint,
    lattice table, error strings) without touching a GPU."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text(r'''
#include <stdio.h>
#include <string.h>
#include "pflbm.h"
int main(void) {
  pflbm_params p;
  memset(&p, 0, sizeof p);
  p.struct_size = sizeof p;
  p.lattice = PFLBM_D2Q9; p.storage = PFLBM_FP32;
  p.nx = 64; p.ny = 32; p.nz = 1; p.periodic[0] = 1;
  p.tau = 0.8; p.mobility = 0.1; p.beta = 3e-3; p.kappa = 6e-3;
  p.rho_l = 10.0; p.rho_g = 1.0; p.theta_deg = 60.0; p.steady_tol = 1e-5;
  size_t bytes = 0;
  if (pflbm_footprint(&p, &bytes) != PFLBM_OK || bytes == 0) return 1;
  int32_t c[27 * 3]; double w[27], k[27]; int32_t opp[27];
  if (pflbm_lattice_table(PFLBM_D2Q9, c, w, opp, k) != 9 || w[0] != 4.0 / 9.0) return 2;
  p.theta_deg = 200.0;
  if (pflbm_footprint(&p, &bytes) != PFLBM_EINVAL) return 3;
  printf("%zu %s %s\n", bytes, pflbm_strerror(PFLBM_EINVAL), pflbm_last_error());
  return 0;
}
''')
    exe = tmp_path / "use"
    inc = os.path.join(ROOT, "include")
    libdir = os.path.dirname(P.LIB_PATH)
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", inc, str(src),
                        "-L", libdir, "-lpflbm", f"-Wl,-rpath,{libdir}", "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert "invalid argument" in r.stdout


def test_theta_map_with_chi_case_refused(P):
    """A per-node contact angle goes with the chi = 0 method only: parameter
    validation refuses it with chi cases 1 and 3 (no device work)."""
    c = workloads.flat_droplet_case(32, 16, 5.0, 60.0)
    c["theta_map"] = np.full((16, 32), 70.0)
    prm = P.params_from_case(c, "f32")
    n = ct.c_size_t(0)
    assert P.lib.pflbm_footprint(ct.byref(prm), ct.byref(n)) == 0
    c["chi_case"] = 1
    prm = P.params_from_case(c, "f32")
    assert P.lib.pflbm_footprint(ct.byref(prm), ct.byref(n)) == -6
    with pytest.raises(ValueError):
        oracle_for(c)


def test_sec33_sphere_geometry(P):
    """The Sec. 3.3 3D input (scaled): a sphere of R_s = 60 k centred at
    (n/2, n/2, n/2 - 50 k), k = n / 256, the drop of R_i = 50 k at the box
    centre, wall sphere of radius R_s - 1 for the angle fit; it classifies."""
    c = workloads.sec33_sphere_case(90.0, n=64)
    m = c["mask"]
    k = 64 / 256.0
    cz = 32 - 50 * k
    assert m[int(cz), 32, 32] == 1 and m[int(cz + 60 * k) + 1, 32, 32] == 0
    assert c["wall"]["kind"] == "ball" and c["wall"]["radius"] == 60 * k - 1
    assert c["phi0"][32, 32, 32] > 0.99 and c["periodic"] == (True, True, False)
    assert P.classify(P.params_from_case(c, "f32"), m).any()


def test_sec32_incline_3d_geometry(P):
    """The Sec. 3.2 3D input (scaled): solid below z = slope x, drop centred
    on the plane at (n/2, n/2, slope n/2), wall plane one node into the solid."""
    import math
    for slope in workloads.SEC32_SLOPES:
        c = workloads.sec32_incline_case_3d(60.0, slope, n=48)
        m = c["mask"]
        x, y = 40, 10
        zc = slope * x
        assert m[int(zc) - 1, y, x] == 1 and m[int(zc) + 2, y, x] == 0
        assert c["phi0"][int(round(slope * 24)), 24, 24] > 0.99         # the drop centre
        n_ = c["wall"]["normal"]
        assert abs(math.hypot(*n_) - 1) < 1e-12 and abs(-n_[0] / n_[2] - slope) < 1e-12
        assert P.classify(P.params_from_case(c, "f32"), m).any()


def test_beta_kappa_from_the_library(P):
    """pflbm_beta_kappa: the planar profile width sqrt(8 kappa/beta) and the
    tension sqrt(2 kappa beta)/6 come back as W and sigma, the values equal the
    oracle's, and non-positive or non-finite inputs are refused."""
    from oracle.model import beta_kappa as oracle_bk
    for sigma, W in ((1e-3, 4.0), (1e-3, 5.0), (5e-2, 3.0), (1e-2, 8.0)):
        b, k = P.beta_kappa(sigma, W)
        assert np.sqrt(8.0 * k / b) == pytest.approx(W, rel=1e-14)
        assert np.sqrt(2.0 * k * b) / 6.0 == pytest.approx(sigma, rel=1e-14)
        assert (b, k) == oracle_bk(sigma, W)
    for sigma, W in ((0.0, 4.0), (1e-3, -1.0), (float("nan"), 4.0), (1e-3, float("inf"))):
        with pytest.raises(P.PflbmError) as e:
            P.beta_kappa(sigma, W)
        assert e.value.code == -1
    assert P.lib.pflbm_beta_kappa(1e-3, 4.0, None, None) == -1
