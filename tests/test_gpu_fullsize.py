"""Parity at the benchmarked sizes, in the launch configuration bench.py times
(tile variant and HIP-graph replay).

The 1024 x 512 case is compared with the FP64 oracle on the whole domain.  The
8192 x 4096 and 256^3 cases are compared on windows: after k steps a node
depends only on the initial state within 3k nodes (one node per step from the
pulls, one from the phi stencils, one from the ghost means), and the initial
g_eq(phi0, mu(phi0)) adds two more.  So the oracle run on a window of
half-width 3k + 4 around a sample node reproduces that node exactly; the
window's cut edges (virtual walls) cannot reach the compared centre.

Tolerances: FP32 storage |dphi|_inf <= 1e-5, p, u, mu within 1e-6 of the FP64
oracle; FP16-deviation storage |dphi|_inf <= 2e-4.
"""
import numpy as np
import pytest

import workloads
from tests.helpers import maxdiff, oracle_for, window

pytestmark = pytest.mark.gpu


def _centre_compare(gf, of, zeta, idx, pos, r, tol_phi, tol_other):
    D = len(idx)
    lo = [max(pos[d] - r, 0) for d in range(D)]                 # clipped at cut domain edges
    hi = [min(pos[d] + r + 1, len(idx[d])) for d in range(D)]
    g_sel = np.ix_(*[idx[d][lo[d]:hi[d]] for d in range(D)][::-1])
    o_sel = tuple(slice(lo[d], hi[d]) for d in range(D))[::-1]
    z = zeta[g_sel]
    assert z.any()
    errs = {"phi": maxdiff(gf["phi"][g_sel], of["phi"][o_sel], z)}
    for k in ("p", "mu"):
        errs[k] = maxdiff(gf[k][g_sel], of[k][o_sel], z)
    errs["u"] = max(maxdiff(gf["u"][d][g_sel], of["u"][d][o_sel], z) for d in range(D))
    assert errs["phi"] <= tol_phi, errs
    for k in ("p", "mu", "u"):
        assert errs[k] <= tol_other, errs
    return errs


def test_fullsize_1024x512_fp32_whole_domain(P):
    """The bench line's case: 1024 x 512 FP32, graph chunk 100, 100 steps, with
    fused tile variant 1 (the library default) and variant 3 (the tuner's choice
    on this shape, which the bench line times); every zeta = 1 node against the
    oracle."""
    c = workloads.flat_1024x512_fp32()
    o = oracle_for(c)
    o.step(100)
    of = o.fields()
    for variant in (1, 3):
        g = P.Case.from_case(c, "f32")
        g.set_graph_chunk(100)
        g.set_step_kernel(variant)
        g.step(100)
        gf = g.fields()
        zeta = (g.classes() & 1).astype(bool)
        g.close()
        e = maxdiff(gf["phi"], of["phi"], zeta)
        ep = maxdiff(gf["p"], of["p"], zeta)
        eu = max(maxdiff(gf["u"][d], of["u"][d], zeta) for d in range(2))
        print(f"1024x512 FP32 variant {variant}, 100 steps: |dphi| {e:.2e}, |dp| {ep:.2e}, "
              f"|du| {eu:.2e}")
        assert e <= 1e-5 and ep <= 1e-6 and eu <= 1e-6


def test_fullsize_8192x4096_fp32_windows(P):
    """The HBM-bound 8192 x 4096 twin, variant 1, graph replay, 6 steps; five
    windows on the drop's interface: both contact points, the apex, two points
    at 45 degrees (one of them across x on the other side)."""
    k = 6
    c = workloads.flat_1024x512_fp32(nx=8192, ny=4096)
    g = P.Case.from_case(c, "f32")
    g.set_graph_chunk(3)
    g.set_step_kernel(1)
    g.step(k)
    gf = g.fields()
    zeta = (g.classes() & 1).astype(bool)
    g.close()
    R = 80.0 * 8192 / 1024
    h = int(R / 2 ** 0.5)
    for pt in [(4096 + int(R), 1), (4096 - int(R), 1), (4096, int(R) - 1), (4096 + h, h),
               (4096 - h, h)]:
        w, idx, pos = window(c, pt, 3 * k + 4)
        o = oracle_for(w)
        o.step(k)
        errs = _centre_compare(gf, o.fields(), zeta, idx, pos, 2, 1e-5, 1e-6)
        print(f"8192x4096 window at {pt}: {errs}")


@pytest.mark.parametrize("storage", ["f32", "f16dev"])
def test_fullsize_256cubed_windows(P, storage):
    """The 3D bench case: 256^3 D3Q19 inclined staircase, default split variant,
    graph replay, 6 steps; windows on the drop's interface: the contact line
    across the slope, up and down the slope, the apex, and inside the drop."""
    k = 6
    c = workloads.inclined_3d_256(storage=storage, n=256)
    g = P.Case.from_case(c, storage)
    g.set_graph_chunk(3)
    g.step(k)
    gf = g.fields()
    zeta = (g.classes() & 1).astype(bool)
    g.close()
    tol_phi, tol_other = (1e-5, 1e-6) if storage == "f32" else (2e-4, 1e-4)
    for pt in [(128, 168, 63), (163, 128, 83), (94, 128, 43), (108, 128, 98), (118, 128, 80)]:
        w, idx, pos = window(c, pt, 3 * k + 4)
        o = oracle_for(w)
        o.step(k)
        errs = _centre_compare(gf, o.fields(), zeta, idx, pos, 2, tol_phi, tol_other)
        print(f"256^3 {storage} window at {pt}: {errs}")


def test_over_4gib_buffers_use_64bit_offsets(P):
    """Maximum sizes: 384^3 D3Q19 FP32 has a g buffer above 4 GiB, so its
    kernels form 64-bit load offsets (the 32-bit form serves every smaller
    case).  Three windows on the interface against the oracle after 6
    graph-replayed steps; a group, whose kernels use 32-bit offsets only,
    refuses it."""
    k = 6
    c = workloads.inclined_droplet_case_3d(n=384, radius=60.0, theta=45.0, width=5.0)
    prm = P.params_from_case(c, "f32")
    assert P.footprint(prm) > 2 * 4 * 2 ** 30
    g = P.Case.from_case(c, "f32")
    g.set_graph_chunk(3)
    g.step(k)
    gf = g.fields()
    zeta = (g.classes() & 1).astype(bool)
    for pt in [(192, 252, 95), (244, 192, 125), (162, 192, 147)]:
        w, idx, pos = window(c, pt, 3 * k + 4)
        o = oracle_for(w)
        o.step(k)
        errs = _centre_compare(gf, o.fields(), zeta, idx, pos, 2, 1e-5, 1e-6)
        print(f"384^3 window at {pt}: {errs}")
    del gf
    grp = P.Group()
    with pytest.raises(P.PflbmError):
        grp.add(g)
    grp.close()
    g.close()
