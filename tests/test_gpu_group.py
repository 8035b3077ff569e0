"""GPU tests of the batched runtime: a persistent launch over a (case, tile)
table gives every member the same bits as running it alone."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _cases2d():
    rng = np.random.default_rng(11)
    out = []
    for k in range(6):
        nx = int(rng.integers(4, 14)) * 16
        c = workloads.cylinder_case(nx, nx // 2, float(rng.uniform(0.2, 0.4)),
                                    float(rng.uniform(30, 150)))
        out.append(c)
    out.append(workloads.flat_droplet_case(37, 19, 5.0, 70.0))      # ragged, tiny
    return out


def _alone(P, c, storage, steps, variant):
    a = P.Case.from_case(c, storage)
    a.set_step_kernel(variant)
    a.step(steps)
    return a.fields()


@pytest.mark.parametrize("storage", ["f32", "f16dev", "f64"])
def test_group_alone_vs_mix_bitwise_2d(P, storage):
    cs = _cases2d()
    g = P.Group()
    g.set_tile(1)
    members = [P.Case.from_case(c, storage) for c in cs]
    for m in members:
        g.add(m)
    g.step(37)
    for c, m in zip(cs, members):
        ref = _alone(P, c, storage, 37, 1)
        f = m.fields()
        assert m.steps == 37
        for k in ("phi", "p", "u", "mu"):
            assert np.array_equal(f[k], ref[k]), k


@pytest.mark.parametrize("variant", [3, 5, 6, 11, 12])
def test_group_alone_vs_mix_bitwise_3d(P, variant):
    """Fused (3), split (5, 6) and fused z-marching (11, 12) batched kernels."""
    cs = [workloads.inclined_droplet_case_3d(n=n, radius=0.25 * n, theta=th, width=4.0)
          for n, th in ((18, 60.0), (26, 120.0), (22, 45.0))]
    g = P.Group()
    g.set_tile(variant)
    members = [P.Case.from_case(c, "f32") for c in cs]
    for m in members:
        g.add(m)
    g.step(21)
    for c, m in zip(cs, members):
        ref = _alone(P, c, "f32", 21, variant)
        assert np.array_equal(m.fields()["phi"], ref["phi"])


@pytest.mark.parametrize("variant", [3, 7, 8, 12])
def test_group_alone_vs_mix_bitwise_d3q7(P, variant):
    """D3Q7 for g: batched fused (3), split (7), z-marching split (8) and fused
    z-marching (12) kernels."""
    cs = [workloads.inclined_droplet_case_3d(n=n, radius=0.25 * n, theta=th, width=4.0)
          for n, th in ((18, 60.0), (26, 120.0))]
    for c in cs:
        c["phase_lattice"] = "D3Q7"
    g = P.Group()
    g.set_tile(variant)
    members = [P.Case.from_case(c, "f32") for c in cs]
    for m in members:
        g.add(m)
    g.step(21)
    for c, m in zip(cs, members):
        ref = _alone(P, c, "f32", 21, variant)
        assert np.array_equal(m.fields()["phi"], ref["phi"])


@pytest.mark.parametrize("variant", [0, 6])
def test_group_other_variants_2d(P, variant):
    """Fused 64 x 4 (0) and split (6) batched kernels against the default fused
    kernel run alone."""
    cs = _cases2d()[:4]
    g = P.Group()
    g.set_tile(variant)
    members = [P.Case.from_case(c, "f32") for c in cs]
    for m in members:
        g.add(m)
    g.step(15)
    for c, m in zip(cs, members):
        ref = _alone(P, c, "f32", 15, 1)
        assert np.array_equal(m.fields()["phi"], ref["phi"])


def test_group_membership_changes(P):
    """Cases join and leave between chunks (with graph replay) and keep their
    own trajectories: a case stepped 10 alone, 40 in a group, removed, 13 alone
    equals 63 alone."""
    cs = _cases2d()[:4]
    a = P.Case.from_case(cs[0], "f32")
    a.step(10)
    g = P.Group()
    g.set_graph_chunk(8)
    others = [P.Case.from_case(c, "f32") for c in cs[1:]]
    g.add(a)
    g.add(others[0])
    g.step(17)
    g.add(others[1])           # joins mid-run
    g.step(23)
    g.remove(others[0])
    g.add(others[2])
    g.remove(a)
    a.step(13)
    g.step(5)
    assert a.steps == 63 and others[1].steps == 28 and others[0].steps == 40
    ref = _alone(P, cs[0], "f32", 63, 1)
    assert np.array_equal(a.fields()["phi"], ref["phi"])
    ref1 = _alone(P, cs[2], "f32", 28, 1)
    assert np.array_equal(others[1].fields()["phi"], ref1["phi"])
    ref0 = _alone(P, cs[1], "f32", 40, 1)
    assert np.array_equal(others[0].fields()["phi"], ref0["phi"])


def test_group_graph_equals_eager(P):
    cs = _cases2d()[:3]
    outs = []
    for chunk in (0, 16):
        g = P.Group()
        g.set_graph_chunk(chunk)
        ms = [P.Case.from_case(c, "f32") for c in cs]
        for m in ms:
            g.add(m)
        g.step(50)
        outs.append([m.fields()["phi"] for m in ms])
        g.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_group_poll_flags(P):
    """Steady flag for a uniform (fixed-point) case; nonfinite flag for a case
    the host drives unstable with an oversized body force."""
    c = workloads.flat_droplet_case(64, 32, 8.0, 60.0)
    calm = dict(c, phi0=np.ones_like(c["phi0"]), theta_deg=90.0)
    g = P.Group()
    a = P.Case.from_case(calm, "f32", steady_tol=1e-7)
    b = P.Case.from_case(c, "f32", body_force=(2.0, -2.0, 0.0))
    g.add(a)
    g.add(b)
    g.step(10)
    d, flags = g.poll()
    g.step(200)
    d, flags = g.poll()
    assert flags[0] & 1 and not flags[0] & 2
    assert flags[1] & 2
    assert d[1]["nonfinite"]


def test_group_rejects_mixed_storage(P):
    c = workloads.flat_droplet_case(32, 16, 5.0, 60.0)
    g = P.Group()
    g.add(P.Case.from_case(c, "f32"))
    with pytest.raises(P.PflbmError):
        g.add(P.Case.from_case(c, "f64"))
    a = P.Case.from_case(c, "f32")
    g.add(a)
    with pytest.raises(P.PflbmError):
        a.step(1)                      # members are stepped through the group


@pytest.mark.parametrize("variant", [1, 6])
def test_group_poll_matches_single_diagnostics(P, variant):
    """The batched reductions (one launch sequence for all members) give each
    member the record its own diagnostics call gives, up to summation order."""
    cs = _cases2d()[:5]
    g = P.Group()
    g.set_tile(variant)
    ms = [P.Case.from_case(c, "f32") for c in cs]
    for m in ms:
        g.add(m)
    g.step(40)
    d, flags = g.poll()
    g.step(40)
    d, flags = g.poll()
    for m, dk in zip(ms, d):
        g.remove(m)
        ref = m.diagnostics()
        assert abs(dk["mass"] - ref["mass"]) <= 1e-12 * abs(ref["mass"])
        assert abs(dk["s_sum"] - ref["s_sum"]) <= 1e-9 * max(1e-12, abs(ref["s_sum"])) + 1e-15
        assert dk["n_points"] == ref["n_points"]
        assert (np.isnan(dk["theta_deg"]) and np.isnan(ref["theta_deg"])) or \
            abs(dk["theta_deg"] - ref["theta_deg"]) < 1e-8
        assert dk["step"] == ref["step"] == 80


@pytest.mark.parametrize("variant", [1, 6])
def test_group_chi_cases_bitwise(P, variant):
    """Members with different Appendix A chi cases (each member's ghost rule and
    wall factor travel in its own parameters) beside a curved-wall case: every
    member matches its run alone bit for bit."""
    cs = []
    for k, th in ((1, 60.0), (3, 120.0), (2, 80.0)):
        c = workloads.flat_droplet_case(70, 33, 8.0, th, 4.0)
        c["chi_case"] = k
        cs.append(c)
    cs.append(workloads.cylinder_case(96, 48, 0.3, 110.0))
    g = P.Group()
    g.set_tile(variant)
    members = [P.Case.from_case(c, "f32") for c in cs]
    for m in members:
        g.add(m)
    g.step(25)
    for c, m in zip(cs, members):
        ref = _alone(P, c, "f32", 25, variant)
        assert np.array_equal(m.fields()["phi"], ref["phi"])


@pytest.mark.parametrize("lattice,variant", [("D2Q9", 1), ("D2Q9", 6), ("D3Q19", 3), ("D3Q19", 7),
                                             ("D3Q19", 8), ("D3Q19", 12)])
def test_group_persistent_grid_equals_per_entry_grid(P, lattice, variant):
    """The persistent grid (a fixed grid striding over the table, blocks_per_cu
    > 0) and one workgroup per table entry (blocks_per_cu = 0) give the same
    bits, with graph replay, across a membership change."""
    if lattice == "D2Q9":
        cs = _cases2d()[:5]
    else:
        cs = [workloads.inclined_droplet_case_3d(n=n, radius=0.25 * n, theta=th, width=4.0)
              for n, th in ((18, 60.0), (26, 120.0), (22, 90.0))]
    out = {}
    for bpc in (0, 1):
        g = P.Group()
        g.set_tile(variant, bpc)
        g.set_graph_chunk(4)
        ms = [P.Case.from_case(c, "f32") for c in cs]
        for m in ms[:-1]:
            g.add(m)
        g.step(8)
        g.add(ms[-1])
        g.step(8)
        g.remove(ms[0])
        g.step(8)
        out[bpc] = [m.fields()["phi"] for m in ms]
        for m in ms[1:]:
            g.remove(m)
        for m in ms:
            m.close()
        g.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_group_poll_fp16_upkeep_matches_alone(P):
    """FP16-deviation scale upkeep inside a group: a member whose scales were
    pushed out of band is rescaled at the poll and continues exactly like the
    same case run alone with a diagnostics call at the same step."""
    c = workloads.flat_droplet_case(96, 40, 9.0, 70.0, 4.0)
    alone = P.Case.from_case(c, "f16dev")
    member = P.Case.from_case(c, "f16dev")
    other = P.Case.from_case(workloads.flat_droplet_case(64, 32, 7.0, 110.0, 4.0), "f16dev")
    sf, sg = alone.fp16_scales()
    for h in (alone, member):
        h.set_fp16_scales(sf / 64, sg / 64)
    g = P.Group()
    g.add(member)
    g.add(other)
    g.step(12)
    g.poll()
    g.step(14)
    alone.step(12)
    alone.diagnostics()
    alone.step(14)
    g.remove(member)
    g.remove(other)
    sf2, sg2 = member.fp16_scales()
    assert sf2 > sf / 64 and sg2 > sg / 64
    assert (sf2, sg2) == alone.fp16_scales()
    assert np.array_equal(member.fields()["phi"], alone.fields()["phi"])
