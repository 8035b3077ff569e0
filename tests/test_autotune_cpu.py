"""Autotuner logic on a stand-in case with a fake timer (no GPU)."""
import json

from paper_2312_00369_amd import autotune


class FakeCase:
    def __init__(self, P):
        self.params = P.make_params("D2Q9", (300, 100), (True, False), 60.0, 3e-3, 6e-3)
        self.shape = (300, 100)
        self.variant = None
        self.xcd = None
        self.state = b"original"
        self.steps_done = 0

    def get_state(self):
        return self.state

    def set_state(self, blob):
        self.state = blob

    def set_step_kernel(self, v):
        self.variant = v

    def set_step_options(self, xcd, nt):
        self.xcd = xcd

    def step(self, n):
        self.steps_done += n
        self.state = b"advanced"


def fake_timer(run, steps, sync):
    case = run.__self__
    run(steps)
    # variant 3 with the chunked XCD order (2) is fastest
    return 1.0 + abs(case.variant - 3) + 0.5 * abs(case.xcd - 2)


def test_tune_case_picks_fastest_restores_and_caches(P, tmp_path):
    cache = autotune.Cache(str(tmp_path / "tune.json"))
    case = FakeCase(P)
    out = autotune.tune_case(case, steps=10, cache=cache, arch="gfx950", timer=fake_timer,
                             sync=lambda: None)
    assert out["variant"] == 3 and out["xcd_order"] == 2
    assert case.variant == 3 and case.xcd == 2
    assert case.state == b"original"                   # state restored after timing
    n_variants = len(P.step_variants("D2Q9"))
    assert len(out["candidates"]) == len(autotune.XCD_ORDERS) * n_variants
    data = json.load(open(tmp_path / "tune.json"))
    key = autotune.cache_key("gfx950", case.params.lattice, case.params.storage, case.shape)
    assert data[key]["variant"] == 3
    # a second case of the same class uses the cache without timing anything
    c2 = FakeCase(P)
    out2 = autotune.tune_case(c2, cache=autotune.Cache(str(tmp_path / "tune.json")),
                              arch="gfx950", timer=None, sync=lambda: None)
    assert out2["cached"] and c2.variant == 3 and c2.steps_done == 0


def test_tune_case_over_fewer_xcd_orders_skips_the_cache(P, tmp_path):
    path = tmp_path / "tune.json"
    cache = autotune.Cache(str(path))
    case = FakeCase(P)
    out = autotune.tune_case(case, steps=10, cache=cache, arch="gfx950", timer=fake_timer,
                             sync=lambda: None, xcd_orders=(0,))
    assert out["variant"] == 3 and out["xcd_order"] == 0 and case.xcd == 0
    assert {c["xcd_order"] for c in out["candidates"]} == {0}
    assert len(out["candidates"]) == len(P.step_variants("D2Q9"))
    assert not path.exists() or json.load(open(path)) == {}


def test_shape_classes():
    assert autotune.shape_class((1024, 512)) == "2d-n2^19"
    assert autotune.shape_class((256, 256, 256)) == "3d-n2^24"
    assert autotune.shape_class((1000, 500)) == autotune.shape_class((1024, 512))


class FakeGroup:
    def __init__(self, members):
        self.members = members
        self.variant = None
        self.bpc = None
        self.steps_done = 0

    def set_tile(self, v, bpc):
        self.variant, self.bpc = v, bpc

    def step(self, n):
        self.steps_done += n
        for m in self.members:
            m.state = b"advanced"


def fake_group_timer(run, steps, sync):
    g = run.__self__
    run(steps)
    # variant 6 on one workgroup per table entry is fastest
    return 1.0 + abs(g.variant - 6) + 0.25 * g.bpc


def test_tune_group_picks_fastest_restores_and_caches(P, tmp_path):
    """The group tuner times (variant, blocks per CU) pairs, restores every
    member, applies the fastest and stores it under the group's shape class; a
    second group of the same class takes the stored choice without timing."""
    cache = autotune.Cache(str(tmp_path / "tune.json"))
    g = FakeGroup([FakeCase(P) for _ in range(3)])
    out = autotune.tune_group(g, steps=10, cache=cache, arch="gfx950", timer=fake_group_timer,
                              sync=lambda: None)
    assert (out["variant"], out["blocks_per_cu"]) == (6, 0) == (g.variant, g.bpc)
    assert all(m.state == b"original" for m in g.members)
    assert len(out["candidates"]) == 4 * len(P.step_variants("D2Q9"))
    data = json.load(open(tmp_path / "tune.json"))
    assert data[out["key"]]["variant"] == 6 and "group-2d-x3-" in out["key"]
    g2 = FakeGroup([FakeCase(P) for _ in range(3)])
    out2 = autotune.tune_group(g2, cache=autotune.Cache(str(tmp_path / "tune.json")),
                               arch="gfx950", timer=None, sync=lambda: None)
    assert out2["cached"] and (g2.variant, g2.bpc) == (6, 0) and g2.steps_done == 0
    # another member count is another class
    g3 = FakeGroup([FakeCase(P) for _ in range(5)])
    assert autotune.group_cache_key("gfx950", g3) != out["key"]
