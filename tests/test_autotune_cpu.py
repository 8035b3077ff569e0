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
    # variant 3 with the XCD order is fastest
    return 1.0 + abs(case.variant - 3) + (0.0 if case.xcd else 0.5)


def test_tune_case_picks_fastest_restores_and_caches(P, tmp_path):
    cache = autotune.Cache(str(tmp_path / "tune.json"))
    case = FakeCase(P)
    out = autotune.tune_case(case, steps=10, cache=cache, arch="gfx950", timer=fake_timer,
                             sync=lambda: None)
    assert out["variant"] == 3 and out["xcd_order"] is True
    assert case.variant == 3 and case.xcd is True
    assert case.state == b"original"                   # state restored after timing
    n_variants = len(P.step_variants("D2Q9"))
    assert len(out["candidates"]) == 2 * n_variants
    data = json.load(open(tmp_path / "tune.json"))
    key = autotune.cache_key("gfx950", case.params.lattice, case.params.storage, case.shape)
    assert data[key]["variant"] == 3
    # a second case of the same class uses the cache without timing anything
    c2 = FakeCase(P)
    out2 = autotune.tune_case(c2, cache=autotune.Cache(str(tmp_path / "tune.json")),
                              arch="gfx950", timer=None, sync=lambda: None)
    assert out2["cached"] and c2.variant == 3 and c2.steps_done == 0


def test_shape_classes():
    assert autotune.shape_class((1024, 512)) == "2d-n2^19"
    assert autotune.shape_class((256, 256, 256)) == "3d-n2^24"
    assert autotune.shape_class((1000, 500)) == autotune.shape_class((1024, 512))
