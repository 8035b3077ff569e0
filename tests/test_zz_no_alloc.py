"""The allocation-free group poll (pflbm_group_poll_static) against
pflbm_group_poll: two identical groups stepped alike give the same records
through either call, on a larger group and then a smaller one (the static
scratch keeps the first call's contents), and the limits are refused."""
import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _cases(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        nx = int(rng.integers(4, 12)) * 16
        out.append(workloads.cylinder_case(nx, nx // 2, float(rng.uniform(0.2, 0.4)),
                                           float(rng.uniform(30, 150))))
    return out


def _same(a, b):
    for k in ("step", "mass", "s_sum", "steady_residual", "theta_deg", "radius", "n_points",
              "nonfinite", "steady"):
        x, y = a[k], b[k]
        if isinstance(x, float) and math.isnan(x):
            assert math.isnan(y), k
        else:
            assert x == y, (k, x, y)


def test_group_poll_static_matches_poll(P):
    for cases, storage in ((_cases(7, 1), "f32"), (_cases(3, 2)[:2], "f16dev")):
        ga, gb = P.Group(), P.Group()
        ma = [P.Case.from_case(c, storage) for c in cases]
        mb = [P.Case.from_case(c, storage) for c in cases]
        for x, y in zip(ma, mb):
            ga.add(x)
            gb.add(y)
        for rnd in range(2):
            ga.step(60)
            gb.step(60)
            da, fa = ga.poll()
            db, fb = gb.poll(static=True)
            assert np.array_equal(fa, fb)
            for x, y in zip(da, db):
                _same(x, y)
        assert all(m.steps == 120 for m in mb)
        for m in ma:
            ga.remove(m)
        for m in mb:
            gb.remove(m)
        ga.close()
        gb.close()


def test_group_poll_static_refusals(P):
    c = workloads.flat_droplet_case(96, 48, 12.0, 70.0, 4.0)
    g = P.Group()
    m = P.Case.from_case(c, "f32")
    g.add(m)
    with pytest.raises(P.PflbmError) as e:       # changed since its last step
        g.poll(static=True)
    assert e.value.code == -5
    g.step(2)
    g.poll(static=True)
    g.remove(m)
    # more table entries than the static scratch holds (32768): a 4096 x 4160 case
    # has 64 x 520 tiles of 64 x 8 nodes
    big = workloads.flat_droplet_case(4096, 4160, 100.0, 70.0, 4.0)
    mb = P.Case.from_case(big, "f32")
    g.add(mb)
    g.step(2)
    with pytest.raises(P.PflbmError) as e:
        g.poll(static=True)
    assert e.value.code == -1
    g.remove(mb)
    g.close()
