"""Launch-shape autotuner for the fused and batched step kernels.

Candidates are the step variants the library exports (`pflbm_step_variants`),
each with the three XCD dispatch orders (round-robin, contiguous, chunked), and for
groups one workgroup per table entry or a persistent grid of 1, 2 or 4
workgroups per CU.  Each candidate
is timed on the real case with graph replay; the case's state is saved before
and restored after, so tuning leaves it exactly as it was (resume is
bit-identical, and no launch shape changes the results).  The best choice is
cached in a JSON file keyed by GPU architecture, lattice, storage and a shape
class (dimension and log2 of the node count).
"""
import json
import math
import os
import time

from . import pflbm as _p

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pflbm_autotune.json")
# XCD dispatch orders of the step kernels (pflbm_set_step_options): round-robin,
# one contiguous run per XCD, chunks of whole tile rows dealt round-robin
XCD_ORDERS = (0, 1, 2)


def gpu_arch():
    import torch
    name = torch.cuda.get_device_properties(0).gcnArchName
    return name.split(":")[0]


def shape_class(shape):
    n = 1
    for v in shape:
        n *= int(v)
    return f"{len(shape)}d-n2^{int(round(math.log2(max(n, 1))))}"


def cache_key(arch, lattice, storage, shape):
    lat = {_p.D2Q9: "D2Q9", _p.D3Q19: "D3Q19", _p.D3Q19_D3Q7: "D3Q19-D3Q7"}.get(lattice,
                                                                             str(lattice))
    st = {_p.FP64: "f64", _p.FP32: "f32", _p.FP16_DEV: "f16dev"}.get(storage, str(storage))
    return f"{arch}/{lat}/{st}/{shape_class(shape)}"


class Cache:
    def __init__(self, path=DEFAULT_CACHE):
        self.path = path
        self.data = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    def get(self, key):
        return self.data.get(key)

    def put(self, key, value):
        self.data[key] = value
        if self.path:
            os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def _wall_timer(run, steps, sync):
    run(max(2, steps // 10))                       # warm-up (and graph capture)
    sync()
    t0 = time.perf_counter()
    run(steps)
    sync()
    return (time.perf_counter() - t0) / steps


def _torch_sync():
    import torch
    torch.cuda.synchronize()


def tune_case(case, steps=200, cache=None, arch=None, timer=None, sync=None,
              xcd_orders=XCD_ORDERS):
    """Pick the fastest (variant, xcd_order) for `case` over every step variant
    and the given XCD orders; applies and returns it.  A search over fewer
    orders than XCD_ORDERS neither reads nor writes the cache."""
    timer = timer or _wall_timer
    sync = sync or _torch_sync
    arch = arch or gpu_arch()
    prm = case.params
    key = cache_key(arch, prm.lattice, prm.storage, case.shape)
    if tuple(xcd_orders) != tuple(XCD_ORDERS):
        cache = None
    if cache is not None and cache.get(key):
        best = cache.get(key)
        case.set_step_kernel(best["variant"])
        case.set_step_options(best["xcd_order"], False)
        return dict(best, cached=True)
    blob = case.get_state()
    lattice = "D2Q9" if prm.lattice == _p.D2Q9 else "D3Q19"
    results = []
    for v in range(len(_p.step_variants(lattice))):
        for xo in xcd_orders:
            case.set_step_kernel(v)
            case.set_step_options(xo, False)
            sec = timer(case.step, steps, sync)
            results.append(dict(variant=v, xcd_order=xo, ms=sec * 1e3))
    case.set_state(blob)
    best = min(results, key=lambda r: r["ms"])
    case.set_step_kernel(best["variant"])
    case.set_step_options(best["xcd_order"], False)
    out = dict(variant=best["variant"], xcd_order=best["xcd_order"], ms=best["ms"],
               candidates=results)
    if cache is not None:
        cache.put(key, {k: out[k] for k in ("variant", "xcd_order", "ms")})
    return out


def group_shape_class(group):
    """Shape class of a group: member count and log2 of its total node count,
    e.g. "2d-x64-n2^23"."""
    ms = group.members
    n = sum(math.prod(int(v) for v in m.shape) for m in ms)
    return f"{len(ms[0].shape)}d-x{len(ms)}-n2^{int(round(math.log2(max(n, 1))))}"


def group_cache_key(arch, group):
    prm = group.members[0].params
    key = cache_key(arch, prm.lattice, prm.storage, (1,))
    return key.rsplit("/", 1)[0] + "/group-" + group_shape_class(group)


def tune_group(group, steps=100, blocks_per_cu=(0, 1, 2, 4), cache=None, arch=None,
               variants=None, timer=None, sync=None):
    """Pick the fastest (variant, blocks per CU) for a group; every member's
    state is restored afterwards.  Applies and returns the choice.  With a
    cache, a stored choice for the same (architecture, lattice, storage, group
    shape class) is applied without timing, and a new choice is stored."""
    timer = timer or _wall_timer
    sync = sync or _torch_sync
    if not group.members:
        return None
    key = None
    if cache is not None:
        arch = arch or gpu_arch()
        key = group_cache_key(arch, group)
        hit = cache.get(key)
        if hit:
            group.set_tile(hit["variant"], hit["blocks_per_cu"])
            return dict(hit, cached=True, key=key)
    blobs = [m.get_state() for m in group.members]
    lattice = "D2Q9" if group.members[0].params.lattice == _p.D2Q9 else "D3Q19"
    if variants is None:
        variants = range(len(_p.step_variants(lattice)))
    results = []
    for v in variants:
        for bpc in blocks_per_cu:
            group.set_tile(v, bpc)
            sec = timer(group.step, steps, sync)
            results.append(dict(variant=v, blocks_per_cu=bpc, ms=sec * 1e3))
    for m, b in zip(group.members, blobs):
        m.set_state(b)
    best = min(results, key=lambda r: r["ms"])
    group.set_tile(best["variant"], best["blocks_per_cu"])
    if cache is not None:
        cache.put(key, {k: best[k] for k in ("variant", "blocks_per_cu", "ms")})
    return dict(best, candidates=results, key=key)
