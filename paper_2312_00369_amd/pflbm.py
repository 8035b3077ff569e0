"""ctypes binding of libpflbm.so (argument marshalling only).

Every function of include/pflbm.h is exposed under the same name on `lib`;
`Case` and `Group` wrap the handles.  All time stepping, stencils, collisions
and reductions run in the HIP library; nothing here computes the method.  If
the library is missing this module raises on import.
"""
import ctypes as ct
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpflbm.so")

D2Q9, D3Q19, D3Q19_D3Q7, D3Q7 = 0, 1, 2, 3
FP64, FP32, FP16_DEV = 0, 1, 2
WALL_NONE, WALL_PLANE, WALL_BALL = 0, 1, 2
STORAGE = {"f64": FP64, "f32": FP32, "f16dev": FP16_DEV, "fp64": FP64, "fp32": FP32,
           "fp16dev": FP16_DEV, FP64: FP64, FP32: FP32, FP16_DEV: FP16_DEV}
LATTICE = {"D2Q9": D2Q9, "D3Q19": D3Q19, "D3Q19/D3Q7": D3Q19_D3Q7, "D3Q7": D3Q7,
           D2Q9: D2Q9, D3Q19: D3Q19, D3Q19_D3Q7: D3Q19_D3Q7, D3Q7: D3Q7}


def case_lattice(c):
    """Lattice id of a `workloads` case dict: its "lattice", with D3Q7 for g when
    c["phase_lattice"] == "D3Q7" (Sec. 2.1.3)."""
    if c.get("phase_lattice") == "D3Q7":
        if c["lattice"] != "D3Q19":
            raise ValueError("D3Q7 for g goes with D3Q19")
        return D3Q19_D3Q7
    return LATTICE[c["lattice"]]
ERRORS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENONFINITE",
          -5: "ESTATE", -6: "EUNSUPPORTED"}


class pflbm_params(ct.Structure):
    _fields_ = [
        ("struct_size", ct.c_uint32),
        ("lattice", ct.c_int32),
        ("storage", ct.c_int32),
        ("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32),
        ("periodic", ct.c_int32 * 3),
        ("tau", ct.c_double), ("tau_phi", ct.c_double), ("mobility", ct.c_double),
        ("beta", ct.c_double), ("kappa", ct.c_double), ("rho_l", ct.c_double),
        ("rho_g", ct.c_double), ("nu_l", ct.c_double), ("nu_g", ct.c_double),
        ("theta_deg", ct.c_double),
        ("body_force", ct.c_double * 3),
        ("wall_kind", ct.c_int32),
        ("wall_point", ct.c_double * 3), ("wall_normal", ct.c_double * 3),
        ("wall_radius", ct.c_double), ("diag_width", ct.c_double),
        ("steady_tol", ct.c_double),
        ("chi_case", ct.c_int32),
        ("theta_map", ct.c_void_p),
    ]


class pflbm_diag(ct.Structure):
    _fields_ = [
        ("step", ct.c_int64), ("mass", ct.c_double), ("s_sum", ct.c_double),
        ("steady_residual", ct.c_double), ("theta_deg", ct.c_double),
        ("centre", ct.c_double * 3), ("radius", ct.c_double),
        ("n_points", ct.c_int64), ("nonfinite", ct.c_int32), ("steady", ct.c_int32),
    ]


class PflbmError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib.pflbm_last_error().decode() if lib is not None else ""
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({code}): {msg}")


def _load():
    # torch ships its own HIP runtime (same soname as ROCm's).  Loading torch
    # first makes this library bind to that runtime, so the process holds a
    # single HIP runtime and torch tensors / streams can be shared with it.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2312_00369_amd.build`")
    L = ct.CDLL(LIB_PATH)
    P = ct.POINTER
    vp, i32, i64, sz = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_size_t
    sig = {
        "pflbm_footprint": (ct.c_int, [P(pflbm_params), P(sz)]),
        "pflbm_classify": (ct.c_int, [P(pflbm_params), vp, vp]),
        "pflbm_lattice_table": (ct.c_int, [i32, vp, vp, vp, vp]),
        "pflbm_beta_kappa": (ct.c_int, [ct.c_double, ct.c_double, P(ct.c_double), P(ct.c_double)]),
        "pflbm_create": (ct.c_int, [P(pflbm_params), vp, vp, vp, P(vp)]),
        "pflbm_create_in": (ct.c_int, [P(pflbm_params), vp, vp, vp, vp, sz, P(vp)]),
        "pflbm_step": (ct.c_int, [vp, i64]),
        "pflbm_set_graph_chunk": (ct.c_int, [vp, i32]),
        "pflbm_set_tile": (ct.c_int, [vp, i32, i32, i32]),
        "pflbm_set_step_kernel": (ct.c_int, [vp, i32]),
        "pflbm_step_variants": (ct.c_int, [i32, vp, i32]),
        "pflbm_set_step_options": (ct.c_int, [vp, i32, i32]),
        "pflbm_fp16_scales": (ct.c_int, [vp, vp, vp]),
        "pflbm_set_fp16_scales": (ct.c_int, [vp, ct.c_double, ct.c_double]),
        "pflbm_fields": (ct.c_int, [vp, vp, vp, vp, vp]),
        "pflbm_node_classes": (ct.c_int, [vp, vp]),
        "pflbm_diagnostics": (ct.c_int, [vp, P(pflbm_diag)]),
        "pflbm_state_size": (ct.c_int, [vp, P(sz)]),
        "pflbm_get_state": (ct.c_int, [vp, vp, sz]),
        "pflbm_set_state": (ct.c_int, [vp, vp, sz]),
        "pflbm_profile": (ct.c_int, [vp, i64, vp, i32]),
        "pflbm_step_count": (i64, [vp]),
        "pflbm_destroy": (None, [vp]),
        "pflbm_group_create": (ct.c_int, [vp, P(vp)]),
        "pflbm_group_add": (ct.c_int, [vp, vp]),
        "pflbm_group_remove": (ct.c_int, [vp, vp]),
        "pflbm_group_size": (ct.c_int, [vp]),
        "pflbm_group_step": (ct.c_int, [vp, i64]),
        "pflbm_group_poll": (ct.c_int, [vp, vp, vp, i32]),
        "pflbm_group_poll_static": (ct.c_int, [vp, vp, vp, i32]),
        "pflbm_group_set_tile": (ct.c_int, [vp, i32, i32]),
        "pflbm_group_set_graph_chunk": (ct.c_int, [vp, i32]),
        "pflbm_group_destroy": (None, [vp]),
        "pflbm_strerror": (ct.c_char_p, [ct.c_int]),
        "pflbm_last_error": (ct.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L, sorted(sig)


lib = None
lib, EXPORTED = _load()


def _check(rc, where):
    if rc != 0:
        raise PflbmError(rc, where)


def _ptr(a):
    return a.ctypes.data_as(ct.c_void_p) if a is not None else None


def beta_kappa(sigma, width):
    """Free-energy coefficients for surface tension and interface width, from the
    library (pflbm_beta_kappa)."""
    b, k = ct.c_double(), ct.c_double()
    _check(lib.pflbm_beta_kappa(float(sigma), float(width), ct.byref(b), ct.byref(k)),
           "pflbm_beta_kappa")
    return b.value, k.value


def make_params(lattice, shape, periodic, theta_deg, beta, kappa, storage="f32", tau=0.8,
                tau_phi=0.0, mobility=0.1, rho_l=10.0, rho_g=1.0, nu_l=0.0, nu_g=0.0,
                body_force=(0.0, 0.0, 0.0), wall=None, diag_width=4.0, steady_tol=1e-5,
                chi_case=2, theta_map=None):
    p = pflbm_params()
    p.struct_size = ct.sizeof(pflbm_params)
    p.lattice = LATTICE[lattice]
    p.storage = STORAGE[storage]
    shp = tuple(shape) + (1,) * (3 - len(shape))
    p.nx, p.ny, p.nz = (int(v) for v in shp)
    per = tuple(periodic) + (True,) * (3 - len(periodic))
    for a in range(3):
        p.periodic[a] = 1 if per[a] else 0
    p.tau, p.tau_phi, p.mobility = tau, tau_phi, mobility
    p.beta, p.kappa = beta, kappa
    p.rho_l, p.rho_g, p.nu_l, p.nu_g = rho_l, rho_g, nu_l, nu_g
    p.theta_deg = theta_deg
    for a in range(3):
        p.body_force[a] = body_force[a] if a < len(body_force) else 0.0
    if wall is None:
        p.wall_kind = WALL_NONE
    elif wall["kind"] == "plane":
        p.wall_kind = WALL_PLANE
        for a, v in enumerate(wall["point"]):
            p.wall_point[a] = v
        for a, v in enumerate(wall["normal"]):
            p.wall_normal[a] = v
    else:
        p.wall_kind = WALL_BALL
        for a, v in enumerate(wall["center"]):
            p.wall_point[a] = v
        p.wall_radius = wall["radius"]
    p.diag_width = diag_width
    p.steady_tol = steady_tol
    p.chi_case = int(chi_case)
    if theta_map is not None:
        # contact angle per node (numpy order (z,) y, x, i.e. x fastest); the
        # array lives as long as the parameter record
        p._theta_map = np.ascontiguousarray(theta_map, dtype=np.float64).ravel()
        if p._theta_map.size != p.nx * p.ny * p.nz:
            raise ValueError("theta_map must have one value per domain node")
        p.theta_map = p._theta_map.ctypes.data
    return p


def params_from_case(c, storage=None, **over):
    """pflbm_params for a case dict of the `workloads` module."""
    beta, kappa = beta_kappa(c["sigma"], c["width"])
    kw = dict(storage=storage or c.get("storage", "f32"), tau=c.get("tau", 0.8),
              mobility=c.get("mobility", 0.1), rho_l=c.get("rho_l", 10.0),
              rho_g=c.get("rho_g", 1.0), wall=c.get("wall"), diag_width=c["width"],
              chi_case=c.get("chi_case", 2), theta_map=c.get("theta_map"))
    kw.update(over)
    return make_params(case_lattice(c), c["shape"], c["periodic"], c["theta_deg"], beta, kappa,
                       **kw)


def footprint(params):
    n = ct.c_size_t(0)
    _check(lib.pflbm_footprint(ct.byref(params), ct.byref(n)), "pflbm_footprint")
    return n.value


def classify(params, mask):
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    out = np.zeros(mask.shape, dtype=np.uint8)
    _check(lib.pflbm_classify(ct.byref(params), _ptr(mask), _ptr(out)), "pflbm_classify")
    return out


def lattice_table(lattice):
    Q = {D2Q9: 9, D3Q7: 7}.get(LATTICE[lattice], 19)
    c = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q)
    opp = np.zeros(Q, dtype=np.int32)
    k = np.zeros(Q)
    rc = lib.pflbm_lattice_table(LATTICE[lattice], _ptr(c), _ptr(w), _ptr(opp), _ptr(k))
    if rc < 0:
        _check(rc, "pflbm_lattice_table")
    return dict(c=c, w=w, opp=opp, k=k)


def step_variants(lattice):
    n = lib.pflbm_step_variants(LATTICE[lattice], None, 0)
    if n < 0:
        _check(n, "pflbm_step_variants")
    t = np.zeros((n, 5), dtype=np.int32)
    lib.pflbm_step_variants(LATTICE[lattice], _ptr(t), n)
    return [dict(block=(64, int(r[0]), int(r[1])), tile=(int(r[2]), int(r[3]), int(r[4]))) for r in t]


def _stream_ptr(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return ct.c_void_p(stream.cuda_stream)
    return ct.c_void_p(int(stream))


class Case:
    """One simulation case resident on the GPU."""

    def __init__(self, params, mask, phi0, stream=None, workspace=False):
        self.params = params
        self.shape = (params.nx, params.ny) if params.lattice == D2Q9 else (params.nx, params.ny, params.nz)
        self.D = len(self.shape)
        self._mask = np.ascontiguousarray(mask, dtype=np.uint8).reshape(self.shape[::-1])
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(self.shape[::-1])
        self._ws = None
        h = ct.c_void_p()
        sp = _stream_ptr(stream)
        if workspace:
            import torch
            nbytes = footprint(params)
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            addr = self._ws.data_ptr()
            addr = (addr + 255) // 256 * 256
            rc = lib.pflbm_create_in(ct.byref(params), _ptr(self._mask), _ptr(phi0), sp,
                                     ct.c_void_p(addr), ct.c_size_t(nbytes), ct.byref(h))
            _check(rc, "pflbm_create_in")
        else:
            _check(lib.pflbm_create(ct.byref(params), _ptr(self._mask), _ptr(phi0), sp, ct.byref(h)),
                   "pflbm_create")
        self.h = h

    @classmethod
    def from_case(cls, c, storage=None, stream=None, workspace=False, **over):
        return cls(params_from_case(c, storage, **over), c["mask"], c["phi0"], stream, workspace)

    def step(self, n=1):
        _check(lib.pflbm_step(self.h, int(n)), "pflbm_step")

    def set_graph_chunk(self, k):
        _check(lib.pflbm_set_graph_chunk(self.h, int(k)), "pflbm_set_graph_chunk")

    def set_tile(self, tx, ty, tz=1):
        _check(lib.pflbm_set_tile(self.h, tx, ty, tz), "pflbm_set_tile")

    def fp16_scales(self):
        """(scale_f, scale_g) of FP16-deviation storage (1, 1 otherwise)."""
        sf, sg = ct.c_double(0), ct.c_double(0)
        _check(lib.pflbm_fp16_scales(self.h, ct.byref(sf), ct.byref(sg)), "pflbm_fp16_scales")
        return sf.value, sg.value

    def set_fp16_scales(self, scale_f, scale_g):
        _check(lib.pflbm_set_fp16_scales(self.h, float(scale_f), float(scale_g)),
               "pflbm_set_fp16_scales")

    def set_step_options(self, xcd_order=True, nontemporal=False):
        _check(lib.pflbm_set_step_options(self.h, int(xcd_order), int(bool(nontemporal))),
               "pflbm_set_step_options")

    def set_step_kernel(self, variant):
        """variant >= 0: fused one-kernel step with that tile shape; -1: three kernels."""
        _check(lib.pflbm_set_step_kernel(self.h, int(variant)), "pflbm_set_step_kernel")

    @property
    def steps(self):
        return int(lib.pflbm_step_count(self.h))

    def fields(self):
        shp = self.shape[::-1]
        phi = np.zeros(shp)
        p = np.zeros(shp)
        mu = np.zeros(shp)
        u = np.zeros((self.D,) + shp)
        _check(lib.pflbm_fields(self.h, _ptr(phi), _ptr(p), _ptr(u), _ptr(mu)), "pflbm_fields")
        return dict(phi=phi, p=p, u=u, mu=mu)

    def classes(self):
        out = np.zeros(self.shape[::-1], dtype=np.uint8)
        _check(lib.pflbm_node_classes(self.h, _ptr(out)), "pflbm_node_classes")
        return out

    def diagnostics(self):
        d = pflbm_diag()
        _check(lib.pflbm_diagnostics(self.h, ct.byref(d)), "pflbm_diagnostics")
        return _diag_dict(d)

    def get_state(self):
        n = ct.c_size_t(0)
        _check(lib.pflbm_state_size(self.h, ct.byref(n)), "pflbm_state_size")
        buf = np.zeros(n.value, dtype=np.uint8)
        _check(lib.pflbm_get_state(self.h, _ptr(buf), n), "pflbm_get_state")
        return buf

    def set_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib.pflbm_set_state(self.h, _ptr(buf), ct.c_size_t(buf.size)), "pflbm_set_state")

    def profile(self, nsteps, nkinds=4):
        out = np.zeros(nkinds)
        _check(lib.pflbm_profile(self.h, int(nsteps), _ptr(out), nkinds), "pflbm_profile")
        return out

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib.pflbm_destroy(self.h)
            self.h = ct.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _diag_dict(d):
    return dict(step=d.step, mass=d.mass, s_sum=d.s_sum, steady_residual=d.steady_residual,
                theta_deg=d.theta_deg, centre=tuple(d.centre), radius=d.radius,
                n_points=d.n_points, nonfinite=bool(d.nonfinite), steady=bool(d.steady))


class Group:
    """Cases advanced together by the batched kernels."""

    def __init__(self, stream=None):
        g = ct.c_void_p()
        _check(lib.pflbm_group_create(_stream_ptr(stream), ct.byref(g)), "pflbm_group_create")
        self.g = g
        self.members = []

    def add(self, case):
        _check(lib.pflbm_group_add(self.g, case.h), "pflbm_group_add")
        self.members.append(case)

    def remove(self, case):
        _check(lib.pflbm_group_remove(self.g, case.h), "pflbm_group_remove")
        self.members.remove(case)

    def __len__(self):
        return int(lib.pflbm_group_size(self.g))

    def step(self, n=1):
        _check(lib.pflbm_group_step(self.g, int(n)), "pflbm_group_step")

    def set_tile(self, variant=-1, blocks_per_cu=0):
        _check(lib.pflbm_group_set_tile(self.g, int(variant), int(blocks_per_cu)),
               "pflbm_group_set_tile")

    def set_graph_chunk(self, k):
        _check(lib.pflbm_group_set_graph_chunk(self.g, int(k)), "pflbm_group_set_graph_chunk")

    def poll(self, static=False):
        """Reductions of every member: (diagnostics dicts, flags).  static=True
        calls the allocation-free variant (pflbm_group_poll_static)."""
        n = len(self.members)
        ds = (pflbm_diag * max(n, 1))()
        flags = np.zeros(max(n, 1), dtype=np.int32)
        fn = lib.pflbm_group_poll_static if static else lib.pflbm_group_poll
        _check(fn(self.g, ds, _ptr(flags), n),
               "pflbm_group_poll_static" if static else "pflbm_group_poll")
        return [_diag_dict(ds[k]) for k in range(n)], flags[:n]

    def close(self):
        if getattr(self, "g", None) is not None and self.g.value:
            lib.pflbm_group_destroy(self.g)
            self.g = ct.c_void_p()
        self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
