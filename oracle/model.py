"""FP64 NumPy oracle of the coupled phase-field / hydrodynamic LBE with the wall
free energy in the chemical potential (test infrastructure only).

Every array holds one value per node of a *padded* grid: each non-periodic axis
gets two layers of virtual solid nodes on both sides, so that every read made
by a ghost node stays inside the array.  Flat index = x + Px*(y + Py*z).

One time step (the paper gives no algorithm box; this is the explicit order the
equations imply, every quantity at time t built from phi(t) and f(t)):
  1. phi = sum_i g_i                                  Eq. (order-parameter)
  2. ghost phi = zeta-weighted mean of its 3^D block  Sec. 2.2.2 (Appendix A
     cases 1 and 3: the ghost solves n_w . grad phi = chi across the wall)
  3. rho(phi), grad phi, lap phi, grad rho            Eq. (gradient), (Laplace)
  4. mu with the wall term a_v sqrt(2 kappa beta) cos(theta) (phi - phi^2)
     (with a per-node theta: the mean cos(theta) of the walls around the node)
                                                      Eq. (chemical_potencial2)
  5. F = mu grad phi + F_b                            Sec. 2.1.1
  6. u from rho u = sum c_i f_i + F/2 (u = 0 on boundary nodes, which lie in
     the solid); then p                               Sec. 2.1.2, after Eq. (GGi)
  7. s = u . grad phi; g collides with G_i and the time derivative of G_i
                                                      Eq. (BGK), (H_i), (F_i)
  8. f collides with F_i                              Eq. (BGK-NS), (feq_i), (GGi)
  9. both sets stream; a population whose source node is solid is replaced by
     the post-collision population of the opposite direction at the same node
     (bounce-back, Sec. 2.2.2).
Readings of points the paper leaves open are marked READING in the comments.
Three of them have no printed number behind them and are pinned by what the
paper states the model recovers: alpha's split of M (only M = c_s^2 alpha
(tau_g - 1/2) is printed; the Cahn-Hilliard rate must depend on M alone), the
backward difference for the time derivative of G_i (an advected mode must decay
at the Cahn-Hilliard rate), and u = 0 on boundary nodes (the wall mode it
suppresses grows under the other reading).

This module is test infrastructure: only the tests, the smoke check and the
CPU baseline of the benchmark use it; the library never does.
"""
from dataclasses import dataclass, field
import math

import numpy as np

from . import lattice as lat


def beta_kappa(sigma, width):
    """beta, kappa from surface tension and interface width.

    READING: the double well psi = beta phi^2 (phi-1)^2 (Eq. bulk_energy) has the
    planar profile 0.5 + 0.5 tanh(2x/W) (Eq. initialphi) with W = sqrt(8 kappa/beta),
    and Young's law with b1 = -sqrt(2 kappa beta) cos(theta) (Eq. b1, sigma_sl =
    b1/6) makes sigma = sqrt(2 kappa beta)/6.  Solving both: beta = 12 sigma / W,
    kappa = 3 sigma W / 2.
    """
    return 12.0 * sigma / width, 1.5 * sigma * width


@dataclass
class Params:
    lattice: str = "D2Q9"
    phase_lattice: str = ""           # velocity set of g; "" = same as `lattice`
    shape: tuple = (128, 64)          # (nx, ny) or (nx, ny, nz)
    periodic: tuple = (True, False)   # per axis
    tau: float = 0.8                  # tau_f when nu_l = nu_g = 0
    tau_phi: float = 0.0              # tau_g; 0 means "same as tau"
    mobility: float = 0.1
    beta: float = 3e-3
    kappa: float = 6e-3
    rho_l: float = 10.0
    rho_g: float = 1.0
    nu_l: float = 0.0
    nu_g: float = 0.0
    theta_deg: float = 60.0
    chi_case: int = 2                 # Appendix A, Table A1: 1, 2 (the method) or 3
    theta_map: object = None          # per-node contact angle (degrees) on solid nodes
    body_force: tuple = (0.0, 0.0, 0.0)
    extra: dict = field(default_factory=dict)


class Grid:
    """Padded node set and neighbour index maps."""

    def __init__(self, shape, periodic):
        self.shape = tuple(int(n) for n in shape)
        self.D = len(self.shape)
        self.periodic = tuple(bool(p) for p in periodic)
        self.pad = [0 if p else 2 for p in self.periodic]
        self.P = [n + 2 * pd for n, pd in zip(self.shape, self.pad)]
        self.N = int(np.prod(self.P))
        rem = np.arange(self.N)
        self.coords = []
        for d in range(self.D):
            self.coords.append(rem % self.P[d])
            rem = rem // self.P[d]
        self.inside = np.ones(self.N, dtype=bool)
        for d in range(self.D):
            q = self.coords[d]
            self.inside &= (q >= self.pad[d]) & (q < self.pad[d] + self.shape[d])
        self._cache = {}

    def shift(self, c):
        """(index of node + c, whether that node exists in the padded array)."""
        key = tuple(int(v) for v in c)
        if key not in self._cache:
            flat = np.zeros(self.N, dtype=np.int64)
            ok = np.ones(self.N, dtype=bool)
            stride = 1
            for d in range(self.D):
                q = self.coords[d] + key[d]
                if self.periodic[d]:
                    q = q % self.P[d]
                else:
                    ok &= (q >= 0) & (q < self.P[d])
                    q = np.clip(q, 0, self.P[d] - 1)
                flat += q * stride
                stride *= self.P[d]
            self._cache[key] = (flat, ok)
        return self._cache[key]

    def to_domain(self, a):
        """Padded flat array -> domain array, numpy shape (nz, ny, nx) / (ny, nx)."""
        a = np.asarray(a).reshape(self.P[::-1])
        sl = tuple(slice(self.pad[d], self.pad[d] + self.shape[d]) for d in range(self.D))
        return a[sl[::-1]]

    def from_domain(self, a, fill=0):
        a = np.asarray(a).reshape(self.shape[::-1])
        out = np.full(self.P[::-1], fill, dtype=a.dtype)
        sl = tuple(slice(self.pad[d], self.pad[d] + self.shape[d]) for d in range(self.D))
        out[sl[::-1]] = a
        return out.ravel()


# ---------------------------------------------------------------- node classes

def classify(grid, L, solid_mask):
    """Node marks of Sec. 2.2.2 and the void fraction of Eq. (avvv) ff.

    READING: the mask is the geometric solid.  A solid node with at least one
    lattice link to a non-solid node is a *boundary* node: it carries f and g and
    takes part in collision and streaming (zeta = 1) but has epsilon = 0.  Fluid
    nodes have zeta = epsilon = 1.  Other solid nodes and the virtual padding
    have zeta = epsilon = 0.  Ghost nodes are zeta = 0 nodes one lattice link
    away from a zeta = 1 node.
    """
    solid = grid.from_domain(np.asarray(solid_mask, dtype=bool), fill=True)
    fluid = grid.inside & ~solid
    near_fluid = np.zeros(grid.N, dtype=bool)
    for i in range(1, L.Q):
        nb, ok = grid.shift(L.c[i])
        near_fluid |= ok & fluid[nb]
    boundary = grid.inside & solid & near_fluid
    zeta = fluid | boundary
    ghost = np.zeros(grid.N, dtype=bool)
    for i in range(1, L.Q):
        nb, ok = grid.shift(L.c[i])
        ghost |= ok & zeta[nb]
    ghost &= ~zeta
    eps = fluid.astype(np.float64)
    return zeta, eps, ghost, boundary


# ---------------------------------------------------------------- stencils

def gradient(grid, L, field_):
    """Eq. (gradient): grad G(x) = sum_{i != 0} w_i c_i G(x + c_i) / c_s^2 (dt = 1)."""
    out = np.zeros((L.D, grid.N))
    for i in range(1, L.Q):
        nb, _ = grid.shift(L.c[i])
        for d in range(L.D):
            out[d] += L.w[i] * L.c[i, d] * field_[nb]
    return out / L.cs2


def laplacian(grid, L, field_):
    """Eq. (Laplace): lap G(x) = sum_{i != 0} 2 w_i [G(x + c_i) - G(x)] / c_s^2."""
    out = np.zeros(grid.N)
    for i in range(1, L.Q):
        nb, _ = grid.shift(L.c[i])
        out += 2.0 * L.w[i] * (field_[nb] - field_)
    return out / L.cs2


def effective_area(grid, L, eps, zeta):
    """Eq. (avvv): a_v ~ |grad epsilon|, with the gradient of Eq. (gradient).
    READING: evaluated once, on zeta = 1 nodes only (zero elsewhere)."""
    g = gradient(grid, L, eps)
    return np.where(zeta, np.sqrt((g ** 2).sum(axis=0)), 0.0)


def ghost_fill(grid, phi, zeta, ghost, chi_a=0.0):
    """Sec. 2.2.2: phi at a ghost node is the mean of phi over the zeta = 1 nodes
    of its 3^D neighbourhood (9 offsets in 2D, 27 in 3D).  Only zeta = 1 values
    enter, so the fill order does not matter.

    chi_a != 0 (Appendix A, cases 1 and 3): the ghost instead satisfies
    Eq. (cubicc), n_w . grad phi = chi(phi_w) with chi(phi) = chi_a (phi - phi^2),
    as a central difference across the wall.  READING: the mean above stands for
    phi at the ghost's mirror node (one lattice spacing away along an axis-aligned
    normal; ghost_normals checks that), and phi_w is the mean of the two values.
    With m the mirror value and g the ghost value, m - g = chi((m + g)/2); in
    terms of phi_w = (m + g)/2 this is
        chi_a phi_w^2 - (chi_a + 2) phi_w + 2 m = 0,
    whose root that tends to m as chi_a -> 0 is taken; then g = 2 phi_w - m."""
    num = np.zeros(grid.N)
    den = np.zeros(grid.N)
    for c in lat.ghost_neighbourhood(grid.D):
        nb, ok = grid.shift(c)
        z = (ok & zeta[nb]).astype(np.float64)
        num += z * phi[nb]
        den += z
    out = np.where(zeta, phi, 0.0)
    sel = ghost & (den > 0)
    m = num[sel] / den[sel]
    if chi_a != 0.0:
        a = chi_a
        phi_w = ((a + 2.0) - np.sqrt((a + 2.0) ** 2 - 8.0 * a * m)) / (2.0 * a)
        m = 2.0 * phi_w - m
    out[sel] = m
    return out


def ghost_normals(grid, zeta, ghost):
    """Direction from each ghost node into the fluid: the sum of the offsets of
    the zeta = 1 nodes in its 3^D neighbourhood (zero rows for non-ghosts)."""
    n = np.zeros((grid.D, grid.N))
    for c in lat.ghost_neighbourhood(grid.D):
        nb, ok = grid.shift(c)
        z = (ok & zeta[nb]).astype(np.float64)
        for d in range(grid.D):
            n[d] += z * c[d]
    n[:, ~ghost] = 0.0
    return n


def chi_coefficient(beta, kappa, theta_deg, chi_case):
    """chi_a of chi(phi) = chi_a (phi - phi^2) in Appendix A, Table A1:
    case 1 -sqrt(2 beta/kappa) cos(theta), case 2 zero, case 3 the opposite of
    case 1."""
    c = {1: -1.0, 2: 0.0, 3: 1.0}[int(chi_case)]
    return c * math.sqrt(2.0 * beta / kappa) * math.cos(math.radians(theta_deg))


# ---------------------------------------------------------------- local physics

def f_equilibrium(L, p, rho, u):
    """Eq. (feq_i) with s_i(u) of Eq. (Siu)."""
    cu = np.einsum("qd,dn->qn", L.c.astype(np.float64), u)
    uu = (u ** 2).sum(axis=0)
    s = L.w[:, None] * (cu / L.cs2 + cu ** 2 / (2 * L.cs2 ** 2) - uu / (2 * L.cs2))
    feq = (p / L.cs2)[None, :] * L.w[:, None] + rho[None, :] * s
    feq[0] -= p / L.cs2                      # i = 0: (p / c_s^2)(w_0 - 1)
    return feq


def g_equilibrium(L, phi, alpha, mu):
    """Eq. (H_i), first form: g_0 = phi - (1 - w_0) alpha mu, g_i = w_i alpha mu."""
    geq = L.w[:, None] * (alpha * mu)[None, :]
    geq[0] = phi - (1.0 - L.w[0]) * alpha * mu
    return geq


def force_distribution(L, tau_f, u, grad_rho, F):
    """Eq. (GGi).  READING: the prefactor uses the relaxation time of the
    hydrodynamic equation, tau_f (printed tau_g), and the broken bracket is read
    as u grad(rho) : (c_i c_i - c_s^2 I) / c_s^2."""
    c = L.c.astype(np.float64)
    u_grho = (u * grad_rho).sum(axis=0)
    cF = np.einsum("qd,dn->qn", c, F)
    cu = np.einsum("qd,dn->qn", c, u)
    cg = np.einsum("qd,dn->qn", c, grad_rho)
    bracket = u_grho[None, :] + cF / L.cs2 + (cu * cg - L.cs2 * u_grho[None, :]) / L.cs2
    return (1.0 - 0.5 / tau_f)[None, :] * L.w[:, None] * bracket


def phase_source(L, s):
    """Eq. (F_i): G_i = w_i s k_i with s = u . grad phi."""
    return (L.w * L.k)[:, None] * s[None, :]


def local_cos_theta(grid, eps, theta_deg, theta_map, solid):
    """Heterogeneous wetting.  READING: the paper has one theta per case; with a
    contact angle per solid node, the wall term at a node uses the mean of
    cos(theta) over the epsilon = 0 nodes (solid or virtual) of its 3^D block.
    Solid nodes take theta_map, virtual nodes the case's theta.  A uniform map
    gives back the single-theta chemical potential."""
    cos_node = np.full(grid.N, math.cos(math.radians(theta_deg)))
    if theta_map is not None:
        tm = grid.from_domain(np.asarray(theta_map, dtype=np.float64), fill=theta_deg)
        cos_node = np.where(solid, np.cos(np.radians(tm)), cos_node)
    num = np.zeros(grid.N)
    den = np.zeros(grid.N)
    for c in lat.ghost_neighbourhood(grid.D):
        nb, ok = grid.shift(c)
        wall = (ok & (eps[nb] == 0.0)).astype(np.float64)
        num += wall * cos_node[nb]
        den += wall
    return np.where(den > 0, num / np.maximum(den, 1.0), math.cos(math.radians(theta_deg)))


def chemical_potential(beta, kappa, theta_deg, phi, lap_phi, a_v, chi_case=2, cos_local=None):
    """Eq. (chemical_potencial2): mu = 4 beta phi (phi-1)(phi-1/2) - kappa lap phi
    - a_v sqrt(2 kappa beta) cos(theta) (phi - phi^2).  Cases 1 and 3 of
    Appendix A use Eq. (chemical_potencial112) with their chi: the wall term is
    a_v [kappa chi + sqrt(2 kappa beta) cos(theta) (phi - phi^2)], i.e. zero
    (case 1) or twice the above (case 3)."""
    cos_t = math.cos(math.radians(theta_deg)) if cos_local is None else cos_local
    wet = math.sqrt(2.0 * kappa * beta) * cos_t
    wet = wet * {1: 0.0, 2: 1.0, 3: 2.0}[int(chi_case)]
    return (4.0 * beta * phi * (phi - 1.0) * (phi - 0.5) - kappa * lap_phi
            - a_v * wet * (phi - phi * phi))


# ---------------------------------------------------------------- the solver

class Oracle:
    """State: f and g *after* streaming at time t (one column per padded node,
    zero on zeta = 0 nodes), plus s(t-1) for the time derivative of G_i."""

    # Coefficient of the time derivative of G_i in Eq. (BGK) (1/2 there).  The
    # pins of the oracle set other values on an instance, on the CPU, to show
    # that they reject them.
    DGDT = 0.5
    # READING of Sec. 2.2.2 (boundary nodes lie in the solid and move with it);
    # False takes the fluid velocity there instead, for the same purpose.
    WALL_VELOCITY_ZERO = True

    def __init__(self, params, solid_mask, phi0):
        self.p = params
        self.L = lat.by_name(params.lattice)
        if self.L.D != len(params.shape):
            raise ValueError("lattice dimension does not match the grid")
        # velocity set of the phase-field LBE (Sec. 2.1.3 names D2Q9 and D3Q7);
        # node classes and the phi stencils stay on the hydrodynamic set
        self.Lg = lat.by_name(params.phase_lattice) if params.phase_lattice else self.L
        if self.Lg.D != self.L.D:
            raise ValueError("phase lattice dimension does not match the grid")
        self.grid = Grid(params.shape, params.periodic)
        self.zeta, self.eps, self.ghost, self.boundary = classify(
            self.grid, self.L, solid_mask)
        self.a_v = effective_area(self.grid, self.L, self.eps, self.zeta)
        solid = self.grid.from_domain(np.asarray(solid_mask, dtype=bool), fill=False)
        self.cos_local = (None if params.theta_map is None else
                          local_cos_theta(self.grid, self.eps, params.theta_deg,
                                          params.theta_map, solid))
        self.chi_a = chi_coefficient(params.beta, params.kappa, params.theta_deg,
                                     params.chi_case)
        if params.theta_map is not None and params.chi_case != 2:
            raise ValueError("a per-node contact angle goes with the chi = 0 method only")
        if params.chi_case != 2:
            # Appendix A tests these cases on a flat plate: every ghost must see
            # the fluid along one lattice axis
            n = ghost_normals(self.grid, self.zeta, self.ghost)[:, self.ghost]
            if (np.count_nonzero(n, axis=0) != 1).any():
                raise ValueError("chi cases 1 and 3 need walls normal to a lattice axis")
        self.tau_g = params.tau_phi if params.tau_phi > 0 else params.tau
        # Eq. (mobility): M = c_s^2 alpha (tau_g - 1/2), c_s^2 of the phase
        # lattice.  READING: tau_g is the given relaxation time and alpha
        # follows from it.
        self.alpha = params.mobility / (self.Lg.cs2 * (self.tau_g - 0.5))
        phi = np.where(self.zeta, self.grid.from_domain(np.asarray(phi0, np.float64)), 0.0)
        mu, _, _ = self._mu(phi)
        self.g = np.where(self.zeta, g_equilibrium(self.Lg, phi, self.alpha, mu), 0.0)
        self.f = np.zeros((self.L.Q, self.grid.N))   # p = 0, u = 0
        self.s_prev = None                           # unset until the first step
        self.t = 0
        # pull maps with bounce-back, built once per velocity set
        self._pull = {}
        for Lx in {self.L.name: self.L, self.Lg.name: self.Lg}.values():
            maps = []
            for i in range(Lx.Q):
                nb, ok = self.grid.shift(-Lx.c[i])
                maps.append((nb, ok & self.zeta[nb]))
            self._pull[Lx.name] = maps

    # --------------------------------------------------------- pieces
    def tau_f(self, phi):
        p = self.p
        if p.nu_l == 0.0 and p.nu_g == 0.0:
            return np.full_like(phi, p.tau)
        nu = phi * (p.nu_l - p.nu_g) + p.nu_g        # Sec. 2.1.1, linear in phi
        return nu / self.L.cs2 + 0.5                 # nu = c_s^2 (tau_f - 1/2)

    def _mu(self, phi):
        p = self.p
        phi_full = ghost_fill(self.grid, phi, self.zeta, self.ghost, self.chi_a)
        lap = laplacian(self.grid, self.L, phi_full)
        mu = chemical_potential(p.beta, p.kappa, p.theta_deg, phi_full, lap, self.a_v,
                                p.chi_case, self.cos_local)
        mu = np.where(self.zeta, mu, 0.0)
        return mu, phi_full, lap

    def macroscopic(self):
        """phi, mu, rho, grad phi, grad rho, F, u, p at the current time."""
        p, L = self.p, self.L
        phi = np.where(self.zeta, self.g.sum(axis=0), 0.0)
        mu, phi_full, _ = self._mu(phi)
        rho_full = phi_full * (p.rho_l - p.rho_g) + p.rho_g
        grad_phi = gradient(self.grid, L, phi_full)
        grad_rho = gradient(self.grid, L, rho_full)
        rho = rho_full
        Fb = np.asarray(p.body_force[:L.D], dtype=np.float64)[:, None]
        F = mu[None, :] * grad_phi + Fb
        mom = np.einsum("qd,qn->dn", L.c.astype(np.float64), self.f) + 0.5 * F
        u = np.where(self.zeta, mom / np.where(self.zeta, rho, 1.0), 0.0)
        # READING: a boundary node is a solid node (Sec. 2.2.2): it collides and
        # streams, but its velocity is the wall's, so u = 0 there wherever u
        # enters (f_eq, F_i, p, s).  With the fluid velocity at these nodes
        # instead, a row-alternating momentum mode along the wall grows slowly
        # at sigma = 0.005 (the Sec. 3.1 parameters) until it breaks the drop.
        if self.WALL_VELOCITY_ZERO:
            u[:, self.boundary] = 0.0
        uu = (u ** 2).sum(axis=0)
        s0 = -L.w[0] * uu / (2.0 * L.cs2)
        pres = L.cs2 / (1.0 - L.w[0]) * (self.f[1:].sum(axis=0)
                                          + 0.5 * (u * grad_rho).sum(axis=0) + rho * s0)
        z = self.zeta
        return dict(phi=phi, phi_full=phi_full, mu=mu, rho=rho, grad_phi=grad_phi,
                    grad_rho=grad_rho, F=F, u=u, p=np.where(z, pres, 0.0))

    # --------------------------------------------------------- one step
    def step(self, n=1):
        for _ in range(n):
            self._step()

    def _step(self):
        p, L, z = self.p, self.L, self.zeta
        m = self.macroscopic()
        s = np.where(z, (m["u"] * m["grad_phi"]).sum(axis=0), 0.0)
        if self.s_prev is None:
            self.s_prev = s.copy()
        s_before = self.s_prev
        # Eq. (BGK) with the time derivative of G_i taken as a backward difference.
        # READING: G_i + (1/2) dG_i/dt ~ w_i k_i (s(t) + (s(t) - s(t-1))/2).
        Lg = self.Lg
        geq = g_equilibrium(Lg, m["phi"], self.alpha, m["mu"])
        src = phase_source(Lg, s) + self.DGDT * (phase_source(Lg, s) - phase_source(Lg, self.s_prev))
        g_post = self.g - (self.g - geq) / self.tau_g + src
        tau_f = self.tau_f(m["phi"])
        feq = f_equilibrium(L, m["p"], m["rho"], m["u"])
        Fi = force_distribution(L, tau_f, m["u"], m["grad_rho"], m["F"])
        f_post = self.f - (self.f - feq) / tau_f[None, :] + Fi
        g_post[:, ~z] = 0.0
        f_post[:, ~z] = 0.0
        self.s_prev = s
        self.g = self._stream(g_post, self.Lg)
        self.f = self._stream(f_post, self.L)
        self.t += 1
        self.last = dict(s=s, s_before=s_before, **m)

    def _stream(self, post, Lx):
        """Pull streaming; a link whose source is a zeta = 0 node bounces back.

        READING: the paper's modified bounce-back (Sec. 2.2.2) is taken as the
        halfway rule in pull form: f_i(x, t+1) = f*_{i'}(x, t) when x - c_i is a
        zeta = 0 node; the wall sits halfway along that link."""
        out = np.zeros_like(post)
        for i in range(Lx.Q):
            nb, take = self._pull[Lx.name][i]
            out[i] = np.where(take, post[i][nb], post[Lx.opp[i]])
        out[:, ~self.zeta] = 0.0
        return out

    # --------------------------------------------------------- outputs
    def fields(self):
        """Domain arrays (numpy shape (nz, ny, nx) or (ny, nx)): phi (ghost value on
        ghost nodes, 0 on other solid nodes), p, u (D components), mu."""
        m = self.macroscopic()
        dom = self.grid.to_domain
        phi = np.where(self.zeta, m["phi"], np.where(self.ghost, m["phi_full"], 0.0))
        return dict(phi=dom(phi), p=dom(m["p"]), mu=dom(m["mu"]),
                    u=np.stack([dom(m["u"][d]) for d in range(self.L.D)]))

    def mass(self):
        return float(self.g.sum(axis=0)[self.zeta].sum())

    def source_sum(self):
        """sum over zeta = 1 nodes of 1.5 s(t) - 0.5 s(t-1) for the step just taken:
        by construction M(t+1) - M(t) equals minus this."""
        s, sb = self.last["s"], self.last["s_before"]
        return float((1.5 * s - 0.5 * sb)[self.zeta].sum())

    def domain(self, a):
        return self.grid.to_domain(a)
