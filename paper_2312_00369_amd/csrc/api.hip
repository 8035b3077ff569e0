// C interface: parameter checks, node classification, device memory layout,
// case lifetime, stepping (eager or HIP-graph replay), fields, diagnostics,
// checkpoints and kernel timing.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>

#include "case.h"

namespace pflbm {

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}
void clear_error() { g_last_error.clear(); }

static size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

dim3 default_tile(int D) { return D == 3 ? dim3(64, 2, 2) : dim3(64, 4, 1); }

// ------------------------------------------------------------------ parameters
int validate_and_derive(const pflbm_params* p, Derived* d) {
  if (!p) return set_error(PFLBM_EINVAL, "params is NULL");
  if (p->struct_size != sizeof(pflbm_params))
    return set_error(PFLBM_EINVAL, "struct_size %u != %zu", p->struct_size, sizeof(pflbm_params));
  if (p->lattice != PFLBM_D2Q9 && p->lattice != PFLBM_D3Q19 && p->lattice != PFLBM_D3Q19_D3Q7)
    return set_error(PFLBM_EUNSUPPORTED, "unknown lattice %d", p->lattice);
  if (p->storage < PFLBM_FP64 || p->storage > PFLBM_FP16_DEV)
    return set_error(PFLBM_EUNSUPPORTED, "unknown storage %d", p->storage);
  const int D = p->lattice == PFLBM_D2Q9 ? 2 : 3;
  if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0)
    return set_error(PFLBM_EINVAL, "grid dims must be positive (%d, %d, %d)", p->nx, p->ny, p->nz);
  if (D == 2 && p->nz != 1) return set_error(PFLBM_EINVAL, "D2Q9 needs nz = 1");
  const bool var = !(p->nu_l == 0.0 && p->nu_g == 0.0);
  if (!var && !(p->tau > 0.5)) return set_error(PFLBM_EINVAL, "tau must exceed 1/2 (got %g)", p->tau);
  if (var && !(p->nu_l > 0.0 && p->nu_g > 0.0))
    return set_error(PFLBM_EINVAL, "nu_l and nu_g must both be positive");
  const double tau_g = p->tau_phi > 0.0 ? p->tau_phi : p->tau;
  if (!(tau_g > 0.5)) return set_error(PFLBM_EINVAL, "tau_phi must exceed 1/2 (got %g)", tau_g);
  if (!(p->mobility > 0.0)) return set_error(PFLBM_EINVAL, "mobility must be positive");
  if (!(p->beta > 0.0) || !(p->kappa > 0.0))
    return set_error(PFLBM_EINVAL, "beta and kappa must be positive");
  if (!(p->rho_l > 0.0) || !(p->rho_g > 0.0))
    return set_error(PFLBM_EINVAL, "densities must be positive");
  if (!(p->theta_deg > 0.0 && p->theta_deg < 180.0))
    return set_error(PFLBM_EINVAL, "theta must lie in (0, 180) degrees (got %g)", p->theta_deg);
  if (p->wall_kind < 0 || p->wall_kind > 2) return set_error(PFLBM_EINVAL, "bad wall_kind");
  if (p->chi_case < 0 || p->chi_case > 3)
    return set_error(PFLBM_EINVAL, "chi_case must be 0..3 (got %d)", p->chi_case);

  d->D = D;
  d->Q = D == 2 ? 9 : 19;
  d->Qg = p->lattice == PFLBM_D3Q19_D3Q7 ? 7 : d->Q;   // populations of g
  Geo& G = d->geo;
  const int n[3] = {p->nx, p->ny, p->nz};
  int P[3];
  for (int a = 0; a < 3; ++a) {
    const bool per = (a >= D) ? true : p->periodic[a] != 0;
    G.per[a] = per ? 1 : 0;
    G.pad[a] = per ? 0 : 1;
    P[a] = n[a] + 2 * G.pad[a];
  }
  G.PX = P[0];
  G.PY = P[1];
  G.PZ = P[2];
  // rows of SX slots; on a walled x axis the first domain node starts a
  // population block (slot offset XO = 63), and the last row's padding node
  // spills into one extra block
  G.SX = (int)round_up((size_t)P[0], kBlk);
  G.XO = G.pad[0] ? kBlk - 1 : 0;
  d->N = (long long)G.SX * G.PY * G.PZ + G.XO;
  if (d->N >= (1LL << 31))
    return set_error(PFLBM_EUNSUPPORTED, "padded grid of %lld nodes exceeds 2^31", d->N);
  G.NQ = (long long)round_up((size_t)d->N, 256);

  Phys& ph = d->phys;
  // nu = c_s^2 (tau_f - 1/2) (Sec. 2.1.2); M = c_s^2 alpha (tau_g - 1/2) (Eq. mobility)
  ph.tau = p->tau;
  ph.inv_tau_g = 1.0 / tau_g;
  // c_s^2 of the velocity set of g: 1/3, or 1/4 for D3Q7 (Sec. 2.1.3)
  const double cs2_g = p->lattice == PFLBM_D3Q19_D3Q7 ? D3Q7::cs2 : kCs2;
  ph.alpha = p->mobility / (cs2_g * (tau_g - 0.5));
  ph.beta = p->beta;
  ph.kappa = p->kappa;
  // wall coefficient of Eq. (chemical_potencial2): sqrt(2 kappa beta) cos(theta)
  ph.wet = std::sqrt(2.0 * p->kappa * p->beta) * std::cos(p->theta_deg * M_PI / 180.0);
  // Appendix A: chi = c sqrt(2 beta/kappa) cos(theta) (phi - phi^2) in the ghost
  // rule, and the wall term of Eq. (chemical_potencial112) becomes (1 + c) wet
  {
    const double c = p->chi_case == 1 ? -1.0 : (p->chi_case == 3 ? 1.0 : 0.0);
    ph.chi_a = c * std::sqrt(2.0 * p->beta / p->kappa) * std::cos(p->theta_deg * M_PI / 180.0);
    ph.wet *= 1.0 + c;
  }
  ph.wet_tab = nullptr;     // set at create (device table of per-node wall coefficients)
  if (p->theta_map && (p->chi_case == 1 || p->chi_case == 3))
    return set_error(PFLBM_EUNSUPPORTED, "a per-node contact angle goes with chi case 2 only");
  ph.rho_l = p->rho_l;
  ph.rho_g = p->rho_g;
  ph.nu_l = p->nu_l;
  ph.nu_g = p->nu_g;
  ph.visc_var = var ? 1 : 0;
  // 3D step kernels: tile rows dealt to the XCDs in chunks (TileOrder mode 2),
  // which lets neighbouring tiles share an L2; 2D: round-robin
  ph.xcd_order = D == 3 ? 2 : 0;
  ph.nt_store = 0;
  for (int a = 0; a < 3; ++a) ph.Fb[a] = (a < D) ? p->body_force[a] : 0.0;
  // FP16 codec scales (powers of two): stored magnitudes of about 2^13 for the
  // largest populations expected from the parameters.
  {
    const double mu_scale = p->beta + 4.0 * p->kappa + std::fabs(ph.wet);
    const double g_est = ph.alpha * mu_scale;
    const double f_est = std::max(p->rho_l, p->rho_g) * 0.02 + 3.0 * mu_scale;
    ph.scale_g = (float)std::ldexp(1.0, (int)std::floor(std::log2(8192.0 / g_est)));
    ph.scale_f = (float)std::ldexp(1.0, (int)std::floor(std::log2(8192.0 / f_est)));
  }

  Wall& w = d->wall;
  w.kind = p->wall_kind;
  double nn = 0.0;
  for (int a = 0; a < 3; ++a) {
    w.p[a] = p->wall_point[a];
    w.nrm[a] = (a < D) ? p->wall_normal[a] : 0.0;
    nn += w.nrm[a] * w.nrm[a];
  }
  if (w.kind == PFLBM_WALL_PLANE) {
    if (!(nn > 0.0)) return set_error(PFLBM_EINVAL, "wall normal must be nonzero");
    for (int a = 0; a < 3; ++a) w.nrm[a] /= std::sqrt(nn);
  }
  if (D == 2) w.p[2] = 0.0;
  w.radius = p->wall_radius;
  w.width = p->diag_width;
  for (int a = 0; a < 3; ++a) w.ref[a] = (a < D) ? 0.5 * n[a] : 0.0;
  return PFLBM_OK;
}

Layout make_layout(const Derived& d, int storage, dim3 tile) {
  Layout L{};
  const size_t NQ = (size_t)d.geo.NQ;
  const size_t cb = storage == PFLBM_FP64 ? 8 : 4;
  L.c_bytes = NQ * cb;
  auto sizes = [&](auto qf, auto qg) {
    constexpr int Qf = decltype(qf)::value, Qg = decltype(qg)::value;
    if (storage == PFLBM_FP64) {
      L.f_bytes = Set<kF64, false, Qf>::bytes(NQ);
      L.g_bytes = Set<kF64, true, Qg>::bytes(NQ);
    } else if (storage == PFLBM_FP32) {
      L.f_bytes = Set<kF32, false, Qf>::bytes(NQ);
      L.g_bytes = Set<kF32, true, Qg>::bytes(NQ);
    } else {
      L.f_bytes = Set<kF16Dev, false, Qf>::bytes(NQ);
      L.g_bytes = Set<kF16Dev, true, Qg>::bytes(NQ);
    }
  };
  using I9 = std::integral_constant<int, 9>;
  using I19 = std::integral_constant<int, 19>;
  using I7 = std::integral_constant<int, 7>;
  if (d.Q == 9) sizes(I9(), I9());
  else if (d.Qg == 7) sizes(I19(), I7());
  else sizes(I19(), I19());
  const Geo& G = d.geo;
  L.nparts = (long long)((G.PX + G.XO + tile.x - 1) / tile.x) * ((G.PY + tile.y - 1) / tile.y) *
             ((G.PZ + tile.z - 1) / tile.z);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = round_up(off + bytes, 256);
    return o;
  };
  L.nodes = take(NQ * 4);
  L.f[0] = take(L.f_bytes);
  L.f[1] = take(L.f_bytes);
  L.g[0] = take(L.g_bytes);
  L.g[1] = take(L.g_bytes);
  L.s = take(L.c_bytes);
  L.phi = take(L.c_bytes);
  L.mu = take(L.c_bytes);
  L.snap = take(L.c_bytes);
  // partial records for the smallest tile the library accepts (64 threads)
  const size_t max_parts = (size_t)((G.PX + G.XO + 63) / 64) * G.PY * G.PZ;
  L.partial = take(max_parts * kRecN * sizeof(double));
  L.rec = take(kRecN * sizeof(double) * 2);
  L.popmax = take(2 * kPopmaxBlocks * sizeof(float));
  L.wet = take(kWetEntries * sizeof(double));
  L.gblocks = take((NQ / kBlk) * sizeof(uint32_t));
  L.total = off;
  return L;
}

// ------------------------------------------------------------------ classification
// Sec. 2.2.2 node marks.  The mask is the geometric solid.  A solid node with a
// lattice link to a non-solid node is a boundary node (zeta = 1, epsilon = 0);
// non-solid nodes are fluid (zeta = epsilon = 1); ghost nodes are zeta = 0 nodes
// one link from a zeta = 1 node.  Non-periodic axes get one padding layer of
// virtual solid (zeta = 0) nodes on each side.
template <class L>
static void classify_t(const Derived& d, const uint8_t* mask, std::vector<uint32_t>& words,
                       uint8_t* classes) {
  const Geo& G = d.geo;
  const int nx = G.PX - 2 * G.pad[0], ny = G.PY - 2 * G.pad[1], nz = G.PZ - 2 * G.pad[2];
  words.assign((size_t)d.N, 0u);
  auto at = [&](int x, int y, int z, int& ok) -> long long {
    const int P3[3] = {G.PX, G.PY, G.PZ};
    int q[3] = {x, y, z};
    ok = 1;
    for (int a = 0; a < 3; ++a) {
      if (G.per[a]) q[a] = ((q[a] % P3[a]) + P3[a]) % P3[a];
      else if (q[a] < 0 || q[a] >= P3[a]) ok = 0;
    }
    return ok ? G.idx(q[0], q[1], q[2]) : -1;
  };
  std::vector<uint8_t> fluid((size_t)d.N, 0), zeta((size_t)d.N, 0);
  auto inside = [&](int x, int y, int z) {
    const int X = x - G.pad[0], Y = y - G.pad[1], Z = z - G.pad[2];
    return X >= 0 && X < nx && Y >= 0 && Y < ny && Z >= 0 && Z < nz;
  };
  auto dom = [&](int x, int y, int z) {
    return (size_t)(x - G.pad[0]) + (size_t)nx * ((size_t)(y - G.pad[1]) + (size_t)ny * (z - G.pad[2]));
  };
  for (int z = 0; z < G.PZ; ++z)
    for (int y = 0; y < G.PY; ++y)
      for (int x = 0; x < G.PX; ++x)
        if (inside(x, y, z) && !mask[dom(x, y, z)]) fluid[G.idx(x, y, z)] = 1;
  for (int z = 0; z < G.PZ; ++z)
    for (int y = 0; y < G.PY; ++y)
      for (int x = 0; x < G.PX; ++x) {
        const long long n = G.idx(x, y, z);
        if (fluid[n]) { zeta[n] = 1; continue; }
        if (!inside(x, y, z)) continue;
        for (int i = 1; i < L::Q; ++i) {
          int ok;
          const long long m = at(x + L::cx(i), y + L::cy(i), z + L::cz(i), ok);
          if (ok && fluid[m]) { zeta[n] = 1; break; }
        }
      }
  for (int z = 0; z < G.PZ; ++z)
    for (int y = 0; y < G.PY; ++y)
      for (int x = 0; x < G.PX; ++x) {
        const long long n = G.idx(x, y, z);
        uint32_t w = 0;
        if (zeta[n]) {
          w |= kZeta;
          if (fluid[n]) w |= kFluid;
          for (int i = 1; i < L::Q; ++i) {
            int ok;
            const long long m = at(x - L::cx(i), y - L::cy(i), z - L::cz(i), ok);
            if (!ok || !zeta[m]) w |= 1u << (kLinkShift + i);
          }
        } else {
          for (int i = 1; i < L::Q; ++i) {
            int ok;
            const long long m = at(x + L::cx(i), y + L::cy(i), z + L::cz(i), ok);
            if (ok && zeta[m]) { w |= kGhost; break; }
          }
        }
        words[n] = w;
      }
  if (classes) {
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
          classes[(size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z)] =
              (uint8_t)(words[G.idx(x + G.pad[0], y + G.pad[1], z + G.pad[2])] & 7u);
  }
}

// The ghost rule of Appendix A cases 1 and 3 puts the ghost's mirror node one
// spacing away along the wall normal, which holds where every ghost node sees
// the zeta = 1 nodes of its 3^D block along one lattice axis (the sum of their
// offsets has one nonzero component).
int check_axis_ghosts(const Derived& d, const std::vector<uint32_t>& words) {
  const Geo& G = d.geo;
  const int P3[3] = {G.PX, G.PY, G.PZ};
  const int dz = d.D == 3 ? 1 : 0;
  for (int z = 0; z < G.PZ; ++z)
    for (int y = 0; y < G.PY; ++y)
      for (int x = 0; x < G.PX; ++x) {
        if (!(words[G.idx(x, y, z)] & kGhost)) continue;
        int s[3] = {0, 0, 0};
        for (int c = -dz; c <= dz; ++c)
          for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a) {
              int q[3] = {x + a, y + b, z + c}, ok = 1;
              for (int k = 0; k < 3; ++k) {
                if (G.per[k]) q[k] = ((q[k] % P3[k]) + P3[k]) % P3[k];
                else if (q[k] < 0 || q[k] >= P3[k]) ok = 0;
              }
              if (ok && (words[G.idx(q[0], q[1], q[2])] & kZeta)) {
                s[0] += a;
                s[1] += b;
                s[2] += c;
              }
            }
        if ((s[0] != 0) + (s[1] != 0) + (s[2] != 0) != 1)
          return set_error(PFLBM_EUNSUPPORTED,
                           "chi cases 1 and 3 need walls normal to a lattice axis; ghost "
                           "node (%d, %d, %d) is not", x, y, z);
      }
  return PFLBM_OK;
}

// Per-node contact angles (theta_map, degrees, read on mask nodes).  READING:
// the wall term of mu at a zeta = 1 node uses the mean cos(theta) over the
// epsilon = 0 nodes of its 3^D block, mask nodes with their own theta and
// virtual nodes with the case's.  The distinct coefficients sqrt(2 kappa beta)
// times that mean go into a table of kWetEntries (entry 0: the case's value);
// each node word carries its entry (wet_bits).
int wet_table(const Derived& d, const pflbm_params* p, const uint8_t* mask,
              std::vector<uint32_t>& words, std::vector<double>& tab) {
  tab.assign(kWetEntries, 0.0);
  tab[0] = d.phys.wet;
  if (!p->theta_map) return PFLBM_OK;
  const Geo& G = d.geo;
  const int nx = G.PX - 2 * G.pad[0], ny = G.PY - 2 * G.pad[1], nz = G.PZ - 2 * G.pad[2];
  const double cos0 = std::cos(p->theta_deg * M_PI / 180.0);
  std::vector<double> cosn((size_t)d.N, cos0);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t dom = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
        if (!mask[dom]) continue;
        const double th = p->theta_map[dom];
        if (!(th > 0.0 && th < 180.0))
          return set_error(PFLBM_EINVAL, "theta_map must lie in (0, 180) degrees on solid nodes "
                           "(got %g at node %zu)", th, dom);
        cosn[G.idx(x + G.pad[0], y + G.pad[1], z + G.pad[2])] = std::cos(th * M_PI / 180.0);
      }
  const double base = std::sqrt(2.0 * p->kappa * p->beta);
  const int P3[3] = {G.PX, G.PY, G.PZ};
  const int dz = d.D == 3 ? 1 : 0;
  int used = 1;
  for (int z = 0; z < G.PZ; ++z)
    for (int y = 0; y < G.PY; ++y)
      for (int x = 0; x < G.PX; ++x) {
        const long long n = G.idx(x, y, z);
        if (!(words[n] & kZeta)) continue;
        double sum = 0.0;
        int cnt = 0;
        for (int c = -dz; c <= dz; ++c)
          for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a) {
              int q[3] = {x + a, y + b, z + c}, ok = 1;
              for (int k = 0; k < 3; ++k) {
                if (G.per[k]) q[k] = ((q[k] % P3[k]) + P3[k]) % P3[k];
                else if (q[k] < 0 || q[k] >= P3[k]) ok = 0;
              }
              if (!ok) continue;
              const long long m = G.idx(q[0], q[1], q[2]);
              if (words[m] & kFluid) continue;
              sum += cosn[m];
              ++cnt;
            }
        if (!cnt) continue;
        const double w = base * (sum / cnt);
        if (w == tab[0]) continue;
        int k = 1;
        while (k < used && tab[k] != w) ++k;
        if (k == used) {
          if (used == kWetEntries)
            return set_error(PFLBM_EUNSUPPORTED, "theta_map gives more than %d distinct wall "
                             "coefficients", kWetEntries - 1);
          tab[used++] = w;
        }
        words[n] |= wet_bits((unsigned)k);
      }
  return PFLBM_OK;
}

void classify_nodes(const Derived& d, const uint8_t* mask, std::vector<uint32_t>& words,
                    uint8_t* classes) {
  if (d.D == 2) classify_t<D2Q9>(d, mask, words, classes);
  else classify_t<D3Q19>(d, mask, words, classes);
}

}  // namespace pflbm

using namespace pflbm;

// ------------------------------------------------------------------ helpers
namespace {

template <class C>
void depad(const pflbm_case_s* h, const C* src, double* dst) {
  const Geo& G = h->dv.geo;
  const int nx = h->prm.nx, ny = h->prm.ny, nz = h->prm.nz;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        dst[(size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z)] =
            (double)src[G.idx(x + G.pad[0], y + G.pad[1], z + G.pad[2])];
}

int upload_phi0(pflbm_case_s* h, const double* phi0, const std::vector<uint32_t>& words) {
  const Geo& G = h->dv.geo;
  const size_t N = (size_t)h->dv.N;
  const bool dbl = h->prm.storage == PFLBM_FP64;
  std::vector<double> vd;
  std::vector<float> vf;
  if (dbl) vd.assign(N, 0.0); else vf.assign(N, 0.0f);
  const int nx = h->prm.nx, ny = h->prm.ny, nz = h->prm.nz;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const long long n = G.idx(x + G.pad[0], y + G.pad[1], z + G.pad[2]);
        if (!(words[n] & kZeta)) continue;
        const double v = phi0[(size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z)];
        if (dbl) vd[n] = v; else vf[n] = (float)v;
      }
  PFLBM_HIP(hipMemcpyAsync(h->phi, dbl ? (const void*)vd.data() : (const void*)vf.data(),
                           N * (dbl ? 8 : 4), hipMemcpyHostToDevice, h->stream));
  PFLBM_HIP(hipStreamSynchronize(h->stream));
  return PFLBM_OK;
}

void drop_graph(pflbm_case_s* h) {
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
    h->gexec_steps = 0;
  }
}

int create_common(const pflbm_params* prm, const uint8_t* mask, const double* phi0,
                  void* stream, void* ws, size_t ws_bytes, pflbm_handle* out) {
  clear_error();
  if (!out) return set_error(PFLBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!mask || !phi0) return set_error(PFLBM_EINVAL, "solid_mask and phi0 are required");
  Derived dv;
  int rc = validate_and_derive(prm, &dv);
  if (rc) return rc;
  pflbm_case_s* h = new (std::nothrow) pflbm_case_s();
  if (!h) return set_error(PFLBM_ENOMEM, "host allocation failed");
  h->prm = *prm;
  h->dv = dv;
  h->tile = default_tile(dv.D);
  h->variant = dv.D == 2 ? 1 : 7;
  h->lay = make_layout(dv, prm->storage, h->tile);
  h->o32 = h->lay.f_bytes < (1ull << 32) && h->lay.g_bytes < (1ull << 32);
  auto fail = [&](int code) {
    pflbm_destroy(h);
    return code;
  };
  if (hipGetDevice(&h->device) != hipSuccess)
    return fail(set_error(PFLBM_EDEVICE, "no HIP device"));
  if (stream) {
    h->stream = static_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreate(&h->stream) != hipSuccess)
      return fail(set_error(PFLBM_EDEVICE, "hipStreamCreate failed"));
    h->own_stream = true;
  }
  if (ws) {
    if (ws_bytes < h->lay.total)
      return fail(set_error(PFLBM_EINVAL, "workspace of %zu bytes is smaller than the %zu needed",
                            ws_bytes, h->lay.total));
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
      return fail(set_error(PFLBM_EINVAL, "workspace must be 256-byte aligned"));
    h->base = static_cast<unsigned char*>(ws);
  } else {
    if (hipMalloc(&h->base, h->lay.total) != hipSuccess) {
      h->base = nullptr;
      (void)hipGetLastError();
      return fail(set_error(PFLBM_ENOMEM, "hipMalloc of %zu bytes failed", h->lay.total));
    }
    h->owns = true;
  }
  const Layout& L = h->lay;
  h->nodes = reinterpret_cast<uint32_t*>(h->base + L.nodes);
  for (int k = 0; k < 2; ++k) {
    h->f[k] = h->base + L.f[k];
    h->g[k] = h->base + L.g[k];
  }
  h->s = h->base + L.s;
  h->phi = h->base + L.phi;
  h->mu = h->base + L.mu;
  h->snap = h->base + L.snap;
  h->partial = reinterpret_cast<double*>(h->base + L.partial);
  h->rec = reinterpret_cast<double*>(h->base + L.rec);
  h->popmax = reinterpret_cast<float*>(h->base + L.popmax);
  h->gblocks = reinterpret_cast<uint32_t*>(h->base + L.gblocks);

  std::vector<uint32_t> words;
  h->classes.assign((size_t)prm->nx * prm->ny * prm->nz, 0);
  classify_nodes(dv, mask, words, h->classes.data());
  // blocks of 64 slots that hold a ghost node off the padding faces of a
  // walled x axis: the split step's ghost pass visits these, and the faces
  // (all of whose ghost nodes it visits directly)
  std::vector<uint32_t> gblocks;
  {
    const Geo& G = dv.geo;
    for (size_t b = 0; b * kBlk < words.size(); ++b) {
      bool any = false;
      for (size_t j = b * kBlk; j < std::min(words.size(), (b + 1) * kBlk); ++j) {
        if (!(words[j] & kGhost)) continue;
        h->nghost += 1;
        const long long x = ((long long)j - G.XO) % G.SX;
        any = any || G.per[0] || (x != 0 && x != G.PX - 1);
      }
      if (any) gblocks.push_back((uint32_t)b);
    }
  }
  h->nghost_blocks = (long long)gblocks.size();
  if (dv.phys.chi_a != 0.0 && (rc = check_axis_ghosts(dv, words))) return fail(rc);
  std::vector<double> wet;
  if ((rc = wet_table(dv, prm, mask, words, wet))) return fail(rc);
  h->dv.phys.wet_tab = reinterpret_cast<const double*>(h->base + L.wet);
  h->prm.theta_map = nullptr;   // the caller's array is read here only
#define CK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return fail(set_error(PFLBM_EDEVICE, "%s: %s", #x, hipGetErrorString(e_))); } while (0)
  CK(hipMemsetAsync(h->base, 0, L.total, h->stream));
  CK(hipMemcpyAsync(h->nodes, words.data(), words.size() * 4, hipMemcpyHostToDevice, h->stream));
  if (!gblocks.empty())
    CK(hipMemcpyAsync(h->gblocks, gblocks.data(), gblocks.size() * 4, hipMemcpyHostToDevice,
                      h->stream));
  CK(hipMemcpyAsync(h->base + L.wet, wet.data(), wet.size() * sizeof(double),
                    hipMemcpyHostToDevice, h->stream));
  if ((rc = upload_phi0(h, phi0, words))) return fail(rc);
  // mu(phi0) with ghosts, g = g_eq(phi0, mu0) placed for the first pull, f = 0.
  if ((rc = run_mu(h))) return fail(rc);
  if ((rc = run_init_g(h))) return fail(rc);
  // phi(0) = sum g and mu(0) exactly as a step forms them, then s(0) for the
  // time-derivative term of the first step (s(-1) := s(0)).
  if ((rc = run_phi(h))) return fail(rc);
  if ((rc = run_mu(h))) return fail(rc);
  if ((rc = run_collide(h, 2, nullptr, nullptr))) return fail(rc);
  CK(hipStreamSynchronize(h->stream));
#undef CK
  *out = h;
  return PFLBM_OK;
}

int check_handle(pflbm_handle h) {
  if (!h) return set_error(PFLBM_EINVAL, "handle is NULL");
  return PFLBM_OK;
}

}  // namespace

namespace pflbm {
int fp16_upkeep(pflbm_case_s* h, int* changed) {
  if (changed) *changed = 0;
  if (h->prm.storage != PFLBM_FP16_DEV) return PFLBM_OK;
  float m[2];
  int rc = run_popmax(h, m);
  if (rc) return rc;
  float* scale[2] = {&h->dv.phys.scale_f, &h->dv.phys.scale_g};
  bool moved = false;
  for (int k = 0; k < 2; ++k) {
    // keep the largest stored magnitude in [2^11, 2^14] (the FP16 maximum is
    // 65504); an all-zero set or a non-finite value (flagged by the
    // diagnostics record) leaves the scale alone
    if (!(m[k] > 0.0f) || !std::isfinite(m[k])) continue;
    if (m[k] >= 2048.0f && m[k] <= 16384.0f) continue;
    int e = (int)std::floor(std::log2(8192.0 / (double)m[k]));
    // the scale stays within [2^-60, 2^60], the range pflbm_set_fp16_scales accepts
    const int e_now = std::ilogb(*scale[k]);
    e = std::max(-60 - e_now, std::min(60 - e_now, e));
    if (e == 0) continue;
    const float factor = std::ldexp(1.0f, e);
    if ((rc = run_rescale(h, k, factor))) return rc;
    *scale[k] *= factor;
    moved = true;
  }
  if (moved) {
    drop_graph(h);
    if (changed) *changed = 1;
  }
  return PFLBM_OK;
}
}  // namespace pflbm

extern "C" {

const char* pflbm_strerror(int code) {
  switch (code) {
    case PFLBM_OK: return "ok";
    case PFLBM_EINVAL: return "invalid argument";
    case PFLBM_ENOMEM: return "out of memory";
    case PFLBM_EDEVICE: return "device error";
    case PFLBM_ENONFINITE: return "non-finite values";
    case PFLBM_ESTATE: return "invalid state";
    case PFLBM_EUNSUPPORTED: return "unsupported";
    default: return "unknown error";
  }
}

const char* pflbm_last_error(void) { return g_last_error.c_str(); }

int pflbm_footprint(const pflbm_params* prm, size_t* bytes) {
  clear_error();
  if (!bytes) return set_error(PFLBM_EINVAL, "bytes is NULL");
  Derived dv;
  int rc = validate_and_derive(prm, &dv);
  if (rc) return rc;
  *bytes = make_layout(dv, prm->storage, default_tile(dv.D)).total;
  return PFLBM_OK;
}

int pflbm_classify(const pflbm_params* prm, const uint8_t* mask, uint8_t* classes) {
  clear_error();
  if (!mask || !classes) return set_error(PFLBM_EINVAL, "mask and classes are required");
  Derived dv;
  int rc = validate_and_derive(prm, &dv);
  if (rc) return rc;
  std::vector<uint32_t> words;
  classify_nodes(dv, mask, words, classes);
  return PFLBM_OK;
}

// Free-energy coefficients from surface tension and interface width: the
// double well beta phi^2 (1 - phi)^2 with gradient energy kappa/2 |grad phi|^2
// has the planar profile 1/2 + 1/2 tanh(2 x / W) with W = sqrt(8 kappa / beta)
// (Eq. initialphi) and tension sigma = sqrt(2 kappa beta) / 6; solved for the
// coefficients, beta = 12 sigma / W and kappa = 3 sigma W / 2.
int pflbm_beta_kappa(double sigma, double width, double* beta, double* kappa) {
  clear_error();
  if (!beta || !kappa) return set_error(PFLBM_EINVAL, "beta and kappa are required");
  if (!(sigma > 0.0) || !(width > 0.0) || !std::isfinite(sigma) || !std::isfinite(width))
    return set_error(PFLBM_EINVAL, "sigma and width must be finite and positive (got %g, %g)",
                     sigma, width);
  *beta = 12.0 * sigma / width;
  *kappa = 1.5 * sigma * width;
  return PFLBM_OK;
}

int pflbm_lattice_table(int32_t lattice, int32_t* c, double* w, int32_t* opp, double* k) {
  clear_error();
  if (lattice != PFLBM_D2Q9 && lattice != PFLBM_D3Q19 && lattice != PFLBM_D3Q19_D3Q7 &&
      lattice != PFLBM_D3Q7)
    return set_error(PFLBM_EUNSUPPORTED, "unknown lattice %d", lattice);
  auto fill = [&](auto L) {
    using LT = decltype(L);
    for (int i = 0; i < LT::Q; ++i) {
      if (c) { c[3 * i] = LT::cx(i); c[3 * i + 1] = LT::cy(i); c[3 * i + 2] = LT::cz(i); }
      if (w) w[i] = LT::w(i);
      if (opp) opp[i] = LT::opp(i);
      if (k) k[i] = LT::k(i);
    }
    return LT::Q;
  };
  if (lattice == PFLBM_D2Q9) return fill(D2Q9{});
  if (lattice == PFLBM_D3Q7) return fill(D3Q7{});
  return fill(D3Q19{});     // PFLBM_D3Q19, and the hydrodynamic set of PFLBM_D3Q19_D3Q7
}

int pflbm_create(const pflbm_params* prm, const uint8_t* mask, const double* phi0, void* stream,
                 pflbm_handle* out) {
  return create_common(prm, mask, phi0, stream, nullptr, 0, out);
}

int pflbm_create_in(const pflbm_params* prm, const uint8_t* mask, const double* phi0,
                    void* stream, void* ws, size_t ws_bytes, pflbm_handle* out) {
  if (!ws) return set_error(PFLBM_EINVAL, "workspace is NULL");
  return create_common(prm, mask, phi0, stream, ws, ws_bytes, out);
}

void pflbm_group_forget(pflbm_handle h);  // group.hip

void pflbm_destroy(pflbm_handle h) {
  if (!h) return;
  if (h->group) pflbm_group_forget(h);
  drop_graph(h);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->owns && h->base) (void)hipFree(h->base);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

int64_t pflbm_step_count(pflbm_handle h) { return h ? h->step : -1; }

int pflbm_set_graph_chunk(pflbm_handle h, int32_t steps) {
  clear_error();
  if (int rc = check_handle(h)) return rc;
  if (steps < 0) return set_error(PFLBM_EINVAL, "chunk must be >= 0");
  if (steps & 1) steps += 1;   // even, so a replay leaves the buffer parity unchanged
  if (steps != h->graph_chunk) drop_graph(h);
  h->graph_chunk = steps;
  return PFLBM_OK;
}

int pflbm_set_tile(pflbm_handle h, int32_t tx, int32_t ty, int32_t tz) {
  clear_error();
  if (int rc = check_handle(h)) return rc;
  if (tx <= 0 || ty <= 0 || tz <= 0 || tx % 64 != 0 || tx * ty * tz > 1024)
    return set_error(PFLBM_EINVAL, "tile (%d,%d,%d): tx must be a multiple of 64, product <= 1024",
                     tx, ty, tz);
  if (h->dv.D == 2 && tz != 1) return set_error(PFLBM_EINVAL, "2D tiles need tz = 1");
  drop_graph(h);
  h->tile = dim3(tx, ty, tz);
  return PFLBM_OK;
}

int pflbm_step(pflbm_handle h, int64_t nsteps) {
  clear_error();
  if (int rc = check_handle(h)) return rc;
  if (nsteps < 0) return set_error(PFLBM_EINVAL, "nsteps must be >= 0");
  if (h->group) return set_error(PFLBM_ESTATE, "case is a group member; step the group");
  int rc;
  const int K = h->graph_chunk;
  if (K > 0 && nsteps >= K) {
    if (h->cur != 0) {           // graphs are captured from parity 0
      if ((rc = run_step_eager(h))) return rc;
      --nsteps;
    }
    if (!h->gexec || h->gexec_steps != K) {
      drop_graph(h);
      hipGraph_t graph = nullptr;
      PFLBM_HIP(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
      const int64_t step0 = h->step;
      for (int k = 0; k < K; ++k) {
        if ((rc = run_step_eager(h))) {
          (void)hipStreamEndCapture(h->stream, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          h->step = step0;
          h->cur = 0;
          return rc;
        }
      }
      h->step = step0;           // capture only recorded the work
      PFLBM_HIP(hipStreamEndCapture(h->stream, &graph));
      hipError_t e = hipGraphInstantiateWithFlags(&h->gexec, graph, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) {
        h->gexec = nullptr;
        return set_error(PFLBM_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
      }
      h->gexec_steps = K;
    }
    while (nsteps >= K) {
      PFLBM_HIP(hipGraphLaunch(h->gexec, h->stream));
      h->step += K;
      nsteps -= K;
    }
  }
  for (int64_t k = 0; k < nsteps; ++k)
    if ((rc = run_step_eager(h))) return rc;
  return PFLBM_OK;
}

int pflbm_fields(pflbm_handle h, double* phi, double* p, double* u, double* mu) {
  clear_error();
  if (int rc = check_handle(h)) return rc;
  int rc;
  // phi(t) and mu(t) with ghosts, then p and u into the idle f buffer.
  if ((rc = run_phi(h))) return rc;
  if ((rc = run_mu(h))) return rc;
  const int D = h->dv.D;
  const size_t cb = h->prm.storage == PFLBM_FP64 ? 8 : 4;
  const size_t NQ = (size_t)h->dv.geo.NQ;
  unsigned char* scratch = static_cast<unsigned char*>(h->f[1 - h->cur]);
  if (p || u) {
    PFLBM_HIP(hipMemsetAsync(scratch, 0, (1 + D) * NQ * cb, h->stream));
    if ((rc = run_collide(h, 1, scratch, scratch + NQ * cb))) return rc;
  }
  std::vector<unsigned char> buf(NQ * cb);
  auto fetch = [&](const void* dev, double* dst) -> int {
    PFLBM_HIP(hipMemcpyAsync(buf.data(), dev, NQ * cb, hipMemcpyDeviceToHost, h->stream));
    PFLBM_HIP(hipStreamSynchronize(h->stream));
    if (cb == 8) depad(h, reinterpret_cast<const double*>(buf.data()), dst);
    else depad(h, reinterpret_cast<const float*>(buf.data()), dst);
    return PFLBM_OK;
  };
  const size_t ncell = (size_t)h->prm.nx * h->prm.ny * h->prm.nz;
  if (phi && (rc = fetch(h->phi, phi))) return rc;
  if (mu && (rc = fetch(h->mu, mu))) return rc;
  if (p && (rc = fetch(scratch, p))) return rc;
  if (u)
    for (int d = 0; d < D; ++d)
      if ((rc = fetch(scratch + (1 + d) * NQ * cb, u + d * ncell))) return rc;
  // zero ghost/solid entries of mu, p and u (phi keeps ghost values)
  for (size_t n = 0; n < ncell; ++n) {
    if (h->classes[n] & kZeta) continue;
    if (mu) mu[n] = 0.0;
    if (p) p[n] = 0.0;
    if (u) for (int d = 0; d < D; ++d) u[d * ncell + n] = 0.0;
    if (phi && !(h->classes[n] & kGhost)) phi[n] = 0.0;
  }
  return PFLBM_OK;
}

int pflbm_node_classes(pflbm_handle h, uint8_t* classes) {
  clear_error();
  if (int rc = check_handle(h)) return rc;
  if (!classes) return set_error(PFLBM_EINVAL, "classes is NULL");
  std::memcpy(classes, h->classes.data(), h->classes.size());
  return PFLBM_OK;
}

}  // extern "C"

// Kasa circle / sphere fit from the moment record, then the contact angle.
void pflbm::finish_diag(const pflbm_case_s* h, const double* r, pflbm_diag* d) {
  std::memset(d, 0, sizeof *d);
  d->step = h->step;
  d->mass = r[kRecMass];
  d->s_sum = r[kRecS];
  d->steady_residual = h->snap_valid ? r[kRecResid] : INFINITY;
  d->nonfinite = r[kRecNonfinite] > 0.0 ? 1 : 0;
  d->n_points = (int64_t)r[kRecCount];
  d->steady = (h->snap_valid && !d->nonfinite && d->steady_residual <= h->prm.steady_tol) ? 1 : 0;
  d->theta_deg = NAN;
  d->radius = NAN;
  const int D = h->dv.D;
  const double n = r[kRecCount];
  if (h->dv.wall.kind == PFLBM_WALL_NONE || n < 2 * D + 2) return;
  // normal equations of min sum (|X|^2 + a.X + b)^2 over the points
  double A[4][5] = {};
  const double S1[3] = {r[kRecX], r[kRecY], r[kRecZ]};
  const double S2[3][3] = {{r[kRecXX], r[kRecXY], r[kRecXZ]},
                           {r[kRecXY], r[kRecYY], r[kRecYZ]},
                           {r[kRecXZ], r[kRecYZ], r[kRecZZ]}};
  const double SR[3] = {r[kRecXR], r[kRecYR], r[kRecZR]};
  const int M = D + 1;
  for (int i = 0; i < D; ++i) {
    for (int j = 0; j < D; ++j) A[i][j] = S2[i][j];
    A[i][D] = S1[i];
    A[i][M] = -SR[i];
  }
  for (int j = 0; j < D; ++j) A[D][j] = S1[j];
  A[D][D] = n;
  A[D][M] = -r[kRecRR];
  for (int c = 0; c < M; ++c) {           // Gaussian elimination, partial pivoting
    int piv = c;
    for (int i = c + 1; i < M; ++i)
      if (std::fabs(A[i][c]) > std::fabs(A[piv][c])) piv = i;
    if (A[piv][c] == 0.0) return;
    if (piv != c)
      for (int j = 0; j <= M; ++j) std::swap(A[c][j], A[piv][j]);
    for (int i = 0; i < M; ++i) {
      if (i == c) continue;
      const double f = A[i][c] / A[c][c];
      for (int j = c; j <= M; ++j) A[i][j] -= f * A[c][j];
    }
  }
  double sol[4];
  for (int i = 0; i < M; ++i) sol[i] = A[i][M] / A[i][i];
  double cen[3] = {0, 0, 0}, cc = 0.0;
  for (int i = 0; i < D; ++i) {
    cen[i] = -0.5 * sol[i];
    cc += cen[i] * cen[i];
  }
  const double R2 = cc - sol[D];
  if (!(R2 > 0.0)) return;
  const double R = std::sqrt(R2);
  const Wall& W = h->dv.wall;
  for (int i = 0; i < 3; ++i) d->centre[i] = (i < D) ? cen[i] + W.ref[i] : 0.0;
  d->radius = R;
  double cost;
  if (W.kind == PFLBM_WALL_PLANE) {
    double hgt = 0.0;
    for (int i = 0; i < D; ++i) hgt += (d->centre[i] - W.p[i]) * W.nrm[i];
    cost = -hgt / R;
  } else {
    double dd = 0.0;
    for (int i = 0; i < D; ++i) dd += (d->centre[i] - W.p[i]) * (d->centre[i] - W.p[i]);
    cost = (R2 + W.radius * W.radius - dd) / (2.0 * R * W.radius);
  }
  cost = std::fmin(1.0, std::fmax(-1.0, cost));
  d->theta_deg = std::acos(cost) * 180.0 / M_PI;
}

extern "C" {

int pflbm_diagnostics(pflbm_handle h, pflbm_diag* d) {
  clear_error();
  if (int rc = check_handle(h)) return rc;
  if (!d) return set_error(PFLBM_EINVAL, "diag is NULL");
  int rc;
  if ((rc = run_phi(h))) return rc;
  double rec[kRecN];
  if ((rc = run_reduce(h, 1, rec))) return rc;
  finish_diag(h, rec, d);
  h->snap_valid = true;
  if (!h->group && (rc = fp16_upkeep(h, nullptr))) return rc;
  return PFLBM_OK;
}


int pflbm_fp16_scales(pflbm_handle h, double* scale_f, double* scale_g) {
  clear_error();
  if (int rc = check_handle(h)) return rc;
  const bool half = h->prm.storage == PFLBM_FP16_DEV;
  if (scale_f) *scale_f = half ? h->dv.phys.scale_f : 1.0;
  if (scale_g) *scale_g = half ? h->dv.phys.scale_g : 1.0;
  return PFLBM_OK;
}

int pflbm_set_fp16_scales(pflbm_handle h, double scale_f, double scale_g) {
  clear_error();
  if (int rc = check_handle(h)) return rc;
  if (h->prm.storage != PFLBM_FP16_DEV)
    return set_error(PFLBM_EUNSUPPORTED, "scales exist for FP16-deviation storage only");
  if (h->group) return set_error(PFLBM_ESTATE, "case is a group member");
  const double want[2] = {scale_f, scale_g};
  for (int k = 0; k < 2; ++k) {
    int e;
    if (!(want[k] > 0.0) || !std::isfinite(want[k]) || std::frexp(want[k], &e) != 0.5 ||
        e < -60 || e > 60)
      return set_error(PFLBM_EINVAL, "scales must be powers of two (got %g)", want[k]);
  }
  float* scale[2] = {&h->dv.phys.scale_f, &h->dv.phys.scale_g};
  for (int k = 0; k < 2; ++k) {
    const double factor = want[k] / (double)*scale[k];
    if (factor == 1.0) continue;
    int rc = run_rescale(h, k, (float)factor);
    if (rc) return rc;
    *scale[k] = (float)want[k];
  }
  PFLBM_HIP(hipStreamSynchronize(h->stream));
  drop_graph(h);
  return PFLBM_OK;
}

namespace {
// Checkpoint blob: a kStateHeader-byte header, then the current f buffer, the
// current g buffer and s.  FP16-deviation buffers hold value * scale, so the
// header carries the scales they were written with.
constexpr size_t kStateHeader = 128;
struct StateHeader {
  char magic[8];
  uint64_t f_bytes, g_bytes, c_bytes;
  int64_t step;
  int32_t lattice, storage, nx, ny, nz, pad_;
  double scale_f, scale_g;     // FP16-deviation scales of the stored buffers (1 otherwise)
};
static_assert(sizeof(StateHeader) <= kStateHeader, "state header");
}  // namespace

int pflbm_state_size(pflbm_handle h, size_t* bytes) {
  clear_error();
  if (int rc = check_handle(h)) return rc;
  if (!bytes) return set_error(PFLBM_EINVAL, "bytes is NULL");
  *bytes = kStateHeader + h->lay.f_bytes + h->lay.g_bytes + h->lay.c_bytes;
  return PFLBM_OK;
}

int pflbm_get_state(pflbm_handle h, void* host, size_t bytes) {
  clear_error();
  if (int rc = check_handle(h)) return rc;
  size_t need;
  pflbm_state_size(h, &need);
  if (!host || bytes < need) return set_error(PFLBM_EINVAL, "state buffer too small (%zu < %zu)", bytes, need);
  StateHeader hd{};
  std::memcpy(hd.magic, "PFLBMST3", 8);
  hd.f_bytes = h->lay.f_bytes;
  hd.g_bytes = h->lay.g_bytes;
  hd.c_bytes = h->lay.c_bytes;
  hd.step = h->step;
  hd.lattice = h->prm.lattice;
  hd.storage = h->prm.storage;
  hd.nx = h->prm.nx; hd.ny = h->prm.ny; hd.nz = h->prm.nz;
  const bool half = h->prm.storage == PFLBM_FP16_DEV;
  hd.scale_f = half ? (double)h->dv.phys.scale_f : 1.0;
  hd.scale_g = half ? (double)h->dv.phys.scale_g : 1.0;
  unsigned char* p = static_cast<unsigned char*>(host);
  std::memset(p, 0, kStateHeader);
  std::memcpy(p, &hd, sizeof hd);
  p += kStateHeader;
  PFLBM_HIP(hipMemcpyAsync(p, h->f[h->cur], h->lay.f_bytes, hipMemcpyDeviceToHost, h->stream));
  PFLBM_HIP(hipMemcpyAsync(p + h->lay.f_bytes, h->g[h->cur], h->lay.g_bytes,
                           hipMemcpyDeviceToHost, h->stream));
  PFLBM_HIP(hipMemcpyAsync(p + h->lay.f_bytes + h->lay.g_bytes, h->s, h->lay.c_bytes,
                           hipMemcpyDeviceToHost, h->stream));
  PFLBM_HIP(hipStreamSynchronize(h->stream));
  return PFLBM_OK;
}

int pflbm_set_state(pflbm_handle h, const void* host, size_t bytes) {
  clear_error();
  if (int rc = check_handle(h)) return rc;
  size_t need;
  pflbm_state_size(h, &need);
  if (!host || bytes < need) return set_error(PFLBM_EINVAL, "state buffer too small (%zu < %zu)", bytes, need);
  StateHeader hd;
  std::memcpy(&hd, host, sizeof hd);
  if (std::memcmp(hd.magic, "PFLBMST3", 8) != 0 || hd.f_bytes != h->lay.f_bytes ||
      hd.g_bytes != h->lay.g_bytes ||
      hd.c_bytes != h->lay.c_bytes || hd.lattice != h->prm.lattice ||
      hd.storage != h->prm.storage || hd.nx != h->prm.nx || hd.ny != h->prm.ny || hd.nz != h->prm.nz)
    return set_error(PFLBM_EINVAL, "state blob does not match this case");
  const bool half = h->prm.storage == PFLBM_FP16_DEV;
  if (half) {
    for (double v : {hd.scale_f, hd.scale_g}) {
      int e;
      if (!(v > 0.0) || !std::isfinite(v) || std::frexp(v, &e) != 0.5 || e < -60 || e > 60)
        return set_error(PFLBM_EINVAL, "state blob holds an invalid FP16 scale (%g)", v);
    }
  }
  const unsigned char* p = static_cast<const unsigned char*>(host) + kStateHeader;
  PFLBM_HIP(hipMemcpyAsync(h->f[h->cur], p, h->lay.f_bytes, hipMemcpyHostToDevice, h->stream));
  PFLBM_HIP(hipMemcpyAsync(h->g[h->cur], p + h->lay.f_bytes, h->lay.g_bytes,
                           hipMemcpyHostToDevice, h->stream));
  PFLBM_HIP(hipMemcpyAsync(h->s, p + h->lay.f_bytes + h->lay.g_bytes, h->lay.c_bytes,
                           hipMemcpyHostToDevice, h->stream));
  PFLBM_HIP(hipStreamSynchronize(h->stream));
  h->step = hd.step;
  h->snap_valid = false;
  if (half && ((float)hd.scale_f != h->dv.phys.scale_f || (float)hd.scale_g != h->dv.phys.scale_g)) {
    // the buffers now hold values at the blob's scales; captured graphs (and a
    // group's member descriptors) carry the old ones
    h->dv.phys.scale_f = (float)hd.scale_f;
    h->dv.phys.scale_g = (float)hd.scale_g;
    drop_graph(h);
  }
  group_member_changed(h);
  return PFLBM_OK;
}

int pflbm_profile(pflbm_handle h, int64_t nsteps, double* avg_ms, int32_t nkinds) {
  clear_error();
  if (int rc = check_handle(h)) return rc;
  if (nsteps <= 0 || nsteps > 100000 || !avg_ms || nkinds <= 0)
    return set_error(PFLBM_EINVAL, "bad profile arguments");
  if (h->group) return set_error(PFLBM_ESTATE, "case is a group member");
  // kinds: 0 k_phi, 1 k_mu, 2 k_collide (three-kernel path), 3 k_step (fused)
  constexpr int K = 4;
  const bool fused = h->variant >= 0;
  const int per = fused ? 1 : 3;
  const int64_t chunk = std::min<int64_t>(nsteps, 256);
  std::vector<hipEvent_t> ev((size_t)chunk * per * 2, nullptr);
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto& x : ev) if (x) (void)hipEventDestroy(x);
      return set_error(PFLBM_EDEVICE, "hipEventCreate failed");
    }
  double tot[K] = {0, 0, 0, 0};
  int rc = PFLBM_OK;
  for (int64_t done = 0; done < nsteps && rc == PFLBM_OK;) {
    const int64_t n = std::min<int64_t>(chunk, nsteps - done);
    for (int64_t s = 0; s < n && rc == PFLBM_OK; ++s) {
      hipEvent_t* e = &ev[(size_t)s * per * 2];
      if (fused) {
        (void)hipEventRecord(e[0], h->stream);
        rc = run_step_fused(h);
        (void)hipEventRecord(e[1], h->stream);
      } else {
        (void)hipEventRecord(e[0], h->stream);
        if (!(rc = run_phi(h))) {
          (void)hipEventRecord(e[1], h->stream);
          (void)hipEventRecord(e[2], h->stream);
          if (!(rc = run_mu(h))) {
            (void)hipEventRecord(e[3], h->stream);
            (void)hipEventRecord(e[4], h->stream);
            rc = run_collide(h, 0, nullptr, nullptr);
            (void)hipEventRecord(e[5], h->stream);
          }
        }
      }
      if (rc) break;
      h->cur ^= 1;
      h->step += 1;
    }
    if (rc) break;
    if (hipStreamSynchronize(h->stream) != hipSuccess) { rc = set_error(PFLBM_EDEVICE, "sync"); break; }
    for (int64_t s = 0; s < n; ++s)
      for (int k = 0; k < per; ++k) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[(size_t)(s * per + k) * 2], ev[(size_t)(s * per + k) * 2 + 1]);
        tot[fused ? 3 : k] += ms;
      }
    done += n;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (rc) return rc;
  for (int k = 0; k < nkinds; ++k) avg_ms[k] = k < K ? tot[k] / (double)nsteps : 0.0;
  return PFLBM_OK;
}

int pflbm_set_step_kernel(pflbm_handle h, int32_t variant) {
  clear_error();
  if (int rc = check_handle(h)) return rc;
  if (variant < -1 || variant >= step_variant_count(h->dv.D))
    return set_error(PFLBM_EINVAL, "step kernel variant %d outside [-1, %d)", variant,
                     step_variant_count(h->dv.D));
  drop_graph(h);
  h->variant = variant;
  return PFLBM_OK;
}

int pflbm_set_step_options(pflbm_handle h, int32_t xcd_order, int32_t nontemporal) {
  clear_error();
  if (int rc = check_handle(h)) return rc;
  drop_graph(h);
  if (xcd_order < 0 || xcd_order > 2)
    return set_error(PFLBM_EINVAL, "xcd_order must be 0, 1 or 2 (got %d)", xcd_order);
  h->dv.phys.xcd_order = xcd_order;
  h->dv.phys.nt_store = nontemporal ? 1 : 0;
  return PFLBM_OK;
}

int pflbm_step_variants(int32_t lattice, int32_t* tiles, int32_t capacity) {
  clear_error();
  if (lattice != PFLBM_D2Q9 && lattice != PFLBM_D3Q19 && lattice != PFLBM_D3Q19_D3Q7)
    return set_error(PFLBM_EUNSUPPORTED, "unknown lattice %d", lattice);
  const int D = lattice == PFLBM_D2Q9 ? 2 : 3;
  const int count = step_variant_count(D);
  for (int v = 0; v < count && v < capacity && tiles; ++v) {
    int t[5];
    step_variant_tile(D, v, t);
    for (int k = 0; k < 5; ++k) tiles[5 * v + k] = t[k];
  }
  return count;
}

}  // extern "C"
