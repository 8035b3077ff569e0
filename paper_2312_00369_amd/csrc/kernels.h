// Device kernels of one time step (templated on lattice and storage).
//
// State kept between steps: post-collision populations f*, g* (ping-pong
// buffers in 64-node blocks, see Set) and s = u . grad(phi) of the previous
// step (one array).  One step is
//   k_phi      phi(x) = sum_i g_i(x), with g_i pulled from x - c_i     Eq. (order-parameter)
//   k_mu       LDS tile with a two-node halo: ghost phi (Sec. 2.2.2), the isotropic
//              Laplacian (Eq. Laplace), a_v = |grad eps| (Eq. avvv) and
//              mu (Eq. chemical_potencial2); writes mu and the ghost phi values
//   k_collide  pulls f and g, forms grad phi (Eq. gradient), rho, F = mu grad phi + F_b,
//              u, p (Sec. 2.1.2), s, and collides both sets: Eq. (BGK-NS) with
//              f_eq of Eq. (feq_i) and F_i of Eq. (GGi); Eq. (BGK) with g_eq of
//              Eq. (H_i) and G_i of Eq. (F_i) plus half its time derivative
// Pulling f_i at x from a zeta = 0 node x - c_i takes f*_opp(i) of x itself
// (bounce-back half-way along the link, Sec. 2.2.2).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lattice.h"

namespace pflbm {

enum Storage { kF64 = 0, kF32 = 1, kF16Dev = 2 };

// ------------------------------------------------------------------ geometry
// Node index within one case (the padded grid has fewer than 2^31 nodes).
using nidx = uint32_t;

// Node (x, y, z) of the padded grid sits in slot x + XO + SX (y + PY z).  On a
// walled x axis XO = 63: the first domain node x = 1 then starts a 64-node
// block, so a row of 64 k domain nodes fills k whole blocks and the two padding
// nodes of consecutive rows share the block between them.  Without the offset
// a 256-node row would spill one node into a fifth block, and every fifth
// wavefront of a step would move whole cache lines for that one node.
struct Geo {
  int PX, PY, PZ;    // padded extents: periodic axes as given, others + 2
  int SX;            // row stride in slots (>= PX, a multiple of 64)
  int per[3];        // periodic flags
  int pad[3];        // 0 periodic, 1 otherwise: domain x = padded x - pad
  int XO;            // slot of x = 0 within its row: 63 on a walled x axis, else 0
  long long NQ;      // node slots (>= SX*PY*PZ + XO, a multiple of 256); stride of u components
  __host__ __device__ nidx idx(int x, int y, int z) const {
    return (nidx)(x + XO) + (nidx)SX * ((nidx)y + (nidx)PY * (nidx)z);
  }
};

// Tiles of TX x TY x TZ nodes; tile b has indices (b % nx, (b / nx) % ny,
// b / (nx ny)).  Along x the tiles start at the first domain node (the
// padding layers of a walled axis hold no fluid or boundary node), so with
// XO = 63 a 64-wide tile row is exactly one population block.  Along y and z
// they start at the padding layer: the tile rows next to the walls then hold
// fewer nodes, and on a small grid, where one round of workgroups makes up
// the launch and its slowest tile sets the time, those wall tiles (which
// also form ghost means) are not the largest.
struct TileGrid {
  int nx, ny, nz, ox, oy, oz, tx, ty, tz;
  __host__ __device__ TileGrid(const Geo& G, int TX, int TY, int TZ)
      : nx((G.PX - 2 * G.pad[0] + TX - 1) / TX), ny((G.PY + TY - 1) / TY),
        nz((G.PZ + TZ - 1) / TZ), ox(G.pad[0]), oy(0), oz(0), tx(TX), ty(TY), tz(TZ) {}
  __host__ __device__ int count() const { return nx * ny * nz; }
  __host__ __device__ void origin(int b, int& x0, int& y0, int& z0) const {
    x0 = ox + (b % nx) * tx;
    y0 = oy + ((b / nx) % ny) * ty;
    z0 = oz + (b / (nx * ny)) * tz;
  }
};

struct Phys {
  double tau, inv_tau_g, alpha, beta, kappa, wet, rho_l, rho_g, nu_l, nu_g;
  double chi_a;            // chi(phi) = chi_a (phi - phi^2) of the ghost rule; 0 = mean only
  const double* wet_tab;   // device table of wall coefficients for per-node contact angles
  double Fb[3];
  int visc_var;
  float scale_f, scale_g;  // FP16 codec: stored = value * scale (power of two)
  int xcd_order;           // step kernels: dispatch order over the XCDs (TileOrder mode)
  int nt_store;            // fused step: non-temporal stores of f*, g*
};

// Streaming store that does not keep the line in the caches (or a plain store).
template <class T>
__device__ inline void st(T* p, T v, int nt) {
  if (nt) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// ------------------------------------------------------------------ storage codec
// One distribution set (f or g) of Q populations in one buffer, laid out in
// blocks of kBlk = 64 node slots: block b holds the rest population of nodes
// 64b .. 64b+63, then population 1 of the same nodes, ..., population Q-1.
// Rows start on a block boundary (the x stride is a multiple of 64), so the 64
// nodes of one wavefront read and write one contiguous block per population
// set; with one array per population the same accesses would land in Q
// regions far apart, which costs HBM efficiency (DRAM page locality).
// The rest population of g carries phi (g_0 ~ phi - (1 - w_0) alpha mu) and
// changes by far less than an FP32 ulp of 1 per step in bulk liquid, so it is
// always stored in FP64; every other population is small and is stored in the
// case's storage type.  FP16-deviation storage keeps value * scale (a power
// of two) in FP16: the rest equilibrium of every FP16 population is 0 (f at
// p = 0, u = 0; g_i, i > 0, at mu = 0), so these are deviations from it.
//   storage   f rest / moving      g rest / moving     compute
//   kF64      f64 / f64            f64 / f64           f64
//   kF32      f32 / f32            f64 / f32           f32
//   kF16Dev   f32 / f16*scale      f64 / f16*scale     f32
constexpr int kBlk = 64;

template <int S> struct ComputeOf { using T = float; };
template <> struct ComputeOf<kF64> { using T = double; };
template <int S> using ComputeT = typename ComputeOf<S>::T;

// O: byte offsets within the buffer are formed in 32 bits (the buffer is
// smaller than 4 GiB), which keeps a pulled address in one register.
template <int S, bool G, int Q, bool O = false>
struct Set {
  using C = ComputeT<S>;
  using R = typename std::conditional<G || S == kF64, double, float>::type;   // rest
  static constexpr bool kHalf = (S == kF16Dev);
  using M = typename std::conditional<S == kF64, double,
            typename std::conditional<kHalf, __half, float>::type>::type;   // moving
  static constexpr size_t kRestBytes = kBlk * sizeof(R);
  static constexpr size_t kBlockBytes = kBlk * (sizeof(R) + (Q - 1) * sizeof(M));
  // buffer bytes for NQ node slots (NQ a multiple of kBlk)
  __host__ __device__ static size_t bytes(long long NQ) {
    return (size_t)(NQ / kBlk) * kBlockBytes;
  }
  // Loads address with a byte offset from the buffer base: 32-bit when O,
  // which the compiler keeps in one register per pending load.
  __device__ static R load_rest(const void* b, nidx n) {
    const unsigned char* p = static_cast<const unsigned char*>(b);
    if constexpr (O) {
      return *reinterpret_cast<const R*>(
          p + ((n / kBlk) * (unsigned)kBlockBytes + (n % kBlk) * (unsigned)sizeof(R)));
    } else {
      return *reinterpret_cast<const R*>(
          p + ((size_t)(n / kBlk) * kBlockBytes + (size_t)(n % kBlk) * sizeof(R)));
    }
  }
  // population i >= 1 of node n
  __device__ static const M* at(const void* b, int i, nidx n) {
    const unsigned char* p = static_cast<const unsigned char*>(b);
    if constexpr (O) {
      return reinterpret_cast<const M*>(
          p + ((n / kBlk) * (unsigned)kBlockBytes + (unsigned)kRestBytes +
               (unsigned)((i - 1) * kBlk * sizeof(M)) + (n % kBlk) * (unsigned)sizeof(M)));
    } else {
      return reinterpret_cast<const M*>(
          p + ((size_t)(n / kBlk) * kBlockBytes + kRestBytes + (size_t)(i - 1) * kBlk * sizeof(M) +
               (size_t)(n % kBlk) * sizeof(M)));
    }
  }
  // stores: block base, then the element
  __device__ static void store_rest(void* b, nidx n, R v, int nt = 0) {
    st(reinterpret_cast<R*>(static_cast<unsigned char*>(b) + (size_t)(n / kBlk) * kBlockBytes) +
           n % kBlk, v, nt);
  }
  __device__ static M* at(void* b, int i, nidx n) {
    return reinterpret_cast<M*>(static_cast<unsigned char*>(b) + (size_t)(n / kBlk) * kBlockBytes +
                                kRestBytes) +
           (i - 1) * kBlk + n % kBlk;
  }
  // v as the next step will read it back after a store (FP16: rounded to the
  // stored half and decoded; otherwise v itself)
  __device__ static C as_stored(C v, float scale) {
    if constexpr (kHalf) return decode(__float2half_rn(v * scale), scale);
    else return C(M(v));
  }
  __device__ static C decode(M v, float scale) {
    if constexpr (kHalf) return __half2float(v) * (1.0f / scale);
    else return C(v);
  }
  __device__ static C load(const void* b, int i, nidx n, float scale) {
    return decode(*at(b, i, n), scale);
  }
  __device__ static void store(void* b, int i, nidx n, C v, float scale, int nt = 0) {
    M* p = at(b, i, n);
    if constexpr (kHalf) {
      const __half h = __float2half_rn(v * scale);
      if (nt) __builtin_nontemporal_store(*reinterpret_cast<const unsigned short*>(&h),
                                          reinterpret_cast<unsigned short*>(p));
      else *p = h;
    } else {
      st(p, M(v), nt);
    }
  }
};

// ------------------------------------------------------------------ indexing
// a * b + c rounded once (the same in every kernel that inlines it, unlike a
// contraction the compiler may or may not form)
template <class C>
__device__ inline C fmac(C a, C b, C c) {
  if constexpr (std::is_same<C, float>::value) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}

// c . (a, b, c3) for a lattice direction with components in {-1, 0, 1}: the
// zero components are left out (a product with 0.0 is not folded away).
template <class C>
__device__ inline C cdot(int cx, int cy, int cz, C a, C b, C c3) {
  C r = C(0);
  bool any = false;
  if (cx) { r = cx > 0 ? a : -a; any = true; }
  if (cy) { r = any ? (cy > 0 ? r + b : r - b) : (cy > 0 ? b : -b); any = true; }
  if (cz) { r = any ? (cz > 0 ? r + c3 : r - c3) : (cz > 0 ? c3 : -c3); }
  return r;
}

// q taken into [0, P) on a periodic axis: entries already inside skip the
// integer division (a few lanes at the edges of a tile take it)
__device__ inline int wrapq(int q, int P) {
  if (q >= 0 && q < P) return q;
  q %= P;
  return q < 0 ? q + P : q;
}

__device__ inline int wrap1(int q, int P, int per) {
  if (per) {
    q += (q < 0) ? P : 0;
    q -= (q >= P) ? P : 0;
  }
  return q;
}

// Flat indices of x + c_i for all i, for a zeta = 1 node (interior along
// non-periodic axes, so only periodic axes can wrap).
template <class L>
__device__ inline void neighbours(const Geo& G, int x, int y, int z, nidx nb[L::Q]) {
  const int xs[3] = {wrap1(x - 1, G.PX, G.per[0]), x, wrap1(x + 1, G.PX, G.per[0])};
  const int ys[3] = {wrap1(y - 1, G.PY, G.per[1]), y, wrap1(y + 1, G.PY, G.per[1])};
  int zs[3] = {z, z, z};
  if (L::D == 3) {
    zs[0] = wrap1(z - 1, G.PZ, G.per[2]);
    zs[2] = wrap1(z + 1, G.PZ, G.per[2]);
  }
#pragma unroll
  for (int i = 0; i < L::Q; ++i)
    nb[i] = G.idx(xs[1 + L::cx(i)], ys[1 + L::cy(i)], zs[1 + L::cz(i)]);
}

// Pull moving population i >= 1 of node n from x - c_i, or take the opposite
// population of n itself when x - c_i is a zeta = 0 node (bounce-back).  The
// rest population never moves.
template <class L, class SetT>
__device__ inline typename SetT::C pull(const void* buf, int i, nidx n, const nidx nb[L::Q],
                                        uint32_t word, float scale) {
  const bool bb = (word >> (kLinkShift + i)) & 1u;
  return bb ? SetT::load(buf, L::opp(i), n, scale) : SetT::load(buf, i, nb[L::opp(i)], scale);
}

// One thread per slot of the padded grid (x counted from slot 0 of the row, so
// a 64-wide workgroup row covers one population block).
__device__ inline bool node_coords(const Geo& G, int& x, int& y, int& z) {
  x = blockIdx.x * blockDim.x + threadIdx.x - G.XO;
  y = blockIdx.y * blockDim.y + threadIdx.y;
  z = blockIdx.z * blockDim.z + threadIdx.z;
  return x >= 0 && x < G.PX && y < G.PY && z < G.PZ;
}

// Inside a loop the compiler hoists every value derived from loop-invariant
// inputs (conversions of the physics constants, products of them with the
// lattice weights, neighbour coordinates) and keeps it in a vector register for
// the whole loop.  Passing these inputs through an empty asm statement at the
// top of each iteration makes them opaque, so derived values are formed next to
// their use, as in straight-line code.
__device__ inline void opaque(Phys& P) {
  asm volatile("" : "+s"(P.tau), "+s"(P.inv_tau_g), "+s"(P.alpha), "+s"(P.beta), "+s"(P.kappa),
               "+s"(P.wet));
  asm volatile("" : "+s"(P.rho_l), "+s"(P.rho_g), "+s"(P.nu_l), "+s"(P.nu_g), "+s"(P.chi_a));
  asm volatile("" : "+s"(P.Fb[0]), "+s"(P.Fb[1]), "+s"(P.Fb[2]), "+s"(P.scale_f),
               "+s"(P.scale_g));
}
__device__ inline void opaque(int& a, int& b) { asm volatile("" : "+v"(a), "+v"(b)); }

// ------------------------------------------------------------------ k_phi
template <class L, int S, bool O = false>
__global__ void k_phi(const uint32_t* __restrict__ nodes, const void* __restrict__ gsrc,
                      ComputeT<S>* __restrict__ phi, Geo G, Phys P) {
  using C = ComputeT<S>;
  int x, y, z;
  if (!node_coords(G, x, y, z)) return;
  const nidx n = G.idx(x, y, z);
  const uint32_t word = nodes[n];
  if (!(word & kZeta)) return;
  nidx nb[L::Q];
  neighbours<L>(G, x, y, z, nb);
  using GS = Set<S, true, L::G::Q, O>;
  // g_0 carries phi; the moving populations are small.  Summing them first and
  // adding g_0 last rounds once, instead of dropping sub-ulp terms one by one.
  C small = C(0);
#pragma unroll
  for (int i = 1; i < L::G::Q; ++i) small += pull<typename L::G, GS>(gsrc, i, n, nb, word, P.scale_g);
  phi[n] = C(GS::load_rest(gsrc, n) + (double)small);
}

// ------------------------------------------------------------------ LDS stencil pieces
// A tile of phi and node words in LDS with strides sx (x) and sxy (x*y).

// Ghost value from the mean m of the zeta = 1 nodes around it.  chi_a = 0: m
// itself (Sec. 2.2.2, zero normal gradient).  Otherwise (Appendix A, cases 1
// and 3) the ghost g meets n_w . grad phi = chi(phi_w) across the wall, m
// standing for the mirror node one spacing away: m - g = chi((m + g)/2) with
// chi(phi) = a (phi - phi^2).  With phi_w = (m + g)/2 that is
// a phi_w^2 - (a + 2) phi_w + 2 m = 0; the root tending to m as a -> 0 is
// taken (a negative discriminant is clamped to zero), and g = 2 phi_w - m.
template <class C>
__device__ inline C ghost_value(C m, C a) {
  if (a == C(0)) return m;
  const C b = a + C(2);
  const C disc = b * b - C(8) * a * m;
  const C w = (b - sqrt(disc > C(0) ? disc : C(0))) / (C(2) * a);
  return C(2) * w - m;
}

// Ghost value over the 3^D block (Sec. 2.2.2); only zeta = 1 entries are read,
// so filling ghosts in place is order-independent.
template <class L, class C>
__device__ inline C ghost_mean(const C* sphi, const uint32_t* sw, int t, int sx, int sxy,
                               C chi_a) {
  C num = C(0);
  int den = 0;
  constexpr int z0 = (L::D == 3) ? -1 : 0, z1 = (L::D == 3) ? 1 : 0;
#pragma unroll
  for (int dz = z0; dz <= z1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int t2 = t + dx + sx * dy + sxy * dz;
        if (sw[t2] & kZeta) {
          num += sphi[t2];
          ++den;
        }
      }
  return den > 0 ? ghost_value(num / C(den), chi_a) : C(0);
}

// The same ghost value read from the phi array (zeta = 1 entries of the 3^D
// block around node (x, y, z), in the order ghost_mean takes them), for the
// ghost pass of the split step.  Entries outside the padded grid, or in the
// padding layer of a walled axis (never zeta = 1), read the node itself (a
// ghost, so never counted): every load of the block is issued before the
// first is used.
template <class L, class C>
__device__ inline C ghost_from(const uint32_t* __restrict__ nodes, const C* __restrict__ phi,
                               const Geo& G, int x, int y, int z, C chi_a) {
  constexpr int NZ = (L::D == 3) ? 3 : 1, NB = 9 * NZ;
  const int P3[3] = {G.PX, G.PY, G.PZ}, c3[3] = {x, y, z};
  const nidx self = G.idx(x, y, z);
  // per axis: coordinates c - 1, c, c + 1 (wrapped on a periodic axis) and
  // whether they are read
  int qq[3][3];
  bool vv[3][3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      int q = c3[d] + s - 1;
      if (d == 2 && L::D == 2) q = c3[d];
      if (G.per[d]) {
        q += (q < 0) ? P3[d] : 0;
        q -= (q >= P3[d]) ? P3[d] : 0;
        vv[d][s] = true;
      } else {
        vv[d][s] = q >= 1 && q < P3[d] - 1;
      }
      qq[d][s] = q;
    }
  }
  nidx at[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int sx = k % 3, sy = (k / 3) % 3, sz = (L::D == 3) ? k / 9 : 1;
    const bool ok = vv[0][sx] && vv[1][sy] && vv[2][sz];
    at[k] = ok ? G.idx(qq[0][sx], qq[1][sy], qq[2][sz]) : self;
  }
  uint32_t w[NB];
  C v[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    w[k] = nodes[at[k]];
    v[k] = phi[at[k]];
  }
  C num = C(0);
  int den = 0;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (w[k] & kZeta) {
      num += v[k];
      ++den;
    }
  }
  return den > 0 ? ghost_value(num / C(den), chi_a) : C(0);
}

// ghost_from for a node of the padding face x = 0 or x = PX - 1 of a walled x
// axis: of its 3^D block only the column at x = 1 (x = PX - 2) lies inside the
// domain, so only those 3^(D-1) entries are read (the others are padding or
// outside, never zeta = 1).  They are summed in ghost_from's order, so the
// value is the same to the bit.
template <class L, class C>
__device__ inline C ghost_face(const uint32_t* __restrict__ nodes, const C* __restrict__ phi,
                               const Geo& G, int x, int y, int z, C chi_a) {
  constexpr int NZ = (L::D == 3) ? 3 : 1, NB = 3 * NZ;
  const int P3[3] = {G.PX, G.PY, G.PZ}, c3[3] = {x, y, z};
  const int xi = x == 0 ? 1 : G.PX - 2;
  const nidx self = G.idx(x, y, z);
  int qq[3][3];
  bool vv[3][3];
#pragma unroll
  for (int d = 1; d < 3; ++d) {
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      int q = c3[d] + s - 1;
      if (d == 2 && L::D == 2) q = c3[d];
      if (G.per[d]) {
        q += (q < 0) ? P3[d] : 0;
        q -= (q >= P3[d]) ? P3[d] : 0;
        vv[d][s] = true;
      } else {
        vv[d][s] = q >= 1 && q < P3[d] - 1;
      }
      qq[d][s] = q;
    }
  }
  nidx at[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int sy = k % 3, sz = (L::D == 3) ? k / 3 : 1;
    at[k] = (vv[1][sy] && vv[2][sz]) ? G.idx(xi, qq[1][sy], qq[2][sz]) : self;
  }
  uint32_t w[NB];
  C v[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    w[k] = nodes[at[k]];
    v[k] = phi[at[k]];
  }
  C num = C(0);
  int den = 0;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (w[k] & kZeta) {
      num += v[k];
      ++den;
    }
  }
  return den > 0 ? ghost_value(num / C(den), chi_a) : C(0);
}

// mu of Eq. (chemical_potencial2) at a zeta = 1 entry: isotropic Laplacian
// (Eq. Laplace) of phi and a_v = |grad eps| (Eq. avvv) from the neighbours.
// Wall coefficient sqrt(2 kappa beta) cos(theta) of Eq. (chemical_potencial2) at
// a node: the case's value, or with a per-node contact angle the table entry
// its word carries (the mean cos(theta) of the walls around it).
// Entry 0 of the table holds the case's value.  The two forms give the same
// value; each is the one that costs the step kernels of its dimension no
// extra registers (2D: skip the load for entry 0; 3D: always load).
template <int D, class C>
__device__ inline C wet_of(uint32_t word, const Phys& P) {
  const uint32_t k = wet_entry(word);
  if constexpr (D == 2) return k ? C(P.wet_tab[k]) : C(P.wet);
  else return C(P.wet_tab[k]);
}

// The same from accessors: phi_at(i) and word_at(i) give phi and the node word
// at x + c_i, wet() the wall coefficient at x (called where the sum needs it).
// Every kernel forms mu through this one function, so their results agree to
// the bit.
template <class L, class C, class PhiAt, class WordAt, class Wet>
__device__ inline C mu_of(C ph, PhiAt&& phi_at, WordAt&& word_at, Wet&& wet, const Phys& P) {
  C lap = C(0), ex = C(0), ey = C(0), ez = C(0);
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    lap = fmac(C(2 * L::w(i)), phi_at(i) - ph, lap);
    // w_i c_i eps: eps is 0 or 1, so each product is exact and the fused form
    // adds what the separate one would; zero components are left out
    const C e = (word_at(i) & kFluid) ? C(1) : C(0);
    if (L::cx(i)) ex = fmac(C(L::w(i) * L::cx(i)), e, ex);
    if (L::cy(i)) ey = fmac(C(L::w(i) * L::cy(i)), e, ey);
    if (L::cz(i)) ez = fmac(C(L::w(i) * L::cz(i)), e, ez);
  }
  const C inv_cs2 = C(3);
  lap *= inv_cs2;
  ex *= inv_cs2;
  ey *= inv_cs2;
  ez *= inv_cs2;
  const C av = sqrt(ex * ex + ey * ey + ez * ez);
  return C(4) * C(P.beta) * ph * (ph - C(1)) * (ph - C(0.5)) - C(P.kappa) * lap -
         av * wet() * (ph - ph * ph);
}

template <class L, class C>
__device__ inline C mu_at(const C* sphi, const uint32_t* sw, int t, int sx, int sxy,
                          const Phys& P) {
  auto off = [&](int i) { return t + L::cx(i) + sx * L::cy(i) + sxy * L::cz(i); };
  return mu_of<L, C>(
      sphi[t], [&](int i) { return sphi[off(i)]; }, [&](int i) { return sw[off(i)]; },
      [&]() { return wet_of<L::D, C>(sw[t], P); }, P);
}

// grad phi of Eq. (gradient) from neighbour values v(i) = phi(x + c_i).
template <class L, class C, class Fn>
__device__ inline void grad_of(Fn v, C& gx, C& gy, C& gz) {
  gx = gy = gz = C(0);
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    const C t = C(L::w(i)) * v(i);
    if (L::cx(i)) gx = L::cx(i) > 0 ? gx + t : gx - t;   // zero components left out
    if (L::cy(i)) gy = L::cy(i) > 0 ? gy + t : gy - t;
    if (L::cz(i)) gz = L::cz(i) > 0 ? gz + t : gz - t;
  }
  gx *= C(3);
  gy *= C(3);
  gz *= C(3);
}

// ------------------------------------------------------------------ k_mu
// Workgroup = one tile of blockDim nodes; LDS holds phi and node words of the
// tile plus two halo layers (ghost nodes of the first halo layer need their own
// neighbours).  Dynamic LDS bytes: (TX+4)(TY+4)(TZ+4 or 1) * (sizeof(C) + 4).
// Writes mu on zeta = 1 nodes and phi on ghost nodes.
template <class L, class C>
__global__ void k_mu(const uint32_t* __restrict__ nodes, C* __restrict__ phi,
                     C* __restrict__ mu, Geo G, Phys P) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int H = 2;
  constexpr int HZ = (L::D == 3) ? H : 0;
  const int TX = blockDim.x, TY = blockDim.y, TZ = blockDim.z;
  const int LX = TX + 2 * H, LY = TY + 2 * H, LZ = TZ + 2 * HZ;
  const int NL = LX * LY * LZ;
  C* sphi = reinterpret_cast<C*>(smem);
  uint32_t* sw = reinterpret_cast<uint32_t*>(sphi + NL);
  const int ox = blockIdx.x * TX - H - G.XO, oy = blockIdx.y * TY - H, oz = blockIdx.z * TZ - HZ;
  const int tid = threadIdx.x + TX * (threadIdx.y + TY * threadIdx.z);
  const int nthr = TX * TY * TZ;

  for (int t = tid; t < NL; t += nthr) {
    const int lx = t % LX, ly = (t / LX) % LY, lz = t / (LX * LY);
    int q[3] = {ox + lx, oy + ly, oz + lz};
    const int P3[3] = {G.PX, G.PY, G.PZ};
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (G.per[d]) {
        q[d] = wrapq(q[d], P3[d]);
      } else {
        ok = ok && q[d] >= 0 && q[d] < P3[d];
      }
    }
    uint32_t w = 0;
    C v = C(0);
    if (ok) {
      const nidx n = G.idx(q[0], q[1], q[2]);
      w = nodes[n];
      if (w & kZeta) v = phi[n];
    }
    sw[t] = w;
    sphi[t] = v;
  }
  __syncthreads();
  for (int t = tid; t < NL; t += nthr) {
    const int lx = t % LX, ly = (t / LX) % LY, lz = t / (LX * LY);
    const bool inner = lx >= 1 && lx < LX - 1 && ly >= 1 && ly < LY - 1 &&
                       (L::D == 2 || (lz >= 1 && lz < LZ - 1));
    if (inner && (sw[t] & kGhost)) sphi[t] = ghost_mean<L, C>(sphi, sw, t, LX, LX * LY, C(P.chi_a));
  }
  __syncthreads();

  int x, y, z;
  if (!node_coords(G, x, y, z)) return;
  const int t = (threadIdx.x + H) + LX * ((threadIdx.y + H) + LY * (threadIdx.z + HZ));
  const uint32_t w = sw[t];
  const nidx n = G.idx(x, y, z);
  if (w & kZeta) mu[n] = mu_at<L, C>(sphi, sw, t, LX, LX * LY, P);
  else if (w & kGhost) phi[n] = sphi[t];
}

// ------------------------------------------------------------------ node update
// Macroscopic quantities of one node from its pulled f, phi, mu and grad phi:
// rho, F = mu grad phi + F_b, u and p (Sec. 2.1.2), s = u . grad phi; u = 0 on
// boundary nodes (they lie in the solid: no slip).
template <class L, int S>
struct Macro {
  using C = ComputeT<S>;
  C rho, rx, ry, rz, Fx, Fy, Fz, ux, uy, uz, uu, ugr, p, s;
  // wall: a boundary node (zeta = 1, not fluid).  It lies in the solid, so its
  // velocity is the wall's: u = 0 wherever u enters (f_eq, F_i, p, s).
  __device__ Macro(const C* f, C ph, C m, C gx, C gy, C gz, bool wall, const Phys& P) {
    constexpr int Q = L::Q;
    const C inv_cs2 = C(3);
    const C drho = C(P.rho_l - P.rho_g);
    rho = C(P.rho_g) + ph * drho;
    rx = drho * gx;                                                // grad rho
    ry = drho * gy;
    rz = drho * gz;
    Fx = m * gx + C(P.Fb[0]);
    Fy = m * gy + C(P.Fb[1]);
    Fz = (L::D == 3) ? m * gz + C(P.Fb[2]) : C(0);
    C mx = C(0), my = C(0), mz = C(0), sumf = C(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      if (L::cx(i)) mx = L::cx(i) > 0 ? mx + f[i] : mx - f[i];   // zero components left out
      if (L::cy(i)) my = L::cy(i) > 0 ? my + f[i] : my - f[i];
      if (L::cz(i)) mz = L::cz(i) > 0 ? mz + f[i] : mz - f[i];
      sumf += f[i];
    }
    const C inv_rho = C(1) / rho;
    ux = wall ? C(0) : (mx + C(0.5) * Fx) * inv_rho;
    uy = wall ? C(0) : (my + C(0.5) * Fy) * inv_rho;
    uz = wall ? C(0) : (mz + C(0.5) * Fz) * inv_rho;
    uu = ux * ux + uy * uy + uz * uz;
    ugr = ux * rx + uy * ry + uz * rz;                             // u . grad rho
    const C w0 = C(L::w(0));
    const C s0 = -w0 * uu * C(0.5) * inv_cs2;
    p = (sumf + C(0.5) * ugr + rho * s0) / (inv_cs2 * (C(1) - w0));
    s = ux * gx + uy * gy + uz * gz;                               // u . grad phi
  }
};

// Collision of both sets at one node (sp = s of the previous step):
// Eq. (BGK) with g_eq of Eq. (H_i) and G_i of Eq. (F_i) plus half its time
// derivative, the latter a backward difference of s, so that
// G_i + dG_i/2 = w_i k_i (1.5 s - 0.5 s_prev); Eq. (BGK-NS) with f_eq of
// Eq. (feq_i) and F_i of Eq. (GGi).  get_sp() gives s_prev.  Each
// post-collision value is handed to the sinks as soon as it is formed:
// put_g0(g*_0), put_g(i, g*_i) for i >= 1, put_f(i, f*_i); returns
// s = u . grad phi (the next step's s_prev).
//
// The collision keeps sum_i g_i = phi and the sources sum to -(1.5 s - 0.5
// s_prev), since sum_i w_i k_i = -1.  With FP32 or FP16 moving populations
// (stored_g(v): v as it will be read back) the FP64 rest population is formed
// from that balance, g*_0 = g_0 + sum_{i>0} (g_i - stored g*_i) - (1.5 s -
// 0.5 s_prev), which equals Eq. (BGK) for i = 0 up to rounding and makes the
// stored sum over a node change by exactly the source in FP64: the storage
// rounding of the moving populations then never changes the phi mass.
template <class L, int S, class GetSp, class PutG0, class PutG, class PutF, class StoredG>
__device__ inline ComputeT<S> collide_post(const ComputeT<S>* f, double g0, const ComputeT<S>* g,
                                           ComputeT<S> ph, ComputeT<S> m, ComputeT<S> gx,
                                           ComputeT<S> gy, ComputeT<S> gz, bool wall,
                                           const Phys& P, GetSp&& get_sp, PutG0&& put_g0, PutG&& put_g,
                                           PutF&& put_f, StoredG&& stored_g) {
  using C = ComputeT<S>;
  constexpr int Q = L::Q;
  const C inv_cs2 = C(3);
  const Macro<L, S> M(f, ph, m, gx, gy, gz, wall, P);
  using LG = typename L::G;          // velocity set of g
  const C w0 = C(LG::w(0));
  const C sp = get_sp();
  const C srcf = C(1.5) * M.s - C(0.5) * sp;
  const C itg = C(P.inv_tau_g);
  const C am = C(P.alpha) * m;
  if constexpr (S == kF64) {
    // g_0 - g_0^eq = g_0 - phi + (1 - w_0) alpha mu = (1 - w_0) alpha mu - sum_{i>0} g_i,
    // formed from small terms only so that g_0 (about phi) is rounded once.
    C gsmall = C(0);
#pragma unroll
    for (int i = 1; i < LG::Q; ++i) gsmall += g[i];
    {
      const C d0 = (C(1) - w0) * am - gsmall;
      const C inc = w0 * C(LG::k(0)) * srcf - d0 * itg;
      put_g0(g0 + (double)inc);
    }
#pragma unroll
    for (int i = 1; i < LG::Q; ++i) {
      const C wi = C(LG::w(i));
      put_g(i, fmac(wi * am - g[i], itg, g[i]) + C(LG::w(i) * LG::k(i)) * srcf);
    }
  } else {
    double dsum = 0.0;          // sum_{i>0} (g_i - stored g*_i), exact in FP64
#pragma unroll
    for (int i = 1; i < LG::Q; ++i) {
      const C wi = C(LG::w(i));
      const C v = fmac(wi * am - g[i], itg, g[i]) + C(LG::w(i) * LG::k(i)) * srcf;
      put_g(i, v);
      dsum += (double)g[i] - (double)stored_g(v);
    }
    put_g0(g0 + dsum - (double)srcf);
  }
  // hydrodynamic collision
  C tau = C(P.tau);
  if (P.visc_var) tau = (ph * C(P.nu_l - P.nu_g) + C(P.nu_g)) * inv_cs2 + C(0.5);
  const C itau = C(1) / tau;
  const C ffac = C(1) - C(0.5) * itau;
  const C pc = M.p * inv_cs2;
  const C uu15 = C(0.5) * inv_cs2 * M.uu;
  const C ffac3 = ffac * inv_cs2;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const C wi = C(L::w(i));
    const C cu = cdot<C>(L::cx(i), L::cy(i), L::cz(i), M.ux, M.uy, M.uz);
    const C cF = cdot<C>(L::cx(i), L::cy(i), L::cz(i), M.Fx, M.Fy, M.Fz);
    const C cr = cdot<C>(L::cx(i), L::cy(i), L::cz(i), M.rx, M.ry, M.rz);
    // velocity part of Eq. (feq_i): w_i [c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2)]
    const C si = wi * fmac(C(4.5) * cu, cu, fmac(inv_cs2, cu, -uu15));
    const C feq = fmac(M.rho, si, pc * C(i == 0 ? L::w(i) - 1.0 : L::w(i)));
    // Eq. (GGi): u.grad rho + c.F/cs2 + [(c.u)(c.grad rho) - cs2 u.grad rho]/cs2,
    // whose u.grad rho terms cancel: (c.F + (c.u)(c.grad rho))/cs2
    const C Fi = (ffac3 * wi) * fmac(cu, cr, cF);
    put_f(i, fmac(feq - f[i], itau, f[i]) + Fi);
  }
  return M.s;
}

// From the pulled populations, phi, mu and grad phi of one zeta = 1 node:
// MODE 0: collide both sets and store f*, g*, s.  MODE 1: store p and u.
// MODE 2: store s only.  MODE 3: as MODE 0 with s_prev passed in.
template <class L, int S, int MODE, bool O = false>
__device__ inline void node_update(const ComputeT<S>* f, double g0, const ComputeT<S>* g,
                                   ComputeT<S> ph, ComputeT<S> m, ComputeT<S> gx,
                                   ComputeT<S> gy, ComputeT<S> gz, uint32_t word, nidx n,
                                   void* __restrict__ fdst, void* __restrict__ gdst,
                                   ComputeT<S>* __restrict__ sprev, ComputeT<S>* __restrict__ out_p,
                                   ComputeT<S>* __restrict__ out_u, const Geo& G, const Phys& P,
                                   int nt = 0, ComputeT<S> sp_pre = ComputeT<S>(0)) {
  using C = ComputeT<S>;
  using FS = Set<S, false, L::Q, O>;
  using GS = Set<S, true, L::G::Q, O>;
  if (MODE == 1 || MODE == 2) {
    const Macro<L, S> M(f, ph, m, gx, gy, gz, !(word & kFluid), P);
    if (MODE == 1) {
      out_p[n] = M.p;
      out_u[n] = M.ux;
      out_u[G.NQ + n] = M.uy;
      if (L::D == 3) out_u[2 * G.NQ + n] = M.uz;
    } else {
      sprev[n] = M.s;
    }
    return;
  }
  const C s = collide_post<L, S>(
      f, g0, g, ph, m, gx, gy, gz, !(word & kFluid), P,
      [&]() { return (MODE == 3) ? sp_pre : sprev[n]; },
      [&](double v) { GS::store_rest(gdst, n, v, nt); },
      [&](int i, C v) { GS::store(gdst, i, n, v, P.scale_g, nt); },
      [&](int i, C v) {
        if (i == 0) FS::store_rest(fdst, n, typename FS::R(v), nt);
        else FS::store(fdst, i, n, v, P.scale_f, nt);
      },
      [&](C v) { return GS::as_stored(v, P.scale_g); });
  sprev[n] = s;
}

// Unfused node update: phi and mu come from the arrays k_phi / k_mu wrote.
template <class L, int S, int MODE>
__global__ void k_collide(const uint32_t* __restrict__ nodes, const void* __restrict__ fsrc,
                          const void* __restrict__ gsrc, void* __restrict__ fdst,
                          void* __restrict__ gdst, const ComputeT<S>* __restrict__ phi,
                          const ComputeT<S>* __restrict__ mu, ComputeT<S>* __restrict__ sprev,
                          ComputeT<S>* __restrict__ out_p, ComputeT<S>* __restrict__ out_u,
                          Geo G, Phys P) {
  using C = ComputeT<S>;
  constexpr int Q = L::Q;
  int x, y, z;
  if (!node_coords(G, x, y, z)) return;
  const nidx n = G.idx(x, y, z);
  const uint32_t word = nodes[n];
  if (!(word & kZeta)) return;
  nidx nb[Q];
  neighbours<L>(G, x, y, z, nb);
  using FS = Set<S, false, L::Q>;
  using GS = Set<S, true, L::G::Q>;
  C f[Q], g[L::G::Q];
  f[0] = C(FS::load_rest(fsrc, n));
  const double g0 = GS::load_rest(gsrc, n);
  g[0] = C(0);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    f[i] = pull<L, FS>(fsrc, i, n, nb, word, P.scale_f);
    if (i < L::G::Q) g[i] = pull<typename L::G, GS>(gsrc, i, n, nb, word, P.scale_g);
  }
  C gx, gy, gz;
  grad_of<L, C>([&](int i) { return phi[nb[i]]; }, gx, gy, gz);
  node_update<L, S, MODE>(f, g0, g, phi[n], mu[n], gx, gy, gz, word, n, fdst, gdst, sprev, out_p,
                          out_u, G, P);
}

// ------------------------------------------------------------------ fused step
// One kernel per time step.  A workgroup of (64, BY, BZ) threads owns a tile of
// 64 x (BY*KY) x (BZ*KZ) nodes (each thread KY*KZ nodes, strided by the block
// size).  It pulls g for the tile and a one-node halo, forms phi there into LDS
// (two halo layers when a ghost node lies within one node of the tile, since
// ghost means need their own neighbours), fills ghosts, and then for every
// tile node evaluates mu and grad phi from LDS, pulls f and collides.  phi and
// mu never go to global memory; the pulled g of the tile stay in registers.
// The arithmetic per node is that of k_phi + k_mu + k_collide, in the same
// order, so both paths give bit-identical results.
template <class L, int S, int BY, int BZ, int KY, int KZ>
struct StepTile {
  using C = ComputeT<S>;
  static constexpr bool D3 = (L::D == 3);
  static constexpr int TX = 64, TY = BY * KY, TZ = D3 ? BZ * KZ : 1;
  static constexpr int LX = TX + 4, LY = TY + 4, LZ = D3 ? TZ + 4 : 1;
  static constexpr int NL = LX * LY * LZ;
};

// Dispatch order of a tile grid over the 8 XCDs.  The hardware deals the
// workgroups of a launch to the XCDs round-robin (workgroup b to XCD b % 8),
// and each XCD has its own L2.
//   mode 0: workgroup b takes tile b (x fastest, then y, then z).
//   mode 1: each XCD takes one contiguous run of tiles.
//   mode 2: tiles are grouped in chunks of whole x-rows of tiles, kXcdRows rows
//           in y at one z position, and the chunks are dealt to the XCDs
//           round-robin: the tiles of a chunk (x- and y-neighbours) run on one
//           XCD at the same time and share its L2 (halo rows, the cache lines
//           that straddle two tiles in x), while every XCD still gets an even
//           share of the domain.  The grid is padded to whole rounds of 8
//           chunks; the extra workgroups get tile -1 and return at once.
constexpr int kXcdRows = 2;
struct TileOrder {
  int nbx, nby, nbz, mode;
  __host__ __device__ int ncy() const { return (nby + kXcdRows - 1) / kXcdRows; }
  __host__ __device__ int chunk() const { return nbx * kXcdRows; }
  __host__ __device__ unsigned grid() const {
    const long long n = (long long)nbx * nby * nbz;
    if (mode != 2) return (unsigned)n;
    const long long nch = (long long)ncy() * nbz;
    return (unsigned)(((nch + 7) / 8) * 8 * chunk());
  }
  __host__ __device__ int tile(int b) const {
    if (mode == 1) {
      const int n = nbx * nby * nbz;
      const int per = n / 8, rem = n % 8, xcd = b % 8, k = b / 8;
      return (xcd < rem) ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
    }
    if (mode == 2) {
      const int cs = chunk(), k = b / 8, c = (k / cs) * 8 + b % 8, p = k % cs;
      if (c >= ncy() * nbz) return -1;
      const int by = (c % ncy()) * kXcdRows + p / nbx;
      if (by >= nby) return -1;
      return p % nbx + nbx * (by + nby * (c / ncy()));
    }
    return b;
  }
};

// Advance the tile with origin (x0, y0, z0) of one case by one step; sphi and
// sw are LDS arrays of StepTile::NL entries.  Every thread of the workgroup
// must call it (it synchronises the workgroup).
template <class L, int S, int BY, int BZ, int KY, int KZ, bool O = false>
__device__ inline void step_tile(int x0, int y0, int z0, const uint32_t* __restrict__ nodes,
                                 const void* __restrict__ fsrc, const void* __restrict__ gsrc,
                                 void* __restrict__ fdst, void* __restrict__ gdst,
                                 ComputeT<S>* __restrict__ sprev, const Geo& G, const Phys& P,
                                 ComputeT<S>* sphi, uint32_t* sw) {
  using C = ComputeT<S>;
  using GS = Set<S, true, L::G::Q, O>;
  using FS = Set<S, false, L::Q, O>;
  constexpr int Q = L::Q;
  constexpr bool D3 = (L::D == 3);
  constexpr int TX = 64, TY = BY * KY, TZ = D3 ? BZ * KZ : 1;
  constexpr int LX = TX + 4, LY = TY + 4, LZ = D3 ? TZ + 4 : 1;
  constexpr int SX = LX, SXY = LX * LY;
  constexpr int NL = LX * LY * LZ;
  constexpr int HZ = D3 ? 2 : 0;
  constexpr int NT = 64 * BY * BZ;
  constexpr int KN = KY * KZ;
  const int lane = threadIdx.x, ty = threadIdx.y, tz = threadIdx.z;
  const int tid = lane + 64 * (ty + BY * tz);
  const int P3[3] = {G.PX, G.PY, G.PZ};

  // global node of LDS entry (lx, ly, lz), or -1 outside the padded grid
  auto gnode = [&](int lx, int ly, int lz, int q[3]) -> long long {
    q[0] = x0 - 2 + lx;
    q[1] = y0 - 2 + ly;
    q[2] = z0 - HZ + lz;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (G.per[d]) {
        q[d] = wrapq(q[d], P3[d]);
      } else if (q[d] < 0 || q[d] >= P3[d]) {
        return -1;
      }
    }
    return G.idx(q[0], q[1], q[2]);
  };
  auto is_tile = [&](int lx, int ly, int lz) {
    return lx >= 2 && lx < 2 + TX && ly >= 2 && ly < 2 + TY && (!D3 || (lz >= 2 && lz < 2 + TZ));
  };
  // phi of a zeta = 1 node from its pulled g (same order as k_phi)
  auto phi_of = [&](nidx n, uint32_t w, const int q[3]) -> C {
    nidx nb[Q];
    neighbours<L>(G, q[0], q[1], q[2], nb);
    C small = C(0);
#pragma unroll
    for (int i = 1; i < L::G::Q; ++i) small += pull<typename L::G, GS>(gsrc, i, n, nb, w, P.scale_g);
    return C(GS::load_rest(gsrc, n) + (double)small);
  };

  // 1. node words of the tile and the first halo layer; any ghost there?
  constexpr int H1X = TX + 2, H1Y = TY + 2, H1Z = D3 ? TZ + 2 : 1;
  constexpr int N1 = H1X * H1Y * H1Z;
  bool ghost_near = false;
  for (int m = tid; m < N1; m += NT) {
    const int lx = 1 + m % H1X, ly = 1 + (m / H1X) % H1Y, lz = (D3 ? 1 : 0) + m / (H1X * H1Y);
    int q[3];
    const long long n = gnode(lx, ly, lz, q);
    const uint32_t w = n >= 0 ? nodes[n] : 0u;
    sw[lx + SX * ly + SXY * lz] = w;
    ghost_near |= (w & kGhost) != 0;
  }
  const bool need2 = __syncthreads_or(ghost_near);

  // 2. own tile nodes: pull g, keep it, phi into LDS
  double g0r[KN];
  C gr[KN][L::G::Q];
#pragma unroll
  for (int k = 0; k < KN; ++k) {
    const int ky = k % KY, kz = k / KY;
    const int lx = 2 + lane, ly = 2 + ty + BY * ky, lz = HZ + (D3 ? tz + BZ * kz : 0);
    const int t = lx + SX * ly + SXY * lz;
    const uint32_t w = sw[t];
    C ph = C(0);
    g0r[k] = 0.0;
    if (w & kZeta) {
      int q[3];
      const long long n = gnode(lx, ly, lz, q);
      nidx nb[Q];
      neighbours<L>(G, q[0], q[1], q[2], nb);
      C small = C(0);
#pragma unroll
      for (int i = 1; i < L::G::Q; ++i) {
        gr[k][i] = pull<typename L::G, GS>(gsrc, i, n, nb, w, P.scale_g);
        small += gr[k][i];
      }
      g0r[k] = GS::load_rest(gsrc, n);
      ph = C(g0r[k] + (double)small);
    }
    sphi[t] = ph;
  }
  // 3. phi on the first halo layer
  for (int m = tid; m < N1; m += NT) {
    const int lx = 1 + m % H1X, ly = 1 + (m / H1X) % H1Y, lz = (D3 ? 1 : 0) + m / (H1X * H1Y);
    if (is_tile(lx, ly, lz)) continue;
    const int t = lx + SX * ly + SXY * lz;
    const uint32_t w = sw[t];
    C ph = C(0);
    if (w & kZeta) {
      int q[3];
      const long long n = gnode(lx, ly, lz, q);
      ph = phi_of(n, w, q);
    }
    sphi[t] = ph;
  }
  // 4. second halo layer, only where ghost means need it: the ghost means of
  // step 5 read a second-layer entry only from the 3^D block of a ghost of
  // the tile or the first layer, so the other entries are left out (a flat
  // wall needs a few entries at the tile's x ends, not a row of phi from g)
  if (need2) {
    for (int m = tid; m < NL; m += NT) {
      const int lx = m % LX, ly = (m / LX) % LY, lz = m / (LX * LY);
      const bool ring2 = lx == 0 || lx == LX - 1 || ly == 0 || ly == LY - 1 ||
                         (D3 && (lz == 0 || lz == LZ - 1));
      if (!ring2) continue;
      bool near = false;
#pragma unroll
      for (int dz = (D3 ? -1 : 0); dz <= (D3 ? 1 : 0); ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            const int ax = lx + dx, ay = ly + dy, az = lz + dz;
            if (ax < 1 || ax > LX - 2 || ay < 1 || ay > LY - 2 || (D3 && (az < 1 || az > LZ - 2)))
              continue;
            near = near || (sw[ax + SX * ay + SXY * az] & kGhost) != 0;
          }
      uint32_t w = 0u;
      C v = C(0);
      if (near) {
        int q[3];
        const long long n = gnode(lx, ly, lz, q);
        w = n >= 0 ? nodes[n] : 0u;
        if (w & kZeta) v = phi_of(n, w, q);
      }
      sw[m] = w;
      sphi[m] = v;
    }
  }
  __syncthreads();
  // 5. ghost means on the tile and the first halo layer
  if (need2) {
    for (int m = tid; m < N1; m += NT) {
      const int lx = 1 + m % H1X, ly = 1 + (m / H1X) % H1Y, lz = (D3 ? 1 : 0) + m / (H1X * H1Y);
      const int t = lx + SX * ly + SXY * lz;
      if (sw[t] & kGhost) sphi[t] = ghost_mean<L, C>(sphi, sw, t, SX, SXY, C(P.chi_a));
    }
    __syncthreads();
  }
  // 6. collide the tile nodes
#pragma unroll
  for (int k = 0; k < KN; ++k) {
    const int ky = k % KY, kz = k / KY;
    const int x = x0 + lane, y = y0 + ty + BY * ky, z = z0 + (D3 ? tz + BZ * kz : 0);
    if (x >= G.PX || y >= G.PY || z >= G.PZ) continue;
    const int lx = 2 + lane, ly = 2 + ty + BY * ky, lz = HZ + (D3 ? tz + BZ * kz : 0);
    const int t = lx + SX * ly + SXY * lz;
    const uint32_t w = sw[t];
    if (!(w & kZeta)) continue;
    const nidx n = G.idx(x, y, z);
    nidx nb[Q];
    neighbours<L>(G, x, y, z, nb);
    C f[Q];
    f[0] = C(FS::load_rest(fsrc, n));
#pragma unroll
    for (int i = 1; i < Q; ++i) f[i] = pull<L, FS>(fsrc, i, n, nb, w, P.scale_f);
    const C m = mu_at<L, C>(sphi, sw, t, SX, SXY, P);
    C gx, gy, gz;
    grad_of<L, C>([&](int i) { return sphi[t + L::cx(i) + SX * L::cy(i) + SXY * L::cz(i)]; },
                  gx, gy, gz);
    node_update<L, S, 0, O>(f, g0r[k], gr[k], sphi[t], m, gx, gy, gz, w, n, fdst, gdst, sprev,
                         nullptr, nullptr, G, P, P.nt_store);
  }
}


// One launch per time step: one workgroup per tile, in the XCD order P.xcd_order
// selects (TileOrder).
template <class L, int S, int BY, int BZ, int KY, int KZ, bool O>
__global__ __launch_bounds__(64 * BY * BZ) void k_step(
    const uint32_t* __restrict__ nodes, const void* __restrict__ fsrc,
    const void* __restrict__ gsrc, void* __restrict__ fdst, void* __restrict__ gdst,
    ComputeT<S>* __restrict__ sprev, Geo G, Phys P) {
  using T = StepTile<L, S, BY, BZ, KY, KZ>;
  __shared__ typename T::C sphi[T::NL];
  __shared__ uint32_t sw[T::NL];
  const TileGrid TG(G, T::TX, T::TY, T::TZ);
  const int b = TileOrder{TG.nx, TG.ny, TG.nz, P.xcd_order}.tile(blockIdx.x);
  if (b < 0) return;
  int x0, y0, z0;
  TG.origin(b, x0, y0, z0);
  step_tile<L, S, BY, BZ, KY, KZ, O>(x0, y0, z0, nodes, fsrc, gsrc, fdst, gdst, sprev, G, P, sphi,
                                  sw);
}

// ------------------------------------------------------------------ split step
// ------------------------------------------------------------------ ghost pass
// Between the phi pass and the collide pass of the split step: the ghost
// nodes' phi (Sec. 2.2.2; Appendix A with chi_a != 0) into the phi array, from
// the zeta = 1 values the phi pass wrote.  The collide pass then reads phi of
// the tile and one halo layer as it stands, with no ghost means of its own.
// A single case uses k_ghost (a block list built with the node classes); a
// group uses k_ghost_group over its tile table:
//
// a workgroup of kGhostThreads takes one tile's box, the tile widened by the
// padding layer where it meets a face of the padded grid, so that the tiles of
// a case cover every ghost node once.  It lists the box's ghost nodes in LDS,
// kGhostChunk entries at a time, and then evaluates them with every lane busy
// (a walled x face holds one ghost node per row, which a one-thread-per-node
// pass would leave alone in its wavefront).
constexpr int kGhostThreads = 256, kGhostChunk = 1024;
template <class L, class C>
__device__ inline void ghost_box(const uint32_t* __restrict__ nodes, C* __restrict__ phi,
                                 const Geo& G, C chi_a, const TileGrid& TG, int b, int* list,
                                 int* count) {
  int o[3];
  TG.origin(b, o[0], o[1], o[2]);
  const int P3[3] = {G.PX, G.PY, G.PZ}, T3[3] = {TG.tx, TG.ty, TG.tz},
            org[3] = {TG.ox, TG.oy, TG.oz};
  int lo[3], ext[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = (o[d] == org[d]) ? 0 : o[d];
    const int hi = (o[d] + T3[d] >= P3[d] - G.pad[d]) ? P3[d] : o[d] + T3[d];
    ext[d] = hi - lo[d];
  }
  const int nbox = ext[0] * ext[1] * ext[2];
  auto coords = [&](int m, int& x, int& y, int& z) {
    x = lo[0] + m % ext[0];
    y = lo[1] + (m / ext[0]) % ext[1];
    z = lo[2] + m / (ext[0] * ext[1]);
  };
  for (int c0 = 0; c0 < nbox; c0 += kGhostChunk) {
    if (threadIdx.x == 0) *count = 0;
    __syncthreads();
    const int c1 = c0 + kGhostChunk < nbox ? c0 + kGhostChunk : nbox;
    for (int m = c0 + (int)threadIdx.x; m < c1; m += kGhostThreads) {
      int x, y, z;
      coords(m, x, y, z);
      if (nodes[G.idx(x, y, z)] & kGhost) list[atomicAdd(count, 1)] = m;
    }
    __syncthreads();
    const int cnt = *count;
    for (int j = threadIdx.x; j < cnt; j += kGhostThreads) {
      int x, y, z;
      coords(list[j], x, y, z);
      phi[G.idx(x, y, z)] = ghost_from<L, C>(nodes, phi, G, x, y, z, chi_a);
    }
    __syncthreads();
  }
}

// Single case, two kinds of workgroup in one launch.  The first nface_wg take
// the padding faces of a walled x axis, one face node per lane (2 per row,
// lanes over consecutive rows); each such face node sits alone in its
// population block.  The others take the listed population blocks (64 slots
// holding a ghost off those faces; the list is built with the node classes),
// one wavefront per block, each lane one slot, wavefronts striding over the
// list two blocks at a time so that the node-word loads of both are in flight
// together.
template <class L, class C>
__global__ __launch_bounds__(kGhostThreads) void k_ghost(const uint32_t* __restrict__ nodes,
                                                          C* __restrict__ phi,
                                                          const uint32_t* __restrict__ blocks,
                                                          int nblocks, int nface_wg, Geo G,
                                                          Phys P) {
  const C chi_a = C(P.chi_a);
  if ((int)blockIdx.x < nface_wg) {
    const int i = blockIdx.x * kGhostThreads + threadIdx.x;
    const int row = i >> 1;
    if (row >= G.PY * G.PZ) return;
    const int x = (i & 1) ? G.PX - 1 : 0, y = row % G.PY, z = row / G.PY;
    const nidx n = G.idx(x, y, z);
    if (nodes[n] & kGhost) phi[n] = ghost_face<L, C>(nodes, phi, G, x, y, z, chi_a);
    return;
  }
  const int lane = threadIdx.x % 64;
  const int nw = (gridDim.x - nface_wg) * (kGhostThreads / 64);
  const int w0 = (blockIdx.x - nface_wg) * (kGhostThreads / 64) + threadIdx.x / 64;
  for (int e = w0; e < nblocks; e += 2 * nw) {
    uint32_t slot[2], w[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int ek = e + k * nw;
      slot[k] = ek < nblocks ? blocks[ek] * (uint32_t)kBlk + lane : 0u;
      w[k] = ek < nblocks ? nodes[slot[k]] : 0u;
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (!(w[k] & kGhost)) continue;
      // (x, y, z) of the slot: slot = x + XO + SX (y + PY z)
      const int r = (int)slot[k] - G.XO;
      const int x = r % G.SX, row = r / G.SX;
      if (nface_wg > 0 && (x == 0 || x == G.PX - 1)) continue;   // the face phase's
      const int y = row % G.PY, z = row / G.PY;
      phi[slot[k]] = ghost_from<L, C>(nodes, phi, G, x, y, z, chi_a);
    }
  }
}

// Split step, second launch: phi and the node words of the tile and a
// one-node halo into LDS (4 bytes per entry, mostly from L2; ghost entries
// carry the ghost pass's values), mu and grad phi from LDS, f and g pulled,
// both sets collided.  One thread per node; workgroup (64, BY, BZ).  g is read
// twice per step (phi pass and here), but nothing is recomputed on the halo.
template <class L, int S, int BY, int BZ, bool O = false>
__device__ inline void stepB_tile(int x0, int y0, int z0, const uint32_t* __restrict__ nodes,
                                  const void* __restrict__ fsrc, const void* __restrict__ gsrc,
                                  void* __restrict__ fdst, void* __restrict__ gdst,
                                  ComputeT<S>* __restrict__ sprev,
                                  const ComputeT<S>* __restrict__ phi, const Geo& G,
                                  const Phys& P, ComputeT<S>* sphi, uint32_t* sw) {
  using C = ComputeT<S>;
  using GS = Set<S, true, L::G::Q, O>;
  using FS = Set<S, false, L::Q, O>;
  constexpr int Q = L::Q;
  constexpr bool D3 = (L::D == 3);
  constexpr int TX = 64, TY = BY, TZ = D3 ? BZ : 1;
  constexpr int LX = TX + 2, LY = TY + 2, LZ = D3 ? TZ + 2 : 1;
  constexpr int SX = LX, SXY = LX * LY, NL = LX * LY * LZ;
  constexpr int HZ = D3 ? 1 : 0;
  constexpr int NT = 64 * BY * (D3 ? BZ : 1);
  const int lane = threadIdx.x, ty = threadIdx.y, tz = D3 ? threadIdx.z : 0;
  const int tid = lane + 64 * (ty + BY * tz);
  const int P3[3] = {G.PX, G.PY, G.PZ};
  // every entry's node word and phi requested before any is stored, so the
  // loads of a thread overlap (phi whatever the word; entries that are neither
  // zeta = 1 nor ghost hold phi = 0 in LDS)
  constexpr int KP = (NL + NT - 1) / NT;
  uint32_t hw[KP];
  C hv[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int m = tid + k * NT;
    hw[k] = 0u;
    hv[k] = C(0);
    if (m >= NL) continue;
    const int lx = m % LX, ly = (m / LX) % LY, lz = m / (LX * LY);
    int q[3] = {x0 - 1 + lx, y0 - 1 + ly, z0 - HZ + lz};
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (G.per[d]) {
        q[d] = wrapq(q[d], P3[d]);
      } else if (q[d] < 0 || q[d] >= P3[d]) {
        ok = false;
      }
    }
    if (ok) {
      const nidx n = G.idx(q[0], q[1], q[2]);
      hw[k] = nodes[n];
      hv[k] = phi[n];
    }
  }
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int m = tid + k * NT;
    if (m >= NL) continue;
    sw[m] = hw[k];
    sphi[m] = (hw[k] & (kZeta | kGhost)) ? hv[k] : C(0);
  }
  __syncthreads();
  const int x = x0 + lane, y = y0 + ty, z = z0 + tz;
  if (x >= G.PX || y >= G.PY || z >= G.PZ) return;
  const int t = (1 + lane) + SX * (1 + ty) + SXY * (HZ + tz);
  const uint32_t w = sw[t];
  if (!(w & kZeta)) return;
  const nidx n = G.idx(x, y, z);
  nidx nb[Q];
  neighbours<L>(G, x, y, z, nb);
  C f[Q], g[L::G::Q];
  f[0] = C(FS::load_rest(fsrc, n));
  const double g0 = GS::load_rest(gsrc, n);
  g[0] = C(0);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    f[i] = pull<L, FS>(fsrc, i, n, nb, w, P.scale_f);
    if (i < L::G::Q) g[i] = pull<typename L::G, GS>(gsrc, i, n, nb, w, P.scale_g);
  }
  const C m = mu_at<L, C>(sphi, sw, t, SX, SXY, P);
  C gx, gy, gz;
  grad_of<L, C>([&](int i) { return sphi[t + L::cx(i) + SX * L::cy(i) + SXY * L::cz(i)]; },
                gx, gy, gz);
  node_update<L, S, 0, O>(f, g0, g, sphi[t], m, gx, gy, gz, w, n, fdst, gdst, sprev, nullptr, nullptr,
                       G, P, P.nt_store);
}

// Waves per SIMD to ask of the register allocator for a workgroup of nt
// threads: the largest multiple of the workgroup's waves per SIMD (nt / 256,
// the four SIMDs of a CU sharing its wavefronts) up to cap.  Workgroups are
// resident whole, so a 512-thread workgroup fits two per CU at 4 or at 5 waves
// per SIMD, and 4 (128 VGPRs) costs nothing against 5 (96).
constexpr int fill_waves(int nt, int cap) {
  return nt <= 256 ? cap : cap / (nt / 256) * (nt / 256);
}

// The collide pass of the split step: FP32 and FP64 take the occupancy-neutral
// bound (a 512-thread workgroup: 80 VGPRs, no spills); FP16-deviation keeps 7
// waves per SIMD (72 VGPRs), measured faster for its instruction-bound pass.
constexpr int stepB_waves(int s, int nt) { return s == kF16Dev ? 7 : fill_waves(nt, 7); }

template <class L, int S, int BY, int BZ, bool O>
__global__ __launch_bounds__(64 * BY * BZ, stepB_waves(S, 64 * BY * BZ)) void k_stepB(
    const uint32_t* __restrict__ nodes, const void* __restrict__ fsrc,
    const void* __restrict__ gsrc, void* __restrict__ fdst, void* __restrict__ gdst,
    ComputeT<S>* __restrict__ sprev, const ComputeT<S>* __restrict__ phi, Geo G, Phys P) {
  constexpr bool D3 = (L::D == 3);
  constexpr int NL = 66 * (BY + 2) * (D3 ? BZ + 2 : 1);
  __shared__ ComputeT<S> sphi[NL];
  __shared__ uint32_t sw[NL];
  const int TZ = D3 ? BZ : 1;
  const TileGrid TG(G, 64, BY, TZ);
  const int b = TileOrder{TG.nx, TG.ny, TG.nz, P.xcd_order}.tile(blockIdx.x);
  if (b < 0) return;
  int x0, y0, z0;
  TG.origin(b, x0, y0, z0);
  stepB_tile<L, S, BY, BZ, O>(x0, y0, z0, nodes, fsrc, gsrc, fdst, gdst, sprev, phi, G, P, sphi, sw);
}

// phi of the tile nodes (64 x BY x BZ) from pulled g, same arithmetic as k_phi.
template <class L, int S, int BY, int BZ, bool O = false>
__device__ inline void phi_tile(int x0, int y0, int z0, const uint32_t* __restrict__ nodes,
                                const void* __restrict__ gsrc, ComputeT<S>* __restrict__ phi,
                                const Geo& G, const Phys& P) {
  using C = ComputeT<S>;
  using GS = Set<S, true, L::G::Q, O>;
  const int x = x0 + threadIdx.x, y = y0 + threadIdx.y, z = z0 + ((L::D == 3) ? threadIdx.z : 0);
  if (x >= G.PX || y >= G.PY || z >= G.PZ) return;
  const nidx n = G.idx(x, y, z);
  const uint32_t w = nodes[n];
  if (!(w & kZeta)) return;
  nidx nb[L::Q];
  neighbours<L>(G, x, y, z, nb);
  C small = C(0);
#pragma unroll
  for (int i = 1; i < L::G::Q; ++i) small += pull<typename L::G, GS>(gsrc, i, n, nb, w, P.scale_g);
  phi[n] = C(GS::load_rest(gsrc, n) + (double)small);
}

// ------------------------------------------------------------------ z-marching split step (3D)
// Second launch of the split step for D3Q19, marching along z.  A workgroup of
// (64, TY) threads owns a column of 64 x TY x TZ nodes and walks it one z
// plane at a time.  LDS holds a ring of four phi / node-word planes, each
// 66 x (TY+2) (the tile and a one-node halo in x and y; ghost entries carry
// the ghost pass's values).  Iteration z stores plane z + 1 (loaded into
// registers during the previous iteration), requests plane z + 2, and after
// one barrier collides plane z from planes z - 1, z, z + 1.  Plane z + 1
// overwrites the slot of plane z - 3, which no thread still reads, so one
// barrier per plane suffices.  Rows shared by consecutive planes of the pulls
// come from cache, so neighbouring tiles along z do not refetch them.
template <class L, int S, int TY, int TZ>
struct ColumnTile {
  static constexpr int LX = 66, LY = TY + 2, PLANE = LX * LY, NL = 4 * PLANE;
};

template <class L, int S, int TY, int TZ, bool O = false>
__device__ inline void stepC_tile(int x0, int y0, int z0, const uint32_t* __restrict__ nodes,
                                  const void* __restrict__ fsrc, const void* __restrict__ gsrc,
                                  void* __restrict__ fdst, void* __restrict__ gdst,
                                  ComputeT<S>* __restrict__ sprev,
                                  const ComputeT<S>* __restrict__ phi, const Geo& G,
                                  const Phys& P, ComputeT<S>* sphi, uint32_t* sw) {
  static_assert(L::D == 3, "z marching is for D3Q19");
  using C = ComputeT<S>;
  using GS = Set<S, true, L::G::Q, O>;
  using FS = Set<S, false, L::Q, O>;
  constexpr int Q = L::Q;
  constexpr int LX = 66, LY = TY + 2, PL = LX * LY;
  constexpr int NT = 64 * TY;
  constexpr int KP = (PL + NT - 1) / NT;   // plane entries per thread
  const int lane = threadIdx.x, ty = threadIdx.y;
  int tid = lane + 64 * ty;            // made opaque once per plane, with x and y
  const int P3[3] = {G.PX, G.PY, G.PZ};
  // ring slot of plane z (z >= z0 - 1)
  auto slot = [&](int z) { return (z - z0 + 1) & 3; };
  // node words and phi of this thread's entries of plane z into registers (phi
  // whatever the word, masked when it goes to LDS, so the loads are independent)
  auto issue_plane = [&](int z, uint32_t (&hw)[KP], C (&hv)[KP]) {
    int qz = z;
    bool zok = true;
    if (G.per[2]) {
      qz = wrapq(qz, P3[2]);
    } else if (qz < 0 || qz >= P3[2]) {
      zok = false;
    }
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int m = tid + k * NT;
      hw[k] = 0u;
      hv[k] = C(0);
      if (m >= PL) continue;
      const int lx = m % LX, ly = m / LX;
      int q[2] = {x0 - 1 + lx, y0 - 1 + ly};
      bool ok = zok;
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        if (G.per[d]) {
          q[d] = wrapq(q[d], P3[d]);
        } else if (q[d] < 0 || q[d] >= P3[d]) {
          ok = false;
        }
      }
      if (ok) {
        const nidx n = G.idx(q[0], q[1], qz);
        hw[k] = nodes[n];
        hv[k] = phi[n];
      }
    }
  };
  // entries that are neither zeta = 1 nor ghost hold phi = 0
  auto commit_plane = [&](int z, const uint32_t (&hw)[KP], const C (&hv)[KP]) {
    C* fp = sphi + slot(z) * PL;
    uint32_t* wp = sw + slot(z) * PL;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int m = tid + k * NT;
      if (m >= PL) continue;
      wp[m] = hw[k];
      fp[m] = (hw[k] & (kZeta | kGhost)) ? hv[k] : C(0);
    }
  };
  uint32_t hw[KP];
  C hv[KP];
  issue_plane(z0 - 1, hw, hv);
  commit_plane(z0 - 1, hw, hv);
  issue_plane(z0, hw, hv);
  commit_plane(z0, hw, hv);
  issue_plane(z0 + 1, hw, hv);
  for (int z = z0; z < z0 + TZ; ++z) {
    tid = lane + 64 * ty;
    asm volatile("" : "+v"(tid));
    commit_plane(z + 1, hw, hv);
    if (z + 2 <= z0 + TZ) issue_plane(z + 2, hw, hv);
    __syncthreads();
    int x = x0 + lane, y = y0 + ty;
    opaque(x, y);
    if (x >= G.PX || y >= G.PY || z >= G.PZ) continue;
    const int t = (1 + lane) + LX * (1 + ty);
    const int s0 = slot(z) * PL, sm = slot(z - 1) * PL, sp = slot(z + 1) * PL;
    const uint32_t w = sw[s0 + t];
    if (!(w & kZeta)) continue;
    const nidx n = G.idx(x, y, z);
    nidx nb[Q];
    neighbours<L>(G, x, y, z, nb);
    C f[Q], g[L::G::Q];
    f[0] = C(FS::load_rest(fsrc, n));
    const double g0 = GS::load_rest(gsrc, n);
    g[0] = C(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      f[i] = pull<L, FS>(fsrc, i, n, nb, w, P.scale_f);
      if (i < L::G::Q) g[i] = pull<typename L::G, GS>(gsrc, i, n, nb, w, P.scale_g);
    }
    // neighbour entry for lattice direction i
    auto at = [&](int i) {
      const int sl = L::cz(i) < 0 ? sm : (L::cz(i) > 0 ? sp : s0);
      return sl + t + L::cx(i) + LX * L::cy(i);
    };
    // mu and grad phi
    const C ph = sphi[s0 + t];
    const C m = mu_of<L, C>(
        ph, [&](int i) { return sphi[at(i)]; }, [&](int i) { return sw[at(i)]; },
        [&]() { return wet_of<L::D, C>(w, P); }, P);
    C gx, gy, gz;
    grad_of<L, C>([&](int i) { return sphi[at(i)]; }, gx, gy, gz);
    node_update<L, S, 0, O>(f, g0, g, ph, m, gx, gy, gz, w, n, fdst, gdst, sprev, nullptr,
                         nullptr, G, P, P.nt_store);
  }
}

// ------------------------------------------------------------------ fused z-marching step (3D)
// One launch per step, g read once.  A workgroup of (64, TY) threads owns a
// column of 64 x TY x TZ nodes and walks it along z; thread (lane, ty) owns
// the nodes (x0 + lane, y0 + ty, z) of every plane.  LDS holds a ring of raw /
// ghost-filled phi planes and a ring of node-word planes, each over the window
// W2 = 68 x (TY + 4) (the tile and two halo layers in x and y).  Iteration j
// collides plane j:
//   S1  node words of plane j + 3 into the word ring (and whether a ghost lies
//       in the window W1 = tile + one halo layer of that plane);
//   S2  raw phi of plane j + 1 over W1 (over W2 when a ghost is in W1 of plane
//       j, j + 1 or j + 2): the owned node pulls its g and keeps it for the
//       collision of the next iteration; halo nodes pull g and keep only phi;
//   S3  raw phi of plane j + 2 at the fluid / boundary nodes the ghosts of plane
//       j + 1 read (their 3 x 3 x 3 blocks reach plane j + 2);
//   S4  ghost means of plane j + 1 over W1;
//   S5  collision of plane j: f pulled, g kept from the previous iteration, mu
//       and grad phi from the phi planes j - 1, j, j + 1.
// The arithmetic per node is that of k_phi + k_mu + k_collide, in the same
// order, so all step kernels give bit-identical results.
template <int TY>
struct MarchTile {
  static constexpr int LX = 68, LY = TY + 4, PL = LX * LY;
  static constexpr int NPHI = 5, NWORD = 6;        // ring slots
  static constexpr int NL_PHI = NPHI * PL, NL_WORD = NWORD * PL;
};

template <class L, int S, int TY, int TZ, bool O = false>
__device__ inline void stepZ_tile(int x0, int y0, int z0, const uint32_t* __restrict__ nodes,
                                  const void* __restrict__ fsrc, const void* __restrict__ gsrc,
                                  void* __restrict__ fdst, void* __restrict__ gdst,
                                  ComputeT<S>* __restrict__ sprev, const Geo& G, const Phys& P0,
                                  ComputeT<S>* sphi, uint32_t* sw) {
  static_assert(L::D == 3, "z marching is for 3D lattices");
  // physics constants and owned coordinates, made opaque once per plane (opaque())
  Phys P = P0;
  int xo = x0 + threadIdx.x, yo = y0 + threadIdx.y;
  using C = ComputeT<S>;
  using GS = Set<S, true, L::G::Q, O>;
  using FS = Set<S, false, L::Q, O>;
  constexpr int Q = L::Q, QG = L::G::Q;
  constexpr int LX = 68, LY = TY + 4, PL = LX * LY, NT = 64 * TY;
  const int lane = threadIdx.x, ty = threadIdx.y;
  const int tid = lane + 64 * ty;
  const int z1 = (z0 + TZ < G.PZ) ? z0 + TZ : G.PZ;     // last plane + 1 of the column
  // ring slots (planes below z0 - 2 are never held)
  auto pslot = [&](int z) { return ((z - z0 + 10) % 5) * PL; };
  auto wslot = [&](int z) { return ((z - z0 + 12) % 6) * PL; };
  // plane z in the padded grid (periodic wrap), or -1 outside a closed axis
  auto zof = [&](int z) -> int {
    if (G.per[2]) {
      return wrapq(z, G.PZ);
    }
    return (z >= 0 && z < G.PZ) ? z : -1;
  };
  // padded coordinates of window entry m (wrapping periodic axes); false outside
  auto exy = [&](int m, int& qx, int& qy) -> bool {
    qx = x0 - 2 + m % LX;
    qy = y0 - 2 + m / LX;
    if (G.per[0]) {
      qx = wrapq(qx, G.PX);
    } else if (qx < 0 || qx >= G.PX) {
      return false;
    }
    if (G.per[1]) {
      qy = wrapq(qy, G.PY);
    } else if (qy < 0 || qy >= G.PY) {
      return false;
    }
    return true;
  };
  // raw phi of window entry m of plane qz (same arithmetic as k_phi); the word
  // of an entry outside the grid is 0
  auto raw_entry = [&](const uint32_t* wp, int m, int qz) -> C {
    const uint32_t w = wp[m];
    if (!(w & kZeta)) return C(0);
    int qx, qy;
    exy(m, qx, qy);
    const nidx n = G.idx(qx, qy, qz);
    nidx nb[Q];
    neighbours<L>(G, qx, qy, qz, nb);
    C small = C(0);
#pragma unroll
    for (int i = 1; i < QG; ++i) small += pull<typename L::G, GS>(gsrc, i, n, nb, w, P.scale_g);
    return C(GS::load_rest(gsrc, n) + (double)small);
  };
  // S1: node words of plane z over W2; returns whether this thread saw a ghost in W1
  auto load_words = [&](int z) -> bool {
    uint32_t* wp = sw + wslot(z);
    const int qz = zof(z);
    bool ghost = false;
    for (int m = tid; m < PL; m += NT) {
      int qx, qy;
      uint32_t w = 0;
      if (qz >= 0 && exy(m, qx, qy)) w = nodes[G.idx(qx, qy, qz)];
      wp[m] = w;
      const int lx = m % LX, ly = m / LX;
      if (lx >= 1 && lx < LX - 1 && ly >= 1 && ly < LY - 1) ghost |= (w & kGhost) != 0;
    }
    return ghost;
  };
  // the tile node (x0 + lane, y0 + ty) is owned (its pulls are kept) when it lies
  // in the padded grid; other tile entries wrap (periodic) or are outside
  const bool own_xy = (xo < G.PX) && (yo < G.PY);
  const int tt = (2 + lane) + LX * (2 + ty);            // window entry of the owned node
  // S2: raw phi of plane z over W1 (and the outer ring when ring2); the owned
  // node's pulled g go to (g0k, gk)
  auto raw_plane = [&](int z, bool ring2, double& g0k, C* gk) {
    C* fp = sphi + pslot(z);
    const uint32_t* wp = sw + wslot(z);
    const int qz = zof(z);
    {
      const uint32_t w = wp[tt];
      C ph = C(0);
      g0k = 0.0;
      if (own_xy && qz >= 0 && (w & kZeta)) {
        const nidx n = G.idx(xo, yo, qz);
        nidx nb[Q];
        neighbours<L>(G, xo, yo, qz, nb);
        C small = C(0);
#pragma unroll
        for (int i = 1; i < QG; ++i) {
          gk[i] = pull<typename L::G, GS>(gsrc, i, n, nb, w, P.scale_g);
          small += gk[i];
        }
        g0k = GS::load_rest(gsrc, n);
        ph = C(g0k + (double)small);
      } else if (!own_xy && qz >= 0) {
        ph = raw_entry(wp, tt, qz);
      }
      fp[tt] = ph;
    }
    // first halo layer: rows 1 and TY + 2 (x 1..66), then x = 1 and 66 of rows 2..TY + 1
    constexpr int NR1 = 2 * 66 + 2 * TY;
    for (int r = tid; r < NR1; r += NT) {
      int lx, ly;
      if (r < 132) {
        ly = r < 66 ? 1 : TY + 2;
        lx = 1 + r % 66;
      } else {
        const int k = r - 132;
        ly = 2 + (k >> 1);
        lx = (k & 1) ? 66 : 1;
      }
      const int m = lx + LX * ly;
      fp[m] = qz >= 0 ? raw_entry(wp, m, qz) : C(0);
    }
    if (ring2) {
      // outer layer: rows 0 and LY - 1, then x = 0 and 67 of rows 1..LY - 2
      constexpr int NR2 = 2 * LX + 2 * (LY - 2);
      for (int r = tid; r < NR2; r += NT) {
        int lx, ly;
        if (r < 2 * LX) {
          ly = r < LX ? 0 : LY - 1;
          lx = r % LX;
        } else {
          const int k = r - 2 * LX;
          ly = 1 + (k >> 1);
          lx = (k & 1) ? LX - 1 : 0;
        }
        const int m = lx + LX * ly;
        fp[m] = qz >= 0 ? raw_entry(wp, m, qz) : C(0);
      }
    }
  };
  // S3: raw phi of plane z at the zeta = 1 entries next to (in x, y) a ghost of
  // the adjacent plane zg inside W1 (the entries that ghost's mean reads)
  auto raw_support = [&](int z, int zg) {
    C* fp = sphi + pslot(z);
    const uint32_t* wp = sw + wslot(z);
    const uint32_t* wq = sw + wslot(zg);
    const int qz = zof(z);
    if (qz < 0) return;
    for (int m = tid; m < PL; m += NT) {
      if (!(wp[m] & kZeta)) continue;
      const int lx = m % LX, ly = m / LX;
      bool near = false;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int ax = lx + dx, ay = ly + dy;
          if (ax >= 1 && ax < LX - 1 && ay >= 1 && ay < LY - 1)
            near |= (wq[ax + LX * ay] & kGhost) != 0;
        }
      if (near) fp[m] = raw_entry(wp, m, qz);
    }
  };
  // S4: ghost means of plane z over W1 (same order as ghost_mean)
  auto fill_ghosts = [&](int z) {
    const int sm = pslot(z - 1), s0 = pslot(z), sp = pslot(z + 1);
    const int wm = wslot(z - 1), w0 = wslot(z), wpl = wslot(z + 1);
    for (int m = tid; m < 66 * (TY + 2); m += NT) {
      const int t = (1 + m % 66) + LX * (1 + m / 66);
      if (!(sw[w0 + t] & kGhost)) continue;
      const int pb[3] = {sm, s0, sp}, wb[3] = {wm, w0, wpl};
      C num = C(0);
      int den = 0;
#pragma unroll
      for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            const int t2 = t + dx + LX * dy;
            if (sw[wb[dz] + t2] & kZeta) {
              num += sphi[pb[dz] + t2];
              ++den;
            }
          }
      if (den > 0) sphi[s0 + t] = ghost_value(num / C(den), C(P.chi_a));
    }
  };

  // prologue: words of planes z0 - 2 .. z0 + 2, with the ghost flags of z0 - 1 .. z0 + 2
  bool gm1, g0f, g1f, g2f;
  {
    (void)load_words(z0 - 2);
    const bool a = load_words(z0 - 1), b = load_words(z0), c = load_words(z0 + 1),
               d = load_words(z0 + 2);
    gm1 = __syncthreads_or(a);
    g0f = __syncthreads_or(b);
    g1f = __syncthreads_or(c);
    g2f = __syncthreads_or(d);
  }
  // raw phi: plane z0 - 2 where the ghosts of z0 - 1 read it, z0 - 1 over W2,
  // z0 over W1 (W2 near ghosts) with the owned pulls kept, and z0 + 1 where the
  // ghosts of z0 read it
  double g0c = 0.0, g0n = 0.0;
  C gc[QG], gn[QG];
#pragma unroll
  for (int i = 0; i < QG; ++i) gc[i] = gn[i] = C(0);
  if (gm1) raw_support(z0 - 2, z0 - 1);
  {
    C* fp = sphi + pslot(z0 - 1);
    const uint32_t* wp = sw + wslot(z0 - 1);
    const int qz = zof(z0 - 1);
    for (int m = tid; m < PL; m += NT) fp[m] = qz >= 0 ? raw_entry(wp, m, qz) : C(0);
  }
  raw_plane(z0, gm1 || g0f || g1f, g0c, gc);
  if (g0f) raw_support(z0 + 1, z0);
  __syncthreads();
  if (gm1) fill_ghosts(z0 - 1);
  if (g0f) fill_ghosts(z0);
  __syncthreads();

  for (int j = z0; j < z1; ++j) {
    P = P0;
    opaque(P);
    xo = x0 + lane;
    yo = y0 + ty;
    opaque(xo, yo);
    // S1
    const bool g3 = load_words(j + 3);
    // S2, S3
    raw_plane(j + 1, g0f || g1f || g2f, g0n, gn);
    if (g1f) raw_support(j + 2, j + 1);
    const bool g3f = __syncthreads_or(g3);
    // S4
    if (g1f) fill_ghosts(j + 1);
    __syncthreads();
    // S5
    const int qz = zof(j);
    const uint32_t w = sw[wslot(j) + tt];
    if (own_xy && (w & kZeta)) {
      const nidx n = G.idx(xo, yo, qz);
      nidx nb[Q];
      neighbours<L>(G, xo, yo, qz, nb);
      C f[Q];
      f[0] = C(FS::load_rest(fsrc, n));
#pragma unroll
      for (int i = 1; i < Q; ++i) f[i] = pull<L, FS>(fsrc, i, n, nb, w, P.scale_f);
      const int sm = pslot(j - 1), s0 = pslot(j), sp = pslot(j + 1);
      const int wm = wslot(j - 1), w0 = wslot(j), wpl = wslot(j + 1);
      auto pat = [&](int i) {
        return (L::cz(i) < 0 ? sm : (L::cz(i) > 0 ? sp : s0)) + tt + L::cx(i) + LX * L::cy(i);
      };
      auto wat = [&](int i) {
        return (L::cz(i) < 0 ? wm : (L::cz(i) > 0 ? wpl : w0)) + tt + L::cx(i) + LX * L::cy(i);
      };
      // mu and grad phi
      const C ph = sphi[s0 + tt];
      const C m = mu_of<L, C>(
          ph, [&](int i) { return sphi[pat(i)]; }, [&](int i) { return sw[wat(i)]; },
          [&]() { return wet_of<L::D, C>(w, P); }, P);
      C gx, gy, gz;
      grad_of<L, C>([&](int i) { return sphi[pat(i)]; }, gx, gy, gz);
      node_update<L, S, 0, O>(f, g0c, gc, ph, m, gx, gy, gz, w, n, fdst, gdst, sprev, nullptr,
                              nullptr, G, P, P.nt_store);
    }
    // the next plane's pulls become the current ones
    g0c = g0n;
#pragma unroll
    for (int i = 0; i < QG; ++i) gc[i] = gn[i];
    g0f = g1f;
    g1f = g2f;
    g2f = g3f;
  }
}


template <class L, int S, int TY, int TZ, bool O>
__global__ __launch_bounds__(64 * TY, fill_waves(64 * TY, 4)) void k_stepZ(
    const uint32_t* __restrict__ nodes, const void* __restrict__ fsrc,
    const void* __restrict__ gsrc, void* __restrict__ fdst, void* __restrict__ gdst,
    ComputeT<S>* __restrict__ sprev, Geo G, Phys P) {
  using T = MarchTile<TY>;
  __shared__ ComputeT<S> sphi[T::NL_PHI];
  __shared__ uint32_t sw[T::NL_WORD];
  const TileGrid TG(G, 64, TY, TZ);
  const int b = TileOrder{TG.nx, TG.ny, TG.nz, P.xcd_order}.tile(blockIdx.x);
  if (b < 0) return;
  int x0, y0, z0;
  TG.origin(b, x0, y0, z0);
  stepZ_tile<L, S, TY, TZ, O>(x0, y0, z0, nodes, fsrc, gsrc, fdst, gdst, sprev, G, P, sphi, sw);
}

template <class L, int S, int TY, int TZ, bool O>
__global__ __launch_bounds__(64 * TY, fill_waves(64 * TY, 5)) void k_stepC(
    const uint32_t* __restrict__ nodes, const void* __restrict__ fsrc,
    const void* __restrict__ gsrc, void* __restrict__ fdst, void* __restrict__ gdst,
    ComputeT<S>* __restrict__ sprev, const ComputeT<S>* __restrict__ phi, Geo G, Phys P) {
  using T = ColumnTile<L, S, TY, TZ>;
  __shared__ ComputeT<S> sphi[T::NL];
  __shared__ uint32_t sw[T::NL];
  const TileGrid TG(G, 64, TY, TZ);
  const int b = TileOrder{TG.nx, TG.ny, TG.nz, P.xcd_order}.tile(blockIdx.x);
  if (b < 0) return;
  int x0, y0, z0;
  TG.origin(b, x0, y0, z0);
  stepC_tile<L, S, TY, TZ, O>(x0, y0, z0, nodes, fsrc, gsrc, fdst, gdst, sprev, phi, G, P, sphi, sw);
}

// ------------------------------------------------------------------ batched step
// Many cases of one lattice and storage advance together over a device table
// of (case, tile) entries; each case has a descriptor with its geometry,
// physics and buffers.  One workgroup takes one entry, or (PERSIST) a fixed
// grid strides over the table.  The table and descriptors live in device
// memory and may change between launches (cases joining or leaving) without
// touching the launch arguments; with the fixed grid captured graphs stay
// valid, with one workgroup per entry the grid follows the table size.
struct Wall {
  int kind;          // 0 none, 1 plane, 2 ball
  double p[3], nrm[3], radius, width;
  double ref[3];     // coordinates are taken relative to this point
};

struct CaseDesc {
  Geo G;
  Phys P;
  const uint32_t* nodes;
  void* f[2];
  void* g[2];
  void* s;
  void* phi;         // phi array (split-step variants, diagnostics)
  void* snap;        // steady-state reference phi
  Wall W;            // wall of the contact-angle fit
  int cur0;          // buffer holding the current state when parity == 0
  int tile0, ntile;  // the member's entries in the tile table
  int pad_;
};

struct TileEntry {
  int case_id;
  int tile;          // tile index within the case, x-fastest
};

// Table entries of one workgroup: its own entry (the grid covers the table),
// or, with PERSIST, a grid-stride walk over the table by a fixed grid.
template <bool PERSIST, class Body>
__device__ inline void for_entries(int n, Body&& body) {
  if constexpr (PERSIST) {
    for (int e = blockIdx.x; e < n; e += gridDim.x) body(e);
  } else {
    if ((int)blockIdx.x < n) body((int)blockIdx.x);
  }
}

template <class L, int S, int BY, int BZ, int KY, int KZ, bool PERSIST = false>
__global__ __launch_bounds__(64 * BY * BZ) void k_step_group(
    const TileEntry* __restrict__ table, const int* __restrict__ ntiles,
    const CaseDesc* __restrict__ cases, int parity) {
  using T = StepTile<L, S, BY, BZ, KY, KZ>;
  __shared__ typename T::C sphi[T::NL];
  __shared__ uint32_t sw[T::NL];
  for_entries<PERSIST>(*ntiles, [&](int e) {
    const TileEntry te = table[e];
    const CaseDesc& cd = cases[te.case_id];
    const Geo G = cd.G;
    const int c = cd.cur0 ^ parity;
    int x0, y0, z0;
    TileGrid(G, T::TX, T::TY, T::TZ).origin(te.tile, x0, y0, z0);
    step_tile<L, S, BY, BZ, KY, KZ, true>(x0, y0, z0, cd.nodes, cd.f[c], cd.g[c],
                                    cd.f[1 - c], cd.g[1 - c], static_cast<ComputeT<S>*>(cd.s), G,
                                    cd.P, sphi, sw);
    __syncthreads();   // the next tile reuses the LDS arrays
  });
}


// Batched split step: the phi pass and the collide pass, each over the table.
template <class L, int S, int BY, int BZ, bool PERSIST = false>
__global__ __launch_bounds__(64 * BY * BZ) void k_phi_group(
    const TileEntry* __restrict__ table, const int* __restrict__ ntiles,
    const CaseDesc* __restrict__ cases, int parity) {
  const int TZ = (L::D == 3) ? BZ : 1;
  for_entries<PERSIST>(*ntiles, [&](int e) {
    const TileEntry te = table[e];
    const CaseDesc& cd = cases[te.case_id];
    const Geo G = cd.G;
    const int c = cd.cur0 ^ parity;
    int x0, y0, z0;
    TileGrid(G, 64, BY, TZ).origin(te.tile, x0, y0, z0);
    phi_tile<L, S, BY, BZ, true>(x0, y0, z0, cd.nodes, cd.g[c], static_cast<ComputeT<S>*>(cd.phi), G, cd.P);
  });
}

template <class L, int S, int BY, int BZ, bool PERSIST = false>
__global__ __launch_bounds__(64 * BY * BZ, stepB_waves(S, 64 * BY * BZ)) void k_stepB_group(
    const TileEntry* __restrict__ table, const int* __restrict__ ntiles,
    const CaseDesc* __restrict__ cases, int parity) {
  constexpr bool D3 = (L::D == 3);
  constexpr int NL = 66 * (BY + 2) * (D3 ? BZ + 2 : 1);
  __shared__ ComputeT<S> sphi[NL];
  __shared__ uint32_t sw[NL];
  const int TZ = D3 ? BZ : 1;
  for_entries<PERSIST>(*ntiles, [&](int e) {
    const TileEntry te = table[e];
    const CaseDesc& cd = cases[te.case_id];
    const Geo G = cd.G;
    const int c = cd.cur0 ^ parity;
    int x0, y0, z0;
    TileGrid(G, 64, BY, TZ).origin(te.tile, x0, y0, z0);
    stepB_tile<L, S, BY, BZ, true>(x0, y0, z0, cd.nodes, cd.f[c], cd.g[c], cd.f[1 - c], cd.g[1 - c],
                             static_cast<ComputeT<S>*>(cd.s),
                             static_cast<const ComputeT<S>*>(cd.phi), G, cd.P, sphi, sw);
    __syncthreads();
  });
}

template <class L, int S, int TY, int TZ, bool PERSIST = false>
__global__ __launch_bounds__(64 * TY, fill_waves(64 * TY, 5)) void k_stepC_group(
    const TileEntry* __restrict__ table, const int* __restrict__ ntiles,
    const CaseDesc* __restrict__ cases, int parity) {
  using T = ColumnTile<L, S, TY, TZ>;
  __shared__ ComputeT<S> sphi[T::NL];
  __shared__ uint32_t sw[T::NL];
  for_entries<PERSIST>(*ntiles, [&](int e) {
    const TileEntry te = table[e];
    const CaseDesc& cd = cases[te.case_id];
    const Geo G = cd.G;
    const int c = cd.cur0 ^ parity;
    int x0, y0, z0;
    TileGrid(G, 64, TY, TZ).origin(te.tile, x0, y0, z0);
    stepC_tile<L, S, TY, TZ, true>(x0, y0, z0, cd.nodes, cd.f[c], cd.g[c], cd.f[1 - c], cd.g[1 - c],
                             static_cast<ComputeT<S>*>(cd.s),
                             static_cast<const ComputeT<S>*>(cd.phi), G, cd.P, sphi, sw);
    __syncthreads();
  });
}

// Batched fused z-marching step: one column segment per table entry.
template <class L, int S, int TY, int TZ, bool PERSIST = false>
__global__ __launch_bounds__(64 * TY, fill_waves(64 * TY, 4)) void k_stepZ_group(
    const TileEntry* __restrict__ table, const int* __restrict__ ntiles,
    const CaseDesc* __restrict__ cases, int parity) {
  using T = MarchTile<TY>;
  __shared__ ComputeT<S> sphi[T::NL_PHI];
  __shared__ uint32_t sw[T::NL_WORD];
  for_entries<PERSIST>(*ntiles, [&](int e) {
    const TileEntry te = table[e];
    const CaseDesc& cd = cases[te.case_id];
    const Geo G = cd.G;
    const int c = cd.cur0 ^ parity;
    int x0, y0, z0;
    TileGrid(G, 64, TY, TZ).origin(te.tile, x0, y0, z0);
    stepZ_tile<L, S, TY, TZ, true>(x0, y0, z0, cd.nodes, cd.f[c], cd.g[c], cd.f[1 - c], cd.g[1 - c],
                                   static_cast<ComputeT<S>*>(cd.s), G, cd.P, sphi, sw);
    __syncthreads();
  });
}

// Batched ghost pass: one table entry's tile box (ghost_box) at a time.
template <class L, int S>
__global__ __launch_bounds__(kGhostThreads) void k_ghost_group(const TileEntry* __restrict__ table,
                                                                const int* __restrict__ ntiles,
                                                                const CaseDesc* __restrict__ cases,
                                                                int tx, int ty, int tz) {
  using C = ComputeT<S>;
  __shared__ int list[kGhostChunk];
  __shared__ int count;
  const int n = *ntiles;
  for (int e = blockIdx.x; e < n; e += gridDim.x) {
    const TileEntry te = table[e];
    const CaseDesc& cd = cases[te.case_id];
    const Geo G = cd.G;
    ghost_box<L, C>(cd.nodes, static_cast<C*>(cd.phi), G, C(cd.P.chi_a), TileGrid(G, tx, ty, tz),
                    te.tile, list, &count);
  }
}

// ------------------------------------------------------------------ init
// g at t = 0 is g_eq(phi0, mu0) after streaming; store it where the first pull
// will find it (the inverse of the pull map).  f = 0 is set by a memset.
template <class L, int S>
__global__ void k_init_g(const uint32_t* __restrict__ nodes, void* __restrict__ gdst,
                         const ComputeT<S>* __restrict__ phi, const ComputeT<S>* __restrict__ mu,
                         Geo G, Phys P) {
  using C = ComputeT<S>;
  int x, y, z;
  if (!node_coords(G, x, y, z)) return;
  const nidx n = G.idx(x, y, z);
  const uint32_t word = nodes[n];
  if (!(word & kZeta)) return;
  nidx nb[L::Q];
  neighbours<L>(G, x, y, z, nb);
  using GS = Set<S, true, L::G::Q>;
  using LG = typename L::G;          // velocity set of g
  const C am = C(P.alpha) * mu[n];
  GS::store_rest(gdst, n, (double)phi[n] - (1.0 - LG::w(0)) * (double)am);
#pragma unroll
  for (int i = 1; i < LG::Q; ++i) {
    const C geq = C(LG::w(i)) * am;
    const bool bb = (word >> (kLinkShift + i)) & 1u;
    if (bb)
      GS::store(gdst, LG::opp(i), n, geq, P.scale_g);
    else
      GS::store(gdst, i, nb[LG::opp(i)], geq, P.scale_g);
  }
}

// ------------------------------------------------------------------ reductions
// Record layout (doubles): see kRec* below.
enum {
  kRecMass = 0, kRecS, kRecResid, kRecNonfinite, kRecCount,
  kRecX, kRecY, kRecZ, kRecXX, kRecXY, kRecXZ, kRecYY, kRecYZ, kRecZZ,
  kRecXR, kRecYR, kRecZR, kRecRR, kRecAbsMax, kRecN
};

__device__ inline double wall_dist(const Wall& W, double x, double y, double z) {
  if (W.kind == 1)
    return (x - W.p[0]) * W.nrm[0] + (y - W.p[1]) * W.nrm[1] + (z - W.p[2]) * W.nrm[2];
  const double dx = x - W.p[0], dy = y - W.p[1], dz = z - W.p[2];
  return sqrt(dx * dx + dy * dy + dz * dz) - W.radius;
}

template <class C>
__device__ inline void add_point(double* acc, const Wall& W, double x, double y, double z) {
  if (W.kind == 0 || wall_dist(W, x, y, z) < W.width) return;
  const double X = x - W.ref[0], Y = y - W.ref[1], Z = z - W.ref[2];
  const double r2 = X * X + Y * Y + Z * Z;
  acc[kRecCount] += 1.0;
  acc[kRecX] += X; acc[kRecY] += Y; acc[kRecZ] += Z;
  acc[kRecXX] += X * X; acc[kRecXY] += X * Y; acc[kRecXZ] += X * Z;
  acc[kRecYY] += Y * Y; acc[kRecYZ] += Y * Z; acc[kRecZZ] += Z * Z;
  acc[kRecXR] += X * r2; acc[kRecYR] += Y * r2; acc[kRecZR] += Z * r2; acc[kRecRR] += r2;
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Mass of node n in FP64 from the stored populations: the FP64 rest population
// of g plus the moving ones (pulled as for phi) summed in FP64.  With FP32 or
// FP16 moving populations this is the exact mass of the stored state, which
// the compute-type phi (rounded to FP32) is not.
template <class L, int S>
__device__ inline double node_mass(const void* __restrict__ gsrc, const Geo& G, int x, int y,
                                   int z, nidx n, uint32_t w, float scale_g) {
  using GS = Set<S, true, L::G::Q, false>;   // 64-bit offsets: any buffer size
  nidx nb[L::Q];
  neighbours<L>(G, x, y, z, nb);
  double small = 0.0;
#pragma unroll
  for (int i = 1; i < L::G::Q; ++i)
    small += (double)pull<typename L::G, GS>(gsrc, i, n, nb, w, scale_g);
  return GS::load_rest(gsrc, n) + small;
}

// Contribution of node (x, y, z) to a diagnostics record.  Interface points lie
// on edges (x, x + e_a) inside the domain between two zeta = 1 nodes where
// exactly one phi is below 1/2 (no periodic seam).  The mass is taken from the
// stored populations (node_mass).
template <class L, int S>
__device__ inline void node_contrib(double* acc, const uint32_t* __restrict__ nodes,
                                    const void* __restrict__ gsrc,
                                    const ComputeT<S>* __restrict__ phi,
                                    const ComputeT<S>* __restrict__ s,
                                    ComputeT<S>* __restrict__ snap, int x, int y, int z,
                                    const Geo& G, float scale_g, const Wall& W, int update_snap) {
  const nidx n = G.idx(x, y, z);
  const uint32_t w = nodes[n];
  if (!(w & kZeta)) return;
  const double ph = (double)phi[n];
  acc[kRecMass] += node_mass<L, S>(gsrc, G, x, y, z, n, w, scale_g);
  acc[kRecS] += (double)s[n];
  const double sn = (double)snap[n];
  acc[kRecResid] = fmax(acc[kRecResid], fabs(ph - sn));
  acc[kRecAbsMax] = fmax(acc[kRecAbsMax], fabs(ph));
  if (!isfinite(ph) || !isfinite((double)s[n])) acc[kRecNonfinite] += 1.0;
  if (update_snap) snap[n] = phi[n];
  const double X = x - G.pad[0], Y = y - G.pad[1], Z = (L::D == 3) ? z - G.pad[2] : 0;
  const int P3[3] = {G.PX, G.PY, G.PZ};
  const int c3[3] = {x, y, z};
#pragma unroll
  for (int a = 0; a < L::D; ++a) {
    if (c3[a] + 1 >= P3[a]) continue;
    const nidx n2 = n + (a == 0 ? 1u : a == 1 ? (nidx)G.SX : (nidx)G.SX * (nidx)G.PY);
    if (!(nodes[n2] & kZeta)) continue;
    const double p2 = (double)phi[n2];
    if ((ph < 0.5) == (p2 < 0.5)) continue;
    const double t = (0.5 - ph) / (p2 - ph);
    add_point<ComputeT<S>>(acc, W, X + (a == 0 ? t : 0.0), Y + (a == 1 ? t : 0.0), Z + (a == 2 ? t : 0.0));
  }
}

// Workgroup reduction of per-thread records into out[0..kRecN) (sums, except
// the residual and |phi| maxima).  blockDim is a multiple of 64, at most 1024.
__device__ inline void block_record(double* acc, double* out) {
  __shared__ double red[16][kRecN];
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int lane = tid & 63, wv = tid >> 6;
  const int nw = (blockDim.x * blockDim.y * blockDim.z + 63) / 64;
#pragma unroll
  for (int k = 0; k < kRecN; ++k) {
    const double v = (k == kRecResid || k == kRecAbsMax) ? wave_max(acc[k]) : wave_sum(acc[k]);
    if (lane == 0) red[wv][k] = v;
  }
  __syncthreads();
  if (tid < kRecN) {
    double v = red[0][tid];
    for (int j = 1; j < nw; ++j)
      v = (tid == kRecResid || tid == kRecAbsMax) ? fmax(v, red[j][tid]) : v + red[j][tid];
    out[tid] = v;
  }
  __syncthreads();
}

// One partial record per workgroup (grid over the padded nodes).
template <class L, int S>
__global__ void k_reduce_partial(const uint32_t* __restrict__ nodes, const void* __restrict__ gsrc,
                                 const ComputeT<S>* __restrict__ phi,
                                 const ComputeT<S>* __restrict__ s, ComputeT<S>* __restrict__ snap,
                                 double* __restrict__ partial, Geo G, float scale_g, Wall W,
                                 int update_snap) {
  double acc[kRecN];
#pragma unroll
  for (int k = 0; k < kRecN; ++k) acc[k] = 0.0;
  int x, y, z;
  if (node_coords(G, x, y, z))
    node_contrib<L, S>(acc, nodes, gsrc, phi, s, snap, x, y, z, G, scale_g, W, update_snap);
  const long long b = blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z);
  block_record(acc, partial + b * kRecN);
}

// Sums nparts partial records in a fixed order (deterministic); one workgroup of 256.
template <int NR>
__global__ void k_reduce_final(const double* __restrict__ partial, long long nparts,
                               double* __restrict__ out) {
  static_assert(NR == kRecN, "record size");
  __shared__ double red[4][kRecN];
  double acc[kRecN];
#pragma unroll
  for (int k = 0; k < kRecN; ++k) acc[k] = 0.0;
  for (long long b = threadIdx.x; b < nparts; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < kRecN; ++k) {
      const double v = partial[b * kRecN + k];
      acc[k] = (k == kRecResid || k == kRecAbsMax) ? fmax(acc[k], v) : acc[k] + v;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kRecN; ++k) {
    const double v = (k == kRecResid || k == kRecAbsMax) ? wave_max(acc[k]) : wave_sum(acc[k]);
    if (lane == 0) red[wv][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < kRecN) {
    const int k = threadIdx.x;
    double v = red[0][k];
    for (int j = 1; j < (int)(blockDim.x / 64); ++j)
      v = (k == kRecResid || k == kRecAbsMax) ? fmax(v, red[j][k]) : v + red[j][k];
    out[k] = v;
  }
}


// ------------------------------------------------------------------ FP16 scale upkeep
// FP16-deviation storage keeps value * 2^k.  At diagnostics the host checks the
// largest stored magnitude of each set and, when it leaves a safe band, moves
// the scale by a power of two and rescales the stored populations in place.

// Largest stored magnitude |h| of the moving populations of f and of g over
// zeta = 1 nodes; one (f, g) pair per workgroup of 256 (grid-stride over the
// node slots).  Non-finite values are reported by the diagnostics record.
template <class L>
__global__ __launch_bounds__(256) void k_popmax(const uint32_t* __restrict__ nodes,
                                                const void* __restrict__ fbuf,
                                                const void* __restrict__ gbuf, long long nslots,
                                                float* __restrict__ partial) {
  using FS = Set<kF16Dev, false, L::Q>;
  using GS = Set<kF16Dev, true, L::G::Q>;
  double mf = 0.0, mg = 0.0;
  for (long long n = blockIdx.x * 256LL + threadIdx.x; n < nslots; n += 256LL * gridDim.x) {
    if (!(nodes[n] & kZeta)) continue;
    for (int i = 1; i < L::Q; ++i)
      mf = fmax(mf, (double)fabsf(__half2float(*FS::at(fbuf, i, (nidx)n))));
    for (int i = 1; i < L::G::Q; ++i)
      mg = fmax(mg, (double)fabsf(__half2float(*GS::at(gbuf, i, (nidx)n))));
  }
  mf = wave_max(mf);
  mg = wave_max(mg);
  __shared__ double red[4][2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[wv][0] = mf;
    red[wv][1] = mg;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double v = red[0][threadIdx.x];
    for (int j = 1; j < 4; ++j) v = fmax(v, red[j][threadIdx.x]);
    partial[2 * blockIdx.x + threadIdx.x] = (float)v;
  }
}

// Multiplies every stored moving population of one FP16 set of Q populations
// (g set when G) by factor, a power of two: exact unless the result leaves the
// FP16 normal range.
template <int Q, bool G>
__global__ __launch_bounds__(256) void k_rescale_half(void* __restrict__ buf, long long nblocks,
                                                      float factor) {
  using SetT = Set<kF16Dev, G, Q>;
  const long long per = (long long)(Q - 1) * kBlk;
  const long long total = nblocks * per;
  for (long long j = blockIdx.x * 256LL + threadIdx.x; j < total; j += 256LL * gridDim.x) {
    const long long b = j / per, r = j % per;
    __half* p = reinterpret_cast<__half*>(static_cast<unsigned char*>(buf) +
                                          b * (long long)SetT::kBlockBytes + SetT::kRestBytes) + r;
    *p = __float2half_rn(__half2float(*p) * factor);
  }
}

// ------------------------------------------------------------------ batched diagnostics
// For a group poll: phi of every member (same arithmetic as k_phi), then one
// partial record per table entry, then per member a fixed-order sum of its
// entries' partials.  Tiles are (tx, ty, tz) nodes, walked by 256 threads.
template <class L, int S>
__global__ __launch_bounds__(256) void k_phi_group_all(const TileEntry* __restrict__ table,
                                                        const int* __restrict__ ntiles,
                                                        const CaseDesc* __restrict__ cases,
                                                        int parity, int tx, int ty, int tz) {
  using C = ComputeT<S>;
  using GS = Set<S, true, L::G::Q, true>;
  const int n = *ntiles;
  const int tid = threadIdx.x;
  for (int e = blockIdx.x; e < n; e += gridDim.x) {
    const TileEntry te = table[e];
    const CaseDesc& cd = cases[te.case_id];
    const Geo G = cd.G;
    const void* gsrc = cd.g[cd.cur0 ^ parity];
    C* phi = static_cast<C*>(cd.phi);
    int x0, y0, z0;
    TileGrid(G, tx, ty, tz).origin(te.tile, x0, y0, z0);
    for (int m = tid; m < tx * ty * tz; m += 256) {
      const int x = x0 + m % tx, y = y0 + (m / tx) % ty, z = z0 + m / (tx * ty);
      if (x >= G.PX || y >= G.PY || z >= G.PZ) continue;
      const nidx nn = G.idx(x, y, z);
      const uint32_t w = cd.nodes[nn];
      if (!(w & kZeta)) continue;
      nidx nb[L::Q];
      neighbours<L>(G, x, y, z, nb);
      C small = C(0);
#pragma unroll
      for (int i = 1; i < L::G::Q; ++i) small += pull<typename L::G, GS>(gsrc, i, nn, nb, w, cd.P.scale_g);
      phi[nn] = C(GS::load_rest(gsrc, nn) + (double)small);
    }
  }
}

template <class L, int S>
__global__ __launch_bounds__(256) void k_reduce_group(const TileEntry* __restrict__ table,
                                                       const int* __restrict__ ntiles,
                                                       const CaseDesc* __restrict__ cases,
                                                       int parity, double* __restrict__ partial,
                                                       int tx, int ty, int tz, int update_snap) {
  using C = ComputeT<S>;
  const int n = *ntiles;
  const int tid = threadIdx.x;
  for (int e = blockIdx.x; e < n; e += gridDim.x) {
    const TileEntry te = table[e];
    const CaseDesc& cd = cases[te.case_id];
    const Geo G = cd.G;
    int x0, y0, z0;
    TileGrid(G, tx, ty, tz).origin(te.tile, x0, y0, z0);
    double acc[kRecN];
#pragma unroll
    for (int k = 0; k < kRecN; ++k) acc[k] = 0.0;
    for (int m = tid; m < tx * ty * tz; m += 256) {
      const int x = x0 + m % tx, y = y0 + (m / tx) % ty, z = z0 + m / (tx * ty);
      if (x >= G.PX || y >= G.PY || z >= G.PZ) continue;
      node_contrib<L, S>(acc, cd.nodes, cd.g[cd.cur0 ^ parity], static_cast<const C*>(cd.phi),
                         static_cast<const C*>(cd.s), static_cast<C*>(cd.snap), x, y, z, G,
                         cd.P.scale_g, cd.W, update_snap);
    }
    block_record(acc, partial + (long long)e * kRecN);
  }
}

// One workgroup of 256 per member: fixed-order sum of its table entries.
template <int NR>
__global__ __launch_bounds__(256) void k_reduce_final_group(const double* __restrict__ partial,
                                                             const CaseDesc* __restrict__ cases,
                                                             double* __restrict__ out) {
  static_assert(NR == kRecN, "record size");
  const CaseDesc& cd = cases[blockIdx.x];
  double acc[kRecN];
#pragma unroll
  for (int k = 0; k < kRecN; ++k) acc[k] = 0.0;
  for (int t = threadIdx.x; t < cd.ntile; t += blockDim.x) {
    const double* p = partial + (long long)(cd.tile0 + t) * kRecN;
#pragma unroll
    for (int k = 0; k < kRecN; ++k)
      acc[k] = (k == kRecResid || k == kRecAbsMax) ? fmax(acc[k], p[k]) : acc[k] + p[k];
  }
  block_record(acc, out + (long long)blockIdx.x * kRecN);
}

}  // namespace pflbm
