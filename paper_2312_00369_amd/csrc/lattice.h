// Velocity sets used by the kernels and the host classifier.
//
// D2Q9 (Sec. 2.1.2, Eq. ci): rest, four axis and four diagonal vectors,
// weights 4/9, 1/9, 1/36.  D3Q19 (Eq. 3ci): rest, six axis and twelve edge
// vectors, weights 1/3, 1/18, 1/36.  c_s^2 = 1/3 for both.  D3Q7 (Sec. 2.1.3,
// the set named for the Cahn-Hilliard LBE in 3D): rest and six axis vectors,
// weights 1/4, 1/8, c_s^2 = 1/4; its vectors are the first seven of D3Q19 in
// the same order, so neighbour indices and link bits are shared.
// k_i is the bracket of the phase source G_i (Eq. F_i):
//   k_i = -1 + (|c_i|^2 - D c_s^2) / (2 c_s^2)
// which is -2, -1/2, 1 for D2Q9, -5/2, -1, 1/2 for D3Q19 and -5/2, -1/2 for D3Q7.
// Each case lattice names the set of its g populations as G.
#pragma once

#include <hip/hip_runtime.h>

namespace pflbm {

struct D2Q9 {
  using G = D2Q9;
  static constexpr int D = 2;
  static constexpr int Q = 9;
  static constexpr double cs2 = 1.0 / 3.0;
  __host__ __device__ static constexpr int cx(int i) {
    constexpr int v[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    return v[i];
  }
  __host__ __device__ static constexpr int cy(int i) {
    constexpr int v[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    return v[i];
  }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr int opp(int i) {
    constexpr int v[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    return v[i];
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
  __host__ __device__ static constexpr double k(int i) {
    return i == 0 ? -2.0 : (i < 5 ? -0.5 : 1.0);
  }
};

struct D3Q19 {
  using G = D3Q19;
  static constexpr int D = 3;
  static constexpr int Q = 19;
  static constexpr double cs2 = 1.0 / 3.0;
  __host__ __device__ static constexpr int cx(int i) {
    constexpr int v[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[i];
  }
  __host__ __device__ static constexpr int cy(int i) {
    constexpr int v[19] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[i];
  }
  __host__ __device__ static constexpr int cz(int i) {
    constexpr int v[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
    return v[i];
  }
  __host__ __device__ static constexpr int opp(int i) {
    constexpr int v[19] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
    return v[i];
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  __host__ __device__ static constexpr double k(int i) {
    return i == 0 ? -2.5 : (i < 7 ? -1.0 : 0.5);
  }
};

struct D3Q7 {
  using G = D3Q7;
  static constexpr int D = 3;
  static constexpr int Q = 7;
  static constexpr double cs2 = 1.0 / 4.0;
  __host__ __device__ static constexpr int cx(int i) { return D3Q19::cx(i); }
  __host__ __device__ static constexpr int cy(int i) { return D3Q19::cy(i); }
  __host__ __device__ static constexpr int cz(int i) { return D3Q19::cz(i); }
  __host__ __device__ static constexpr int opp(int i) { return D3Q19::opp(i); }
  __host__ __device__ static constexpr double w(int i) { return i == 0 ? 0.25 : 0.125; }
  __host__ __device__ static constexpr double k(int i) { return i == 0 ? -2.5 : -0.5; }
};

// D3Q19 for f and the stencils, D3Q7 for g.
struct D3Q19G7 : D3Q19 {
  using G = D3Q7;
};

// hydrodynamic c_s^2 (both hydrodynamic sets)
constexpr double kCs2 = 1.0 / 3.0;

// Node word bits (one uint32 per padded node).
constexpr unsigned kZeta = 1u;        // fluid or boundary node: carries f and g
constexpr unsigned kFluid = 2u;       // epsilon = 1
constexpr unsigned kGhost = 4u;       // zeta = 0 node one link from a zeta = 1 node
constexpr int kLinkShift = 8;         // bit kLinkShift + i: node - c_i is zeta = 0
// Wall-wetting table entry of a node (0: the case's value): 10 bits, the low 5
// in bits 27..31 and the high 5 in bits 3..7 (both unused otherwise).
constexpr int kWetEntries = 1024;
__host__ __device__ constexpr unsigned wet_entry(unsigned word) {
  return (word >> 27) | ((word << 2) & 0x3e0u);
}
__host__ __device__ constexpr unsigned wet_bits(unsigned k) {
  return ((k & 31u) << 27) | ((k >> 5) << 3);
}

}  // namespace pflbm
