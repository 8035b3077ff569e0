// Kernel launchers for one case, dispatched on (lattice, storage).
#include "case.h"

namespace pflbm {

namespace {

dim3 grid_of(const Geo& G, dim3 t) {
  return dim3((G.PX + t.x - 1) / t.x, (G.PY + t.y - 1) / t.y, (G.PZ + t.z - 1) / t.z);
}

template <class L, int S>
struct Engine {
  using C = ComputeT<S>;

  static int phi(pflbm_case_s* h) {
    const Geo& G = h->dv.geo;
    if (h->o32)
      hipLaunchKernelGGL((k_phi<L, S, true>), grid_of(G, h->tile), h->tile, 0, h->stream, h->nodes,
                         h->g[h->cur], static_cast<C*>(h->phi), G, h->dv.phys);
    else
      hipLaunchKernelGGL((k_phi<L, S, false>), grid_of(G, h->tile), h->tile, 0, h->stream,
                         h->nodes, h->g[h->cur], static_cast<C*>(h->phi), G, h->dv.phys);
    PFLBM_HIP(hipGetLastError());
    return PFLBM_OK;
  }

  static size_t mu_lds(dim3 t) {
    const size_t lz = (L::D == 3) ? t.z + 4 : 1;
    return (size_t)(t.x + 4) * (t.y + 4) * lz * (sizeof(C) + sizeof(uint32_t));
  }

  static int mu(pflbm_case_s* h) {
    const Geo& G = h->dv.geo;
    hipLaunchKernelGGL((k_mu<L, C>), grid_of(G, h->tile), h->tile, mu_lds(h->tile), h->stream,
                       h->nodes, static_cast<C*>(h->phi), static_cast<C*>(h->mu), G, h->dv.phys);
    PFLBM_HIP(hipGetLastError());
    return PFLBM_OK;
  }

  static int collide(pflbm_case_s* h, int mode, void* out_p, void* out_u) {
    const Geo& G = h->dv.geo;
    const int c = h->cur;
    auto args = [&](auto kern) {
      hipLaunchKernelGGL(kern, grid_of(G, h->tile), h->tile, 0, h->stream, h->nodes, h->f[c],
                         h->g[c], h->f[1 - c], h->g[1 - c], static_cast<const C*>(h->phi),
                         static_cast<const C*>(h->mu), static_cast<C*>(h->s),
                         static_cast<C*>(out_p), static_cast<C*>(out_u), G, h->dv.phys);
    };
    if (mode == 0)
      args(k_collide<L, S, 0>);
    else if (mode == 1)
      args(k_collide<L, S, 1>);
    else
      args(k_collide<L, S, 2>);
    PFLBM_HIP(hipGetLastError());
    return PFLBM_OK;
  }

  template <int BY, int BZ, int KY, int KZ>
  static int step_v(pflbm_case_s* h) {
    const Geo& G = h->dv.geo;
    constexpr int TY = BY * KY, TZ = (L::D == 3) ? BZ * KZ : 1;
    const unsigned nbx = (G.PX + 63) / 64, nby = (G.PY + TY - 1) / TY, nbz = (G.PZ + TZ - 1) / TZ;
    const dim3 grid(nbx * nby * nbz, 1, 1);
    const dim3 block(64, BY, (L::D == 3) ? BZ : 1);
    const int c = h->cur;
    constexpr int bz = (L::D == 3) ? BZ : 1, kz = (L::D == 3) ? KZ : 1;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, grid, block, 0, h->stream, h->nodes, h->f[c], h->g[c], h->f[1 - c],
                         h->g[1 - c], static_cast<C*>(h->s), G, h->dv.phys);
    };
    if (h->o32) go(k_step<L, S, BY, bz, KY, kz, true>);
    else go(k_step<L, S, BY, bz, KY, kz, false>);
    PFLBM_HIP(hipGetLastError());
    return PFLBM_OK;
  }

  template <int BY, int BZ>
  static int split_v(pflbm_case_s* h) {
    const Geo& G = h->dv.geo;
    int rc = phi(h);
    if (rc) return rc;
    constexpr int bz = (L::D == 3) ? BZ : 1;
    const unsigned nbx = (G.PX + 63) / 64, nby = (G.PY + BY - 1) / BY, nbz = (G.PZ + bz - 1) / bz;
    const int c = h->cur;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(nbx * nby * nbz), dim3(64, BY, bz), 0, h->stream, h->nodes,
                         h->f[c], h->g[c], h->f[1 - c], h->g[1 - c], static_cast<C*>(h->s),
                         static_cast<const C*>(h->phi), G, h->dv.phys);
    };
    if (h->o32) go(k_stepB<L, S, BY, bz, true>);
    else go(k_stepB<L, S, BY, bz, false>);
    PFLBM_HIP(hipGetLastError());
    return PFLBM_OK;
  }

  template <int TY, int TZ>
  static int column_v(pflbm_case_s* h) {
    if constexpr (L::D == 3) {
      const Geo& G = h->dv.geo;
      int rc = phi(h);
      if (rc) return rc;
      const unsigned nbx = (G.PX + 63) / 64, nby = (G.PY + TY - 1) / TY, nbz = (G.PZ + TZ - 1) / TZ;
      const int c = h->cur;
      auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(nbx * nby * nbz), dim3(64, TY), 0, h->stream, h->nodes,
                           h->f[c], h->g[c], h->f[1 - c], h->g[1 - c], static_cast<C*>(h->s),
                           static_cast<const C*>(h->phi), G, h->dv.phys);
      };
      if (h->o32) go(k_stepC<L, S, TY, TZ, true>);
      else go(k_stepC<L, S, TY, TZ, false>);
      PFLBM_HIP(hipGetLastError());
      return PFLBM_OK;
    }
    return set_error(PFLBM_EINVAL, "z-marching variants are for D3Q19");
  }

  static int step_fused(pflbm_case_s* h) {
    if (L::D == 2) {
      switch (h->variant) {
        case 5: return split_v<4, 1>(h);
        case 6: return split_v<8, 1>(h);
        case 7: return split_v<16, 1>(h);
        case 0: return step_v<4, 1, 1, 1>(h);
        case 1: return step_v<4, 1, 2, 1>(h);
        case 2: return step_v<4, 1, 4, 1>(h);
        case 3: return step_v<8, 1, 2, 1>(h);
        case 4: return step_v<2, 1, 4, 1>(h);
        default: break;
      }
    } else {
      switch (h->variant) {
        case 0: return step_v<2, 2, 1, 1>(h);
        case 1: return step_v<2, 2, 2, 1>(h);
        case 2: return step_v<2, 2, 2, 2>(h);
        case 3: return step_v<4, 4, 1, 1>(h);
        case 4: return step_v<4, 2, 1, 2>(h);
        case 5: return split_v<4, 4>(h);
        case 6: return split_v<2, 2>(h);
        case 7: return split_v<4, 2>(h);
        case 8: return column_v<4, 16>(h);
        case 9: return column_v<8, 16>(h);
        case 10: return column_v<8, 32>(h);
        default: break;
      }
    }
    return set_error(PFLBM_EINVAL, "unknown step variant %d", h->variant);
  }

  static int init_g(pflbm_case_s* h) {
    const Geo& G = h->dv.geo;
    hipLaunchKernelGGL((k_init_g<L, S>), grid_of(G, h->tile), h->tile, 0, h->stream, h->nodes,
                       h->g[h->cur], static_cast<const C*>(h->phi), static_cast<const C*>(h->mu),
                       G, h->dv.phys);
    PFLBM_HIP(hipGetLastError());
    return PFLBM_OK;
  }

  static int reduce(pflbm_case_s* h, int update_snap) {
    const Geo& G = h->dv.geo;
    const dim3 t = h->tile;
    const dim3 gr = grid_of(G, t);
    hipLaunchKernelGGL((k_reduce_partial<L, C>), gr, t, 0, h->stream, h->nodes,
                       static_cast<const C*>(h->phi), static_cast<const C*>(h->s),
                       static_cast<C*>(h->snap), h->partial, G, h->dv.wall, update_snap);
    PFLBM_HIP(hipGetLastError());
    const long long nparts = (long long)gr.x * gr.y * gr.z;
    hipLaunchKernelGGL(k_reduce_final<kRecN>, dim3(1), dim3(256), 0, h->stream, h->partial, nparts,
                       h->rec);
    PFLBM_HIP(hipGetLastError());
    return PFLBM_OK;
  }
};

template <class L, int S>
struct GroupEngine {
  template <int BY, int BZ, int KY, int KZ>
  static int launch(const GroupLaunch& gl, int parity) {
    constexpr int bz = (L::D == 3) ? BZ : 1, kz = (L::D == 3) ? KZ : 1;
    hipLaunchKernelGGL((k_step_group<L, S, BY, bz, KY, kz>), dim3(gl.grid), dim3(64, BY, bz), 0,
                       gl.stream, gl.table, gl.ntiles, gl.cases, parity);
    PFLBM_HIP(hipGetLastError());
    return PFLBM_OK;
  }
  template <int BY, int BZ, int KY, int KZ>
  static int occupancy(int* blocks) {
    constexpr int bz = (L::D == 3) ? BZ : 1, kz = (L::D == 3) ? KZ : 1;
    PFLBM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, reinterpret_cast<const void*>(&k_step_group<L, S, BY, bz, KY, kz>), 64 * BY * bz, 0));
    return PFLBM_OK;
  }
  template <int BY, int BZ>
  static int launch_split(const GroupLaunch& gl, int parity) {
    constexpr int bz = (L::D == 3) ? BZ : 1;
    hipLaunchKernelGGL((k_phi_group<L, S, BY, bz>), dim3(gl.grid), dim3(64, BY, bz), 0, gl.stream,
                       gl.table, gl.ntiles, gl.cases, parity);
    PFLBM_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_stepB_group<L, S, BY, bz>), dim3(gl.grid), dim3(64, BY, bz), 0,
                       gl.stream, gl.table, gl.ntiles, gl.cases, parity);
    PFLBM_HIP(hipGetLastError());
    return PFLBM_OK;
  }
  template <int TY, int TZ>
  static int launch_column(const GroupLaunch& gl, int parity) {
    if constexpr (L::D == 3) {
      hipLaunchKernelGGL((k_phi_group_all<L, S>), dim3(gl.grid), dim3(256), 0, gl.stream,
                         gl.table, gl.ntiles, gl.cases, parity, 64, TY, TZ);
      PFLBM_HIP(hipGetLastError());
      hipLaunchKernelGGL((k_stepC_group<L, S, TY, TZ>), dim3(gl.grid), dim3(64, TY), 0, gl.stream,
                         gl.table, gl.ntiles, gl.cases, parity);
      PFLBM_HIP(hipGetLastError());
      return PFLBM_OK;
    }
    return set_error(PFLBM_EINVAL, "z-marching variants are for D3Q19");
  }
  template <int TY, int TZ>
  static int occupancy_column(int* blocks) {
    if constexpr (L::D == 3) {
      PFLBM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          blocks, reinterpret_cast<const void*>(&k_stepC_group<L, S, TY, TZ>), 64 * TY, 0));
      return PFLBM_OK;
    }
    return set_error(PFLBM_EINVAL, "z-marching variants are for D3Q19");
  }
  template <int BY, int BZ>
  static int occupancy_split(int* blocks) {
    constexpr int bz = (L::D == 3) ? BZ : 1;
    PFLBM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, reinterpret_cast<const void*>(&k_stepB_group<L, S, BY, bz>), 64 * BY * bz, 0));
    return PFLBM_OK;
  }
  static int go(const GroupLaunch& gl, int parity, int* occ) {
#define PFLBM_SPLIT(V, BY, BZ) \
  case V: return occ ? occupancy_split<BY, BZ>(occ) : launch_split<BY, BZ>(gl, parity);
#define PFLBM_COLUMN(V, TY, TZ) \
  case V: return occ ? occupancy_column<TY, TZ>(occ) : launch_column<TY, TZ>(gl, parity);
#define PFLBM_VARIANT(V, BY, BZ, KY, KZ) \
  case V: return occ ? occupancy<BY, BZ, KY, KZ>(occ) : launch<BY, BZ, KY, KZ>(gl, parity);
    if (L::D == 2) {
      switch (gl.variant) {
        PFLBM_VARIANT(0, 4, 1, 1, 1)
        PFLBM_VARIANT(1, 4, 1, 2, 1)
        PFLBM_VARIANT(2, 4, 1, 4, 1)
        PFLBM_VARIANT(3, 8, 1, 2, 1)
        PFLBM_VARIANT(4, 2, 1, 4, 1)
        PFLBM_SPLIT(5, 4, 1)
        PFLBM_SPLIT(6, 8, 1)
        PFLBM_SPLIT(7, 16, 1)
        default: break;
      }
    } else {
      switch (gl.variant) {
        PFLBM_VARIANT(0, 2, 2, 1, 1)
        PFLBM_VARIANT(1, 2, 2, 2, 1)
        PFLBM_VARIANT(2, 2, 2, 2, 2)
        PFLBM_VARIANT(3, 4, 4, 1, 1)
        PFLBM_VARIANT(4, 4, 2, 1, 2)
        PFLBM_SPLIT(5, 4, 4)
        PFLBM_SPLIT(6, 2, 2)
        PFLBM_SPLIT(7, 4, 2)
        PFLBM_COLUMN(8, 4, 16)
        PFLBM_COLUMN(9, 8, 16)
        PFLBM_COLUMN(10, 8, 32)
        default: break;
      }
    }
#undef PFLBM_VARIANT
#undef PFLBM_SPLIT
#undef PFLBM_COLUMN
    return set_error(PFLBM_EINVAL, "unknown step variant %d", gl.variant);
  }
};

template <template <class, int> class Fn, class... A>
int dispatch(pflbm_case_s* h, A... a) {
  const int lat = h->prm.lattice, st = h->prm.storage;
  if (lat == PFLBM_D2Q9) {
    if (st == PFLBM_FP64) return Fn<D2Q9, kF64>::go(h, a...);
    if (st == PFLBM_FP32) return Fn<D2Q9, kF32>::go(h, a...);
    if (st == PFLBM_FP16_DEV) return Fn<D2Q9, kF16Dev>::go(h, a...);
  } else {
    if (st == PFLBM_FP64) return Fn<D3Q19, kF64>::go(h, a...);
    if (st == PFLBM_FP32) return Fn<D3Q19, kF32>::go(h, a...);
    if (st == PFLBM_FP16_DEV) return Fn<D3Q19, kF16Dev>::go(h, a...);
  }
  return set_error(PFLBM_EUNSUPPORTED, "unsupported lattice/storage %d/%d", lat, st);
}

template <class L, int S> struct DoPhi { static int go(pflbm_case_s* h) { return Engine<L, S>::phi(h); } };
template <class L, int S> struct DoMu { static int go(pflbm_case_s* h) { return Engine<L, S>::mu(h); } };
template <class L, int S> struct DoCollide {
  static int go(pflbm_case_s* h, int m, void* p, void* u) { return Engine<L, S>::collide(h, m, p, u); }
};
template <class L, int S> struct DoStep { static int go(pflbm_case_s* h) { return Engine<L, S>::step_fused(h); } };
template <class L, int S> struct DoInit { static int go(pflbm_case_s* h) { return Engine<L, S>::init_g(h); } };
template <class L, int S> struct DoReduce {
  static int go(pflbm_case_s* h, int up) { return Engine<L, S>::reduce(h, up); }
};

}  // namespace

int run_phi(pflbm_case_s* h) { return dispatch<DoPhi>(h); }
int run_mu(pflbm_case_s* h) { return dispatch<DoMu>(h); }
int run_collide(pflbm_case_s* h, int mode, void* out_p, void* out_u) {
  return dispatch<DoCollide>(h, mode, out_p, out_u);
}
int run_init_g(pflbm_case_s* h) { return dispatch<DoInit>(h); }
int run_step_fused(pflbm_case_s* h) { return dispatch<DoStep>(h); }

namespace {
template <class L, int S>
int group_diag_t(const GroupLaunch& gl, int parity, int tx, int ty, int tz, double* partial,
                 double* out, int ncases, int update_snap) {
  using C = ComputeT<S>;
  hipLaunchKernelGGL((k_phi_group_all<L, S>), dim3(gl.grid), dim3(256), 0, gl.stream, gl.table,
                     gl.ntiles, gl.cases, parity, tx, ty, tz);
  PFLBM_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_reduce_group<L, C>), dim3(gl.grid), dim3(256), 0, gl.stream, gl.table,
                     gl.ntiles, gl.cases, partial, tx, ty, tz, update_snap);
  PFLBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_final_group<kRecN>, dim3(ncases), dim3(256), 0, gl.stream, partial,
                     gl.cases, out);
  PFLBM_HIP(hipGetLastError());
  return PFLBM_OK;
}
}  // namespace

int run_group_diag(const GroupLaunch& gl, int parity, int tx, int ty, int tz, double* partial,
                   double* out, int ncases, int update_snap) {
  if (ncases <= 0) return PFLBM_OK;
#define PFLBM_GD(LT, ST) \
  return group_diag_t<LT, ST>(gl, parity, tx, ty, tz, partial, out, ncases, update_snap)
  if (gl.lattice == PFLBM_D2Q9) {
    if (gl.storage == PFLBM_FP64) PFLBM_GD(D2Q9, kF64);
    if (gl.storage == PFLBM_FP32) PFLBM_GD(D2Q9, kF32);
    if (gl.storage == PFLBM_FP16_DEV) PFLBM_GD(D2Q9, kF16Dev);
  } else {
    if (gl.storage == PFLBM_FP64) PFLBM_GD(D3Q19, kF64);
    if (gl.storage == PFLBM_FP32) PFLBM_GD(D3Q19, kF32);
    if (gl.storage == PFLBM_FP16_DEV) PFLBM_GD(D3Q19, kF16Dev);
  }
#undef PFLBM_GD
  return set_error(PFLBM_EUNSUPPORTED, "unsupported lattice/storage %d/%d", gl.lattice, gl.storage);
}

int run_step_group(const GroupLaunch& gl, int parity, int* occupancy_blocks) {
  if (gl.lattice == PFLBM_D2Q9) {
    if (gl.storage == PFLBM_FP64) return GroupEngine<D2Q9, kF64>::go(gl, parity, occupancy_blocks);
    if (gl.storage == PFLBM_FP32) return GroupEngine<D2Q9, kF32>::go(gl, parity, occupancy_blocks);
    if (gl.storage == PFLBM_FP16_DEV) return GroupEngine<D2Q9, kF16Dev>::go(gl, parity, occupancy_blocks);
  } else {
    if (gl.storage == PFLBM_FP64) return GroupEngine<D3Q19, kF64>::go(gl, parity, occupancy_blocks);
    if (gl.storage == PFLBM_FP32) return GroupEngine<D3Q19, kF32>::go(gl, parity, occupancy_blocks);
    if (gl.storage == PFLBM_FP16_DEV) return GroupEngine<D3Q19, kF16Dev>::go(gl, parity, occupancy_blocks);
  }
  return set_error(PFLBM_EUNSUPPORTED, "unsupported lattice/storage %d/%d", gl.lattice, gl.storage);
}

int step_variant_count(int D) { return D == 2 ? 8 : 11; }

// Tile of each step variant: threads (64, by, bz), nodes (64, ty, tz).
int step_variant_tile(int D, int v, int tile[5]) {
  // variants 0-4: fused one-kernel step; 5-7: split step (phi pass + collide
  // pass); 8-10 (D3Q19 only): split step marching along z
  static const int t2[8][5] = {
      {4, 1, 64, 4, 1}, {4, 1, 64, 8, 1}, {4, 1, 64, 16, 1}, {8, 1, 64, 16, 1}, {2, 1, 64, 8, 1},
      {4, 1, 64, 4, 1}, {8, 1, 64, 8, 1}, {16, 1, 64, 16, 1}};
  static const int t3[11][5] = {
      {2, 2, 64, 2, 2}, {2, 2, 64, 4, 2}, {2, 2, 64, 4, 4}, {4, 4, 64, 4, 4}, {4, 2, 64, 4, 4},
      {4, 4, 64, 4, 4}, {2, 2, 64, 2, 2}, {4, 2, 64, 4, 2},
      {4, 1, 64, 4, 16}, {8, 1, 64, 8, 16}, {8, 1, 64, 8, 32}};
  if (v < 0 || v >= step_variant_count(D)) return -1;
  for (int k = 0; k < 5; ++k) tile[k] = D == 2 ? t2[v][k] : t3[v][k];
  return 0;
}

int run_reduce(pflbm_case_s* h, int update_snap, double* host_rec) {
  int rc = dispatch<DoReduce>(h, update_snap);
  if (rc) return rc;
  if (host_rec) {
    PFLBM_HIP(hipMemcpyAsync(host_rec, h->rec, kRecN * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream));
    PFLBM_HIP(hipStreamSynchronize(h->stream));
  }
  return PFLBM_OK;
}

int run_step_eager(pflbm_case_s* h) {
  int rc;
  if (h->variant >= 0) {
    if ((rc = run_step_fused(h))) return rc;
    h->cur ^= 1;
    h->step += 1;
    return PFLBM_OK;
  }
  if ((rc = run_phi(h))) return rc;
  if ((rc = run_mu(h))) return rc;
  if ((rc = run_collide(h, 0, nullptr, nullptr))) return rc;
  h->cur ^= 1;
  h->step += 1;
  return PFLBM_OK;
}

}  // namespace pflbm
