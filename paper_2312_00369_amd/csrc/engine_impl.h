// Kernel launchers of one lattice: Engine (one case) and GroupEngine (a
// batch), templated on lattice and storage, and the table of entry points
// each per-lattice source file instantiates (engine_<lattice>.hip).
#pragma once
#include <algorithm>

#include "case.h"

namespace pflbm {

namespace {

// Grid of the one-thread-per-slot kernels: x runs over slots XO .. XO + PX - 1
// of each row (node_coords subtracts XO).
dim3 grid_of(const Geo& G, dim3 t) {
  return dim3((G.PX + G.XO + t.x - 1) / t.x, (G.PY + t.y - 1) / t.y, (G.PZ + t.z - 1) / t.z);
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

  // ghost phi into the phi array (split step, after phi)
  static int ghost(pflbm_case_s* h) {
    if (!h->nghost) return PFLBM_OK;
    const Geo& G = h->dv.geo;
    const long long nb = h->nghost_blocks;
    const int face_wg = G.per[0] ? 0 : (2 * G.PY * G.PZ + kGhostThreads - 1) / kGhostThreads;
    const int list_wg = (int)std::min<long long>((nb + 7) / 8, 2048);
    hipLaunchKernelGGL((k_ghost<L, C>), dim3(face_wg + list_wg), dim3(kGhostThreads), 0,
                       h->stream, h->nodes, static_cast<C*>(h->phi), h->gblocks, (int)nb, face_wg,
                       G, h->dv.phys);
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
    const TileGrid TG(G, 64, TY, TZ);
    const dim3 grid(TileOrder{TG.nx, TG.ny, TG.nz, h->dv.phys.xcd_order}.grid(), 1, 1);
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
    if (!rc) rc = ghost(h);
    if (rc) return rc;
    constexpr int bz = (L::D == 3) ? BZ : 1;
    const TileGrid TG(G, 64, BY, bz);
    const unsigned ngrid = TileOrder{TG.nx, TG.ny, TG.nz, h->dv.phys.xcd_order}.grid();
    const int c = h->cur;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(ngrid), dim3(64, BY, bz), 0, h->stream, h->nodes,
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
      if (!rc) rc = ghost(h);
      if (rc) return rc;
      const TileGrid TG(G, 64, TY, TZ);
      const unsigned ngrid = TileOrder{TG.nx, TG.ny, TG.nz, h->dv.phys.xcd_order}.grid();
      const int c = h->cur;
      auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(ngrid), dim3(64, TY), 0, h->stream, h->nodes,
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

  template <int TY, int TZ>
  static int march_v(pflbm_case_s* h) {
    if constexpr (L::D == 3) {
      const Geo& G = h->dv.geo;
      const TileGrid TG(G, 64, TY, TZ);
      const unsigned ngrid = TileOrder{TG.nx, TG.ny, TG.nz, h->dv.phys.xcd_order}.grid();
      const int c = h->cur;
      auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(ngrid), dim3(64, TY), 0, h->stream, h->nodes,
                           h->f[c], h->g[c], h->f[1 - c], h->g[1 - c], static_cast<C*>(h->s), G,
                           h->dv.phys);
      };
      if (h->o32) go(k_stepZ<L, S, TY, TZ, true>);
      else go(k_stepZ<L, S, TY, TZ, false>);
      PFLBM_HIP(hipGetLastError());
      return PFLBM_OK;
    }
    return set_error(PFLBM_EINVAL, "z-marching variants are for 3D lattices");
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
        case 11: return march_v<4, 32>(h);
        case 12: return march_v<8, 32>(h);
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
    hipLaunchKernelGGL((k_reduce_partial<L, S>), gr, t, 0, h->stream, h->nodes, h->g[h->cur],
                       static_cast<const C*>(h->phi), static_cast<const C*>(h->s),
                       static_cast<C*>(h->snap), h->partial, G, h->dv.phys.scale_g, h->dv.wall,
                       update_snap);
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
  // gl.persist: a fixed grid strides over the table (the PERSIST kernels);
  // otherwise one workgroup per table entry.  The occupancy queries are for
  // the persistent kernels, whose grid they size.
  template <int BY, int BZ, int KY, int KZ>
  static int launch(const GroupLaunch& gl, int parity) {
    constexpr int bz = (L::D == 3) ? BZ : 1, kz = (L::D == 3) ? KZ : 1;
    if (gl.persist)
      hipLaunchKernelGGL((k_step_group<L, S, BY, bz, KY, kz, true>), dim3(gl.grid),
                         dim3(64, BY, bz), 0, gl.stream, gl.table, gl.ntiles, gl.cases, parity);
    else
      hipLaunchKernelGGL((k_step_group<L, S, BY, bz, KY, kz, false>), dim3(gl.grid),
                         dim3(64, BY, bz), 0, gl.stream, gl.table, gl.ntiles, gl.cases, parity);
    PFLBM_HIP(hipGetLastError());
    return PFLBM_OK;
  }
  template <int BY, int BZ, int KY, int KZ>
  static int occupancy(int* blocks) {
    constexpr int bz = (L::D == 3) ? BZ : 1, kz = (L::D == 3) ? KZ : 1;
    PFLBM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, reinterpret_cast<const void*>(&k_step_group<L, S, BY, bz, KY, kz, true>),
        64 * BY * bz, 0));
    return PFLBM_OK;
  }
  template <int BY, int BZ>
  static int launch_split(const GroupLaunch& gl, int parity) {
    constexpr int bz = (L::D == 3) ? BZ : 1;
    if (gl.persist)
      hipLaunchKernelGGL((k_phi_group<L, S, BY, bz, true>), dim3(gl.grid), dim3(64, BY, bz), 0,
                         gl.stream, gl.table, gl.ntiles, gl.cases, parity);
    else
      hipLaunchKernelGGL((k_phi_group<L, S, BY, bz, false>), dim3(gl.grid), dim3(64, BY, bz), 0,
                         gl.stream, gl.table, gl.ntiles, gl.cases, parity);
    PFLBM_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_ghost_group<L, S>), dim3(gl.grid), dim3(kGhostThreads), 0, gl.stream,
                       gl.table, gl.ntiles, gl.cases, 64, BY, bz);
    PFLBM_HIP(hipGetLastError());
    if (gl.persist)
      hipLaunchKernelGGL((k_stepB_group<L, S, BY, bz, true>), dim3(gl.grid), dim3(64, BY, bz), 0,
                         gl.stream, gl.table, gl.ntiles, gl.cases, parity);
    else
      hipLaunchKernelGGL((k_stepB_group<L, S, BY, bz, false>), dim3(gl.grid), dim3(64, BY, bz),
                         0, gl.stream, gl.table, gl.ntiles, gl.cases, parity);
    PFLBM_HIP(hipGetLastError());
    return PFLBM_OK;
  }
  template <int TY, int TZ>
  static int launch_column(const GroupLaunch& gl, int parity) {
    if constexpr (L::D == 3) {
      hipLaunchKernelGGL((k_phi_group_all<L, S>), dim3(gl.grid), dim3(256), 0, gl.stream,
                         gl.table, gl.ntiles, gl.cases, parity, 64, TY, TZ);
      PFLBM_HIP(hipGetLastError());
      hipLaunchKernelGGL((k_ghost_group<L, S>), dim3(gl.grid), dim3(kGhostThreads), 0, gl.stream,
                         gl.table, gl.ntiles, gl.cases, 64, TY, TZ);
      PFLBM_HIP(hipGetLastError());
      if (gl.persist)
        hipLaunchKernelGGL((k_stepC_group<L, S, TY, TZ, true>), dim3(gl.grid), dim3(64, TY), 0,
                           gl.stream, gl.table, gl.ntiles, gl.cases, parity);
      else
        hipLaunchKernelGGL((k_stepC_group<L, S, TY, TZ, false>), dim3(gl.grid), dim3(64, TY), 0,
                           gl.stream, gl.table, gl.ntiles, gl.cases, parity);
      PFLBM_HIP(hipGetLastError());
      return PFLBM_OK;
    }
    return set_error(PFLBM_EINVAL, "z-marching variants are for D3Q19");
  }
  template <int TY, int TZ>
  static int launch_march(const GroupLaunch& gl, int parity) {
    if constexpr (L::D == 3) {
      if (gl.persist)
        hipLaunchKernelGGL((k_stepZ_group<L, S, TY, TZ, true>), dim3(gl.grid), dim3(64, TY), 0,
                           gl.stream, gl.table, gl.ntiles, gl.cases, parity);
      else
        hipLaunchKernelGGL((k_stepZ_group<L, S, TY, TZ, false>), dim3(gl.grid), dim3(64, TY), 0,
                           gl.stream, gl.table, gl.ntiles, gl.cases, parity);
      PFLBM_HIP(hipGetLastError());
      return PFLBM_OK;
    }
    return set_error(PFLBM_EINVAL, "z-marching variants are for 3D lattices");
  }
  template <int TY, int TZ>
  static int occupancy_march(int* blocks) {
    if constexpr (L::D == 3) {
      PFLBM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          blocks, reinterpret_cast<const void*>(&k_stepZ_group<L, S, TY, TZ, true>), 64 * TY, 0));
      return PFLBM_OK;
    }
    return set_error(PFLBM_EINVAL, "z-marching variants are for 3D lattices");
  }
  template <int TY, int TZ>
  static int occupancy_column(int* blocks) {
    if constexpr (L::D == 3) {
      PFLBM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          blocks, reinterpret_cast<const void*>(&k_stepC_group<L, S, TY, TZ, true>), 64 * TY, 0));
      return PFLBM_OK;
    }
    return set_error(PFLBM_EINVAL, "z-marching variants are for D3Q19");
  }
  template <int BY, int BZ>
  static int occupancy_split(int* blocks) {
    constexpr int bz = (L::D == 3) ? BZ : 1;
    PFLBM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, reinterpret_cast<const void*>(&k_stepB_group<L, S, BY, bz, true>), 64 * BY * bz,
        0));
    return PFLBM_OK;
  }
  static int go(const GroupLaunch& gl, int parity, int* occ) {
#define PFLBM_SPLIT(V, BY, BZ) \
  case V: return occ ? occupancy_split<BY, BZ>(occ) : launch_split<BY, BZ>(gl, parity);
#define PFLBM_COLUMN(V, TY, TZ) \
  case V: return occ ? occupancy_column<TY, TZ>(occ) : launch_column<TY, TZ>(gl, parity);
#define PFLBM_MARCH(V, TY, TZ) \
  case V: return occ ? occupancy_march<TY, TZ>(occ) : launch_march<TY, TZ>(gl, parity);
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
        PFLBM_MARCH(11, 4, 32)
        PFLBM_MARCH(12, 8, 32)
        default: break;
      }
    }
#undef PFLBM_VARIANT
#undef PFLBM_SPLIT
#undef PFLBM_COLUMN
#undef PFLBM_MARCH
    return set_error(PFLBM_EINVAL, "unknown step variant %d", gl.variant);
  }
};

template <class L, int S>
int group_diag_t(const GroupLaunch& gl, int parity, int tx, int ty, int tz, double* partial,
                 double* out, int ncases, int update_snap) {
  hipLaunchKernelGGL((k_phi_group_all<L, S>), dim3(gl.grid), dim3(256), 0, gl.stream, gl.table,
                     gl.ntiles, gl.cases, parity, tx, ty, tz);
  PFLBM_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_reduce_group<L, S>), dim3(gl.grid), dim3(256), 0, gl.stream, gl.table,
                     gl.ntiles, gl.cases, parity, partial, tx, ty, tz, update_snap);
  PFLBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_final_group<kRecN>, dim3(ncases), dim3(256), 0, gl.stream, partial,
                     gl.cases, out);
  PFLBM_HIP(hipGetLastError());
  return PFLBM_OK;
}

// Entry points of lattice L, dispatched on the storage type.
template <class L>
struct LatticeImpl {
  template <template <class, int> class Fn, class... A>
  static int by_storage(int st, A... a) {
    if (st == PFLBM_FP64) return Fn<L, kF64>::go(a...);
    if (st == PFLBM_FP32) return Fn<L, kF32>::go(a...);
    if (st == PFLBM_FP16_DEV) return Fn<L, kF16Dev>::go(a...);
    return set_error(PFLBM_EUNSUPPORTED, "unsupported storage %d", st);
  }
  template <class L2, int S> struct Phi { static int go(pflbm_case_s* h) { return Engine<L2, S>::phi(h); } };
  template <class L2, int S> struct Mu { static int go(pflbm_case_s* h) { return Engine<L2, S>::mu(h); } };
  template <class L2, int S> struct Collide {
    static int go(pflbm_case_s* h, int m, void* p, void* u) { return Engine<L2, S>::collide(h, m, p, u); }
  };
  template <class L2, int S> struct Step { static int go(pflbm_case_s* h) { return Engine<L2, S>::step_fused(h); } };
  template <class L2, int S> struct Init { static int go(pflbm_case_s* h) { return Engine<L2, S>::init_g(h); } };
  template <class L2, int S> struct Reduce {
    static int go(pflbm_case_s* h, int up) { return Engine<L2, S>::reduce(h, up); }
  };
  template <class L2, int S> struct GStep {
    static int go(const GroupLaunch* gl, int parity, int* occ) {
      return GroupEngine<L2, S>::go(*gl, parity, occ);
    }
  };
  template <class L2, int S> struct GDiag {
    static int go(const GroupLaunch* gl, int parity, int tx, int ty, int tz, double* partial,
                  double* out, int ncases, int update_snap) {
      return group_diag_t<L2, S>(*gl, parity, tx, ty, tz, partial, out, ncases, update_snap);
    }
  };
  static int phi(pflbm_case_s* h) { return by_storage<Phi>(h->prm.storage, h); }
  static int mu(pflbm_case_s* h) { return by_storage<Mu>(h->prm.storage, h); }
  static int collide(pflbm_case_s* h, int m, void* p, void* u) {
    return by_storage<Collide>(h->prm.storage, h, m, p, u);
  }
  static int step(pflbm_case_s* h) { return by_storage<Step>(h->prm.storage, h); }
  static int init_g(pflbm_case_s* h) { return by_storage<Init>(h->prm.storage, h); }
  static int reduce(pflbm_case_s* h, int up) { return by_storage<Reduce>(h->prm.storage, h, up); }
  static int group_step(const GroupLaunch& gl, int parity, int* occ) {
    return by_storage<GStep>(gl.storage, &gl, parity, occ);
  }
  static int group_diag(const GroupLaunch& gl, int parity, int tx, int ty, int tz, double* partial,
                        double* out, int ncases, int update_snap) {
    return by_storage<GDiag>(gl.storage, &gl, parity, tx, ty, tz, partial, out, ncases,
                             update_snap);
  }
  // FP16-deviation storage: per-workgroup maxima of the stored magnitudes
  // (kPopmaxBlocks pairs in h->popmax), and the in-place rescale of one set.
  static int popmax(pflbm_case_s* h) {
    const int c = h->cur;
    hipLaunchKernelGGL((k_popmax<L>), dim3(kPopmaxBlocks), dim3(256), 0, h->stream, h->nodes,
                       h->f[c], h->g[c], h->dv.N, h->popmax);
    PFLBM_HIP(hipGetLastError());
    return PFLBM_OK;
  }
  static int rescale(pflbm_case_s* h, int set_g, float factor) {
    const long long nblocks = h->dv.geo.NQ / kBlk;
    void* buf = set_g ? h->g[h->cur] : h->f[h->cur];
    if (set_g)
      hipLaunchKernelGGL((k_rescale_half<L::G::Q, true>), dim3(1024), dim3(256), 0, h->stream, buf,
                         nblocks, factor);
    else
      hipLaunchKernelGGL((k_rescale_half<L::Q, false>), dim3(1024), dim3(256), 0, h->stream, buf,
                         nblocks, factor);
    PFLBM_HIP(hipGetLastError());
    return PFLBM_OK;
  }
  static const LatticeEntry* entry() {
    static const LatticeEntry e = {phi, mu, collide, step, init_g, reduce, group_step, group_diag,
                                   popmax, rescale};
    return &e;
  }
};

}  // namespace

}  // namespace pflbm
