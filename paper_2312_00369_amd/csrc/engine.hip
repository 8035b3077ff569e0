// Kernel launchers for one case or a group, dispatched on the lattice (each
// lattice's launchers live in engine_<lattice>.hip) and the storage type.
#include <algorithm>

#include "case.h"

namespace pflbm {

const LatticeEntry* lattice_entry_d2q9();
const LatticeEntry* lattice_entry_d3q19();
const LatticeEntry* lattice_entry_d3q19g7();

namespace {
const LatticeEntry* entry_of(int lattice) {
  if (lattice == PFLBM_D2Q9) return lattice_entry_d2q9();
  if (lattice == PFLBM_D3Q19) return lattice_entry_d3q19();
  if (lattice == PFLBM_D3Q19_D3Q7) return lattice_entry_d3q19g7();
  return nullptr;
}
}  // namespace

#define PFLBM_ENTRY(lat)                                                           \
  const LatticeEntry* e = entry_of(lat);                                          \
  if (!e) return set_error(PFLBM_EUNSUPPORTED, "unsupported lattice %d", (lat));

int run_phi(pflbm_case_s* h) { PFLBM_ENTRY(h->prm.lattice) return e->phi(h); }
int run_mu(pflbm_case_s* h) { PFLBM_ENTRY(h->prm.lattice) return e->mu(h); }
int run_collide(pflbm_case_s* h, int mode, void* out_p, void* out_u) {
  PFLBM_ENTRY(h->prm.lattice) return e->collide(h, mode, out_p, out_u);
}
int run_init_g(pflbm_case_s* h) { PFLBM_ENTRY(h->prm.lattice) return e->init_g(h); }
int run_step_fused(pflbm_case_s* h) { PFLBM_ENTRY(h->prm.lattice) return e->step(h); }

int run_group_diag(const GroupLaunch& gl, int parity, int tx, int ty, int tz, double* partial,
                   double* out, int ncases, int update_snap) {
  if (ncases <= 0) return PFLBM_OK;
  PFLBM_ENTRY(gl.lattice) return e->group_diag(gl, parity, tx, ty, tz, partial, out, ncases,
                                               update_snap);
}

int run_step_group(const GroupLaunch& gl, int parity, int* occupancy_blocks) {
  PFLBM_ENTRY(gl.lattice) return e->group_step(gl, parity, occupancy_blocks);
}

int run_popmax(pflbm_case_s* h, float out[2]) {
  PFLBM_ENTRY(h->prm.lattice)
  int rc = e->popmax(h);
  if (rc) return rc;
  float part[2 * kPopmaxBlocks];
  PFLBM_HIP(hipMemcpyAsync(part, h->popmax, sizeof part, hipMemcpyDeviceToHost, h->stream));
  PFLBM_HIP(hipStreamSynchronize(h->stream));
  out[0] = out[1] = 0.0f;
  for (int b = 0; b < kPopmaxBlocks; ++b) {
    out[0] = std::max(out[0], part[2 * b]);
    out[1] = std::max(out[1], part[2 * b + 1]);
  }
  return PFLBM_OK;
}

int run_rescale(pflbm_case_s* h, int set_g, float factor) {
  PFLBM_ENTRY(h->prm.lattice) return e->rescale(h, set_g, factor);
}

#undef PFLBM_ENTRY

int step_variant_count(int D) { return D == 2 ? 8 : 13; }

// Tile of each step variant: threads (64, by, bz), nodes (64, ty, tz).
int step_variant_tile(int D, int v, int tile[5]) {
  // variants 0-4: fused one-kernel step; 5-7: split step (phi pass + collide
  // pass); 8-10 (3D only): split step marching along z; 11-12 (3D only): fused
  // one-kernel step marching along z
  static const int t2[8][5] = {
      {4, 1, 64, 4, 1}, {4, 1, 64, 8, 1}, {4, 1, 64, 16, 1}, {8, 1, 64, 16, 1}, {2, 1, 64, 8, 1},
      {4, 1, 64, 4, 1}, {8, 1, 64, 8, 1}, {16, 1, 64, 16, 1}};
  static const int t3[13][5] = {
      {2, 2, 64, 2, 2}, {2, 2, 64, 4, 2}, {2, 2, 64, 4, 4}, {4, 4, 64, 4, 4}, {4, 2, 64, 4, 4},
      {4, 4, 64, 4, 4}, {2, 2, 64, 2, 2}, {4, 2, 64, 4, 2},
      {4, 1, 64, 4, 16}, {8, 1, 64, 8, 16}, {8, 1, 64, 8, 32},
      {4, 1, 64, 4, 32}, {8, 1, 64, 8, 32}};
  if (v < 0 || v >= step_variant_count(D)) return -1;
  for (int k = 0; k < 5; ++k) tile[k] = D == 2 ? t2[v][k] : t3[v][k];
  return 0;
}

int run_reduce(pflbm_case_s* h, int update_snap, double* host_rec) {
  const LatticeEntry* e = entry_of(h->prm.lattice);
  if (!e) return set_error(PFLBM_EUNSUPPORTED, "unsupported lattice %d", h->prm.lattice);
  int rc = e->reduce(h, update_snap);
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
