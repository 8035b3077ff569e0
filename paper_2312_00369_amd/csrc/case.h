// Internal host-side definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pflbm.h"
#include "kernels.h"

namespace pflbm {

// Thread-local error text; set_error returns its code so call sites can
// `return set_error(...)`.
int set_error(int code, const char* fmt, ...);
void clear_error();

#define PFLBM_HIP(call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::pflbm::set_error(PFLBM_EDEVICE, "%s failed: %s (%s:%d)", #call,       \
                                hipGetErrorString(e_), __FILE__, __LINE__);          \
  } while (0)

struct Layout {
  size_t nodes, f[2], g[2], s, phi, mu, snap, partial, rec, popmax, wet, gblocks, total;
  size_t f_bytes, g_bytes;   // one f buffer, one g buffer
  size_t c_bytes;     // one compute-type field
  long long nparts;   // reduction partial records
};

// Geometry, physics constants and node classes derived on the host.
struct Derived {
  int D, Q;           // dimension; populations of f (and of the stencils' set)
  int Qg;             // populations of g (7 with D3Q7, else Q)
  Geo geo;
  Phys phys;
  Wall wall;
  long long N;        // SX * PY * PZ node slots
};

int validate_and_derive(const pflbm_params* prm, Derived* d);
Layout make_layout(const Derived& d, int storage, dim3 tile);
// Node words on the padded grid; also fills `classes` (nx*ny*nz bytes) if non-null.
void classify_nodes(const Derived& d, const uint8_t* mask, std::vector<uint32_t>& words,
                    uint8_t* classes);
dim3 default_tile(int D);

}  // namespace pflbm

struct pflbm_group_s;

struct pflbm_case_s {
  pflbm_params prm;
  pflbm::Derived dv;
  pflbm::Layout lay;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  bool owns = false;
  unsigned char* base = nullptr;
  uint32_t* nodes = nullptr;
  void* f[2] = {nullptr, nullptr};
  void* g[2] = {nullptr, nullptr};
  void* s = nullptr;
  void* phi = nullptr;
  void* mu = nullptr;
  void* snap = nullptr;
  double* partial = nullptr;
  double* rec = nullptr;
  float* popmax = nullptr;        // kPopmaxBlocks (f, g) pairs
  std::vector<uint8_t> classes;   // host copy of the domain classes
  long long nghost = 0;           // ghost nodes (the split step's ghost pass is skipped at 0)
  uint32_t* gblocks = nullptr;    // population blocks (64 slots) holding a ghost node off the
  long long nghost_blocks = 0;    // padding faces of a walled x axis, ascending; their number
  int cur = 0;                    // buffer holding the current post-collision state
  int64_t step = 0;
  bool snap_valid = false;
  dim3 tile;
  int graph_chunk = 64;
  int variant = 1;                // fused step kernel variant; -1 = three-kernel path
  bool o32 = false;               // f and g buffers below 4 GiB: 32-bit population offsets
  hipGraphExec_t gexec = nullptr;
  int gexec_steps = 0;
  pflbm_group_s* group = nullptr;
};

namespace pflbm {
// Per-(lattice, storage) launchers; defined in engine.hip.
int run_phi(pflbm_case_s* h);
int run_mu(pflbm_case_s* h);
int run_collide(pflbm_case_s* h, int mode, void* out_p, void* out_u);
int run_init_g(pflbm_case_s* h);
int run_reduce(pflbm_case_s* h, int update_snap, double* host_rec);
int run_step_eager(pflbm_case_s* h);
int run_step_fused(pflbm_case_s* h);
constexpr int kStepVariants = 13;   // largest count over the lattices
int step_variant_count(int D);
int step_variant_tile(int D, int v, int tile[5]);

// One launch of the batched step kernel.
struct GroupLaunch {
  int lattice, storage, variant, grid;
  int persist;           // 1: fixed grid striding over the table; 0: one workgroup per entry
  hipStream_t stream;
  const TileEntry* table;
  const int* ntiles;
  const CaseDesc* cases;
};
// Launches one batched step with the given parity, or (occupancy_blocks != 0)
// only reports how many workgroups of the kernel fit on one CU.
int run_step_group(const GroupLaunch& gl, int parity, int* occupancy_blocks);
void group_member_changed(pflbm_case_s* h);
// Batched phi + diagnostics reductions over a group's table: out[k * kRecN ..]
// receives member k's record.
int run_group_diag(const GroupLaunch& gl, int parity, int tx, int ty, int tz, double* partial,
                   double* out, int ncases, int update_snap);

// Launchers of one lattice for every storage type (engine_<lattice>.hip).
struct LatticeEntry {
  int (*phi)(pflbm_case_s*);
  int (*mu)(pflbm_case_s*);
  int (*collide)(pflbm_case_s*, int, void*, void*);
  int (*step)(pflbm_case_s*);
  int (*init_g)(pflbm_case_s*);
  int (*reduce)(pflbm_case_s*, int);
  int (*group_step)(const GroupLaunch&, int, int*);
  int (*group_diag)(const GroupLaunch&, int, int, int, int, double*, double*, int, int);
  int (*popmax)(pflbm_case_s*);
  int (*rescale)(pflbm_case_s*, int, float);
};
constexpr int kPopmaxBlocks = 64;   // workgroups of the stored-magnitude reduction
// FP16-deviation storage: keeps each set's largest stored magnitude in a safe
// band by moving its scale by a power of two (rescaling the current buffer);
// *changed (may be NULL) is set when a scale moved.  No-op for other storage.
int fp16_upkeep(pflbm_case_s* h, int* changed);
int run_popmax(pflbm_case_s* h, float out[2]);
int run_rescale(pflbm_case_s* h, int set_g, float factor);
// Contact-angle fit and flags from a reduction record.
void finish_diag(const pflbm_case_s* h, const double* rec, pflbm_diag* d);
}  // namespace pflbm
