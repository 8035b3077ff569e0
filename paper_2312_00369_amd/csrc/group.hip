// Groups: many cases of one lattice and storage advanced by one launch per
// step over a device (case, tile) table (one workgroup per entry, or a
// persistent grid striding over it).
//
// Buffer parity.  Each member's descriptor records which of its two buffers
// held the current state when the table was last built (cur0); launch k after
// the build runs with parity k & 1.  Host-side step counters and buffer indices
// of the members are brought up to date after every group call.  Graph chunks
// are captured with an even step count starting at parity 0, so a replay leaves
// the parity where it found it; membership changes rewrite the device table
// and descriptors in place (same addresses) between replays.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "case.h"

using namespace pflbm;

// Scratch of the allocation-free poll (pflbm_group_poll_static): the partial
// records of the batched reductions (one per table entry) followed by the
// member records.  A file-scope device array, so that poll allocates nothing;
// every GPU the library runs on holds its own copy until the process ends.
// The kernels write every partial and record before it is read, so nothing in
// it has to start at zero; calls that overlap on one GPU share it and race.
constexpr int kStaticEntries = 32768;   // table entries of one group
constexpr int kStaticMembers = 1024;    // members of one group
static __device__ __align__(256) double scratch[(size_t)(kStaticEntries + kStaticMembers) * kRecN];

struct pflbm_group_s {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<pflbm_case_s*> members;
  std::vector<hipStream_t> home_stream;   // each member's own stream
  std::vector<int64_t> step0;
  std::vector<int> cur0;
  int lattice = -1, storage = -1, D = 0;
  int variant = -1;        // -1: library default for the lattice
  int blocks_per_cu = 0;   // 0: one workgroup per table entry; > 0: persistent grid
  int cus = 0;
  // device table (capacity-managed; addresses change only on growth)
  TileEntry* d_table = nullptr;
  int* d_ntiles = nullptr;
  CaseDesc* d_cases = nullptr;
  size_t cap_tiles = 0, cap_cases = 0;
  int ntiles = 0;
  bool dirty = true;
  int64_t since_build = 0;
  int graph_chunk = 64;
  hipGraphExec_t gexec = nullptr;
  int gexec_steps = 0;
  int grid = 0;
  // batched diagnostics buffers (partials per table entry, records per member)
  double* d_partial = nullptr;
  double* d_rec = nullptr;
  size_t cap_partial = 0, cap_rec = 0;
};

namespace {

int default_variant(int D) { return D == 2 ? 1 : 7; }

void drop_graph(pflbm_group_s* g) {
  if (g->gexec) {
    (void)hipGraphExecDestroy(g->gexec);
    g->gexec = nullptr;
    g->gexec_steps = 0;
  }
}

// Bring every member's step count and buffer index up to date.
void sync_members(pflbm_group_s* g) {
  for (size_t k = 0; k < g->members.size(); ++k) {
    pflbm_case_s* h = g->members[k];
    h->step = g->step0[k] + g->since_build;
    h->cur = g->cur0[k] ^ (int)(g->since_build & 1);
  }
}

GroupLaunch launch_of(const pflbm_group_s* g) {
  GroupLaunch gl;
  gl.lattice = g->lattice;
  gl.storage = g->storage;
  gl.variant = g->variant;
  gl.grid = g->grid;
  gl.persist = g->blocks_per_cu > 0 ? 1 : 0;
  gl.stream = g->stream;
  gl.table = g->d_table;
  gl.ntiles = g->d_ntiles;
  gl.cases = g->d_cases;
  return gl;
}

int tiles_of(const pflbm_case_s* h, int variant) {
  int t[5];
  step_variant_tile(h->dv.D, variant, t);
  const Geo& G = h->dv.geo;
  return TileGrid(G, t[2], t[3], t[4]).count();
}

int rebuild(pflbm_group_s* g) {
  sync_members(g);
  g->since_build = 0;
  if (g->variant < 0 && g->D) g->variant = default_variant(g->D);
  if (g->D && g->variant >= step_variant_count(g->D))
    return set_error(PFLBM_EINVAL, "step variant %d does not exist for this lattice", g->variant);
  std::vector<TileEntry> table;
  std::vector<CaseDesc> cases(g->members.size());
  for (size_t k = 0; k < g->members.size(); ++k) {
    pflbm_case_s* h = g->members[k];
    g->step0[k] = h->step;
    g->cur0[k] = h->cur;
    CaseDesc& cd = cases[k];
    std::memset(&cd, 0, sizeof cd);
    cd.G = h->dv.geo;
    cd.P = h->dv.phys;
    cd.nodes = h->nodes;
    cd.f[0] = h->f[0];
    cd.f[1] = h->f[1];
    cd.g[0] = h->g[0];
    cd.g[1] = h->g[1];
    cd.s = h->s;
    cd.phi = h->phi;
    cd.snap = h->snap;
    cd.W = h->dv.wall;
    cd.cur0 = h->cur;
    const int nt = tiles_of(h, g->variant);
    cd.tile0 = (int)table.size();
    cd.ntile = nt;
    for (int t = 0; t < nt; ++t) table.push_back(TileEntry{(int)k, t});
  }
  bool moved = false;
  if (table.size() > g->cap_tiles || !g->d_table) {
    const size_t cap = std::max<size_t>(1024, table.size() * 3 / 2);
    if (g->d_table) (void)hipFree(g->d_table);
    g->d_table = nullptr;
    if (hipMalloc(&g->d_table, cap * sizeof(TileEntry)) != hipSuccess) {
      (void)hipGetLastError();
      g->cap_tiles = 0;
      return set_error(PFLBM_ENOMEM, "group table allocation failed");
    }
    g->cap_tiles = cap;
    moved = true;
  }
  if (cases.size() > g->cap_cases || !g->d_cases) {
    const size_t cap = std::max<size_t>(64, cases.size() * 3 / 2);
    if (g->d_cases) (void)hipFree(g->d_cases);
    g->d_cases = nullptr;
    if (hipMalloc(&g->d_cases, cap * sizeof(CaseDesc)) != hipSuccess) {
      (void)hipGetLastError();
      g->cap_cases = 0;
      return set_error(PFLBM_ENOMEM, "group descriptor allocation failed");
    }
    g->cap_cases = cap;
    moved = true;
  }
  if (!g->d_ntiles) {
    if (hipMalloc(&g->d_ntiles, sizeof(int)) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(PFLBM_ENOMEM, "group counter allocation failed");
    }
    moved = true;
  }
  if (table.size() > g->cap_partial || !g->d_partial) {
    const size_t cap = std::max<size_t>(1024, table.size() * 3 / 2);
    if (g->d_partial) (void)hipFree(g->d_partial);
    g->d_partial = nullptr;
    if (hipMalloc(&g->d_partial, cap * kRecN * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      g->cap_partial = 0;
      return set_error(PFLBM_ENOMEM, "group partial records allocation failed");
    }
    g->cap_partial = cap;
  }
  if (cases.size() > g->cap_rec || !g->d_rec) {
    const size_t cap = std::max<size_t>(64, cases.size() * 3 / 2);
    if (g->d_rec) (void)hipFree(g->d_rec);
    g->d_rec = nullptr;
    if (hipMalloc(&g->d_rec, cap * kRecN * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      g->cap_rec = 0;
      return set_error(PFLBM_ENOMEM, "group records allocation failed");
    }
    g->cap_rec = cap;
  }
  if (moved) drop_graph(g);
  g->ntiles = (int)table.size();
  if (!table.empty())
    PFLBM_HIP(hipMemcpyAsync(g->d_table, table.data(), table.size() * sizeof(TileEntry),
                             hipMemcpyHostToDevice, g->stream));
  if (!cases.empty())
    PFLBM_HIP(hipMemcpyAsync(g->d_cases, cases.data(), cases.size() * sizeof(CaseDesc),
                             hipMemcpyHostToDevice, g->stream));
  PFLBM_HIP(hipMemcpyAsync(g->d_ntiles, &g->ntiles, sizeof(int), hipMemcpyHostToDevice, g->stream));
  // the host vectors go out of scope: wait for the copies
  PFLBM_HIP(hipStreamSynchronize(g->stream));
  // blocks_per_cu > 0: a persistent grid of that many workgroups per CU (capped
  // by occupancy) strides over the table; 0: one workgroup per table entry
  // (fewer registers, more waves per SIMD; measured faster)
  int grid = std::max(1, g->ntiles);
  if (g->blocks_per_cu > 0) {
    if (!g->cus)
      PFLBM_HIP(hipDeviceGetAttribute(&g->cus, hipDeviceAttributeMultiprocessorCount, 0));
    int occ = 0;
    if (int rc = run_step_group(launch_of(g), 0, &occ)) return rc;
    occ = std::max(1, std::min(occ, g->blocks_per_cu));
    grid = std::max(1, g->cus * occ);
  }
  if (grid != g->grid) drop_graph(g);
  g->grid = grid;
  g->dirty = false;
  return PFLBM_OK;
}

int launch_eager(pflbm_group_s* g) {
  int rc = run_step_group(launch_of(g), (int)(g->since_build & 1), nullptr);
  if (rc) return rc;
  g->since_build += 1;
  return PFLBM_OK;
}

}  // namespace

namespace pflbm {
// A member's state was set from outside (checkpoint restore): re-base its
// entry so that the group's bookkeeping reproduces its step count, and rebuild
// the member descriptors before the next launch (they carry its FP16 scales).
void group_member_changed(pflbm_case_s* h) {
  pflbm_group_s* g = h->group;
  if (!g) return;
  for (size_t k = 0; k < g->members.size(); ++k)
    if (g->members[k] == h) {
      g->step0[k] = h->step - g->since_build;
      g->cur0[k] = h->cur ^ (int)(g->since_build & 1);
    }
  g->dirty = true;
}
}  // namespace pflbm

extern "C" {

void pflbm_group_forget(pflbm_handle h) {
  if (!h || !h->group) return;
  pflbm_group_s* g = h->group;
  (void)hipStreamSynchronize(g->stream);
  sync_members(g);
  auto it = std::find(g->members.begin(), g->members.end(), h);
  if (it != g->members.end()) {
    const size_t k = (size_t)(it - g->members.begin());
    h->stream = g->home_stream[k];
    g->members.erase(it);
    g->home_stream.erase(g->home_stream.begin() + k);
    g->step0.erase(g->step0.begin() + k);
    g->cur0.erase(g->cur0.begin() + k);
    // re-base the survivors so that their descriptors can be rebuilt
    for (size_t j = 0; j < g->members.size(); ++j) {
      g->step0[j] = g->members[j]->step;
      g->cur0[j] = g->members[j]->cur;
    }
    g->since_build = 0;
  }
  h->group = nullptr;
  g->dirty = true;
}

int pflbm_group_create(void* stream, pflbm_group* out) {
  clear_error();
  if (!out) return set_error(PFLBM_EINVAL, "out is NULL");
  *out = nullptr;
  auto* g = new (std::nothrow) pflbm_group_s();
  if (!g) return set_error(PFLBM_ENOMEM, "host allocation failed");
  if (stream) {
    g->stream = static_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreate(&g->stream) != hipSuccess) {
      delete g;
      return set_error(PFLBM_EDEVICE, "hipStreamCreate failed");
    }
    g->own_stream = true;
  }
  *out = g;
  return PFLBM_OK;
}

int pflbm_group_add(pflbm_group g, pflbm_handle h) {
  clear_error();
  if (!g || !h) return set_error(PFLBM_EINVAL, "NULL group or handle");
  if (h->group) return set_error(PFLBM_ESTATE, "case already belongs to a group");
  if (!g->members.empty() && (h->prm.lattice != g->lattice || h->prm.storage != g->storage))
    return set_error(PFLBM_EINVAL, "group members must share lattice and storage");
  if (!h->o32)
    return set_error(PFLBM_EUNSUPPORTED,
                     "case too large for a group (an f or g buffer of 4 GiB or more)");
  PFLBM_HIP(hipStreamSynchronize(h->stream));
  PFLBM_HIP(hipStreamSynchronize(g->stream));
  sync_members(g);
  for (size_t j = 0; j < g->members.size(); ++j) {
    g->step0[j] = g->members[j]->step;
    g->cur0[j] = g->members[j]->cur;
  }
  g->since_build = 0;
  if (g->members.empty()) {
    g->lattice = h->prm.lattice;
    g->storage = h->prm.storage;
    g->D = h->dv.D;
  }
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
    h->gexec_steps = 0;
  }
  g->members.push_back(h);
  g->home_stream.push_back(h->stream);
  g->step0.push_back(h->step);
  g->cur0.push_back(h->cur);
  h->stream = g->stream;
  h->group = g;
  g->dirty = true;
  return PFLBM_OK;
}

int pflbm_group_remove(pflbm_group g, pflbm_handle h) {
  clear_error();
  if (!g || !h) return set_error(PFLBM_EINVAL, "NULL group or handle");
  if (h->group != g) return set_error(PFLBM_ESTATE, "case is not a member of this group");
  pflbm_group_forget(h);
  return PFLBM_OK;
}

int pflbm_group_size(pflbm_group g) { return g ? (int)g->members.size() : -1; }

int pflbm_group_step(pflbm_group g, int64_t nsteps) {
  clear_error();
  if (!g) return set_error(PFLBM_EINVAL, "group is NULL");
  if (nsteps < 0) return set_error(PFLBM_EINVAL, "nsteps must be >= 0");
  if (g->members.empty() || nsteps == 0) return PFLBM_OK;
  int rc;
  if (g->dirty && (rc = rebuild(g))) return rc;
  const int K = g->graph_chunk;
  if (K > 0 && nsteps >= K) {
    if (g->since_build & 1) {
      if ((rc = launch_eager(g))) return rc;
      --nsteps;
    }
    if (!g->gexec || g->gexec_steps != K) {
      drop_graph(g);
      hipGraph_t graph = nullptr;
      PFLBM_HIP(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < K; ++k) {
        if ((rc = run_step_group(launch_of(g), k & 1, nullptr))) {
          (void)hipStreamEndCapture(g->stream, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          return rc;
        }
      }
      PFLBM_HIP(hipStreamEndCapture(g->stream, &graph));
      hipError_t e = hipGraphInstantiateWithFlags(&g->gexec, graph, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) {
        g->gexec = nullptr;
        return set_error(PFLBM_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
      }
      g->gexec_steps = K;
    }
    while (nsteps >= K && !(g->since_build & 1)) {
      PFLBM_HIP(hipGraphLaunch(g->gexec, g->stream));
      g->since_build += K;
      nsteps -= K;
    }
  }
  for (int64_t k = 0; k < nsteps; ++k)
    if ((rc = launch_eager(g))) return rc;
  sync_members(g);
  return PFLBM_OK;
}

int pflbm_group_poll(pflbm_group g, pflbm_diag* d, int32_t* flags, int32_t capacity) {
  clear_error();
  if (!g) return set_error(PFLBM_EINVAL, "group is NULL");
  if (capacity < (int)g->members.size()) return set_error(PFLBM_EINVAL, "capacity too small");
  if (g->members.empty()) return PFLBM_OK;
  int rc;
  if (g->dirty && (rc = rebuild(g))) return rc;
  int t[5];
  step_variant_tile(g->D, g->variant, t);
  const int nc = (int)g->members.size();
  if ((rc = run_group_diag(launch_of(g), (int)(g->since_build & 1), t[2], t[3], t[4], g->d_partial,
                           g->d_rec, nc, 1)))
    return rc;
  std::vector<double> rec((size_t)nc * kRecN);
  PFLBM_HIP(hipMemcpyAsync(rec.data(), g->d_rec, rec.size() * sizeof(double),
                           hipMemcpyDeviceToHost, g->stream));
  PFLBM_HIP(hipStreamSynchronize(g->stream));
  sync_members(g);
  for (int k = 0; k < nc; ++k) {
    pflbm_case_s* h = g->members[k];
    pflbm_diag tmp;
    finish_diag(h, &rec[(size_t)k * kRecN], &tmp);
    h->snap_valid = true;
    if (d) d[k] = tmp;
    if (flags) flags[k] = (tmp.steady ? 1 : 0) | (tmp.nonfinite ? 2 : 0);
  }
  // FP16 scale upkeep per member; a moved scale reaches the kernels through the
  // member descriptors, which the next step rebuilds
  for (int k = 0; k < nc; ++k) {
    int changed = 0;
    if ((rc = fp16_upkeep(g->members[k], &changed))) return rc;
    if (changed) g->dirty = true;
  }
  return PFLBM_OK;
}

}  // extern "C"

namespace {
// Device address of `scratch` on the current device, looked up once per device
// (hipGetSymbolAddress with that device current) and kept: host code passes
// this address to the kernels, never the array's name.
constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
double* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

int scratch_address(double** out) {
  int dev = 0;
  PFLBM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(PFLBM_EUNSUPPORTED, "device %d is beyond the %d the library tracks", dev,
                     kMaxDevices);
  std::call_once(g_scratch_once[dev], [dev] {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (g_scratch_err[dev] == hipSuccess) g_scratch_ptr[dev] = static_cast<double*>(p);
  });
  if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev])
    return set_error(PFLBM_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                     hipGetErrorString(g_scratch_err[dev]));
  *out = g_scratch_ptr[dev];
  return PFLBM_OK;
}
}  // namespace

extern "C" {

int pflbm_group_poll_static(pflbm_group g, pflbm_diag* d, int32_t* flags, int32_t capacity) {
  clear_error();
  if (!g) return set_error(PFLBM_EINVAL, "group is NULL");
  if (capacity < (int)g->members.size()) return set_error(PFLBM_EINVAL, "capacity too small");
  if (g->members.empty()) return PFLBM_OK;
  // a changed group needs its table rebuilt, which may allocate
  if (g->dirty)
    return set_error(PFLBM_ESTATE, "the group changed since its last step: step it (which "
                     "rebuilds its table) before an allocation-free poll");
  const int nc = (int)g->members.size();
  if (g->ntiles > kStaticEntries || nc > kStaticMembers)
    return set_error(PFLBM_EINVAL, "a group of %d table entries and %d members exceeds the "
                     "allocation-free poll's scratch (%d entries, %d members)", g->ntiles, nc,
                     kStaticEntries, kStaticMembers);
  double* scr = nullptr;
  int rc = scratch_address(&scr);
  if (rc) return rc;
  double* partial = scr;
  double* recs = scr + (size_t)kStaticEntries * kRecN;
  int t[5];
  step_variant_tile(g->D, g->variant, t);
  if ((rc = run_group_diag(launch_of(g), (int)(g->since_build & 1), t[2], t[3], t[4], partial,
                           recs, nc, 1)))
    return rc;
  sync_members(g);
  // member records through a small host buffer on the stack
  constexpr int kBatch = 32;
  double buf[kBatch * kRecN];
  for (int k0 = 0; k0 < nc; k0 += kBatch) {
    const int nb = std::min(kBatch, nc - k0);
    PFLBM_HIP(hipMemcpyAsync(buf, recs + (size_t)k0 * kRecN, (size_t)nb * kRecN * sizeof(double),
                             hipMemcpyDeviceToHost, g->stream));
    PFLBM_HIP(hipStreamSynchronize(g->stream));
    for (int j = 0; j < nb; ++j) {
      pflbm_case_s* h = g->members[k0 + j];
      pflbm_diag tmp;
      finish_diag(h, buf + (size_t)j * kRecN, &tmp);
      h->snap_valid = true;
      if (d) d[k0 + j] = tmp;
      if (flags) flags[k0 + j] = (tmp.steady ? 1 : 0) | (tmp.nonfinite ? 2 : 0);
    }
  }
  // FP16 scale upkeep per member, as pflbm_group_poll (in place, no allocation)
  for (int k = 0; k < nc; ++k) {
    int changed = 0;
    if ((rc = fp16_upkeep(g->members[k], &changed))) return rc;
    if (changed) g->dirty = true;
  }
  return PFLBM_OK;
}

int pflbm_group_set_tile(pflbm_group g, int32_t variant, int32_t blocks_per_cu) {
  clear_error();
  if (!g) return set_error(PFLBM_EINVAL, "group is NULL");
  if (variant < -1 || variant >= kStepVariants || blocks_per_cu < 0)
    return set_error(PFLBM_EINVAL, "bad group launch shape (%d, %d)", variant, blocks_per_cu);
  (void)hipStreamSynchronize(g->stream);
  sync_members(g);
  drop_graph(g);
  g->variant = variant;
  g->blocks_per_cu = blocks_per_cu;
  g->dirty = true;
  return PFLBM_OK;
}

int pflbm_group_set_graph_chunk(pflbm_group g, int32_t steps) {
  clear_error();
  if (!g) return set_error(PFLBM_EINVAL, "group is NULL");
  if (steps < 0) return set_error(PFLBM_EINVAL, "chunk must be >= 0");
  if (steps & 1) steps += 1;
  if (steps != g->graph_chunk) drop_graph(g);
  g->graph_chunk = steps;
  return PFLBM_OK;
}

void pflbm_group_destroy(pflbm_group g) {
  if (!g) return;
  (void)hipStreamSynchronize(g->stream);
  sync_members(g);
  for (size_t k = 0; k < g->members.size(); ++k) {
    g->members[k]->stream = g->home_stream[k];
    g->members[k]->group = nullptr;
  }
  drop_graph(g);
  if (g->d_table) (void)hipFree(g->d_table);
  if (g->d_cases) (void)hipFree(g->d_cases);
  if (g->d_ntiles) (void)hipFree(g->d_ntiles);
  if (g->d_partial) (void)hipFree(g->d_partial);
  if (g->d_rec) (void)hipFree(g->d_rec);
  if (g->own_stream) (void)hipStreamDestroy(g->stream);
  delete g;
}

}  // extern "C"
