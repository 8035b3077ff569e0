// Groups of cases stepped together (placeholder: members step one after another).
#include <algorithm>
#include <vector>

#include "case.h"

using namespace pflbm;

struct pflbm_group_s {
  hipStream_t stream = nullptr;
  std::vector<pflbm_case_s*> members;
};

extern "C" {

void pflbm_group_forget(pflbm_handle h) {
  if (!h || !h->group) return;
  auto& m = h->group->members;
  m.erase(std::remove(m.begin(), m.end(), h), m.end());
  h->group = nullptr;
}

int pflbm_group_create(void* stream, pflbm_group* out) {
  clear_error();
  if (!out) return set_error(PFLBM_EINVAL, "out is NULL");
  auto* g = new (std::nothrow) pflbm_group_s();
  if (!g) return set_error(PFLBM_ENOMEM, "host allocation failed");
  g->stream = static_cast<hipStream_t>(stream);
  *out = g;
  return PFLBM_OK;
}

int pflbm_group_add(pflbm_group g, pflbm_handle h) {
  clear_error();
  if (!g || !h) return set_error(PFLBM_EINVAL, "NULL group or handle");
  if (h->group) return set_error(PFLBM_ESTATE, "case already belongs to a group");
  g->members.push_back(h);
  h->group = g;
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
  for (auto* h : g->members)
    for (int64_t k = 0; k < nsteps; ++k)
      if (int rc = run_step_eager(h)) return rc;
  return PFLBM_OK;
}

int pflbm_diagnostics(pflbm_handle h, pflbm_diag* d);

int pflbm_group_poll(pflbm_group g, pflbm_diag* d, int32_t* flags, int32_t capacity) {
  clear_error();
  if (!g) return set_error(PFLBM_EINVAL, "group is NULL");
  if (capacity < (int)g->members.size()) return set_error(PFLBM_EINVAL, "capacity too small");
  for (size_t k = 0; k < g->members.size(); ++k) {
    pflbm_diag tmp;
    if (int rc = pflbm_diagnostics(g->members[k], &tmp)) return rc;
    if (d) d[k] = tmp;
    if (flags) flags[k] = (tmp.steady ? 1 : 0) | (tmp.nonfinite ? 2 : 0);
  }
  return PFLBM_OK;
}

int pflbm_group_set_tile(pflbm_group g, int32_t, int32_t, int32_t, int32_t) {
  clear_error();
  if (!g) return set_error(PFLBM_EINVAL, "group is NULL");
  return PFLBM_OK;
}

void pflbm_group_destroy(pflbm_group g) {
  if (!g) return;
  for (auto* h : g->members) h->group = nullptr;
  delete g;
}

}  // extern "C"
