// C-ABI entry points for partitions, error reporting and versioning.
#include <cstring>
#include <new>
#include <string>

#include "internal.h"

namespace addns {
thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace addns

using addns::set_error;

extern "C" {

const char* addns_last_error(void) { return addns::g_last_error.c_str(); }

const char* addns_version(void) { return "libaddns 0.1 (gfx950)"; }

int addns_build_partition(int32_t N, const int32_t* rowptr, const int32_t* colidx,
                          const double* vals, int32_t m, int32_t sz, addns_partition_t* out) {
  addns::g_last_error.clear();
  if (!out || !rowptr || (N > 0 && (!colidx || !vals))) {
    set_error("addns_build_partition: null argument");
    return ADDNS_ERR_ARG;
  }
  if (N < 1 || m < 1 || sz < 1) {
    set_error("addns_build_partition: need N >= 1, m >= 1, sz >= 1");
    return ADDNS_ERR_ARG;
  }
  if (rowptr[0] != 0) {
    set_error("addns_build_partition: rowptr[0] must be 0");
    return ADDNS_ERR_ARG;
  }
  for (int32_t i = 0; i < N; ++i) {
    if (rowptr[i + 1] < rowptr[i]) {
      set_error("addns_build_partition: rowptr not monotone at row " + std::to_string(i));
      return ADDNS_ERR_ARG;
    }
  }
  for (int32_t e = 0; e < rowptr[N]; ++e) {
    if (colidx[e] < 0 || colidx[e] >= N) {
      set_error("addns_build_partition: column index out of range at entry " + std::to_string(e));
      return ADDNS_ERR_ARG;
    }
  }
  try {
    auto* p = new addns_partition();
    int st = addns::build_partition(N, rowptr, colidx, vals, m, sz, p->d);
    if (st < 0) {
      delete p;
      return st;
    }
    *out = p;
    return st;
  } catch (const std::bad_alloc&) {
    set_error("addns_build_partition: out of host memory");
    return ADDNS_ERR_NOMEM;
  } catch (const std::exception& e) {
    set_error(std::string("addns_build_partition: ") + e.what());
    return ADDNS_ERR_PARTITION;
  }
}

int addns_partition_info(addns_partition_t p, int32_t* N, int32_t* m, int32_t* n_interior,
                         int32_t* sep_size, int32_t* k, int32_t* drange_total) {
  if (!p) {
    set_error("addns_partition_info: null handle");
    return ADDNS_ERR_ARG;
  }
  const auto& d = p->d;
  if (N) *N = d.N;
  if (m) *m = d.m;
  if (n_interior) *n_interior = d.n_int();
  if (sep_size) *sep_size = d.sep_size();
  if (k) *k = d.k();
  if (drange_total) *drange_total = (int32_t)d.drange_nodes.size();
  return ADDNS_OK;
}

int addns_partition_export(addns_partition_t p, int32_t* perm, int32_t* part,
                           int32_t* int_offsets, int32_t* agg_offsets, int32_t* drange_offsets,
                           int32_t* drange_nodes, int32_t* pair) {
  if (!p) {
    set_error("addns_partition_export: null handle");
    return ADDNS_ERR_ARG;
  }
  const auto& d = p->d;
  auto cp = [](int32_t* dst, const std::vector<int32_t>& src) {
    if (dst && !src.empty()) std::memcpy(dst, src.data(), src.size() * sizeof(int32_t));
  };
  cp(perm, d.perm);
  cp(part, d.part);
  cp(int_offsets, d.int_offsets);
  cp(agg_offsets, d.agg_offsets);
  cp(drange_offsets, d.drange_offsets);
  cp(drange_nodes, d.drange_nodes);
  cp(pair, d.pair);
  return ADDNS_OK;
}

void addns_partition_destroy(addns_partition_t p) { delete p; }

}  // extern "C"
