// C-ABI entry points for partitions, error reporting and versioning.
#include <climits>
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

int addns_partition_concat(const addns_partition_t* parts, int32_t nsys, addns_partition_t* out) {
  addns::g_last_error.clear();
  if (!parts || !out || nsys < 1) {
    set_error("addns_partition_concat: need nsys >= 1 partitions and an output handle");
    return ADDNS_ERR_ARG;
  }
  for (int32_t s = 0; s < nsys; ++s)
    if (!parts[s]) {
      set_error("addns_partition_concat: null partition " + std::to_string(s));
      return ADDNS_ERR_ARG;
    }
  try {
    auto* c = new addns_partition();
    addns::PartitionData& D = c->d;
    int64_t N = 0, nnz = 0, m = 0;
    for (int32_t s = 0; s < nsys; ++s) {
      N += parts[s]->d.N;
      nnz += (int64_t)parts[s]->d.colidx.size();
      m += parts[s]->d.m;
    }
    if (N > INT32_MAX || nnz > INT32_MAX || m > INT32_MAX) {
      delete c;
      set_error("addns_partition_concat: concatenated system exceeds int32 sizes");
      return ADDNS_ERR_ARG;
    }
    D.N = (int32_t)N;
    D.m = (int32_t)m;
    D.sz = parts[0]->d.sz;
    D.rowptr.assign(1, 0);
    D.int_offsets.assign(1, 0);
    D.agg_offsets.assign(1, 0);
    D.drange_offsets.assign(1, 0);
    D.part.reserve(N);
    // interiors of every system first (system order), then every separator
    int32_t node0 = 0, sub0 = 0, sep0 = 0;
    std::vector<int32_t> seps;
    for (int32_t s = 0; s < nsys; ++s) {
      const addns::PartitionData& P = parts[s]->d;
      for (int32_t i = 0; i < P.N; ++i)
        for (int32_t e = P.rowptr[i]; e < P.rowptr[i + 1]; ++e) D.colidx.push_back(P.colidx[e] + node0);
      for (int32_t i = 0; i < P.N; ++i) D.rowptr.push_back(D.rowptr.back() + P.rowptr[i + 1] - P.rowptr[i]);
      D.is_p.insert(D.is_p.end(), P.is_p.begin(), P.is_p.end());
      for (int32_t i = 0; i < P.N; ++i) D.part.push_back(P.part[i] < 0 ? -1 : P.part[i] + sub0);
      for (int32_t r = 0; r < P.n_int(); ++r) D.perm.push_back(P.perm[r] + node0);
      for (int32_t j = 0; j < P.m; ++j) D.int_offsets.push_back(D.int_offsets.back() + P.int_offsets[j + 1] - P.int_offsets[j]);
      for (int32_t r = P.n_int(); r < P.N; ++r) seps.push_back(P.perm[r] + node0);
      for (int32_t t = 0; t < P.sep_size(); ++t) D.pair.push_back(P.pair[t] < 0 ? -1 : P.pair[t] + node0);
      for (int32_t i = 0; i < P.k(); ++i) {
        D.agg_offsets.push_back(P.agg_offsets[i + 1] + sep0);
        for (int32_t t = P.drange_offsets[i]; t < P.drange_offsets[i + 1]; ++t)
          D.drange_nodes.push_back(P.drange_nodes[t] + node0);
        D.drange_offsets.push_back((int32_t)D.drange_nodes.size());
      }
      if (P.status > D.status) D.status = P.status;
      node0 += P.N;
      sub0 += P.m;
      sep0 += P.sep_size();
    }
    D.perm.insert(D.perm.end(), seps.begin(), seps.end());
    *out = c;
    return ADDNS_OK;
  } catch (const std::bad_alloc&) {
    set_error("addns_partition_concat: out of host memory");
    return ADDNS_ERR_NOMEM;
  }
}

void addns_partition_destroy(addns_partition_t p) { delete p; }

}  // extern "C"
