// Internal declarations of libaddns (not part of the C ABI).
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/addns.h"

namespace addns {

void set_error(const std::string& msg);

// Host-side result of the substructuring (section 1; section 3.3).
struct PartitionData {
  int32_t N = 0, m = 0, sz = 0;
  std::vector<int32_t> rowptr, colidx;  // pattern of C (kept for the setup plan)
  std::vector<uint8_t> is_p;            // pressure-like rows (zero/absent diagonal)
  std::vector<int32_t> perm;            // new -> old
  std::vector<int32_t> part;            // old -> subdomain, -1 separator
  std::vector<int32_t> int_offsets;     // m+1
  std::vector<int32_t> agg_offsets;     // k+1 (separator positions)
  std::vector<int32_t> drange_offsets;  // k+1
  std::vector<int32_t> drange_nodes;    // original indices
  std::vector<int32_t> pair;            // per separator position
  int status = 0;
  int32_t n_int() const { return int_offsets.back(); }
  int32_t sep_size() const { return N - n_int(); }
  int32_t k() const { return (int32_t)agg_offsets.size() - 1; }
};

int build_partition(int32_t N, const int32_t* rowptr, const int32_t* colidx, const double* vals,
                    int32_t m, int32_t sz, PartitionData& out);

}  // namespace addns

namespace addns {
struct PlanCache;  // host plans built from this partition (precond.h)
}

struct addns_partition {
  addns::PartitionData d;
  // Integer setup plans derived from the partition and the options (the
  // gather maps, sweep geometry and coarse-space structure), kept so that a
  // new setup on the same partition with the same options does not redo
  // them.  Not shared between threads, like the handle itself.
  std::shared_ptr<addns::PlanCache> cache;
};
