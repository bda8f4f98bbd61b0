// Host-side planning under AddressSanitizer and UndefinedBehaviorSanitizer
// (test infrastructure: built by tests/test_host_sanitizers.py with g++ from
// the library's host sources, no GPU).  For each matrix file
//   int32 N, int32 nnz, int32 m, int32 sz, rowptr[N+1], colidx[nnz], double vals[nnz]
// it builds the partition, then the setup plan for every interface mode,
// block multiplier, overlap width and block sizing, and the coarse space and
// its plan for two piece sizes, and prints one summary line.
#include <cstdio>
#include <exception>
#include <string>
#include <vector>

#include "precond.h"

namespace addns {
// the C interface's error text is not part of this build
void set_error(const std::string&) {}
}  // namespace addns

using namespace addns;

static bool read_matrix(const char* path, int32_t& N, int32_t& m, int32_t& sz, std::vector<int32_t>& rp,
                        std::vector<int32_t>& ci, std::vector<double>& v) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return false;
  int32_t h[4];
  bool ok = std::fread(h, sizeof(int32_t), 4, f) == 4;
  if (ok) {
    N = h[0];
    m = h[2];
    sz = h[3];
    rp.resize(N + 1);
    ci.resize(h[1]);
    v.resize(h[1]);
    ok = std::fread(rp.data(), sizeof(int32_t), N + 1, f) == (size_t)(N + 1) &&
         std::fread(ci.data(), sizeof(int32_t), h[1], f) == (size_t)h[1] &&
         std::fread(v.data(), sizeof(double), h[1], f) == (size_t)h[1];
  }
  std::fclose(f);
  return ok;
}

int main(int argc, char** argv) {
  int failures = 0;
  for (int a = 1; a < argc; ++a) {
    int32_t N = 0, m = 0, sz = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> v;
    if (!read_matrix(argv[a], N, m, sz, rp, ci, v)) {
      std::printf("cannot read %s\n", argv[a]);
      return 2;
    }
    PartitionData P;
    const int st = build_partition(N, rp.data(), ci.data(), v.data(), m, sz, P);
    if (st < 0) {
      std::printf("%s: partition status %d\n", argv[a], st);
      ++failures;
      continue;
    }
    int plans = 0, refused = 0;
    const int modes[] = {ADDNS_SCHUR_MSCN, ADDNS_SCHUR_LUM, ADDNS_SCHUR_MSCNR, ADDNS_SCHUR_EXACT_BJ};
    for (int mode : modes)
      for (int mult = 1; mult <= 2; ++mult)
        for (int ovl : {0, sz - 1})
          for (int per = 0; per <= 1; ++per) {
            if (ovl > 0 && mode == ADDNS_SCHUR_EXACT_BJ) continue;
            try {
              Plan pl;
              build_plan(P, pl, mode, mult, ovl, per != 0);
              ++plans;
              if (ovl == 0 && mode == ADDNS_SCHUR_MSCN && mult == 1) {
                for (int piece : {8, 32}) {
                  CoarsePlan cp;
                  build_coarse_plan(P, pl, piece, cp);
                }
              }
            } catch (const std::exception&) {
              ++refused;  // e.g. aggregates too large for the overlap chain
            }
          }
    std::printf("%s: N %d m %d separator %d plans %d refused %d\n", argv[a], N, P.m, P.sep_size(), plans, refused);
  }
  return failures == 0 ? 0 : 1;
}
