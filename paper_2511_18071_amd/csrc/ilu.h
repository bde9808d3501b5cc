// Host-side ILU(0) of the still-water operator and the level schedule of its triangular solves.
#pragma once
#include <vector>

#include "tables.h"

namespace sa {

struct IluFactors {
  int n = 0;
  std::vector<int> lptr, lcol;    // strictly lower part of L by row (unit diagonal implied)
  std::vector<double> lval;
  std::vector<int> uptr, ucol;    // strictly upper part of U by row
  std::vector<double> uval;
  std::vector<double> dinv;       // 1 / u_ii
  int nlev_f = 0, nlev_b = 0;     // levels of the forward and the backward substitution
  std::vector<int> fptr, frows;   // rows of forward level l: frows[fptr[l] .. fptr[l+1])
  std::vector<int> bptr, brows;   // rows of backward level l
};

// ILU(0) of A(0, 0) assembled from the problem's sixth-order tables. 0 on success, -1 for a
// row without a diagonal entry, -2 for a zero or non-finite pivot.
int ilu_still_water(int ncol, int nl, int periodic, const OperatorTables& tb, IluFactors& f);

}  // namespace sa
