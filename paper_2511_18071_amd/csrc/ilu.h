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
  // the device layout: each level split into steps of ILU_SLOTS rows (padding rows -1); slot s
  // of step t is row frow[t * ILU_SLOTS + s] with one record of ILU_REC entries, column -1 past
  // its end (the strictly lower part of L for the forward substitution, the strictly upper part
  // of U for the backward one)
  int nstep_f = 0, nstep_b = 0;
  std::vector<int> frow, brow, fcol, bcol;
  std::vector<double> fval, bval;
  std::vector<double> bdinv;  // 1 / u_ii of the row in each backward slot (0 for padding)
};

constexpr int ILU_REC = 64;    // one wavefront lane per entry of a row
constexpr int ILU_SLOTS = 16;  // rows per substitution step: two per wavefront of a 512-thread workgroup

// ILU(0) of A(0, 0) assembled from the problem's sixth-order tables. 0 on success, -1 for a
// row without a diagonal entry, -2 for a zero or non-finite pivot, -3 for a row of L or U with
// more than ILU_REC entries.
int ilu_still_water(int ncol, int nl, int periodic, const OperatorTables& tb, IluFactors& f);

}  // namespace sa
