// Host-side tables of the sixth-order mixed-stage operator (plain C++, shared by the problem
// set-up and the allocation-free operator entry point).
#pragma once
#include <vector>

namespace sa {

struct OperatorTables {
  std::vector<double> wsig;  // nl x 7 first-derivative weights in sigma, 1/dsigma included
  std::vector<int> ssig;     // nl window starts in sigma
  std::vector<double> wchi;  // 7 x 7 x weights, 1/dx included: rows 0-2 left windows, 3 centred,
                             // 4-6 right windows
  std::vector<double> sig;   // nl sigma values (level 0: the ghost level below the bed)
  std::vector<double> hext;  // ncol depths, ghost columns by even reflection
  std::vector<double> hchi;  // ncol sixth-order dh/dchi on the surface subgrid
};

// values at the physical columns extended to the column grid (walls: even reflection into
// the two ghost columns)
std::vector<double> extend_columns(const double* v, int nphys, int periodic);

void operator_tables(int ncol, int nl, int nphys, int periodic, double dx, double dsig, const double* h,
                     OperatorTables& t);

}  // namespace sa
