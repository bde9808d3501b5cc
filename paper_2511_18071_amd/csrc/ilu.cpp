// Incomplete LU factorisation with zero fill of the still-water operator, the preconditioner of
// Sec. 3 (a fixed incomplete LU of the operator generated at eta = 0), and the level schedule
// of its two triangular solves. Host code, run once per problem at creation.
//
// The operator A(0, 0) is assembled row by row from the sixth-order tables of the problem (the
// composed first-derivative form of the mixed-stage operator with both stages at still water,
// where d = h, d_chi = h_chi and sigma_x = h_chi (1 - sigma) / h), with the same boundary rows
// as the device operator: identity on the free surface and at the grid corners, the bed row
// -h_chi G_chi - G_z of the bed node on the ghost level, -+G_chi of the wall node on the wall
// ghost columns. Its pattern is structural: every node pair the stencils reach, whatever the
// value of the coefficient (sigma_x vanishes on a flat bed and at the surface).
//
// ILU(0) (Saad, Sec. 10.3): L unit lower and U upper on that pattern with (L U)_ij = a_ij on
// it, row by row: for each k < i of row i in increasing order, l_ik = a_ik / u_kk and
// a_ij -= l_ik u_kj for the j > k of row k that row i holds.
//
// Level schedule: the forward solve of row i needs the rows k < i of its L pattern, so row i
// goes one level after the deepest of them; the backward solve likewise over U from the last
// row up. Rows of one level are independent. The device reads each substitution as steps of
// ILU_SLOTS rows in level order (a level split over several steps where it has more rows), one
// record of ILU_REC (column, value) pairs per row: every address follows from the step number,
// so a wavefront loads the rows of later steps before the current step's results exist.
#include <math.h>

#include <algorithm>
#include <vector>

#include "ilu.h"

namespace sa {

namespace {

void chi_win(int c, int ncol, int periodic, int& row, int& start) {
  if (periodic) { row = 3; start = c - 3; return; }
  if (c < 3) { row = c; start = 0; }
  else if (c > ncol - 4) { row = 4 + c - (ncol - 3); start = ncol - 7; }
  else { row = 3; start = c - 3; }
}

}  // namespace

int ilu_still_water(int ncol, int nl, int periodic, const OperatorTables& tb, IluFactors& f) {
  const int nz = nl - 1;
  const int n = ncol * nl;
  f = IluFactors();
  f.n = n;
  // ---- assemble A(0, 0), one row at a time into a dense accumulator
  std::vector<int> ptr(n + 1, 0), col;
  std::vector<double> val;
  col.reserve((size_t)n * 56);
  val.reserve((size_t)n * 56);
  std::vector<double> acc(n, 0.0);
  std::vector<int> mark(n, -1), touched;
  touched.reserve(256);
  int cur = -1;
  auto add = [&](int j, int c, double v) {
    if (periodic) c = ((c % ncol) + ncol) % ncol;
    const int k = j * ncol + c;
    if (mark[k] != cur) { mark[k] = cur; acc[k] = 0.0; touched.push_back(k); }
    acc[k] += v;
  };
  const std::vector<double>& h = tb.hext;
  const std::vector<double>& hx = tb.hchi;
  auto sx = [&](int j, int c) { return hx[c] * (1.0 - tb.sig[j]) / h[c]; };
  // s times row (j, c) of G_chi = D_chi + sigma_x D_sigma, and of G_z = D_sigma / d
  auto g_chi = [&](int j, int c, double s) {
    int row, st;
    chi_win(c, ncol, periodic, row, st);
    for (int b = 0; b < 7; ++b) add(j, st + b, s * tb.wchi[row * 7 + b]);
    const double a = s * sx(j, c);
    for (int m = 0; m < 7; ++m) add(tb.ssig[j] + m, c, a * tb.wsig[j * 7 + m]);
  };
  auto g_z = [&](int j, int c, double s) {
    const double a = s / h[c];
    for (int m = 0; m < 7; ++m) add(tb.ssig[j] + m, c, a * tb.wsig[j * 7 + m]);
  };
  for (int i = 0; i < n; ++i) {
    cur = i;
    touched.clear();
    const int j = i / ncol, c = i % ncol;
    const bool ghost_c = !periodic && (c == 0 || c == ncol - 1);
    if (j == nz || (ghost_c && (j == 0 || j == nz))) {
      add(j, c, 1.0);
    } else if (j == 0) {  // bed: n . grad p at the bed node above, n = (-h_chi, -1)
      g_chi(1, c, -hx[c]);
      g_z(1, c, -1.0);
    } else if (ghost_c) {  // wall: -+ G_chi at the wall node
      if (c == 0) g_chi(j, 1, -1.0);
      else g_chi(j, ncol - 2, 1.0);
    } else {
      int row, st;
      chi_win(c, ncol, periodic, row, st);
      for (int a = 0; a < 7; ++a) {
        const int ca = periodic ? ((st + a) % ncol + ncol) % ncol : st + a;
        g_chi(j, ca, tb.wchi[row * 7 + a]);
      }
      const double s = sx(j, c), id = 1.0 / h[c];
      for (int m = 0; m < 7; ++m) {
        const int jm = tb.ssig[j] + m;
        const double w = tb.wsig[j * 7 + m];
        g_chi(jm, c, s * w);
        g_z(jm, c, id * w);
      }
    }
    std::sort(touched.begin(), touched.end());
    for (int k : touched) {
      col.push_back(k);
      val.push_back(acc[k]);
    }
    ptr[i + 1] = (int)col.size();
  }
  // ---- ILU(0) in place, row by row
  std::vector<int> diag(n, -1);
  for (int i = 0; i < n; ++i)
    for (int e = ptr[i]; e < ptr[i + 1]; ++e)
      if (col[e] == i) diag[i] = e;
  for (int i = 0; i < n; ++i)
    if (diag[i] < 0) return -1;
  std::vector<int> where(n, -1);
  for (int i = 0; i < n; ++i) {
    for (int e = ptr[i]; e < ptr[i + 1]; ++e) where[col[e]] = e;
    for (int e = ptr[i]; e < diag[i]; ++e) {
      const int k = col[e];
      const double piv = val[diag[k]];
      if (piv == 0.0 || !isfinite(piv)) return -2;
      const double l = val[e] / piv;
      val[e] = l;
      for (int q = diag[k] + 1; q < ptr[k + 1]; ++q) {
        const int p = where[col[q]];
        if (p >= 0) val[p] -= l * val[q];
      }
    }
    for (int e = ptr[i]; e < ptr[i + 1]; ++e) where[col[e]] = -1;
  }
  // ---- split into the strictly lower part of L, the strictly upper part of U, 1/u_ii
  f.lptr.assign(n + 1, 0);
  f.uptr.assign(n + 1, 0);
  f.dinv.resize(n);
  for (int i = 0; i < n; ++i) {
    for (int e = ptr[i]; e < diag[i]; ++e) { f.lcol.push_back(col[e]); f.lval.push_back(val[e]); }
    for (int e = diag[i] + 1; e < ptr[i + 1]; ++e) { f.ucol.push_back(col[e]); f.uval.push_back(val[e]); }
    f.lptr[i + 1] = (int)f.lcol.size();
    f.uptr[i + 1] = (int)f.ucol.size();
    f.dinv[i] = 1.0 / val[diag[i]];
  }
  // ---- level schedules
  auto schedule = [&](bool forward, std::vector<int>& lptr, std::vector<int>& rows) {
    std::vector<int> lev(n, 0);
    int nlev = 0;
    for (int t = 0; t < n; ++t) {
      const int i = forward ? t : n - 1 - t;
      int d = 0;
      const std::vector<int>& p = forward ? f.lptr : f.uptr;
      const std::vector<int>& cidx = forward ? f.lcol : f.ucol;
      for (int e = p[i]; e < p[i + 1]; ++e) d = std::max(d, lev[cidx[e]] + 1);
      lev[i] = d;
      nlev = std::max(nlev, d + 1);
    }
    lptr.assign(nlev + 1, 0);
    for (int i = 0; i < n; ++i) lptr[lev[i] + 1]++;
    for (int l = 0; l < nlev; ++l) lptr[l + 1] += lptr[l];
    rows.resize(n);
    std::vector<int> fill(lptr.begin(), lptr.end() - 1);
    for (int i = 0; i < n; ++i) rows[fill[lev[i]]++] = i;  // increasing i within a level
    return nlev;
  };
  f.nlev_f = schedule(true, f.fptr, f.frows);
  f.nlev_b = schedule(false, f.bptr, f.brows);
  // steps of ILU_SLOTS rows (a level with more rows takes several steps: its rows are
  // independent), one record per row
  auto pack = [&](int nlev, const std::vector<int>& lp, const std::vector<int>& rows, const std::vector<int>& p,
                  const std::vector<int>& cidx, const std::vector<double>& v, int& nstep, std::vector<int>& srow,
                  std::vector<int>& pc, std::vector<double>& pv) {
    nstep = 0;
    for (int l = 0; l < nlev; ++l) nstep += (lp[l + 1] - lp[l] + ILU_SLOTS - 1) / ILU_SLOTS;
    const size_t slots = (size_t)nstep * ILU_SLOTS;
    srow.assign(slots, -1);
    pc.assign(slots * ILU_REC, -1);
    pv.assign(slots * ILU_REC, 0.0);
    size_t s = 0;
    for (int l = 0; l < nlev; ++l) {
      const int cnt = lp[l + 1] - lp[l];
      for (int q = 0; q < cnt; ++q, ++s) {
        const int i = rows[lp[l] + q];
        if (p[i + 1] - p[i] > ILU_REC) return false;
        srow[s] = i;
        for (int e = p[i]; e < p[i + 1]; ++e) {
          pc[s * ILU_REC + (e - p[i])] = cidx[e];
          pv[s * ILU_REC + (e - p[i])] = v[e];
        }
      }
      s = (s + ILU_SLOTS - 1) / ILU_SLOTS * ILU_SLOTS;  // the next level starts a new step
    }
    return true;
  };
  if (!pack(f.nlev_f, f.fptr, f.frows, f.lptr, f.lcol, f.lval, f.nstep_f, f.frow, f.fcol, f.fval)) return -3;
  if (!pack(f.nlev_b, f.bptr, f.brows, f.uptr, f.ucol, f.uval, f.nstep_b, f.brow, f.bcol, f.bval)) return -3;
  f.bdinv.assign(f.brow.size(), 0.0);
  for (size_t s = 0; s < f.brow.size(); ++s)
    if (f.brow[s] >= 0) f.bdinv[s] = f.dinv[f.brow[s]];
  return 0;
}

}  // namespace sa
