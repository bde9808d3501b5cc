// Host-side setup of a problem: difference weights, still-water coarse-grid inverse and the
// sketch random stream. Plain C++ (no device code).
#include <atomic>
#include <algorithm>
#include <thread>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "internal.h"
#include "tables.h"

namespace sa {

// Fornberg's recursion for finite-difference weights on arbitrary nodes (Fornberg 1988):
// c[i*(mmax+1) + m] weights node i for the m-th derivative at z.
void fornberg(double z, const double* x, int n, int mmax, double* c) {
  const int M = mmax + 1;
  for (int i = 0; i < n * M; ++i) c[i] = 0.0;
  double c1 = 1.0, c4 = x[0] - z;
  c[0] = 1.0;
  for (int i = 1; i < n; ++i) {
    const int mn = i < mmax ? i : mmax;
    double c2 = 1.0;
    const double c5 = c4;
    c4 = x[i] - z;
    for (int j = 0; j < i; ++j) {
      const double c3 = x[i] - x[j];
      c2 *= c3;
      if (j == i - 1) {
        for (int k = mn; k >= 1; --k) c[i * M + k] = c1 * (k * c[(i - 1) * M + k - 1] - c5 * c[(i - 1) * M + k]) / c2;
        c[i * M] = -c1 * c5 * c[(i - 1) * M] / c2;
      }
      for (int k = mn; k >= 1; --k) c[j * M + k] = (c4 * c[j * M + k] - k * c[j * M + k - 1]) / c3;
      c[j * M] = c4 * c[j * M] / c3;
    }
    c1 = c2;
  }
}

int window_start(int i, int npts, int width) {
  int s = i - width / 2;
  if (s > npts - width) s = npts - width;
  if (s < 0) s = 0;
  return s;
}

std::vector<double> extend_columns(const double* v, int nphys, int periodic) {
  std::vector<double> e;
  if (periodic) {
    e.assign(v, v + nphys);
  } else {
    e.resize(nphys + 2);
    e[0] = v[1];
    for (int i = 0; i < nphys; ++i) e[i + 1] = v[i];
    e[nphys + 1] = v[nphys - 2];
  }
  return e;
}

void operator_tables(int ncol, int nl, int nphys, int periodic, double dx, double dsig, const double* h,
                     OperatorTables& t) {
  double nodes[7], c[14];
  // sigma: seven-point windows, centred where the levels allow, shifted inside at the ends
  t.wsig.assign((size_t)nl * 7, 0.0);
  t.ssig.assign(nl, 0);
  for (int j = 0; j < nl; ++j) {
    const int st = window_start(j, nl, 7);
    for (int m = 0; m < 7; ++m) nodes[m] = (double)(st + m);
    fornberg((double)j, nodes, 7, 1, c);
    for (int m = 0; m < 7; ++m) t.wsig[(size_t)j * 7 + m] = c[m * 2 + 1] / dsig;
    t.ssig[j] = st;
  }
  // x: the seven windows a column can need (rows 0-2: node 0, 1, 2 of a left window; 3:
  // centre; 4-6: node 4, 5, 6 of a right window)
  t.wchi.assign(49, 0.0);
  for (int m = 0; m < 7; ++m) nodes[m] = (double)m;
  for (int row = 0; row < 7; ++row) {
    fornberg((double)row, nodes, 7, 1, c);
    for (int m = 0; m < 7; ++m) t.wchi[row * 7 + m] = c[m * 2 + 1] / dx;
  }
  t.sig.resize(nl);
  for (int j = 0; j < nl; ++j) t.sig[j] = (j - 1) * dsig;
  t.hext = extend_columns(h, nphys, periodic);
  t.hchi.assign(ncol, 0.0);
  for (int col = 0; col < ncol; ++col) {
    int row, start;
    if (periodic) { row = 3; start = col - 3; }
    else if (col < 3) { row = col; start = 0; }
    else if (col > ncol - 4) { row = 4 + col - (ncol - 3); start = ncol - 7; }
    else { row = 3; start = col - 3; }
    double s = 0.0;
    for (int m = 0; m < 7; ++m) s += t.wchi[row * 7 + m] * t.hext[((start + m) % ncol + ncol) % ncol];
    t.hchi[col] = s;
  }
}

// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based stream: output i of seed s is
// mix(s + i * golden_gamma). Draw a of stored solution `index` takes outputs 2(64 index + a) + 1
// and + 2, maps them to (0, 1] and applies the Box-Muller transform.
static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline double unit_interval(uint64_t seed, uint64_t i) {
  const uint64_t v = mix64(seed + i * 0x9E3779B97F4A7C15ULL);
  return (double)((v >> 11) + 1) * 0x1.0p-53;
}

void splitmix_gaussians(uint64_t seed, int64_t index, int k, double* out) {
  for (int a = 0; a < k; ++a) {
    const uint64_t i = 2ULL * (64ULL * (uint64_t)index + (uint64_t)a) + 1ULL;
    const double u1 = unit_interval(seed, i), u2 = unit_interval(seed, i + 1);
    out[a] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
  }
}

// Still-water operator rows (second-order direct form, same row kinds as the mixed-stage
// operator), assembled densely for the coarsest multigrid grid.
int dense_still_water_inverse(int ncol, int nx, int nl, int periodic, double dx, double dsig,
                              const double* h, const double* hx, const double* hxx, double* inv) {
  const int nz = nl - 1, n = ncol * nl;
  std::vector<double> a((size_t)n * n, 0.0);
  auto at = [&](int row, int c, int j, double v) {
    if (periodic) c = (c % ncol + ncol) % ncol;
    a[(size_t)row * n + (size_t)j * ncol + c] += v;
  };
  const double rdx = 1.0 / dx, rds = 1.0 / dsig;
  for (int j = 0; j < nl; ++j) {
    const double sg = (j - 1) * dsig;
    for (int c = 0; c < ncol; ++c) {
      const int row = j * ncol + c;
      const bool ghostcol = !periodic && (c == 0 || c == ncol - 1);
      if (j == nz || (ghostcol && j == 0)) {
        at(row, c, j, 1.0);
        continue;
      }
      if (ghostcol) {  // -G_x at the left wall node, +G_x at the right wall node
        const int w = c == 0 ? 1 : ncol - 2;
        const double sgn = c == 0 ? -1.0 : 1.0;
        const double s = hx[w] * (1.0 - sg) / h[w];
        at(row, w + 1, j, sgn * 0.5 * rdx);
        at(row, w - 1, j, -sgn * 0.5 * rdx);
        at(row, w, j + 1, sgn * s * 0.5 * rds);
        at(row, w, j - 1, -sgn * s * 0.5 * rds);
        continue;
      }
      if (j == 0) {  // bed: -h_x G_x - G_z at the bed node (level 1)
        const double s1 = hx[c] / h[c];
        at(row, c + 1, 1, -hx[c] * 0.5 * rdx);
        at(row, c - 1, 1, hx[c] * 0.5 * rdx);
        const double q = hx[c] * s1 + 1.0 / h[c];
        at(row, c, 2, -q * 0.5 * rds);
        at(row, c, 0, q * 0.5 * rds);
        continue;
      }
      const double oms = 1.0 - sg, hh = h[c], hc = hx[c];
      const double s = hc * oms / hh;
      const double sxx = oms * hxx[c] / hh - 2.0 * oms * hc * hc / (hh * hh);
      const double azz = (s * s + 1.0 / (hh * hh)) * rds * rds;
      at(row, c + 1, j, rdx * rdx);
      at(row, c - 1, j, rdx * rdx);
      at(row, c, j, -2.0 * rdx * rdx - 2.0 * azz);
      const double cx = 2.0 * s * 0.25 * rdx * rds;
      at(row, c + 1, j + 1, cx);
      at(row, c + 1, j - 1, -cx);
      at(row, c - 1, j + 1, -cx);
      at(row, c - 1, j - 1, cx);
      at(row, c, j + 1, azz + sxx * 0.5 * rds);
      at(row, c, j - 1, azz - sxx * 0.5 * rds);
    }
  }
  // Gauss-Jordan elimination with partial pivoting: inv = a^-1. The row updates of each
  // column step are split over host threads (the rows are independent within a step, so the
  // result does not depend on the split); a spin barrier separates the steps.
  std::vector<double> e((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) e[(size_t)i * n + i] = 1.0;
  const unsigned hw = std::thread::hardware_concurrency();
  const int nthr = std::max(1, std::min({(int)(hw ? hw : 1), 16, n / 128}));
  std::atomic<int> arrived{0}, phase{0}, failed{0};
  auto barrier = [&]() {
    const int ph = phase.load(std::memory_order_acquire);
    if (arrived.fetch_add(1, std::memory_order_acq_rel) == nthr - 1) {
      arrived.store(0, std::memory_order_relaxed);
      phase.fetch_add(1, std::memory_order_release);
    } else {
      while (phase.load(std::memory_order_acquire) == ph) std::this_thread::yield();
    }
  };
  auto work = [&](int t) {
    const int r0 = (int)((long)n * t / nthr), r1 = (int)((long)n * (t + 1) / nthr);
    for (int col = 0; col < n; ++col) {
      if (t == 0) {
        int piv = col;
        double best = fabs(a[(size_t)col * n + col]);
        for (int r = col + 1; r < n; ++r) {
          const double v = fabs(a[(size_t)r * n + col]);
          if (v > best) best = v, piv = r;
        }
        if (!(best > 0.0)) {
          failed.store(1, std::memory_order_relaxed);
        } else {
          if (piv != col) {
            for (int q = 0; q < n; ++q) {
              double v = a[(size_t)col * n + q]; a[(size_t)col * n + q] = a[(size_t)piv * n + q]; a[(size_t)piv * n + q] = v;
              v = e[(size_t)col * n + q]; e[(size_t)col * n + q] = e[(size_t)piv * n + q]; e[(size_t)piv * n + q] = v;
            }
          }
          const double d = 1.0 / a[(size_t)col * n + col];
          for (int q = 0; q < n; ++q) a[(size_t)col * n + q] *= d, e[(size_t)col * n + q] *= d;
        }
      }
      barrier();
      if (failed.load(std::memory_order_relaxed)) return;
      // columns left of col are zero in the pivot row: their updates would subtract zeros
      for (int r = r0; r < r1; ++r) {
        if (r == col) continue;
        const double f = a[(size_t)r * n + col];
        if (f == 0.0) continue;
        for (int q = col; q < n; ++q) a[(size_t)r * n + q] -= f * a[(size_t)col * n + q];
        for (int q = 0; q < n; ++q) e[(size_t)r * n + q] -= f * e[(size_t)col * n + q];
      }
      barrier();
    }
  };
  {
    std::vector<std::thread> pool;
    for (int t = 1; t < nthr; ++t) pool.emplace_back(work, t);
    work(0);
    for (auto& th : pool) th.join();
  }
  if (failed.load()) return -1;
  // stored transposed: inv[j * n + i] = (a^-1)[i][j], so device rows read coalesced
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) inv[(size_t)j * n + i] = e[(size_t)i * n + j];
  (void)nx;
  return 0;
}

}  // namespace sa
