// The mixed-stage operator on a three-dimensional (chi, gamma, sigma) grid: Sec. 2.1 writes the
// sigma-transform and the push-forward of the gradient in three dimensions, Sec. 3 the pressure
// operator grad^(i) . grad^(i-1) with ghost-node Neumann rows. In composed first-derivative form
//
//   y = D_chi G_chi + s_x^cur D_sig G_chi + D_gam G_gam + s_y^cur D_sig G_gam + (1/d^cur) D_sig G_z,
//   G_chi = D_chi x + s_x^prev xs,  G_gam = D_gam x + s_y^prev xs,  G_z = xs / d^prev,  xs = D_sig x,
//
// with s_x = (h_chi - sigma d_chi)/d and s_y = (h_gam - sigma d_gam)/d per column and level.
// Because D_sig acts along sigma and D_chi, D_gam within a level, D_sig G_chi = D_chi xs +
// D_sig(s_x^prev xs) (likewise for gamma); the kernel evaluates the terms at a level from
// values at that level (x with a six-column halo, xs with a three-column halo) and the terms
// along sigma from the xs of its own column at the seven levels of the sigma window.
//
// One workgroup owns a tile of 32 chi-columns x 8 gamma-rows and walks up its columns level by
// level: x of each level is staged once into a ring of seven levels in LDS (the first seven in
// one batch of loads, then each level's loads issued a level ahead), xs of each level is formed
// once and kept for seven levels, and the output of level j is written as soon as the xs of the
// top of its sigma window exists. Every input is read from HBM once (the halo from
// neighbours' tiles, mostly from the caches), y written once: the kernel is bound by HBM traffic
// and by its FP64 arithmetic (about 85 fused multiply-adds per node).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "host.h"

using namespace sa;

namespace {

constexpr int T3X = 32;                 // tile columns (chi)
constexpr int T3Y = 8;                  // tile rows (gamma)
constexpr int NT3 = T3X * T3Y;          // threads per workgroup, one per tile column
constexpr int RW = T3X + 6;             // width of the staged rectangle (three-column halo)
constexpr int RH = T3Y + 6;             // height of the staged rectangle
constexpr int RING = 7;                 // levels kept: one sigma window
constexpr int NHALO = 2 * 3 * T3Y + 2 * 3 * T3X;  // halo positions of the plus-shaped region
static_assert(NHALO <= NT3, "one halo position per thread");
constexpr int NGEO = 12;                // per-column geometry arrays

// geometry array indices (per plane column, both stages)
enum { G_HX, G_HY, G_IP, G_AXP, G_BXP, G_AYP, G_BYP, G_IC, G_AXC, G_BXC, G_AYC, G_BYC };

struct Op3 {
  int ncol, nrow, nl, nz, nxp, nyp, per_x, per_y;
  int c_shift, r_shift, ntx;           // tile origins: c0 = bx * T3X - c_shift
  long long nplane;
  const double* wsig;                   // nl x 7, 1/dsigma included
  const int* ssig;                      // nl window starts
  const double* wx;                     // 7 x 7 chi windows (1/dx)
  const double* wy;                     // 7 x 7 gamma windows (1/dy)
  const double* sig;                    // nl
  const double* hext;                   // nplane, ghost columns/rows by even reflection
  double* geo;                          // NGEO x nplane
  int* flags;
};

// LDS layout (doubles), one workgroup
struct Lds3 {
  static constexpr int WSIG = 0;                            // NLMAX * 7
  static constexpr int SIG = WSIG + NLMAX * 7;              // NLMAX
  static constexpr int WX = SIG + NLMAX;                    // 49
  static constexpr int WY = WX + 49;                        // 49
  static constexpr int XR = WY + 49;                        // RING x RH x RW
  static constexpr int XSC = XR + RING * RH * RW;           // RH x RW, xs of the current level
  static constexpr int XSR = XSC + RH * RW;                 // RING x NT3, xs of the tile columns
  static constexpr int T1R = XSR + RING * NT3;              // RING x NT3, the level terms of y
  static constexpr int XAX = T1R + RING * NT3;              // T3Y x 6, x at chi offsets -6..-4, +3..+5
  static constexpr int XAY = XAX + T3Y * 6;                 // 6 x T3X, x at gamma offsets
  static constexpr int GX = XAY + 6 * T3X;                  // T3Y x RW
  static constexpr int GY = GX + T3Y * RW;                  // RH x T3X
  static constexpr int GHX = GY + RH * T3X;                 // T3Y x 6 x 2: s_x^prev of the chi halo
  static constexpr int GHY = GHX + T3Y * 6 * 2;             // 6 x T3X x 2: s_y^prev of the gamma halo
  static constexpr int END = GHY + 6 * T3X * 2;
};
constexpr size_t LDS3_BYTES = (size_t)Lds3::END * 8 + (size_t)NLMAX * 4;

// window of a first derivative at node i of a line of n nodes: weight row and first node
__device__ __host__ inline void win7(int i, int n, int periodic, int& row, int& start) {
  if (periodic) { row = 3; start = i - 3; return; }
  if (i < 3) { row = i; start = 0; }
  else if (i > n - 4) { row = 4 + i - (n - 3); start = n - 7; }
  else { row = 3; start = i - 3; }
}

__device__ inline int wrap(int i, int n) { return ((i % n) + n) % n; }

// level whose xs completes the sigma window of level j (the window's top)
__device__ inline int win_top(int j, int nl) { return min(max(j + 3, 6), nl - 1); }

// physical index of an extended column/row (walls: ghosts reflect the first interior node)
__device__ inline int phys_of(int i, int n, int periodic) {
  if (periodic) return i;
  if (i == 0) return 1;
  if (i == n - 1) return n - 4;
  return i - 1;
}

}  // namespace

extern "C" __global__ void __launch_bounds__(NT3) sa_geometry3_kernel(Op3 P, const double* __restrict__ eta_p,
                                                                     const double* __restrict__ eta_c) {
  const long long pi = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (pi >= P.nplane) return;
  const int c = (int)(pi % P.ncol), r = (int)(pi / P.ncol);
  auto ext = [&](const double* e, int cc, int rr) {
    const int pc = phys_of(cc, P.ncol, P.per_x), pr = phys_of(rr, P.nrow, P.per_y);
    return e[(long long)pr * P.nxp + pc];
  };
  int rx, sx, ry, sy;
  win7(c, P.ncol, P.per_x, rx, sx);
  win7(r, P.nrow, P.per_y, ry, sy);
  double hx = 0, hy = 0, dxp = 0, dyp = 0, dxc = 0, dyc = 0;
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    const int cc = P.per_x ? wrap(sx + m, P.ncol) : sx + m;
    const int rr = P.per_y ? wrap(sy + m, P.nrow) : sy + m;
    const double w1 = P.wx[rx * 7 + m], w2 = P.wy[ry * 7 + m];
    const double h1 = P.hext[(long long)r * P.ncol + cc], h2 = P.hext[(long long)rr * P.ncol + c];
    hx += w1 * h1;
    hy += w2 * h2;
    dxp += w1 * (h1 + ext(eta_p, cc, r));
    dxc += w1 * (h1 + ext(eta_c, cc, r));
    dyp += w2 * (h2 + ext(eta_p, c, rr));
    dyc += w2 * (h2 + ext(eta_c, c, rr));
  }
  const double h = P.hext[pi];
  const double d_p = h + ext(eta_p, c, r), d_c = h + ext(eta_c, c, r);
  if (!(d_p > 0.0) || !(d_c > 0.0) || !isfinite(d_p) || !isfinite(d_c) || !isfinite(dxp) || !isfinite(dyp) ||
      !isfinite(dxc) || !isfinite(dyc))
    atomicOr(P.flags + FLAG_GEOM, 1);
  const double ip = 1.0 / d_p, ic = 1.0 / d_c;
  const long long np = P.nplane;
  double* g = P.geo;
  g[G_HX * np + pi] = hx;
  g[G_HY * np + pi] = hy;
  g[G_IP * np + pi] = ip;
  g[G_AXP * np + pi] = hx * ip;
  g[G_BXP * np + pi] = dxp * ip;
  g[G_AYP * np + pi] = hy * ip;
  g[G_BYP * np + pi] = dyp * ip;
  g[G_IC * np + pi] = ic;
  g[G_AXC * np + pi] = hx * ic;
  g[G_BXC * np + pi] = dxc * ic;
  g[G_AYC * np + pi] = hy * ic;
  g[G_BYC * np + pi] = dyc * ic;
}

extern "C" __global__ void __launch_bounds__(NT3) sa_operator3_kernel(Op3 P, const double* __restrict__ x,
                                                                     double* __restrict__ y) {
  extern __shared__ double lds3[];
  double* wsig = lds3 + Lds3::WSIG;
  double* sig = lds3 + Lds3::SIG;
  double* wx = lds3 + Lds3::WX;
  double* wy = lds3 + Lds3::WY;
  double* XR = lds3 + Lds3::XR;
  double* XSC = lds3 + Lds3::XSC;
  double* XSR = lds3 + Lds3::XSR;
  double* T1R = lds3 + Lds3::T1R;
  double* XAX = lds3 + Lds3::XAX;
  double* XAY = lds3 + Lds3::XAY;
  double* GXB = lds3 + Lds3::GX;
  double* GYB = lds3 + Lds3::GY;
  double* GHX = lds3 + Lds3::GHX;
  double* GHY = lds3 + Lds3::GHY;
  int* ssig = (int*)(lds3 + Lds3::END);

  const int t = threadIdx.x;
  const int ncol = P.ncol, nrow = P.nrow, nl = P.nl, nz = P.nz;
  const long long np = P.nplane;
  // the hardware hands consecutive workgroups to the eight XCDs in turn: give each XCD a
  // contiguous run of tiles, so that neighbouring tiles meet in its L2
  const int nb = gridDim.x, xcd = blockIdx.x % 8, per = nb / 8, extra = nb % 8;
  const int tile = xcd * per + min(xcd, extra) + blockIdx.x / 8;
  const int bx = tile % P.ntx, by = tile / P.ntx;
  const int c0 = bx * T3X - P.c_shift, r0 = by * T3Y - P.r_shift;

  for (int i = t; i < nl * 7; i += NT3) wsig[i] = P.wsig[i];
  for (int i = t; i < nl; i += NT3) { sig[i] = P.sig[i]; ssig[i] = P.ssig[i]; }
  if (t < 49) { wx[t] = P.wx[t]; wy[t] = P.wy[t]; }

  // global column / row of a tile-relative position; -1 beyond a wall
  auto gcol = [&](int cc) { const int c = c0 + cc; return P.per_x ? wrap(c, ncol) : (c >= 0 && c < ncol ? c : -1); };
  auto grow = [&](int rr) { const int r = r0 + rr; return P.per_y ? wrap(r, nrow) : (r >= 0 && r < nrow ? r : -1); };

  // this thread's tile column and its halo position (plus-shaped region around the tile)
  const int tc = t % T3X, tr = t / T3X;
  int hc = 0, hr = 0;
  if (t < 24) { hr = t / 3; hc = -3 + t % 3; }
  else if (t < 48) { hr = (t - 24) / 3; hc = T3X + (t - 24) % 3; }
  else if (t < 48 + 3 * T3X) { hr = -3 + (t - 48) / T3X; hc = (t - 48) % T3X; }
  else if (t < NHALO) { hr = T3Y + (t - 48 - 3 * T3X) / T3X; hc = (t - 48 - 3 * T3X) % T3X; }
  const int gc = gcol(tc), gr = grow(tr);
  const bool tile_ok = gc >= 0 && gr >= 0;
  const bool out_ok = tile_ok && c0 + tc >= 0 && c0 + tc < ncol && r0 + tr >= 0 && r0 + tr < nrow;
  const long long tplane = tile_ok ? (long long)gr * ncol + gc : 0;
  const int hgc = t < NHALO ? gcol(hc) : -1, hgr = t < NHALO ? grow(hr) : -1;
  const bool halo_ok = hgc >= 0 && hgr >= 0;
  const long long hplane = halo_ok ? (long long)hgr * ncol + hgc : 0;
  // arms: x at chi offsets -6..-4 and +3..+5 of the tile rows, gamma offsets of the tile columns
  int ac = 0, ar = 0;
  if (t < T3Y * 6) { ar = t / 6; const int k = t % 6; ac = k < 3 ? -6 + k : T3X + k; }
  else if (t < NHALO) { const int k = (t - T3Y * 6) / T3X; ac = (t - T3Y * 6) % T3X; ar = k < 3 ? -6 + k : T3Y + k; }
  const int agc = t < NHALO ? gcol(ac) : -1, agr = t < NHALO ? grow(ar) : -1;
  const bool arm_ok = agc >= 0 && agr >= 0;
  const long long aplane = arm_ok ? (long long)agr * ncol + agc : 0;

  // geometry of the tile column (registers) and of the halo columns that need it (LDS)
  double hx = 0, hy = 0, ip = 0, axp = 0, bxp = 0, ayp = 0, byp = 0, ic = 0, axc = 0, bxc = 0, ayc = 0, byc = 0;
  if (tile_ok) {
    const double* g = P.geo;
    hx = g[G_HX * np + tplane]; hy = g[G_HY * np + tplane]; ip = g[G_IP * np + tplane];
    axp = g[G_AXP * np + tplane]; bxp = g[G_BXP * np + tplane]; ayp = g[G_AYP * np + tplane];
    byp = g[G_BYP * np + tplane]; ic = g[G_IC * np + tplane]; axc = g[G_AXC * np + tplane];
    bxc = g[G_BXC * np + tplane]; ayc = g[G_AYC * np + tplane]; byc = g[G_BYC * np + tplane];
  }
  if (t < 48) {  // chi halo: rows of the tile, columns -3..-1 and T3X..T3X+2
    const int k = t < 24 ? t % 3 : 3 + (t - 24) % 3;
    const int i = (hr * 6 + k) * 2;
    GHX[i] = halo_ok ? P.geo[G_AXP * np + hplane] : 0.0;
    GHX[i + 1] = halo_ok ? P.geo[G_BXP * np + hplane] : 0.0;
  } else if (t < NHALO) {  // gamma halo: columns of the tile, rows -3..-1 and T3Y..T3Y+2
    const int k = hr < 0 ? hr + 3 : 3 + hr - T3Y;
    const int i = (k * T3X + hc) * 2;
    GHY[i] = halo_ok ? P.geo[G_AYP * np + hplane] : 0.0;
    GHY[i + 1] = halo_ok ? P.geo[G_BYP * np + hplane] : 0.0;
  }

  // the chi and gamma windows of the tile column, as offsets into the staged rectangle
  int rowx, stx, rowy, sty;
  win7(P.per_x ? tc : gc, ncol, P.per_x, rowx, stx);
  win7(P.per_y ? tr : gr, nrow, P.per_y, rowy, sty);
  const int ox = P.per_x ? tc - 3 : stx - c0;  // tile-relative first node of the chi window
  const int oy = P.per_y ? tr - 3 : sty - r0;
  const bool ghost_c = !P.per_x && (gc == 0 || gc == ncol - 1);
  const bool ghost_r = !P.per_y && (gr == 0 || gr == nrow - 1);

  const int rect_t = (tr + 3) * RW + tc + 3;
  const int rect_h = (hr + 3) * RW + hc + 3;
  // the first seven levels (the window of the first outputs, nl >= 7) in one batch of loads,
  // the arms of level 0 with them
  {
    double pt[RING], ph[RING];
#pragma unroll
    for (int m = 0; m < RING; ++m) {
      pt[m] = tile_ok ? x[(long long)m * np + tplane] : 0.0;
      ph[m] = halo_ok ? x[(long long)m * np + hplane] : 0.0;
    }
#pragma unroll
    for (int m = 0; m < RING; ++m) {
      XR[m * (RH * RW) + rect_t] = pt[m];
      if (t < NHALO) XR[m * (RH * RW) + rect_h] = ph[m];
    }
  }
  double arm_next = arm_ok ? x[aplane] : 0.0;  // arms of the next level w to be formed
  double pre_t = 0.0, pre_h = 0.0;              // the level after the staged ones
  if (nl > RING) {
    pre_t = tile_ok ? x[(long long)RING * np + tplane] : 0.0;
    pre_h = halo_ok ? x[(long long)RING * np + hplane] : 0.0;
  }
  int next_w = 0, next_j = 0;
  __syncthreads();

  for (int lt = RING - 1; lt < nl; ++lt) {
    if (lt >= RING) {
      // stage level lt, then start the loads of level lt + 1
      double* xr = XR + (lt % RING) * (RH * RW);
      xr[rect_t] = pre_t;
      if (t < NHALO) xr[rect_h] = pre_h;
      if (lt + 1 < nl) {
        const long long off = (long long)(lt + 1) * np;
        pre_t = tile_ok ? x[off + tplane] : 0.0;
        pre_h = halo_ok ? x[off + hplane] : 0.0;
      }
      __syncthreads();
    }
    while (next_w < nl && win_top(next_w, nl) == lt) {
      const int w = next_w++;
      // xs = D_sig x at level w over the tile and its three-column halo; x of the arms
      {
        const int s0 = ssig[w];
        const double* ws = wsig + w * 7;
        double st = 0.0, sh = 0.0;
#pragma unroll
        for (int m = 0; m < 7; ++m) {
          const double* lv = XR + ((s0 + m) % RING) * (RH * RW);
          st += ws[m] * lv[rect_t];
          if (t < NHALO) sh += ws[m] * lv[rect_h];
        }
        XSC[rect_t] = st;
        XSR[(w % RING) * NT3 + t] = st;
        if (t < NHALO) XSC[rect_h] = sh;
        if (t < T3Y * 6) XAX[t] = arm_next;
        else if (t < NHALO) XAY[t - T3Y * 6] = arm_next;
        if (w + 1 < nl) arm_next = arm_ok ? x[(long long)(w + 1) * np + aplane] : 0.0;
      }
      __syncthreads();
      const double* xw = XR + (w % RING) * (RH * RW);
      const double sw = sig[w];
      // x at a tile-row position of the six-column neighbourhood, and at a tile-column one
      auto x_row = [&](int cc, int rr) {
        if (cc >= -3 && cc < T3X + 3) return xw[(rr + 3) * RW + cc + 3];
        return XAX[rr * 6 + (cc < -3 ? cc + 6 : cc - T3X)];
      };
      auto x_col = [&](int cc, int rr) {
        if (rr >= -3 && rr < T3Y + 3) return xw[(rr + 3) * RW + cc + 3];
        return XAY[(rr < -3 ? rr + 6 : rr - T3Y) * T3X + cc];
      };
      // G_chi at the tile rows x (tile + chi halo), G_gam at the tile columns x (tile + gamma halo)
      auto g_chi = [&](int cc, int rr, int gcc, double a, double b) {
        int row, st;
        win7(P.per_x ? cc : gcc, ncol, P.per_x, row, st);
        const int o = P.per_x ? cc - 3 : st - c0;
        double d = 0.0;
#pragma unroll
        for (int m = 0; m < 7; ++m) d += wx[row * 7 + m] * x_row(o + m, rr);
        return d + (a - sw * b) * XSC[(rr + 3) * RW + cc + 3];
      };
      auto g_gam = [&](int cc, int rr, int grr, double a, double b) {
        int row, st;
        win7(P.per_y ? rr : grr, nrow, P.per_y, row, st);
        const int o = P.per_y ? rr - 3 : st - r0;
        double d = 0.0;
#pragma unroll
        for (int m = 0; m < 7; ++m) d += wy[row * 7 + m] * x_col(cc, o + m);
        return d + (a - sw * b) * XSC[(rr + 3) * RW + cc + 3];
      };
      if (tile_ok) {
        GXB[tr * RW + tc + 3] = g_chi(tc, tr, gc, axp, bxp);
        GYB[(tr + 3) * T3X + tc] = g_gam(tc, tr, gr, ayp, byp);
      }
      if (t < 48) {
        const int k = t < 24 ? t % 3 : 3 + (t - 24) % 3;
        GXB[hr * RW + hc + 3] = halo_ok ? g_chi(hc, hr, hgc, GHX[(hr * 6 + k) * 2], GHX[(hr * 6 + k) * 2 + 1]) : 0.0;
      } else if (t < NHALO) {
        const int k = hr < 0 ? hr + 3 : 3 + hr - T3Y;
        GYB[(hr + 3) * T3X + hc] =
            halo_ok ? g_gam(hc, hr, hgr, GHY[(k * T3X + hc) * 2], GHY[(k * T3X + hc) * 2 + 1]) : 0.0;
      }
      __syncthreads();
      // the level terms of y at level w (the full row where it is a boundary row)
      if (tile_ok) {
        double v;
        if (w == nz || (ghost_c && ghost_r) || (w == 0 && (ghost_c || ghost_r))) {
          v = xw[rect_t];
        } else if (w == 0) {
          v = 0.0;  // the bed row is formed at level 1
        } else if (ghost_c) {
          v = gc == 0 ? -GXB[tr * RW + tc + 4] : GXB[tr * RW + tc + 2];
        } else if (ghost_r) {
          v = gr == 0 ? -GYB[(tr + 4) * T3X + tc] : GYB[(tr + 2) * T3X + tc];
        } else {
          double dgx = 0.0, dxs = 0.0, dgy = 0.0, dys = 0.0;
#pragma unroll
          for (int m = 0; m < 7; ++m) {
            const double a = wx[rowx * 7 + m], b = wy[rowy * 7 + m];
            dgx += a * GXB[tr * RW + ox + m + 3];
            dxs += a * XSC[(tr + 3) * RW + ox + m + 3];
            dgy += b * GYB[(oy + m + 3) * T3X + tc];
            dys += b * XSC[(oy + m + 3) * RW + tc + 3];
          }
          v = dgx + (axc - sw * bxc) * dxs + dgy + (ayc - sw * byc) * dys;
          if (w == 1) {
            // bed row of the ghost node below: n . grad^(i-1) p with n = (-h_chi, -h_gam, -1)
            T1R[t] = -hx * GXB[tr * RW + tc + 3] - hy * GYB[(tr + 3) * T3X + tc] - ip * XSC[rect_t];
          }
        }
        T1R[(w % RING) * NT3 + t] = v;
      }
      // outputs whose sigma window is complete: the terms along sigma from this column's xs
      while (next_j < nl && win_top(next_j, nl) == w) {
        const int j = next_j++;
        if (!out_ok) continue;
        double v = T1R[(j % RING) * NT3 + t];
        if (j > 0 && j < nz && !ghost_c && !ghost_r) {
          const int s0 = ssig[j];
          double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
          for (int m = 0; m < 7; ++m) {
            const int lv = s0 + m;
            const double xs = XSR[(lv % RING) * NT3 + t] * wsig[j * 7 + m];
            sx += (axp - sig[lv] * bxp) * xs;
            sy += (ayp - sig[lv] * byp) * xs;
            sz += xs;
          }
          v += (axc - sig[j] * bxc) * sx + (ayc - sig[j] * byc) * sy + ic * ip * sz;
        }
        y[(long long)j * np + tplane] = v;
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------------------------------
// host side

struct sa_op3d {
  sa_grid3 grid;
  int ncol = 0, nrow = 0, nl = 0, nxp = 0, nyp = 0;
  long long nplane = 0, n = 0;
  hipStream_t stream = nullptr;
  char* arena = nullptr;
  Op3 P{};
  double* eta = nullptr;  // 2 x nyp x nxp (host surfaces are staged here)
  double* xs = nullptr;   // n, staging of host x
  double* ys = nullptr;   // n, staging of host y
  int* flags = nullptr;
  int blocks = 0;
  bool have_surface = false;
};

static int op3_flags(sa_op3d* op) {
  int f[NFLAGS];
  HIPCHK(hipMemcpyAsync(f, op->flags, sizeof f, hipMemcpyDeviceToHost, op->stream));
  HIPCHK(hipStreamSynchronize(op->stream));
  if (f[FLAG_GEOM]) {
    const int z[NFLAGS] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(op->flags, z, sizeof z, hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipStreamSynchronize(op->stream));
    op->have_surface = false;
    return sa_fail(SA_EGEOM, "sa_op3d: h + eta <= 0 or non-finite surface");
  }
  return SA_OK;
}

extern "C" int sa_op3d_create(const sa_grid3* grid, const double* h, void* hip_stream, sa_op3d** out) {
  if (!grid || !h || !out) return sa_fail(SA_EARG, "sa_op3d_create: null argument");
  *out = nullptr;
  for (int bc : {grid->bc_x, grid->bc_y})
    if (bc != SA_PERIODIC && bc != SA_WALLS) return sa_fail(SA_EARG, "sa_op3d_create: bad bc");
  const int per_x = grid->bc_x == SA_PERIODIC, per_y = grid->bc_y == SA_PERIODIC;
  if (grid->nz < 6 || grid->nz + 1 > NLMAX) return sa_fail(SA_EARG, "sa_op3d_create: nz must be in [6, %d]", NLMAX - 1);
  if ((per_x && grid->nx < 9) || (!per_x && grid->nx < 7) || (per_y && grid->ny < 9) || (!per_y && grid->ny < 7))
    return sa_fail(SA_EARG, "sa_op3d_create: nx, ny too small for seven-point stencils");
  if (!(grid->length_x > 0.0) || !(grid->length_y > 0.0) || !isfinite(grid->length_x) || !isfinite(grid->length_y))
    return sa_fail(SA_EARG, "sa_op3d_create: lengths must be positive");
  sa_op3d* op = new sa_op3d();
  op->grid = *grid;
  op->ncol = per_x ? grid->nx - 1 : grid->nx + 2;
  op->nrow = per_y ? grid->ny - 1 : grid->ny + 2;
  op->nxp = per_x ? grid->nx - 1 : grid->nx;
  op->nyp = per_y ? grid->ny - 1 : grid->ny;
  op->nl = grid->nz + 1;
  op->nplane = (long long)op->ncol * op->nrow;
  op->n = op->nplane * op->nl;
  if (op->n > (long long)1 << 31) {
    delete op;
    return sa_fail(SA_EARG, "sa_op3d_create: more than 2^31 unknowns");
  }
  for (long long i = 0; i < (long long)op->nxp * op->nyp; ++i)
    if (!(h[i] > 0.0) || !isfinite(h[i])) {
      delete op;
      return sa_fail(SA_EGEOM, "sa_op3d_create: depth must be positive and finite");
    }
  op->stream = (hipStream_t)hip_stream;
  const int nl = op->nl, ncol = op->ncol, nrow = op->nrow;
  const double dx = grid->length_x / (grid->nx - 1), dy = grid->length_y / (grid->ny - 1), dsig = 1.0 / (grid->nz - 1);
  // tables: sigma windows, chi and gamma windows, sigma values, extended depth
  std::vector<double> wsig((size_t)nl * 7), wxv(49), wyv(49), sigv(nl), hext((size_t)op->nplane);
  std::vector<int> ssig(nl);
  double nodes[7], c[14];
  for (int j = 0; j < nl; ++j) {
    const int st = window_start(j, nl, 7);
    for (int m = 0; m < 7; ++m) nodes[m] = (double)(st + m);
    fornberg((double)j, nodes, 7, 1, c);
    for (int m = 0; m < 7; ++m) wsig[(size_t)j * 7 + m] = c[m * 2 + 1] / dsig;
    ssig[j] = st;
    sigv[j] = (j - 1) * dsig;
  }
  for (int m = 0; m < 7; ++m) nodes[m] = (double)m;
  for (int row = 0; row < 7; ++row) {
    fornberg((double)row, nodes, 7, 1, c);
    for (int m = 0; m < 7; ++m) {
      wxv[row * 7 + m] = c[m * 2 + 1] / dx;
      wyv[row * 7 + m] = c[m * 2 + 1] / dy;
    }
  }
  auto phys = [](int i, int n, int periodic) { return periodic ? i : (i == 0 ? 1 : (i == n - 1 ? n - 4 : i - 1)); };
  for (int r = 0; r < nrow; ++r)
    for (int cc = 0; cc < ncol; ++cc)
      hext[(size_t)r * ncol + cc] = h[(size_t)phys(r, nrow, per_y) * op->nxp + phys(cc, ncol, per_x)];
  // one device arena
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += (bytes + 255) & ~(size_t)255; return o; };
  const size_t o_wsig = take(wsig.size() * 8), o_ssig = take((size_t)nl * 4), o_wx = take(49 * 8), o_wy = take(49 * 8),
               o_sig = take((size_t)nl * 8), o_h = take(hext.size() * 8), o_geo = take((size_t)NGEO * op->nplane * 8),
               o_flags = take(NFLAGS * 4), o_eta = take((size_t)2 * op->nxp * op->nyp * 8),
               o_xs = take((size_t)op->n * 8), o_ys = take((size_t)op->n * 8);
  if (hipMalloc((void**)&op->arena, off) != hipSuccess) {
    delete op;
    return sa_fail(SA_EOOM, "sa_op3d_create: %zu bytes of device memory", off);
  }
  char* A = op->arena;
  std::vector<char> img(o_geo, 0);
  memcpy(img.data() + o_wsig, wsig.data(), wsig.size() * 8);
  memcpy(img.data() + o_ssig, ssig.data(), (size_t)nl * 4);
  memcpy(img.data() + o_wx, wxv.data(), 49 * 8);
  memcpy(img.data() + o_wy, wyv.data(), 49 * 8);
  memcpy(img.data() + o_sig, sigv.data(), (size_t)nl * 8);
  memcpy(img.data() + o_h, hext.data(), hext.size() * 8);
  const int z[NFLAGS] = {0, 0, 0, 0};
  if (hipMemcpyAsync(A, img.data(), img.size(), hipMemcpyHostToDevice, op->stream) != hipSuccess ||
      hipMemcpyAsync(A + o_flags, z, sizeof z, hipMemcpyHostToDevice, op->stream) != hipSuccess ||
      hipStreamSynchronize(op->stream) != hipSuccess) {
    (void)hipFree(op->arena);
    delete op;
    return sa_fail(SA_EDEVICE, "sa_op3d_create: upload failed");
  }
  Op3& P = op->P;
  P.ncol = ncol; P.nrow = nrow; P.nl = nl; P.nz = grid->nz; P.nxp = op->nxp; P.nyp = op->nyp;
  P.per_x = per_x; P.per_y = per_y;
  // tiles next to a wall keep at least four columns (rows): their shifted windows stay inside
  // the staged halo
  P.c_shift = (!per_x && ncol % T3X >= 1 && ncol % T3X <= 3) ? T3X / 2 : 0;
  P.r_shift = (!per_y && nrow % T3Y >= 1 && nrow % T3Y <= 3) ? T3Y / 2 : 0;
  P.ntx = (ncol + P.c_shift + T3X - 1) / T3X;
  const int nty = (nrow + P.r_shift + T3Y - 1) / T3Y;
  op->blocks = P.ntx * nty;
  P.nplane = op->nplane;
  P.wsig = (const double*)(A + o_wsig); P.ssig = (const int*)(A + o_ssig);
  P.wx = (const double*)(A + o_wx); P.wy = (const double*)(A + o_wy); P.sig = (const double*)(A + o_sig);
  P.hext = (const double*)(A + o_h); P.geo = (double*)(A + o_geo); P.flags = (int*)(A + o_flags);
  op->flags = P.flags;
  op->eta = (double*)(A + o_eta);
  op->xs = (double*)(A + o_xs);
  op->ys = (double*)(A + o_ys);
  if (hipFuncSetAttribute((const void*)sa_operator3_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)LDS3_BYTES) != hipSuccess) {
    (void)hipFree(op->arena);
    delete op;
    return sa_fail(SA_EDEVICE, "sa_op3d_create: LDS attribute");
  }
  *out = op;
  return SA_OK;
}

extern "C" int sa_op3d_set_surface(sa_op3d* op, const double* eta_prev, const double* eta_cur, int32_t mem) {
  if (!op || !eta_prev || !eta_cur) return sa_fail(SA_EARG, "sa_op3d_set_surface: null argument");
  const size_t np = (size_t)op->nxp * op->nyp;
  const double *ep = eta_prev, *ec = eta_cur;
  if (mem == SA_MEM_HOST) {
    for (size_t i = 0; i < np; ++i)
      if (!isfinite(eta_prev[i]) || !isfinite(eta_cur[i])) return sa_fail(SA_EGEOM, "sa_op3d_set_surface: non-finite surface");
    HIPCHK(hipMemcpyAsync(op->eta, eta_prev, np * 8, hipMemcpyHostToDevice, op->stream));
    HIPCHK(hipMemcpyAsync(op->eta + np, eta_cur, np * 8, hipMemcpyHostToDevice, op->stream));
    ep = op->eta;
    ec = op->eta + np;
  } else if (mem != SA_MEM_DEVICE) {
    return sa_fail(SA_EARG, "sa_op3d_set_surface: bad mem");
  }
  const int gb = (int)((op->nplane + NT3 - 1) / NT3);
  hipLaunchKernelGGL(sa_geometry3_kernel, dim3(gb), dim3(NT3), 0, op->stream, op->P, ep, ec);
  HIPCHK(hipGetLastError());
  op->have_surface = true;
  if (mem == SA_MEM_HOST) return op3_flags(op);
  return SA_OK;
}

extern "C" int sa_op3d_apply(sa_op3d* op, const double* x, double* y, int32_t mem) {
  if (!op || !x || !y) return sa_fail(SA_EARG, "sa_op3d_apply: null argument");
  if (!op->have_surface) return sa_fail(SA_EARG, "sa_op3d_apply: set the surfaces first");
  if (mem != SA_MEM_HOST && mem != SA_MEM_DEVICE) return sa_fail(SA_EARG, "sa_op3d_apply: bad mem");
  const double* xd = x;
  double* yd = y;
  if (mem == SA_MEM_HOST) {
    HIPCHK(hipMemcpyAsync(op->xs, x, (size_t)op->n * 8, hipMemcpyHostToDevice, op->stream));
    xd = op->xs;
    yd = op->ys;
  }
  hipLaunchKernelGGL(sa_operator3_kernel, dim3(op->blocks), dim3(NT3), LDS3_BYTES, op->stream, op->P, xd, yd);
  HIPCHK(hipGetLastError());
  if (mem == SA_MEM_DEVICE) return SA_OK;
  HIPCHK(hipMemcpyAsync(y, yd, (size_t)op->n * 8, hipMemcpyDeviceToHost, op->stream));
  return op3_flags(op);
}

extern "C" int sa_op3d_sync(sa_op3d* op) {
  if (!op) return sa_fail(SA_EARG, "sa_op3d_sync: null argument");
  return op3_flags(op);
}

extern "C" int64_t sa_op3d_size(const sa_op3d* op) { return op ? op->n : -1; }

extern "C" int sa_op3d_workgroups(const sa_op3d* op) { return op ? op->blocks : -1; }

extern "C" void sa_op3d_destroy(sa_op3d* op) {
  if (!op) return;
  if (op->stream) (void)hipStreamSynchronize(op->stream);
  if (op->arena) (void)hipFree(op->arena);
  delete op;
}
