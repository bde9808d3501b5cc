// C ABI of the solver library (declared in include/sawave.h): problem set-up, buffer
// ownership, kernel launches and the per-solve report log.
#include "host.h"
#include "ilu.h"

static_assert(sa::ILU_SLOTS == 2 * sa::NWAVE, "an ILU(0) step holds two rows per wavefront");

using namespace sa;

static thread_local std::string g_err;

static size_t g_solve_lds = 0;  // dynamic-LDS limit set on the solve kernel so far

const void* sa_solve_fn(int precision) {
  return precision == SA_FP32_IR ? (const void*)sa_solve_ir_kernel : (const void*)sa_solve_kernel;
}

int sa_reserve_solve_lds(size_t bytes) {
  if (bytes <= g_solve_lds) return SA_OK;
  HIPCHK(hipFuncSetAttribute(sa_solve_fn(SA_FP64), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  HIPCHK(hipFuncSetAttribute(sa_solve_fn(SA_FP32_IR), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  g_solve_lds = bytes;
  return SA_OK;
}

int sa_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

extern "C" void sa_default_options(sa_options* o) {
  memset(o, 0, sizeof *o);
  o->restart = 30;
  o->max_restarts = 200;
  o->rtol = 1e-8;
  o->precond = SA_PC_MG;
  o->nu1 = 1;
  o->nu2 = 1;
  o->omega = 0.5;
  o->max_levels = 32;
  o->guess = SA_GUESS_EWMA;
  o->k = 8;
  o->r = 0.9;
  o->seed = 0;
  o->n_init = 0;
  o->tau_drop = 1e-7;
  o->precision = SA_FP64;
  o->rtol_inner = 1e-4;
  o->max_refine = 200;
  o->cluster = 0;
  o->profile = 0;
  o->coarse_max = 700;
  o->window = 16;
  o->decay = SA_DECAY_SOLVES;
  o->decay_dtau = 1.0;
}

extern "C" const char* sa_last_error(void) { return g_err.c_str(); }

extern "C" const char* sa_build_info(void) {
  static char info[128];
  snprintf(info, sizeof info, "sawave gfx950 HIP %d.%d block=%d kmax=%d", HIP_VERSION_MAJOR, HIP_VERSION_MINOR,
           BLOCK, KMAX);
  return info;
}

extern "C" int sa_sketch_draws(uint64_t seed, int64_t index, int32_t k, double* out) {
  if (!out || k < 1 || k > 64 || index < 0) return sa_fail(SA_EARG, "sa_sketch_draws: bad arguments");
  splitmix_gaussians(seed, index, k, out);
  return SA_OK;
}

// ---------------------------------------------------------------------------------------
// host-side tables

// second-order centred dh/dx, d2h/dx2 on the extended column grid
static void centred_h(const std::vector<double>& h, int periodic, double dx, std::vector<double>& hx,
                      std::vector<double>& hxx) {
  const int nc = (int)h.size();
  hx.assign(nc, 0.0);
  hxx.assign(nc, 0.0);
  for (int c = 0; c < nc; ++c) {
    int cm = c - 1, cp = c + 1;
    if (periodic) {
      cm = (cm + nc) % nc;
      cp = cp % nc;
    } else if (c == 0 || c == nc - 1) {
      continue;  // ghost columns: never used by a row that survives
    }
    hx[c] = (h[cp] - h[cm]) / (2.0 * dx);
    hxx[c] = (h[cp] - 2.0 * h[c] + h[cm]) / (dx * dx);
  }
}

static constexpr int TM_HOST = 64;  // the V-cycle's default tile width (device TM)

static size_t round_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Elimination factors of the vertical line systems of the still-water operator on one level:
// after combining the bed row with row 1 (factor gam) each column is tridiagonal; pc are the
// elimination ratios and inv the inverse pivots of its LU factorisation. Ghost columns of
// wall grids are diagonal (pc = 0, gam = 0). uniform: every column has the same factors.
static void line_factors(int ncol, int nl, int periodic, double dx, double dsig, const std::vector<double>& ihv,
                         const std::vector<double>& hxv, const std::vector<double>& hxxv, bool uniform,
                         std::vector<double>& pc, std::vector<double>& inv, std::vector<double>& lov,
                         std::vector<double>& gam) {
  const int nz = nl - 1, ncf = uniform ? 1 : ncol;
  const double rds = 1.0 / dsig, rdx = 1.0 / dx;
  pc.assign((size_t)nl * ncf, 0.0);
  inv.assign((size_t)nl * ncf, 1.0);
  lov.assign((size_t)nl * ncf, 0.0);
  gam.assign(ncf, 0.0);
  for (int c = 0; c < ncf; ++c) {
    if (!periodic && (c == 0 || c == ncol - 1)) {
      for (int j = 1; j < nz; ++j) inv[(size_t)j * ncf + c] = 1.0 / (0.5 * rdx);
      continue;
    }
    const double ih = ihv[c], hx = hxv[c], hxx = hxxv[c];
    auto coefs = [&](int j, double& lo, double& di, double& up) {
      const double oms = 1.0 - (j - 1) * dsig;
      const double sv = hx * oms * ih;
      const double sxx = oms * hxx * ih - 2.0 * oms * hx * hx * ih * ih;
      const double a = (sv * sv + ih * ih) * rds * rds, b = sxx * 0.5 * rds;
      lo = a - b;
      up = a + b;
      di = -2.0 * rdx * rdx - 2.0 * a;
    };
    const double q = hx * (hx * ih) + ih;
    const double a0 = 0.5 * rds * q, c0 = -0.5 * rds * q;
    double l1, d1, u1;
    coefs(1, l1, d1, u1);
    const double a0p = a0 - c0 * l1 / u1;
    const double b0p = -c0 * d1 / u1;
    gam[c] = c0 / u1;
    double pcp = b0p / a0p;
    pc[c] = pcp;
    inv[c] = 1.0 / a0p;
    for (int j = 1; j < nz; ++j) {
      double lo, di, up;
      coefs(j, lo, di, up);
      const double iv = 1.0 / (di - lo * pcp);
      pcp = up * iv;
      pc[(size_t)j * ncf + c] = pcp;
      inv[(size_t)j * ncf + c] = iv;
      lov[(size_t)j * ncf + c] = lo;
    }
  }
}

static int tiles_host(int ncol, int periodic, int tw) {
  int nt = (ncol + tw - 1) / tw;
  if (!periodic && nt > 1 && ncol - (nt - 1) * tw < 4) --nt;
  return nt;
}

// ---------------------------------------------------------------------------------------

// Builds a problem; with bytes_only set it validates, sizes the device arena, stores its size
// there and returns without touching the device.
static int create_impl(const sa_grid* grid, const double* h, const sa_options* optin, void* hip_stream,
                       sa_problem** out, int64_t* bytes_only) {
  if (!grid || !h || (!out && !bytes_only)) return sa_fail(SA_EARG, "sa_create: null argument");
  if (out) *out = nullptr;
  sa_options opt;
  if (optin) opt = *optin; else sa_default_options(&opt);
  const int periodic = grid->bc == SA_PERIODIC;
  if (grid->bc != SA_PERIODIC && grid->bc != SA_WALLS) return sa_fail(SA_EARG, "sa_create: bc must be SA_PERIODIC or SA_WALLS");
  if (grid->nz < 6 || grid->nz + 1 > NLMAX) return sa_fail(SA_EARG, "sa_create: nz must be in [6, %d]", NLMAX - 1);
  const int ncol = periodic ? grid->nx - 1 : grid->nx + 2;
  if ((periodic && ncol < 8) || (!periodic && grid->nx < 7))
    return sa_fail(SA_EARG, "sa_create: nx too small for seven-point stencils");
  if (!(grid->length > 0.0) || !isfinite(grid->length)) return sa_fail(SA_EARG, "sa_create: length must be positive");
  if (opt.restart < 1 || opt.restart > MMAX) return sa_fail(SA_EARG, "sa_create: restart must be in [1, %d]", MMAX);
  if (opt.max_restarts < 0) return sa_fail(SA_EARG, "sa_create: max_restarts < 0");
  if (!(opt.rtol >= 0.0)) return sa_fail(SA_EARG, "sa_create: rtol must be >= 0");
  if (opt.precond < SA_PC_NONE || opt.precond > SA_PC_ILU0) return sa_fail(SA_EARG, "sa_create: unknown precond");
  if (opt.precond == SA_PC_ILU0 && opt.precision != SA_FP64)
    return sa_fail(SA_EARG, "sa_create: the ILU(0) preconditioner runs in FP64 only");
  if (opt.nu1 < 0 || opt.nu2 < 0 || opt.nu1 > 8 || opt.nu2 > 8) return sa_fail(SA_EARG, "sa_create: sweeps in [0, 8]");
  if (opt.precond == SA_PC_LINE && opt.nu1 < 1) return sa_fail(SA_EARG, "sa_create: line preconditioner needs nu1 >= 1");
  if (opt.guess < SA_GUESS_COLD || opt.guess > SA_GUESS_RANGE) return sa_fail(SA_EARG, "sa_create: unknown guess mode");
  if (opt.k < 1 || opt.k > KMAX) return sa_fail(SA_EARG, "sa_create: k must be in [1, %d]", KMAX);
  if (opt.guess == SA_GUESS_RANGE && (opt.window < opt.k || opt.window > KWIN))
    return sa_fail(SA_EARG, "sa_create: window must be in [k, %d]", KWIN);
  if (!(opt.r >= 0.0 && opt.r <= 1.0)) return sa_fail(SA_EARG, "sa_create: r must be in [0, 1]");
  if (opt.decay != SA_DECAY_SOLVES && opt.decay != SA_DECAY_TIME) return sa_fail(SA_EARG, "sa_create: unknown decay");
  if (opt.orthonormalize != 0 && opt.orthonormalize != 1) return sa_fail(SA_EARG, "sa_create: orthonormalize is 0 or 1");
  if (opt.orthonormalize && opt.guess != SA_GUESS_RANGE)
    return sa_fail(SA_EARG, "sa_create: orthonormalize applies to the range finder only");
  if (opt.decay == SA_DECAY_TIME && opt.guess != SA_GUESS_EWMA)
    return sa_fail(SA_EARG, "sa_create: SA_DECAY_TIME applies to the EWMA sketch only");
  if (opt.decay == SA_DECAY_TIME && !(opt.decay_dtau > 0.0 && isfinite(opt.decay_dtau)))
    return sa_fail(SA_EARG, "sa_create: decay_dtau must be positive");
  if (opt.precision != SA_FP64 && opt.precision != SA_FP32_IR) return sa_fail(SA_EARG, "sa_create: unknown precision");
  if (opt.precision == SA_FP32_IR && !(opt.rtol_inner > 0.0 && opt.rtol_inner < 1.0))
    return sa_fail(SA_EARG, "sa_create: rtol_inner must be in (0, 1)");
  if (opt.precision == SA_FP32_IR && opt.max_refine < 1) return sa_fail(SA_EARG, "sa_create: max_refine >= 1");
  if (opt.max_levels < 1) return sa_fail(SA_EARG, "sa_create: max_levels >= 1");
  if (opt.coarse_max < 1 || opt.coarse_max > COARSE_MAX) return sa_fail(SA_EARG, "sa_create: coarse_max in [1, %d]", COARSE_MAX);
  const int nphys = periodic ? grid->nx - 1 : grid->nx;
  for (int i = 0; i < nphys; ++i)
    if (!(h[i] > 0.0) || !isfinite(h[i])) return sa_fail(SA_EGEOM, "sa_create: depth must be positive and finite");

  int ndev = 0;
  if (!bytes_only && (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1))
    return sa_fail(SA_ENOTBUILT, "sa_create: no HIP device");

  sa_problem* p = new sa_problem();
  p->grid = *grid;
  p->opt = opt;
  p->stream = (hipStream_t)hip_stream;
  if (!bytes_only) (void)hipGetDevice(&p->device);
  p->ncol = ncol;
  p->nl = grid->nz + 1;
  p->n = ncol * p->nl;
  p->nphys = nphys;
  const int nl = p->nl, n = p->n;
  const double dx = grid->length / (grid->nx - 1), dsig = 1.0 / (grid->nz - 1);

  // ---- tables
  OperatorTables tb;
  operator_tables(ncol, nl, nphys, periodic, dx, dsig, h, tb);
  const std::vector<double>&wsig = tb.wsig, &wchi = tb.wchi, &sig = tb.sig, &hext = tb.hext, &hchi = tb.hchi;
  const std::vector<int>& ssig = tb.ssig;
  IluFactors ilu;
  if (opt.precond == SA_PC_ILU0) {
    const int rc = ilu_still_water(ncol, nl, periodic, tb, ilu);
    if (rc != 0) {
      delete p;
      return sa_fail(SA_EARG, "sa_create: ILU(0) of the still-water operator failed (%s)",
                     rc == -1 ? "missing diagonal" : rc == -2 ? "zero pivot" : "a factor row longer than 64");
    }
  }

  // ---- still-water hierarchy
  struct HL { int nx, ncol; double dx; std::vector<double> h, ih, hx, hxx, fpc, finv, flo, fgam; int fstride; };
  std::vector<HL> levs;
  {
    HL l0;
    l0.nx = grid->nx; l0.ncol = ncol; l0.dx = dx;
    l0.h = hext;
    for (double v : l0.h) l0.ih.push_back(1.0 / v);
    centred_h(l0.h, periodic, dx, l0.hx, l0.hxx);
    levs.push_back(l0);
    std::vector<double> hphys(h, h + nphys);
    const int maxlev = opt.precond == SA_PC_MG ? (opt.max_levels < MAXLEV ? opt.max_levels : MAXLEV) : 1;
    while ((int)levs.size() < maxlev) {
      const HL& f = levs.back();
      if ((long)f.ncol * nl <= opt.coarse_max) break;
      HL c;
      if (periodic) {
        if (f.ncol % 2 || f.ncol / 2 < 4) break;
        c.ncol = f.ncol / 2; c.nx = c.ncol + 1;
      } else {
        if ((f.nx - 1) % 2 || (f.nx - 1) / 2 + 1 < 3) break;
        c.nx = (f.nx - 1) / 2 + 1; c.ncol = c.nx + 2;
      }
      c.dx = grid->length / (c.nx - 1);
      std::vector<double> hc;
      for (size_t i = 0; i < hphys.size(); i += 2) hc.push_back(hphys[i]);
      hphys = hc;
      c.h = extend_columns(hphys.data(), (int)hphys.size(), periodic);
      for (double v : c.h) c.ih.push_back(1.0 / v);
      centred_h(c.h, periodic, c.dx, c.hx, c.hxx);
      levs.push_back(c);
    }
  }
  const int nlev = (int)levs.size();
  const int cn = levs.back().ncol * nl;
  int tail = nlev - 1;  // first level one preconditioner tile wide (run by one workgroup)
  for (int l = 0; l < nlev - 1; ++l)
    if (levs[l].ncol <= 64) { tail = l; break; }
  for (auto& L : levs) {
    bool uniform = periodic != 0;
    for (int c = 1; c < L.ncol && uniform; ++c)
      uniform = L.h[c] == L.h[0] && L.hx[c] == L.hx[0] && L.hxx[c] == L.hxx[0];
    line_factors(L.ncol, nl, periodic, L.dx, dsig, L.ih, L.hx, L.hxx, uniform, L.fpc, L.finv, L.flo, L.fgam);
    L.fstride = uniform ? 0 : L.ncol;
  }
  std::vector<double> cinv;
  size_t cinv_n = 0;
  if (opt.precond == SA_PC_MG) {
    if (cn > COARSE_MAX) {
      delete p;
      return sa_fail(SA_EARG, "sa_create: coarsest grid has %d unknowns (> %d); allow more levels", cn, COARSE_MAX);
    }
    cinv_n = (size_t)cn * cn;
  }

  // ---- cluster size and LDS
  const int m = opt.restart, k = opt.k;
  // default cluster: one 64-column preconditioner tile of the finest level per workgroup
  // (the passes of the V-cycle then take one tile-latency each), at most 64 workgroups
  int G = opt.cluster;
  // one 32-column tile of the finest level per workgroup, at most 256 (one per CU: the
  // cluster sums spread their loads over the workgroup and the coarse V-cycle levels meet
  // at sub-cluster barriers, so the whole chip pays on the large grids)
  if (G <= 0) G = (ncol + 31) / 32 < 256 ? (ncol + 31) / 32 : 256;
  if (opt.precond == SA_PC_ILU0) G = 1;  // the substitutions run on one workgroup
  hipDeviceProp_t prop{};
  if (!bytes_only && hipGetDeviceProperties(&prop, p->device) != hipSuccess) {
    delete p;
    return sa_fail(SA_EDEVICE, "hipGetDeviceProperties failed");
  }
  const size_t head = (size_t)PSTRIDE + NWAVE * (MMAX + 2) + (size_t)(m + 1) * m + 2 * m + 2 * (m + 1) + m + KMAX +
                      4 * KMAX * KMAX + 8 + 16;
  const int TWMh = TX + 3;
  auto opcoef = [&](int W) { return (size_t)(49 + 9 * nl + 5 * (W + 6)); };
  const size_t need_op = (size_t)(TWMh + 12 + 2 * (TWMh + 6)) * nl + opcoef(TWMh) + NWAVE;
  // block operator of the guess on tiles of tg columns (widest tile tg + 3)
  auto need_gram_of = [&](int tg) {
    const int Wg = tg + 3;
    const bool sk = opt.guess == SA_GUESS_EWMA || opt.guess == SA_GUESS_RANGE;
    return sk ? (size_t)(k * Wg + Wg + Wg + 12 + 2 * (Wg + 6)) * nl + opcoef(Wg) : 0;
  };
  const int TMSh = 64 + 4;  // preconditioner tile with its 2-column halo
  size_t need_pc = (size_t)5 * TMSh * nl + 5 * TMSh;
  if (opt.precond == SA_PC_MG && need_pc < (size_t)cn + BLOCK)
    need_pc = (size_t)cn + BLOCK;  // coarsest solve: f and partial sums
  // ILU(0): z in the phase scratch during the substitutions where it fits
  const bool ilu_lds = opt.precond == SA_PC_ILU0 && n <= ILU_LDS_MAX;
  if (ilu_lds && need_pc < (size_t)n) need_pc = (size_t)n;
  // V = Q of the range finder: the sketch's Gram stages chunks of 512 elements of its k columns
  const size_t need_qr = (opt.guess == SA_GUESS_RANGE && opt.orthonormalize) ? (size_t)k * 512 : 0;
  auto big_of = [&](size_t need_gram) {
    size_t big = need_op;
    if (need_gram > big) big = need_gram;
    if (need_qr > big) big = need_qr;
    if (need_pc > big) big = need_pc;
    if (big < 2 * (size_t)BLOCK) big = 2 * (size_t)BLOCK;  // the Gram pass combines per-thread partials
    return big;
  };
  // the widest guess tiles (64, 32 or 16 columns: fewer tiles per workgroup) whose block
  // operator fits the 160 KB of LDS
  int txg = 64;
  size_t big = big_of(need_gram_of(txg));
  while (txg > 16 && (head + big) * sizeof(double) > 160 * 1024) {
    txg /= 2;
    big = big_of(need_gram_of(txg));
  }
  // Line-solve constants (column data, factors, gamma) of the cluster levels on which every
  // workgroup owns at most one tile, kept in LDS for a whole solve where there is room (staged
  // once per solve instead of in every V-cycle pass), in the solve's precision (floats for the
  // FP32 V-cycle of the refinement path). The block lives in the part of the phase scratch that
  // only the guess uses (the Gram tiles): while GMRES runs, the scratch holds at most an
  // operator tile or a preconditioner tile.
  std::vector<int> res_off(nlev, -1);
  size_t res_total = 0;
  const size_t res_esz = opt.precision == SA_FP32_IR ? sizeof(float) : sizeof(double);
  const size_t gmres_scratch = need_op > need_pc ? need_op : need_pc;
  if (opt.precond == SA_PC_MG && opt.nu1 == 1 && opt.nu2 >= 1) {
    const int lt = (G > 1 && tail < nlev - 1) ? tail : nlev - 1;
    for (int l = 0; l < lt; ++l) {
      const int tw = (levs[l].ncol + 31) / 32 <= G ? 32 : TM_HOST;
      if ((levs[l].ncol + tw - 1) / tw > G) continue;
      // a uniform level keeps its column data and one shared set of factors and gamma
      const size_t sz = levs[l].fstride == 0 ? (size_t)4 * (tw + 4) + 3 * nl + 1 : (size_t)(5 + 3 * nl) * (tw + 4);
      if ((head + gmres_scratch) * sizeof(double) + (res_total + sz) * res_esz > 160 * 1024) continue;
      res_off[l] = (int)res_total;
      res_total += sz;
    }
  }
  const size_t res_end = (head + gmres_scratch) * sizeof(double) + (res_total * res_esz + 7) / 8 * 8;
  p->lds_solve = (head + big) * sizeof(double);
  if (res_total > 0 && res_end > p->lds_solve) p->lds_solve = res_end;
  p->lds_op = need_op * sizeof(double);
  p->lds_pc = need_pc * sizeof(double);
  if (p->lds_solve > 160 * 1024 && (bytes_only || p->lds_solve > (size_t)prop.sharedMemPerBlock)) {
    delete p;
    return sa_fail(SA_EARG, "sa_create: %zu bytes of LDS needed (nz, k or restart too large)", p->lds_solve);
  }
  if (!bytes_only && sa_reserve_solve_lds(p->lds_solve) != SA_OK) {
    delete p;
    return SA_EDEVICE;
  }
  if (G > 1 && !bytes_only) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sa_solve_fn(opt.precision), BLOCK, p->lds_solve) != hipSuccess ||
        per_cu < 1 || G > per_cu * prop.multiProcessorCount) {
      delete p;
      return sa_fail(SA_EARG, "sa_create: cluster of %d workgroups cannot be co-resident", G);
    }
  }
  p->G = G;

  // ---- device arena
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += round_up(bytes); return o; };
  const size_t o_wsig = take(wsig.size() * 8), o_ssig = take(ssig.size() * 4), o_wchi = take(49 * 8),
               o_sig = take(nl * 8), o_h = take(ncol * 8), o_hchi = take(ncol * 8), o_geo = take(4 * (size_t)ncol * 8);
  std::vector<size_t> o_lh(nlev), o_lih(nlev), o_lhx(nlev), o_lhxx(nlev), o_lf(nlev), o_lu(nlev), o_lo(nlev),
      o_fpc(nlev), o_finv(nlev), o_flo(nlev), o_fgam(nlev);
  const bool ir = opt.precision == SA_FP32_IR;
  std::vector<size_t> o_lf32(nlev, 0), o_lu32(nlev, 0), o_lo32(nlev, 0), o_fpc32(nlev, 0), o_finv32(nlev, 0),
      o_flo32(nlev, 0), o_fgam32(nlev, 0);
  for (int l = 0; l < nlev; ++l) {
    const size_t nlv = (size_t)levs[l].ncol * nl;
    // column data h | 1/h | h_x | h_xx and factors lo | pc | inv in one block each, so that a
    // kernel reaches part q at base + q * stride
    const size_t nc8 = (size_t)levs[l].ncol * 8, fs8 = levs[l].fpc.size() * 8;
    o_lh[l] = take(4 * nc8); o_lih[l] = o_lh[l] + nc8; o_lhx[l] = o_lh[l] + 2 * nc8; o_lhxx[l] = o_lh[l] + 3 * nc8;
    o_flo[l] = take(3 * fs8); o_fpc[l] = o_flo[l] + fs8; o_finv[l] = o_flo[l] + 2 * fs8;
    o_fgam[l] = take(levs[l].fgam.size() * 8);
    o_lf[l] = take(nlv * 8); o_lu[l] = take(nlv * 8); o_lo[l] = take(nlv * 8);
    if (ir) {
      const size_t fs4 = levs[l].fpc.size() * 4;
      o_flo32[l] = take(3 * fs4); o_fpc32[l] = o_flo32[l] + fs4; o_finv32[l] = o_flo32[l] + 2 * fs4;
      o_fgam32[l] = take(levs[l].fgam.size() * 4);
      o_lf32[l] = take(nlv * 4); o_lu32[l] = take(nlv * 4); o_lo32[l] = take(nlv * 4);
    }
  }
  const size_t o_cinv = take(cinv_n * 8 + 8);
  const size_t o_cinv32 = ir ? take(cinv_n * 4 + 8) : 0;
  const size_t o_V32 = ir ? take((size_t)(m + 1) * n * 4) : 0, o_t32 = ir ? take((size_t)n * 4) : 0,
               o_r32 = ir ? take((size_t)n * 4) : 0;
  const size_t o_x = take((size_t)n * 8), o_xc = take((size_t)n * 8), o_r = take((size_t)n * 8),
               o_rc = take((size_t)n * 8), o_t = take((size_t)n * 8), o_V = take((size_t)(m + 1) * n * 8);
  const bool range = opt.guess == SA_GUESS_RANGE;
  const size_t ysz = opt.guess == SA_GUESS_EWMA || range ? (size_t)k * n * 8 : 8;
  const size_t o_Y0 = take(ysz), o_Y1 = take(range ? 8 : ysz);
  const size_t o_Xr = take(range ? (size_t)opt.window * n * 8 : 8), o_Om = take((size_t)KWIN * KMAX * 8);
  const size_t o_part = take((size_t)2 * (G + 1) * PSTRIDE * 8), o_bar = take(64 * (1 + MAXLEV)), o_flags = take(NFLAGS * 4),
               o_log = take(LOGCAP * sizeof(sa_solve_info)), o_b = take((size_t)n * 8), o_eta = take(2 * (size_t)nphys * 8),
               o_prob = take(sizeof(Problem)), o_prof = take(NPROF * 8);
  const bool il = opt.precond == SA_PC_ILU0;
  const size_t o_ifr = take(il ? ilu.frow.size() * 4 : 8), o_ifc = take(il ? ilu.fcol.size() * 4 : 8),
               o_ifv = take(il ? ilu.fval.size() * 8 : 8), o_ibr = take(il ? ilu.brow.size() * 4 : 8),
               o_ibc = take(il ? ilu.bcol.size() * 4 : 8), o_ibv = take(il ? ilu.bval.size() * 8 : 8),
               o_idi = take(il ? ilu.bdinv.size() * 8 : 8);
  p->arena_bytes = off;
  if (bytes_only) {
    *bytes_only = (int64_t)off;
    delete p;
    return SA_OK;
  }
  if (cinv_n) {
    cinv.resize(cinv_n);
    const HL& L = levs.back();
    if (dense_still_water_inverse(L.ncol, L.nx, nl, periodic, L.dx, dsig, L.h.data(), L.hx.data(), L.hxx.data(),
                                  cinv.data()) != 0) {
      delete p;
      return sa_fail(SA_EARG, "sa_create: singular coarsest operator");
    }
    // few rows per workgroup: keep the inverse row by row (each workgroup then streams its own
    // rows with coalesced loads); else transposed (a thread per row, coalesced across rows)
    if ((cn + G - 1) / G <= CN_ROWS) {
      std::vector<double> rm(cinv_n);
      for (int i = 0; i < cn; ++i)
        for (int j = 0; j < cn; ++j) rm[(size_t)i * cn + j] = cinv[(size_t)j * cn + i];
      cinv.swap(rm);
    }
  }
  if (hipMalloc((void**)&p->arena, off) != hipSuccess) {
    delete p;
    return sa_fail(SA_EOOM, "sa_create: cannot allocate %zu bytes of device memory", off);
  }
  char* A = p->arena;
  auto up = [&](size_t o, const void* src, size_t bytes) {
    return hipMemcpy(A + o, src, bytes, hipMemcpyHostToDevice);
  };
  hipError_t e = hipMemsetAsync(A, 0, off, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e == hipSuccess) e = up(o_wsig, wsig.data(), wsig.size() * 8);
  if (e == hipSuccess) e = up(o_ssig, ssig.data(), ssig.size() * 4);
  if (e == hipSuccess) e = up(o_wchi, wchi.data(), 49 * 8);
  if (e == hipSuccess) e = up(o_sig, sig.data(), nl * 8);
  if (e == hipSuccess) e = up(o_h, hext.data(), ncol * 8);
  if (e == hipSuccess) e = up(o_hchi, hchi.data(), ncol * 8);
  for (int l = 0; l < nlev && e == hipSuccess; ++l) {
    e = up(o_lh[l], levs[l].h.data(), levs[l].ncol * 8);
    if (e == hipSuccess) e = up(o_lhx[l], levs[l].hx.data(), levs[l].ncol * 8);
    if (e == hipSuccess) e = up(o_lhxx[l], levs[l].hxx.data(), levs[l].ncol * 8);
    if (e == hipSuccess) e = up(o_lih[l], levs[l].ih.data(), levs[l].ncol * 8);
    if (e == hipSuccess) e = up(o_fpc[l], levs[l].fpc.data(), levs[l].fpc.size() * 8);
    if (e == hipSuccess) e = up(o_finv[l], levs[l].finv.data(), levs[l].finv.size() * 8);
    if (e == hipSuccess) e = up(o_flo[l], levs[l].flo.data(), levs[l].flo.size() * 8);
    if (e == hipSuccess) e = up(o_fgam[l], levs[l].fgam.data(), levs[l].fgam.size() * 8);
  }
  if (e == hipSuccess && !cinv.empty()) e = up(o_cinv, cinv.data(), cinv.size() * 8);
  if (il) {
    if (e == hipSuccess) e = up(o_ifr, ilu.frow.data(), ilu.frow.size() * 4);
    if (e == hipSuccess) e = up(o_ifc, ilu.fcol.data(), ilu.fcol.size() * 4);
    if (e == hipSuccess) e = up(o_ifv, ilu.fval.data(), ilu.fval.size() * 8);
    if (e == hipSuccess) e = up(o_ibr, ilu.brow.data(), ilu.brow.size() * 4);
    if (e == hipSuccess) e = up(o_ibc, ilu.bcol.data(), ilu.bcol.size() * 4);
    if (e == hipSuccess) e = up(o_ibv, ilu.bval.data(), ilu.bval.size() * 8);
    if (e == hipSuccess) e = up(o_idi, ilu.bdinv.data(), ilu.bdinv.size() * 8);
  }
  if (ir) {
    auto up32 = [&](size_t o, const std::vector<double>& v) {
      std::vector<float> f(v.begin(), v.end());
      return f.empty() ? hipSuccess : up(o, f.data(), f.size() * 4);
    };
    for (int l = 0; l < nlev && e == hipSuccess; ++l) {
      e = up32(o_fpc32[l], levs[l].fpc);
      if (e == hipSuccess) e = up32(o_finv32[l], levs[l].finv);
      if (e == hipSuccess) e = up32(o_flo32[l], levs[l].flo);
      if (e == hipSuccess) e = up32(o_fgam32[l], levs[l].fgam);
    }
    if (e == hipSuccess) e = up32(o_cinv32, cinv);
  }

  Problem& P = p->hp;
  P.ncol = ncol; P.nl = nl; P.nz = grid->nz; P.n = n; P.nphys = nphys; P.periodic = periodic;
  P.dx = dx; P.dsig = dsig;
  P.wsig = (decltype(P.wsig))(A + o_wsig); P.ssig = (decltype(P.ssig))(A + o_ssig); P.wchi = (decltype(P.wchi))(A + o_wchi);
  P.sig = (decltype(P.sig))(A + o_sig); P.h = (decltype(P.h))(A + o_h); P.hchi = (decltype(P.hchi))(A + o_hchi);
  P.geo = (decltype(P.geo))(A + o_geo);
  P.pc = opt.precond; P.nu1 = opt.nu1; P.nu2 = opt.nu2; P.nlev = nlev; P.omega = opt.omega; P.tail = tail;
  P.res_base = res_total > 0 ? (int)(head + gmres_scratch) : -1;
  P.tx = (ncol + 31) / 32 <= G ? 32 : TM_HOST;
  for (int l = 0; l < nlev; ++l) {
    Level& L = P.lev[l];
    L.ncol = levs[l].ncol; L.nx = levs[l].nx; L.dx = levs[l].dx;
    L.h = (decltype(L.h))(A + o_lh[l]); L.hx = (decltype(L.hx))(A + o_lhx[l]); L.hxx = (decltype(L.hxx))(A + o_lhxx[l]);
    L.ih = (decltype(L.ih))(A + o_lih[l]);
    L.fpc = (decltype(L.fpc))(A + o_fpc[l]); L.finv = (decltype(L.finv))(A + o_finv[l]);
    L.fgam = (decltype(L.fgam))(A + o_fgam[l]); L.fstride = levs[l].fstride;
    L.flo = (decltype(L.flo))(A + o_flo[l]);
    L.facstride = (int)levs[l].fpc.size();
    // 32-column tiles where the cluster has a workgroup for each of them (one round of tiles
    // either way, more workgroups busy), else 64 (not on the levels the rank-0 workgroup runs
    // alone)
    L.tm = (l < tail && (levs[l].ncol + 31) / 32 <= G) ? 32 : TM_HOST;
    L.res = res_off[l];
    L.f = (decltype(L.f))(A + o_lf[l]); L.u = (decltype(L.u))(A + o_lu[l]); L.o = (decltype(L.o))(A + o_lo[l]);
    if (ir) {
      L.fpc32 = (decltype(L.fpc32))(A + o_fpc32[l]); L.finv32 = (decltype(L.finv32))(A + o_finv32[l]);
      L.flo32 = (decltype(L.flo32))(A + o_flo32[l]); L.fgam32 = (decltype(L.fgam32))(A + o_fgam32[l]);
      L.f32 = (decltype(L.f32))(A + o_lf32[l]); L.u32 = (decltype(L.u32))(A + o_lu32[l]); L.o32 = (decltype(L.o32))(A + o_lo32[l]);
    } else {
      L.fpc32 = L.finv32 = L.flo32 = L.fgam32 = nullptr;
      L.f32 = L.u32 = L.o32 = nullptr;
    }
  }
  P.ilu_frow = (decltype(P.ilu_frow))(A + o_ifr);
  P.ilu_fcol = (decltype(P.ilu_fcol))(A + o_ifc); P.ilu_fval = (decltype(P.ilu_fval))(A + o_ifv);
  P.ilu_brow = (decltype(P.ilu_brow))(A + o_ibr);
  P.ilu_bcol = (decltype(P.ilu_bcol))(A + o_ibc); P.ilu_bval = (decltype(P.ilu_bval))(A + o_ibv);
  P.ilu_dinv = (decltype(P.ilu_dinv))(A + o_idi);
  P.ilu_nf = il ? ilu.nstep_f : 0; P.ilu_nb = il ? ilu.nstep_b : 0; P.ilu_lds = ilu_lds ? 1 : 0;
  P.cinv = (decltype(P.cinv))(A + o_cinv); P.cn = cn; P.cinv_rows = (cn + G - 1) / G <= CN_ROWS ? 1 : 0;
  P.cinv32 = ir ? (decltype(P.cinv32))(A + o_cinv32) : nullptr;
  P.V32 = ir ? (decltype(P.V32))(A + o_V32) : nullptr;
  P.t32 = ir ? (decltype(P.t32))(A + o_t32) : nullptr;
  P.r32 = ir ? (decltype(P.r32))(A + o_r32) : nullptr;
  P.precision = opt.precision; P.max_refine = opt.max_refine; P.rtol_inner = opt.rtol_inner;
  P.x = (decltype(P.x))(A + o_x); P.xc = (decltype(P.xc))(A + o_xc); P.r = (decltype(P.r))(A + o_r); P.rc = (decltype(P.rc))(A + o_rc);
  P.t = (decltype(P.t))(A + o_t); P.V = (decltype(P.V))(A + o_V);
  P.Y[0] = (std::remove_reference_t<decltype(P.Y[0])>)(A + o_Y0); P.Y[1] = (std::remove_reference_t<decltype(P.Y[1])>)(A + o_Y1);
  P.Xr = (decltype(P.Xr))(A + o_Xr); P.Om = (decltype(P.Om))(A + o_Om); P.K = range ? opt.window : 0;
  P.k = k; P.m = m; P.max_restarts = opt.max_restarts; P.tau_drop = opt.tau_drop; P.txg = txg;
  P.orth = opt.orthonormalize ? 1 : 0;
  P.partials = (decltype(P.partials))(A + o_part); P.bar = (decltype(P.bar))(A + o_bar); P.flags = (decltype(P.flags))(A + o_flags);
  P.log = (decltype(P.log))(A + o_log); P.G = G;
  p->dp = (Problem*)(A + o_prob);
  p->b_own = (double*)(A + o_b);
  p->eta_own = (double*)(A + o_eta);
  if (opt.profile) p->prof = (unsigned long long*)(A + o_prof);
  {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, p->device) == hipSuccess && khz > 0) p->clock_khz = khz;
  }
  if (e == hipSuccess) e = up(o_prob, &P, sizeof(Problem));
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)sa_operator_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p->lds_op);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)sa_precond_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p->lds_pc);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)sa_operator32_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p->lds_op);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)sa_precond32_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p->lds_pc);
  if (e != hipSuccess) {
    (void)hipFree(p->arena);
    delete p;
    return sa_fail(SA_EDEVICE, "sa_create: %s", hipGetErrorString(e));
  }
  *out = p;
  return SA_OK;
}

extern "C" int sa_create(const sa_grid* grid, const double* h, const sa_options* opt, void* hip_stream,
                         sa_problem** out) {
  if (!out) return sa_fail(SA_EARG, "sa_create: null argument");
  return create_impl(grid, h, opt, hip_stream, out, nullptr);
}

int64_t sa_problem_bytes(const sa_grid* grid, const double* h, const sa_options* opt) {
  int64_t bytes = 0;
  const int rc = create_impl(grid, h, opt, nullptr, nullptr, &bytes);
  return rc < 0 ? rc : bytes;
}

extern "C" int sa_problem_footprint(const sa_grid* grid, const double* h, const sa_options* opt, int64_t* bytes) {
  if (!bytes) return sa_fail(SA_EARG, "sa_problem_footprint: null argument");
  const int64_t b = sa_problem_bytes(grid, h, opt);
  if (b < 0) return (int)b;
  *bytes = b;
  return SA_OK;
}

extern "C" void sa_destroy(sa_problem* p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream); else (void)hipDeviceSynchronize();
  (void)hipFree(p->arena);
  delete p;
}

extern "C" int64_t sa_size(const sa_problem* p) { return p ? p->n : -1; }
extern "C" int32_t sa_ncol(const sa_problem* p) { return p ? p->ncol : -1; }
extern "C" int64_t sa_sketch_count(const sa_problem* p) { return p ? p->pushes + (p->unpushed ? 1 : 0) : -1; }

int sa_check_flags(sa_problem* p) {
  int f[NFLAGS];
  HIPCHK(hipMemcpyAsync(f, p->hp.flags, sizeof f, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  if (f[FLAG_ABORT]) {
    p->broken = true;
    return sa_fail(SA_EDEVICE, "device barrier timed out; problem unusable");
  }
  int code = SA_OK;
  if (f[FLAG_GEOM]) code = sa_fail(SA_EGEOM, "h + eta <= 0 or non-finite surface");
  else if (f[FLAG_NONFINITE]) code = sa_fail(SA_ENONFINITE, "non-finite value in the right-hand side or solve");
  if (code != SA_OK) {
    int z[NFLAGS] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(p->hp.flags, z, sizeof z, hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
  }
  return code;
}

extern "C" int sa_set_surface(sa_problem* p, const double* eta_prev, const double* eta_cur, int32_t mem) {
  if (!p || !eta_prev || !eta_cur) return sa_fail(SA_EARG, "sa_set_surface: null argument");
  if (p->broken) return sa_fail(SA_EDEVICE, "problem unusable after a device error");
  if (mem == SA_MEM_HOST) {
    for (int i = 0; i < p->nphys; ++i) {
      const double hp = eta_prev[i], hc = eta_cur[i];
      if (!isfinite(hp) || !isfinite(hc)) return sa_fail(SA_EGEOM, "sa_set_surface: non-finite surface");
    }
    HIPCHK(hipMemcpyAsync(p->eta_own, eta_prev, p->nphys * 8, hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipMemcpyAsync(p->eta_own + p->nphys, eta_cur, p->nphys * 8, hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    p->eta_p = p->eta_own;
    p->eta_c = p->eta_own + p->nphys;
  } else if (mem == SA_MEM_DEVICE) {
    p->eta_p = eta_prev;
    p->eta_c = eta_cur;
  } else {
    return sa_fail(SA_EARG, "sa_set_surface: bad mem");
  }
  return SA_OK;
}

extern "C" int sa_push_rhs(sa_problem* p, const double* b, int32_t mem) {
  if (!p || !b) return sa_fail(SA_EARG, "sa_push_rhs: null argument");
  if (p->broken) return sa_fail(SA_EDEVICE, "problem unusable after a device error");
  if (mem == SA_MEM_HOST) {
    HIPCHK(hipMemcpyAsync(p->b_own, b, (size_t)p->n * 8, hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    p->b = p->b_own;
  } else if (mem == SA_MEM_DEVICE) {
    p->b = b;
  } else {
    return sa_fail(SA_EARG, "sa_push_rhs: bad mem");
  }
  return SA_OK;
}

// Forgetting factor of the solution about to enter the sketch: r per stored solution, or r to
// the time since the last stored solution in units of decay_dtau (an empty sketch takes any
// factor).
static double push_factor(const sa_problem* p) {
  const sa_options& o = p->opt;
  if (o.decay == SA_DECAY_TIME && p->pushes > 0) return pow(o.r, (p->t_unpushed - p->t_pushed) / o.decay_dtau);
  return o.r;
}

static SolveArgs base_args(sa_problem* p) {
  SolveArgs a;
  memset(&a, 0, sizeof a);
  a.ycur = p->ycur;
  a.r = p->opt.r;
  a.rtol = p->opt.rtol;
  a.b = (decltype(a.b))p->b;
  a.eta_p = (decltype(a.eta_p))p->eta_p;
  a.eta_c = (decltype(a.eta_c))p->eta_c;
  a.prof = (decltype(a.prof))p->prof;
  return a;
}

static hipError_t launch_cluster(sa_problem* p, const void* fn, void** args, size_t lds) {
  if (p->G == 1) return hipLaunchKernel(fn, dim3(1), dim3(BLOCK), args, lds, p->stream);
  return hipLaunchCooperativeKernel(fn, dim3(p->G), dim3(BLOCK), args, (unsigned)lds, p->stream);
}

SolveArgs sa_prepare_solve(sa_problem* p, bool* ewma_out) {
  SolveArgs a = base_args(p);
  const sa_options& o = p->opt;
  const bool ewma = o.guess == SA_GUESS_EWMA, range = o.guess == SA_GUESS_RANGE;
  const bool sk = ewma || range;
  a.push = sk && p->unpushed;
  if (a.push) splitmix_gaussians(o.seed, p->pushes, o.k, a.om);
  if (a.push) a.r = push_factor(p);
  const int64_t pushes_after = p->pushes + (a.push ? 1 : 0);
  a.sketch_guess = sk && pushes_after > 0 && p->solves >= o.n_init;
  a.prev_guess = p->have_solution && (o.guess == SA_GUESS_PREVIOUS || (sk && !a.sketch_guess));
  a.range = range ? 1 : 0;
  a.range_slot = (range && a.push) ? (int)(p->pushes % o.window) : -1;
  a.window = range ? (int)(pushes_after < o.window ? pushes_after : o.window) : 0;
  a.log_slot = (int)(p->log_pos % LOGCAP);
  *ewma_out = ewma;
  return a;
}

void sa_commit_solve(sa_problem* p, const SolveArgs& a) {
  if (a.push) {
    if (!a.range) p->ycur ^= 1;  // the EWMA sketch ping-pongs; the range finder's ring does not
    p->pushes += 1;
    p->t_pushed = p->t_unpushed;
  }
  p->t_unpushed = p->t_next;
  p->t_set = false;
  p->unpushed = p->opt.guess == SA_GUESS_EWMA || p->opt.guess == SA_GUESS_RANGE;
  p->have_solution = true;
  p->solves += 1;
  p->log_pos += 1;
}

extern "C" int sa_set_time(sa_problem* p, double tau) {
  if (!p) return sa_fail(SA_EARG, "sa_set_time: null problem");
  if (p->opt.decay != SA_DECAY_TIME) return sa_fail(SA_EARG, "sa_set_time: the problem counts solutions, not time");
  if (!isfinite(tau)) return sa_fail(SA_EARG, "sa_set_time: tau must be finite");
  if (p->solves > 0 && tau < p->t_unpushed) return sa_fail(SA_EARG, "sa_set_time: time labels must not decrease");
  p->t_next = tau;
  p->t_set = true;
  return SA_OK;
}

extern "C" int sa_solve(sa_problem* p, sa_solve_info* info, int32_t flags) {
  if (!p) return sa_fail(SA_EARG, "sa_solve: null problem");
  if (p->broken) return sa_fail(SA_EDEVICE, "problem unusable after a device error");
  if (!p->b || !p->eta_p || !p->eta_c) return sa_fail(SA_EARG, "sa_solve: set the surfaces and the right-hand side first");
  if (p->opt.decay == SA_DECAY_TIME && !p->t_set) return sa_fail(SA_EARG, "sa_solve: SA_DECAY_TIME needs sa_set_time first");
  bool ewma = false;
  SolveArgs a = sa_prepare_solve(p, &ewma);
  BatchItem one;
  one.P = (decltype(one.P))p->dp;
  one.first = 0;
  one.sketch = ewma ? 1 : 0;
  one.a = a;
  const BatchItem* none = nullptr;
  int zero = 0;
  void* args[] = {(void*)&none, (void*)&zero, (void*)&one};
  HIPCHK(launch_cluster(p, sa_solve_fn(p->opt.precision), args, p->lds_solve));
  sa_commit_solve(p, a);
  if (flags & SA_ASYNC) return SA_OK;
  HIPCHK(hipStreamSynchronize(p->stream));
  int code = sa_check_flags(p);
  sa_solve_info rep;
  HIPCHK(hipMemcpy(&rep, p->hp.log + a.log_slot, sizeof rep, hipMemcpyDeviceToHost));
  p->log_read = p->log_pos;
  if (info) *info = rep;
  if (code != SA_OK) return code;
  if (rep.status == SA_EDEVICE) {
    p->broken = true;
    return sa_fail(SA_EDEVICE, "device barrier timed out");
  }
  return rep.status;
}

extern "C" int sa_read_log(sa_problem* p, sa_solve_info* out, int32_t max, int32_t* n_out) {
  if (!p || !n_out || (max > 0 && !out)) return sa_fail(SA_EARG, "sa_read_log: bad arguments");
  HIPCHK(hipStreamSynchronize(p->stream));
  int code = sa_check_flags(p);
  int64_t avail = p->log_pos - p->log_read;
  if (avail > LOGCAP) {
    p->log_read = p->log_pos - LOGCAP;
    avail = LOGCAP;
  }
  int32_t cnt = 0;
  while (cnt < max && p->log_read < p->log_pos) {
    HIPCHK(hipMemcpy(out + cnt, p->hp.log + (p->log_read % LOGCAP), sizeof(sa_solve_info), hipMemcpyDeviceToHost));
    ++cnt;
    ++p->log_read;
  }
  *n_out = cnt;
  return code;
}

static hipMemcpyKind kind_from(int32_t mem, bool to_device) {
  if (mem == SA_MEM_HOST) return to_device ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost;
  return hipMemcpyDeviceToDevice;
}

extern "C" int sa_get_solution(sa_problem* p, double* x, int32_t mem) {
  if (!p || !x || (mem != SA_MEM_HOST && mem != SA_MEM_DEVICE)) return sa_fail(SA_EARG, "sa_get_solution: bad arguments");
  HIPCHK(hipMemcpyAsync(x, p->hp.x, (size_t)p->n * 8, kind_from(mem, false), p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return SA_OK;
}

// ---- checkpoint of the solver state ----------------------------------------------------
// Layout: a fixed header (what must match the problem it is loaded into, and the counters),
// then the last solution x (n doubles), then the sketch: Y (k x n, EWMA) or the ring of the
// range finder (K x n) followed by its rows of Omega (KWIN x KMAX).
namespace {
struct StateHeader {
  char magic[8];
  int32_t version, guess, precision, k, window, nx, nz, bc;
  int64_t n, pushes, solves, log_pos;
  int32_t unpushed, have_solution, decay, orth;
  double r;
  uint64_t seed;
  double decay_dtau, t_unpushed, t_pushed;
};
constexpr char STATE_MAGIC[8] = {'S', 'A', 'W', 'A', 'V', 'E', 'S', 'T'};

size_t state_doubles(const sa_problem* p) {
  size_t d = (size_t)p->n;
  if (p->opt.guess == SA_GUESS_EWMA) d += (size_t)p->opt.k * p->n;
  if (p->opt.guess == SA_GUESS_RANGE) d += (size_t)p->opt.window * p->n + (size_t)KWIN * KMAX;
  return d;
}
}  // namespace

extern "C" int sa_save_state(const sa_problem* pc, void* buf, size_t* len) {
  if (!pc || !len) return sa_fail(SA_EARG, "sa_save_state: null argument");
  sa_problem* p = const_cast<sa_problem*>(pc);
  const size_t need = sizeof(StateHeader) + state_doubles(p) * 8;
  if (!buf) {
    *len = need;
    return SA_OK;
  }
  if (*len < need) {
    *len = need;
    return sa_fail(SA_EARG, "sa_save_state: buffer of %zu bytes, %zu needed", *len, need);
  }
  if (p->broken) return sa_fail(SA_EDEVICE, "problem unusable after a device error");
  StateHeader h;
  memset(&h, 0, sizeof h);
  memcpy(h.magic, STATE_MAGIC, 8);
  h.version = 2;
  h.guess = p->opt.guess; h.precision = p->opt.precision; h.k = p->opt.k; h.window = p->opt.window;
  h.nx = p->grid.nx; h.nz = p->grid.nz; h.bc = p->grid.bc;
  h.n = p->n; h.pushes = p->pushes; h.solves = p->solves; h.log_pos = p->log_pos;
  h.unpushed = p->unpushed ? 1 : 0; h.have_solution = p->have_solution ? 1 : 0;
  h.r = p->opt.r; h.seed = p->opt.seed;
  h.decay = p->opt.decay; h.decay_dtau = p->opt.decay_dtau; h.orth = p->opt.orthonormalize; h.t_unpushed = p->t_unpushed; h.t_pushed = p->t_pushed;
  char* out = (char*)buf;
  memcpy(out, &h, sizeof h);
  double* d = (double*)(out + sizeof h);
  const size_t n = (size_t)p->n;
  HIPCHK(hipMemcpyAsync(d, p->hp.x, n * 8, hipMemcpyDeviceToHost, p->stream));
  if (p->opt.guess == SA_GUESS_EWMA)
    HIPCHK(hipMemcpyAsync(d + n, p->hp.Y[p->ycur], (size_t)p->opt.k * n * 8, hipMemcpyDeviceToHost, p->stream));
  if (p->opt.guess == SA_GUESS_RANGE) {
    HIPCHK(hipMemcpyAsync(d + n, p->hp.Xr, (size_t)p->opt.window * n * 8, hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipMemcpyAsync(d + n + (size_t)p->opt.window * n, p->hp.Om, (size_t)KWIN * KMAX * 8,
                          hipMemcpyDeviceToHost, p->stream));
  }
  HIPCHK(hipStreamSynchronize(p->stream));
  *len = need;
  return SA_OK;
}

extern "C" int sa_load_state(sa_problem* p, const void* buf, size_t len) {
  if (!p || !buf) return sa_fail(SA_EARG, "sa_load_state: null argument");
  if (p->broken) return sa_fail(SA_EDEVICE, "problem unusable after a device error");
  StateHeader h;
  if (len < sizeof h) return sa_fail(SA_EARG, "sa_load_state: %zu bytes is no saved state", len);
  memcpy(&h, buf, sizeof h);
  if (memcmp(h.magic, STATE_MAGIC, 8) != 0 || h.version != 2) return sa_fail(SA_EARG, "sa_load_state: not a saved state");
  if (h.n != p->n || h.nx != p->grid.nx || h.nz != p->grid.nz || h.bc != p->grid.bc || h.guess != p->opt.guess ||
      h.k != p->opt.k || (h.guess == SA_GUESS_RANGE && h.window != p->opt.window) || h.r != p->opt.r ||
      h.seed != p->opt.seed || h.precision != p->opt.precision || h.decay != p->opt.decay ||
      h.orth != p->opt.orthonormalize ||
      (h.decay == SA_DECAY_TIME && h.decay_dtau != p->opt.decay_dtau))
    return sa_fail(SA_EARG, "sa_load_state: the state belongs to another grid or other options");
  if (len != sizeof h + state_doubles(p) * 8) return sa_fail(SA_EARG, "sa_load_state: truncated state");
  const double* d = (const double*)((const char*)buf + sizeof h);
  const size_t n = (size_t)p->n;
  HIPCHK(hipMemcpyAsync(p->hp.x, d, n * 8, hipMemcpyHostToDevice, p->stream));
  if (p->opt.guess == SA_GUESS_EWMA)
    HIPCHK(hipMemcpyAsync(p->hp.Y[0], d + n, (size_t)p->opt.k * n * 8, hipMemcpyHostToDevice, p->stream));
  if (p->opt.guess == SA_GUESS_RANGE) {
    HIPCHK(hipMemcpyAsync(p->hp.Xr, d + n, (size_t)p->opt.window * n * 8, hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipMemcpyAsync(p->hp.Om, d + n + (size_t)p->opt.window * n, (size_t)KWIN * KMAX * 8,
                          hipMemcpyHostToDevice, p->stream));
  }
  HIPCHK(hipStreamSynchronize(p->stream));
  p->ycur = 0;
  p->pushes = h.pushes;
  p->solves = h.solves;
  p->log_pos = p->log_read = h.log_pos;
  p->unpushed = h.unpushed != 0;
  p->have_solution = h.have_solution != 0;
  p->t_unpushed = h.t_unpushed;
  p->t_pushed = h.t_pushed;
  p->t_set = false;
  return SA_OK;
}

extern "C" int sa_debug_abort(sa_problem* p) {
  if (!p) return sa_fail(SA_EARG, "sa_debug_abort: null problem");
  const int one = 1;
  HIPCHK(hipMemcpyAsync(p->hp.flags + FLAG_ABORT, &one, sizeof one, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return SA_OK;
}

extern "C" int sa_get_solution_async(sa_problem* p, double* x) {
  if (!p || !x) return sa_fail(SA_EARG, "sa_get_solution_async: null argument");
  HIPCHK(hipMemcpyAsync(x, p->hp.x, (size_t)p->n * 8, hipMemcpyDeviceToDevice, p->stream));
  return SA_OK;
}

// copy an input into a device scratch vector when it lives on the host
static int stage_in(sa_problem* p, const double* src, int32_t mem, double* scratch, const double** dev) {
  if (mem == SA_MEM_DEVICE) { *dev = src; return SA_OK; }
  if (mem != SA_MEM_HOST) return sa_fail(SA_EARG, "bad mem");
  HIPCHK(hipMemcpyAsync(scratch, src, (size_t)p->n * 8, hipMemcpyHostToDevice, p->stream));
  *dev = scratch;
  return SA_OK;
}

int sa_apply_operator_enqueue(sa_problem* p, const double* x, double* y) {
  if (!p->eta_p || !p->eta_c) return sa_fail(SA_EARG, "sa_apply_operator: set the surfaces first");
  const int gb = (p->ncol + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL(sa_geometry_kernel, dim3(gb), dim3(BLOCK), 0, p->stream, p->dp, p->eta_p, p->eta_c);
  HIPCHK(hipGetLastError());
  const int nt = tiles_host(p->ncol, p->grid.bc == SA_PERIODIC, TX);
  hipLaunchKernelGGL(sa_operator_kernel, dim3(nt), dim3(BLOCK), p->lds_op, p->stream, p->dp, x, y);
  HIPCHK(hipGetLastError());
  return SA_OK;
}

extern "C" int sa_apply_operator(sa_problem* p, const double* x, double* y, int32_t mem) {
  if (!p || !x || !y) return sa_fail(SA_EARG, "sa_apply_operator: null argument");
  if (!p->eta_p || !p->eta_c) return sa_fail(SA_EARG, "sa_apply_operator: set the surfaces first");
  const double* xd;
  int rc = stage_in(p, x, mem, p->hp.xc, &xd);
  if (rc) return rc;
  double* yd = mem == SA_MEM_DEVICE ? y : p->hp.rc;
  const int gb = (p->ncol + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL(sa_geometry_kernel, dim3(gb), dim3(BLOCK), 0, p->stream, p->dp, p->eta_p, p->eta_c);
  HIPCHK(hipGetLastError());
  const int nt = tiles_host(p->ncol, p->grid.bc == SA_PERIODIC, TX);
  hipLaunchKernelGGL(sa_operator_kernel, dim3(nt), dim3(BLOCK), p->lds_op, p->stream, p->dp, xd, yd);
  HIPCHK(hipGetLastError());
  if (mem == SA_MEM_HOST) HIPCHK(hipMemcpyAsync(y, yd, (size_t)p->n * 8, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return sa_check_flags(p);
}

extern "C" int sa_apply_precond(sa_problem* p, const double* x, double* y, int32_t mem) {
  if (!p || !x || !y) return sa_fail(SA_EARG, "sa_apply_precond: null argument");
  const double* xd;
  int rc = stage_in(p, x, mem, p->hp.xc, &xd);
  if (rc) return rc;
  double* yd = mem == SA_MEM_DEVICE ? y : p->hp.rc;
  void* args[] = {(void*)&p->dp, (void*)&xd, (void*)&yd, (void*)&p->prof};
  HIPCHK(launch_cluster(p, (const void*)sa_precond_kernel, args, p->lds_pc));
  if (mem == SA_MEM_HOST) HIPCHK(hipMemcpyAsync(y, yd, (size_t)p->n * 8, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return sa_check_flags(p);
}

// FP32 inner kernels of the refinement path, for tests: host arrays are staged through the
// problem's FP32 work vectors.
static int fp32_io(sa_problem* p, const float* x, float* y, int32_t mem, const char* who, const float** xd, float** yd) {
  if (!p || !x || !y) return sa_fail(SA_EARG, "%s: null argument", who);
  if (p->opt.precision != SA_FP32_IR) return sa_fail(SA_EARG, "%s: problem created without SA_FP32_IR", who);
  if (mem == SA_MEM_DEVICE) { *xd = x; *yd = y; return SA_OK; }
  if (mem != SA_MEM_HOST) return sa_fail(SA_EARG, "%s: bad mem", who);
  HIPCHK(hipMemcpyAsync(p->hp.r32, x, (size_t)p->n * 4, hipMemcpyHostToDevice, p->stream));
  *xd = p->hp.r32;
  *yd = p->hp.t32;
  return SA_OK;
}

extern "C" int sa_apply_operator_f32(sa_problem* p, const float* x, float* y, int32_t mem) {
  const float* xd;
  float* yd;
  int rc = fp32_io(p, x, y, mem, "sa_apply_operator_f32", &xd, &yd);
  if (rc) return rc;
  if (!p->eta_p || !p->eta_c) return sa_fail(SA_EARG, "sa_apply_operator_f32: set the surfaces first");
  const int gb = (p->ncol + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL(sa_geometry_kernel, dim3(gb), dim3(BLOCK), 0, p->stream, p->dp, p->eta_p, p->eta_c);
  HIPCHK(hipGetLastError());
  const int nt = tiles_host(p->ncol, p->grid.bc == SA_PERIODIC, TX);
  hipLaunchKernelGGL(sa_operator32_kernel, dim3(nt), dim3(BLOCK), p->lds_op, p->stream, p->dp, xd, yd);
  HIPCHK(hipGetLastError());
  if (mem == SA_MEM_HOST) HIPCHK(hipMemcpyAsync(y, yd, (size_t)p->n * 4, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return sa_check_flags(p);
}

extern "C" int sa_apply_precond_f32(sa_problem* p, const float* x, float* y, int32_t mem) {
  const float* xd;
  float* yd;
  int rc = fp32_io(p, x, y, mem, "sa_apply_precond_f32", &xd, &yd);
  if (rc) return rc;
  void* args[] = {(void*)&p->dp, (void*)&xd, (void*)&yd};
  HIPCHK(launch_cluster(p, (const void*)sa_precond32_kernel, args, p->lds_pc));
  if (mem == SA_MEM_HOST) HIPCHK(hipMemcpyAsync(y, yd, (size_t)p->n * 4, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return sa_check_flags(p);
}

// store a solution that is still waiting for the next solve's fused push
static int flush_push(sa_problem* p) {
  if (!p->unpushed || p->opt.guess != SA_GUESS_EWMA) return SA_OK;
  SolveArgs a = base_args(p);
  a.push = 1;
  a.r = push_factor(p);
  splitmix_gaussians(p->opt.seed, p->pushes, p->opt.k, a.om);
  const int gb = (p->n + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL(sa_push_kernel, dim3(gb < 1024 ? gb : 1024), dim3(BLOCK), 0, p->stream, p->dp, a);
  HIPCHK(hipGetLastError());
  p->ycur ^= 1;
  p->pushes += 1;
  p->t_pushed = p->t_unpushed;
  p->unpushed = false;
  return SA_OK;
}

extern "C" int sa_get_sketch(sa_problem* p, double* y, int32_t mem) {
  if (!p || !y || (mem != SA_MEM_HOST && mem != SA_MEM_DEVICE)) return sa_fail(SA_EARG, "sa_get_sketch: bad arguments");
  if (p->opt.guess != SA_GUESS_EWMA) return sa_fail(SA_EARG, "sa_get_sketch: no sketch in this guess mode");
  int rc = flush_push(p);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(y, p->hp.Y[p->ycur], (size_t)p->n * p->opt.k * 8, kind_from(mem, false), p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return SA_OK;
}

extern "C" int sa_get_phase_times(sa_problem* p, double* out, int32_t n) {
  if (!p || !out || n < 1 || n > NPROF) return sa_fail(SA_EARG, "sa_get_phase_times: bad arguments");
  if (!p->prof) return sa_fail(SA_EARG, "sa_get_phase_times: problem created without profile = 1");
  unsigned long long t[NPROF];
  HIPCHK(hipMemcpyAsync(t, p->prof, sizeof t, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  for (int i = 0; i < n; ++i) out[i] = (double)t[i] / p->clock_khz;
  return SA_OK;
}
