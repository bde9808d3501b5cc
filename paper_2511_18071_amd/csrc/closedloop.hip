// The closed loop of Alg. 1 on the GPU: low-storage Runge-Kutta (LSERK45) stepping of the
// velocity field and the free surface of a periodic simulation, whose mixed-stage pressure
// systems go to the problem's solver one stage after another (Sec. 3). With rho = 1, zero
// viscosity and gravity F = (0, -g), stage i (coefficients alpha_i, beta_i):
//
//   f_eta = w - u D_chi eta at the surface; K_eta = alpha_i K_eta + dtau f_eta;
//   eta^(i) = eta^(i-1) + beta_i K_eta;
//   R = F - (u . grad^(i-1)) u + (sigma / d^(i-1)) f_eta D_sigma u;
//   Q = u / (beta_i dtau) + alpha_i K_u / dtau + R;
//   rhs = grad^(i) . Q (PDE rows), n . Q at the bed node (bed rows, n = (-h_chi, -1)), 0 (surface);
//   p = p_s + p_d, p_s = g d^(i-1) (1 - sigma) the hydrostatic pressure under the previous
//     stage's surface and p_d = A(eta^(i-1), eta^(i))^-1 (rhs - A p_s) the dynamic pressure
//     (the problem's solve, with its guess: the sequence it sees is the dynamic part);
//   K_u = alpha_i K_u + dtau (R - grad^(i-1) p); u^(i) = u^(i-1) + beta_i K_u,
//
// with grad = (D_chi + sigma_x D_sigma, (1/d) D_sigma) at the stated stage. Velocities live on
// every node of the pressure grid (the ghost level included) and every node takes the same
// update. The kernels are plain one-thread-per-node stencils over global memory: the loop's
// own arithmetic is a few passes over the state per stage, the solve dominates.
#include <hip/hip_runtime.h>
#include <math.h>

#include "host.h"

using namespace sa;

namespace {

constexpr int LB = 256;
constexpr double GRAV = 9.81;

// LSERK45 (Carpenter & Kennedy 1994), the published 2N-storage coefficients
constexpr double LA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                          -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
constexpr double LB5[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                           1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                           2277821191437.0 / 14882151754819.0};
// stage times tau_n + c_i dtau (the time labels of the stage systems, for forgetting in time)
constexpr double LC5[5] = {0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                           2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0};

struct LoopArgs {
  int ncol, nl, nz, n;
  const double* wsig;  // nl x 7
  const int* ssig;     // nl
  const double* wchi;  // 7 x 7 (row 3: centred)
  const double* sig;   // nl
  const double* h;     // ncol
  const double* hchi;  // ncol
  double *u, *w, *ku, *kw, *rx, *rz, *qx, *qz, *rhs, *p, *ps;
  double *eta, *eta_new, *keta, *feta;
  double* geo;  // 5 x ncol: 1/d prev, d_chi prev, 1/d cur, d_chi cur, h_chi
  double a, b, dt;
};

__device__ inline int wrapc(int c, int n) { return ((c % n) + n) % n; }

// centred seven-point D_chi of a level row (periodic)
__device__ inline double dchi(const LoopArgs& A, const double* row, int c) {
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < 7; ++m) s += A.wchi[21 + m] * row[wrapc(c - 3 + m, A.ncol)];
  return s;
}

// D_sigma of a column at level j
__device__ inline double dsig(const LoopArgs& A, const double* v, int j, int c) {
  const int s0 = A.ssig[j];
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < 7; ++m) s += A.wsig[j * 7 + m] * v[(s0 + m) * A.ncol + c];
  return s;
}

}  // namespace

// surface: f_eta, K_eta, eta^(i)
extern "C" __global__ void __launch_bounds__(LB) sa_loop_surface_kernel(LoopArgs A) {
  const int c = blockIdx.x * LB + threadIdx.x;
  if (c >= A.ncol) return;
  const int top = A.nz * A.ncol;
  const double f = A.w[top + c] - A.u[top + c] * dchi(A, A.eta, c);
  const double k = A.a * A.keta[c] + A.dt * f;
  A.feta[c] = f;
  A.keta[c] = k;
  A.eta_new[c] = A.eta[c] + A.b * k;
}

// per-column geometry of both stages
extern "C" __global__ void __launch_bounds__(LB) sa_loop_geometry_kernel(LoopArgs A) {
  const int c = blockIdx.x * LB + threadIdx.x;
  if (c >= A.ncol) return;
  const int nc = A.ncol;
  double dp = 0.0, dc = 0.0;
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    const int cc = wrapc(c - 3 + m, nc);
    dp += A.wchi[21 + m] * (A.h[cc] + A.eta[cc]);
    dc += A.wchi[21 + m] * (A.h[cc] + A.eta_new[cc]);
  }
  A.geo[c] = 1.0 / (A.h[c] + A.eta[c]);
  A.geo[nc + c] = dp;
  A.geo[2 * nc + c] = 1.0 / (A.h[c] + A.eta_new[c]);
  A.geo[3 * nc + c] = dc;
  A.geo[4 * nc + c] = A.hchi[c];
}

// R and Q at every node (geometry of stage i - 1)
extern "C" __global__ void __launch_bounds__(LB) sa_loop_force_kernel(LoopArgs A) {
  const int i = blockIdx.x * LB + threadIdx.x;
  if (i >= A.n) return;
  const int nc = A.ncol, j = i / nc, c = i - j * nc;
  const double id = A.geo[c], sx = (A.geo[4 * nc + c] - A.sig[j] * A.geo[nc + c]) * id;
  const double* urow = A.u + (size_t)j * nc;
  const double* wrow = A.w + (size_t)j * nc;
  const double us = dsig(A, A.u, j, c), ws = dsig(A, A.w, j, c);
  const double ux = dchi(A, urow, c) + sx * us, uz = id * us;
  const double wx = dchi(A, wrow, c) + sx * ws, wz = id * ws;
  const double uu = A.u[i], ww = A.w[i];
  const double move = A.sig[j] * A.feta[c] * id;
  const double rx = -(uu * ux + ww * uz) + move * us;
  const double rz = -GRAV - (uu * wx + ww * wz) + move * ws;
  A.rx[i] = rx;
  A.rz[i] = rz;
  A.qx[i] = uu / (A.b * A.dt) + A.a * A.ku[i] / A.dt + rx;
  A.qz[i] = ww / (A.b * A.dt) + A.a * A.kw[i] / A.dt + rz;
}

// right-hand side: grad^(i) . Q, the bed rows n . Q, zero on the surface
extern "C" __global__ void __launch_bounds__(LB) sa_loop_rhs_kernel(LoopArgs A) {
  const int i = blockIdx.x * LB + threadIdx.x;
  if (i >= A.n) return;
  const int nc = A.ncol, j = i / nc, c = i - j * nc;
  double v;
  if (j == A.nz) {
    v = 0.0;
  } else if (j == 0) {
    v = -A.geo[4 * nc + c] * A.qx[nc + c] - A.qz[nc + c];
  } else {
    const double id = A.geo[2 * nc + c], sx = (A.geo[4 * nc + c] - A.sig[j] * A.geo[3 * nc + c]) * id;
    v = dchi(A, A.qx + (size_t)j * nc, c) + sx * dsig(A, A.qx, j, c) + id * dsig(A, A.qz, j, c);
  }
  A.rhs[i] = v;
}

// p_s = g d^(i-1) (1 - sigma) at every node
extern "C" __global__ void __launch_bounds__(LB) sa_loop_hydrostatic_kernel(LoopArgs A) {
  const int i = blockIdx.x * LB + threadIdx.x;
  if (i >= A.n) return;
  const int nc = A.ncol, j = i / nc, c = i - j * nc;
  A.ps[i] = GRAV * (A.h[c] + A.eta[c]) * (1.0 - A.sig[j]);
}

// rhs -= A p_s (A p_s in qx, which the right-hand side no longer needs)
extern "C" __global__ void __launch_bounds__(LB) sa_loop_dynamic_rhs_kernel(LoopArgs A) {
  const int i = blockIdx.x * LB + threadIdx.x;
  if (i >= A.n) return;
  A.rhs[i] -= A.qx[i];
}

// K_u = alpha K_u + dt (R - grad^(i-1) p), u += beta K_u (geometry of stage i - 1), p = p_s + p_d
extern "C" __global__ void __launch_bounds__(LB) sa_loop_update_kernel(LoopArgs A) {
  const int i = blockIdx.x * LB + threadIdx.x;
  if (i >= A.n) return;
  const int nc = A.ncol, j = i / nc, c = i - j * nc;
  const double id = A.geo[c], sx = (A.geo[4 * nc + c] - A.sig[j] * A.geo[nc + c]) * id;
  const double psg = dsig(A, A.p, j, c) + dsig(A, A.ps, j, c);
  const double px = dchi(A, A.p + (size_t)j * nc, c) + dchi(A, A.ps + (size_t)j * nc, c) + sx * psg, pz = id * psg;
  const double ku = A.a * A.ku[i] + A.dt * (A.rx[i] - px);
  const double kw = A.a * A.kw[i] + A.dt * (A.rz[i] - pz);
  A.ku[i] = ku;
  A.kw[i] = kw;
  A.u[i] += A.b * ku;
  A.w[i] += A.b * kw;
}

struct sa_loop {
  sa_problem* p = nullptr;
  double dt = 0.0;
  long long steps = 0;  // completed steps
  double* arena = nullptr;
  LoopArgs A{};
};

extern "C" int sa_loop_create(sa_problem* p, double dtau, sa_loop** out) {
  if (!p || !out) return sa_fail(SA_EARG, "sa_loop_create: null argument");
  *out = nullptr;
  if (p->grid.bc != SA_PERIODIC) return sa_fail(SA_EARG, "sa_loop_create: the closed loop runs on periodic problems");
  if (!(dtau > 0.0) || !isfinite(dtau)) return sa_fail(SA_EARG, "sa_loop_create: dtau must be positive");
  sa_loop* L = new sa_loop();
  L->p = p;
  L->dt = dtau;
  const size_t n = (size_t)p->n, nc = (size_t)p->ncol;
  // u w ku kw rx rz qx qz rhs p ps (n each), eta eta_new keta feta (nc each), geo (5 nc)
  const size_t doubles = 11 * n + 9 * nc;
  if (hipMalloc((void**)&L->arena, doubles * 8) != hipSuccess) {
    delete L;
    return sa_fail(SA_EOOM, "sa_loop_create: %zu bytes of device memory", doubles * 8);
  }
  if (hipMemsetAsync(L->arena, 0, doubles * 8, p->stream) != hipSuccess || hipStreamSynchronize(p->stream) != hipSuccess) {
    (void)hipFree(L->arena);
    delete L;
    return sa_fail(SA_EDEVICE, "sa_loop_create: clearing the state failed");
  }
  LoopArgs& A = L->A;
  A.ncol = p->ncol; A.nl = p->nl; A.nz = p->grid.nz; A.n = p->n;
  A.wsig = (const double*)p->hp.wsig; A.ssig = (const int*)p->hp.ssig; A.wchi = (const double*)p->hp.wchi;
  A.sig = (const double*)p->hp.sig; A.h = (const double*)p->hp.h; A.hchi = (const double*)p->hp.hchi;
  double* q = L->arena;
  A.u = q; q += n; A.w = q; q += n; A.ku = q; q += n; A.kw = q; q += n; A.rx = q; q += n; A.rz = q; q += n;
  A.qx = q; q += n; A.qz = q; q += n; A.rhs = q; q += n; A.p = q; q += n; A.ps = q; q += n;
  A.eta = q; q += nc; A.eta_new = q; q += nc; A.keta = q; q += nc; A.feta = q; q += nc; A.geo = q;
  A.dt = dtau;
  *out = L;
  return SA_OK;
}

extern "C" int sa_loop_set_state(sa_loop* L, const double* eta, const double* u, const double* w, int32_t mem) {
  if (!L || !eta || !u || !w) return sa_fail(SA_EARG, "sa_loop_set_state: null argument");
  if (mem != SA_MEM_HOST && mem != SA_MEM_DEVICE) return sa_fail(SA_EARG, "sa_loop_set_state: bad mem");
  const hipMemcpyKind k = mem == SA_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  sa_problem* p = L->p;
  const size_t n = (size_t)p->n, nc = (size_t)p->ncol;
  HIPCHK(hipMemcpyAsync(L->A.eta, eta, nc * 8, k, p->stream));
  HIPCHK(hipMemcpyAsync(L->A.u, u, n * 8, k, p->stream));
  HIPCHK(hipMemcpyAsync(L->A.w, w, n * 8, k, p->stream));
  HIPCHK(hipMemsetAsync(L->A.ku, 0, 2 * n * 8, p->stream));
  HIPCHK(hipMemsetAsync(L->A.keta, 0, nc * 8, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return SA_OK;
}

extern "C" int sa_loop_get_state(sa_loop* L, double* eta, double* u, double* w, int32_t mem) {
  if (!L || !eta || !u || !w) return sa_fail(SA_EARG, "sa_loop_get_state: null argument");
  if (mem != SA_MEM_HOST && mem != SA_MEM_DEVICE) return sa_fail(SA_EARG, "sa_loop_get_state: bad mem");
  const hipMemcpyKind k = mem == SA_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  sa_problem* p = L->p;
  const size_t n = (size_t)p->n, nc = (size_t)p->ncol;
  HIPCHK(hipMemcpyAsync(eta, L->A.eta, nc * 8, k, p->stream));
  HIPCHK(hipMemcpyAsync(u, L->A.u, n * 8, k, p->stream));
  HIPCHK(hipMemcpyAsync(w, L->A.w, n * 8, k, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return SA_OK;
}

extern "C" int sa_loop_step(sa_loop* L, sa_solve_info* infos) {
  if (!L) return sa_fail(SA_EARG, "sa_loop_step: null argument");
  sa_problem* p = L->p;
  LoopArgs& A = L->A;
  const int gn = (A.n + LB - 1) / LB, gc = (A.ncol + LB - 1) / LB;
  const int64_t first = p->log_pos;  // the log slot of this step's first solve
  for (int s = 0; s < 5; ++s) {
    A.a = LA[s];
    A.b = LB5[s];
    hipLaunchKernelGGL(sa_loop_surface_kernel, dim3(gc), dim3(LB), 0, p->stream, A);
    hipLaunchKernelGGL(sa_loop_geometry_kernel, dim3(gc), dim3(LB), 0, p->stream, A);
    hipLaunchKernelGGL(sa_loop_force_kernel, dim3(gn), dim3(LB), 0, p->stream, A);
    hipLaunchKernelGGL(sa_loop_rhs_kernel, dim3(gn), dim3(LB), 0, p->stream, A);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(sa_loop_hydrostatic_kernel, dim3(gn), dim3(LB), 0, p->stream, A);
    HIPCHK(hipGetLastError());
    int rc = sa_set_surface(p, A.eta, A.eta_new, SA_MEM_DEVICE);
    if (rc == SA_OK) rc = sa_apply_operator_enqueue(p, A.ps, A.qx);
    if (rc == SA_OK) {
      hipLaunchKernelGGL(sa_loop_dynamic_rhs_kernel, dim3(gn), dim3(LB), 0, p->stream, A);
      HIPCHK(hipGetLastError());
      rc = sa_push_rhs(p, A.rhs, SA_MEM_DEVICE);
    }
    if (rc == SA_OK && p->opt.decay == SA_DECAY_TIME) rc = sa_set_time(p, ((double)L->steps + LC5[s]) * L->dt);
    if (rc == SA_OK) rc = sa_solve(p, nullptr, SA_ASYNC);
    if (rc == SA_OK) rc = sa_get_solution_async(p, A.p);
    if (rc) return rc;
    hipLaunchKernelGGL(sa_loop_update_kernel, dim3(gn), dim3(LB), 0, p->stream, A);
    HIPCHK(hipGetLastError());
    double* t = A.eta;  // eta^(i) becomes the current surface
    A.eta = A.eta_new;
    A.eta_new = t;
  }
  L->steps += 1;
  // the five reports (the only wait of the step)
  sa_solve_info rep[5];
  int32_t got = 0;
  p->log_read = first;
  const int rc = sa_read_log(p, rep, 5, &got);
  if (infos)
    for (int s = 0; s < got; ++s) infos[s] = rep[s];
  if (rc != SA_OK) return rc;
  for (int s = 0; s < got; ++s) {
    if (rep[s].status == SA_EDEVICE) {
      p->broken = true;
      return sa_fail(SA_EDEVICE, "sa_loop_step: device barrier timed out");
    }
    if (rep[s].status != SA_OK) return sa_fail(SA_NOCONV, "sa_loop_step: stage %d did not converge", s);
  }
  return SA_OK;
}

extern "C" void sa_loop_destroy(sa_loop* L) {
  if (!L) return;
  if (L->p && L->p->stream) (void)hipStreamSynchronize(L->p->stream);
  if (L->arena) (void)hipFree(L->arena);
  delete L;
}
