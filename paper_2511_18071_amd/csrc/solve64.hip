// gfx950 kernels of the FP64 path: one solve (or a batch of solves) per launch, and the
// standalone operator, preconditioner, geometry and sketch-push kernels.
#include "device.h"

namespace sa {

// one FP64 solve per cluster: guess, restarted GMRES, report
extern "C" __global__ void __launch_bounds__(BLOCK) sa_solve_kernel(const BatchItem* __restrict__ items, int nitems,
                                                                    BatchItem one) {
  solve_entry<SA_FP64>(items, nitems, one);
}

extern "C" __global__ void __launch_bounds__(BLOCK) sa_geometry_kernel(const Problem* __restrict__ PP,
                                                                       const double* eta_p, const double* eta_c) {
  const Problem& P = *PP;
  Cl cl = make_cl(P, (int)blockIdx.x, (int)gridDim.x);
  phase_geometry(P, cl, eta_p, eta_c);
}

extern "C" __global__ void __launch_bounds__(BLOCK) sa_operator_kernel(const Problem* __restrict__ PP,
                                                                       const double* x, double* y) {
  const Problem& P = *PP;
  double* smem = dyn_lds;
  Cl cl = make_cl(P, (int)blockIdx.x, (int)gridDim.x);
  phase_operator(P, cl, x, 1.0, y, nullptr, smem, smem, 0);
}

extern "C" __global__ void __launch_bounds__(BLOCK) sa_precond_kernel(const Problem* __restrict__ PP,
                                                                      const double* v, double* z,
                                                                      unsigned long long* prof) {
  const Problem& P = *PP;
  double* smem = dyn_lds;
  Cl cl = make_cl(P, (int)blockIdx.x, P.G);
  PhaseClock clk;
  clk.begin(prof != nullptr, cl.rank, prof);
  precond<double>(P, cl, v, z, smem, &clk);
  clk.flush(prof);
}

extern "C" __global__ void __launch_bounds__(BLOCK) sa_push_kernel(const Problem* __restrict__ PP, SolveArgs a) {
  const Problem& P = *PP;
  Cl cl = make_cl(P, (int)blockIdx.x, (int)gridDim.x);
  phase_push(P, cl, a, P.Y[a.ycur], P.Y[a.ycur ^ 1]);
}

}  // namespace sa
