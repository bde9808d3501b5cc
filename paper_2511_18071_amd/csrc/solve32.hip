// gfx950 kernels of the mixed-precision path: FP64 refinement around FP32 GMRES cycles, one
// solve (or a batch of solves) per launch, and the standalone FP32 operator and
// preconditioner kernels.
#include "device.h"

namespace sa {

// one refinement solve per cluster: guess, FP32 cycles with FP64 residual checks, report
extern "C" __global__ void __launch_bounds__(BLOCK) sa_solve_ir_kernel(const BatchItem* __restrict__ items,
                                                                       int nitems, BatchItem one) {
  solve_entry<SA_FP32_IR>(items, nitems, one);
}

// y = A x with FP32 input, output and arithmetic (the inner operator of the refinement path)
extern "C" __global__ void __launch_bounds__(BLOCK) sa_operator32_kernel(const Problem* __restrict__ PP,
                                                                         const float* x, float* y) {
  const Problem& P = *PP;
  double* smem = dyn_lds;
  Cl cl = make_cl(P, (int)blockIdx.x, (int)gridDim.x);
  phase_operator_s<float>(P, cl, x, 1.0f, y, (float*)smem);
}

// z = M^-1 v in FP32 (the inner preconditioner of the refinement path)
extern "C" __global__ void __launch_bounds__(BLOCK) sa_precond32_kernel(const Problem* __restrict__ PP,
                                                                        const float* v, float* z) {
  const Problem& P = *PP;
  double* smem = dyn_lds;
  Cl cl = make_cl(P, (int)blockIdx.x, P.G);
  precond<float>(P, cl, v, z, (float*)smem, nullptr);
}

}  // namespace sa
