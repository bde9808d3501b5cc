// Host-side state shared by the C-ABI translation units (problems and the server).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <type_traits>
#include <vector>

#include "internal.h"
#include "tables.h"

namespace sa {
extern "C" __global__ void sa_solve_kernel(const BatchItem*, int, BatchItem);
extern "C" __global__ void sa_solve_ir_kernel(const BatchItem*, int, BatchItem);
extern "C" __global__ void sa_geometry_kernel(const Problem*, const double*, const double*);
extern "C" __global__ void sa_operator_kernel(const Problem*, const double*, double*);
extern "C" __global__ void sa_precond_kernel(const Problem*, const double*, double*, unsigned long long*);
extern "C" __global__ void sa_push_kernel(const Problem*, SolveArgs);
extern "C" __global__ void sa_operator32_kernel(const Problem*, const float*, float*);
extern "C" __global__ void sa_precond32_kernel(const Problem*, const float*, float*);
}  // namespace sa

// record the message of a hard error (thread-local, read by sa_last_error) and return code
int sa_fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return sa_fail(SA_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct sa_problem {
  sa_grid grid;
  sa_options opt;
  hipStream_t stream = nullptr;
  int device = 0;
  int ncol = 0, nl = 0, n = 0, nphys = 0;
  sa::Problem hp{};              // host copy of the device descriptor
  sa::Problem* dp = nullptr;     // device descriptor
  char* arena = nullptr;         // one device allocation holding every buffer
  size_t arena_bytes = 0;
  double* b_own = nullptr;       // internal right-hand side (host pushes)
  double* eta_own = nullptr;     // 2 x nphys internal surfaces (host pushes)
  const double* b = nullptr;     // current right-hand side (device)
  const double* eta_p = nullptr;
  const double* eta_c = nullptr;
  size_t lds_solve = 0, lds_op = 0, lds_pc = 0;
  int G = 1;
  int ycur = 0;
  int64_t pushes = 0, solves = 0;
  bool unpushed = false;         // the last solution is not in the sketch yet
  // SA_DECAY_TIME: the label given for the next solve, the label of the solution not yet in
  // the sketch and of the last solution pushed into it
  double t_next = 0.0, t_unpushed = 0.0, t_pushed = 0.0;
  bool t_set = false;
  bool have_solution = false;
  int64_t log_pos = 0, log_read = 0;
  bool broken = false;
  unsigned long long* prof = nullptr;  // NPHASE device counters (opt.profile)
  double clock_khz = 100000.0;
};

// The host steps around one solve launch: arguments of the next solve of p (push of the
// previous solution, guess selection, sketch draws, log slot) and the bookkeeping once it is
// enqueued. `ewma` tells which solve kernel variant runs it.
sa::SolveArgs sa_prepare_solve(sa_problem* p, bool* ewma);
void sa_commit_solve(sa_problem* p, const sa::SolveArgs& a);
// device flags of p folded into a status (and cleared), SA_EDEVICE after a barrier time-out
int sa_check_flags(sa_problem* p);
// y = A x of p's current surfaces, device vectors, enqueued on p's stream (no wait)
int sa_apply_operator_enqueue(sa_problem* p, const double* x, double* y);
// raise the dynamic-LDS limit of the solve kernels to at least `bytes` (never lowers it)
int sa_reserve_solve_lds(size_t bytes);
// the solve kernel of a precision (SA_FP64 or SA_FP32_IR)
const void* sa_solve_fn(int precision);
// bytes of device memory sa_create would allocate for these arguments (< 0: invalid)
int64_t sa_problem_bytes(const sa_grid* grid, const double* h, const sa_options* opt);
