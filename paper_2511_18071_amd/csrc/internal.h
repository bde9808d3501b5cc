// Internal data structures shared by the host setup code and the gfx950 kernels.
#pragma once
#include <stdint.h>

#include "../../include/sawave.h"

// Device memory pointers stored in the structures below. The device pass gives them the
// global address space so that every load and store through them is a global (not flat)
// access; the host pass sees plain pointers (set them with a cast to decltype(field)).
#if defined(__HIP_DEVICE_COMPILE__)
#define SA_GLOBAL __attribute__((address_space(1)))
#else
#define SA_GLOBAL
#endif

namespace sa {

constexpr int BLOCK = 512;        // threads per workgroup
constexpr int NWAVE = BLOCK / 64; // wave64s per workgroup (a power of two)
constexpr int KMAX = 16;          // largest sketch rank handled on the device
constexpr int MMAX = 64;          // largest restart length
constexpr int MAXLEV = 24;        // multigrid levels
constexpr int TX = 64;            // columns per operator tile
constexpr int HW = 3;             // stencil half width (seven-point first derivatives)
constexpr int NLMAX = 66;         // largest number of levels nz + 1
constexpr int PSTRIDE = 320;      // doubles per workgroup in the reduction scratch
constexpr int LOGCAP = 4096;      // solve reports kept on the device
constexpr int COARSE_MAX = 4096;  // largest coarsest-grid size solved by a dense inverse
constexpr int CN_ROWS = 16;       // at most this many coarse rows per workgroup: the inverse is kept row by row
constexpr int KWIN = 32;          // largest window of the randomized range finder
constexpr int ILU_LDS_MAX = 16384; // unknowns up to which the ILU(0) substitutions keep z in LDS

// Flags written by kernels (device int array).
enum { FLAG_GEOM = 0, FLAG_NONFINITE = 1, FLAG_ABORT = 2, NFLAGS = 4 };

// One level of the still-water preconditioner hierarchy (level 0 = the problem grid).
struct Level {
  int ncol, nx;              // columns (ghosts included), physical points
  double dx;
  const double SA_GLOBAL* h;           // depth per column (ghost columns by reflection)
  const double SA_GLOBAL* ih;          // 1/h per column
  const double SA_GLOBAL* hx;          // second-order centred dh/dx per column
  const double SA_GLOBAL* hxx;        // second-order centred d2h/dx2 per column
  // line-solve factors of the fixed still-water operator: ratio pc and inverse pivot at
  // [j * fstride + c] (fstride = 0: every column has the same factors), bed-row combination
  // factor per column
  const double SA_GLOBAL* fpc;
  const double SA_GLOBAL* finv;
  const double SA_GLOBAL* flo;         // sub-diagonal of the column systems (same layout)
  const double SA_GLOBAL* fgam;
  int fstride;
  int tm;                    // tile width of the default V-cycle passes (32 on levels whose
                             // 32-column tiles each get a cluster workgroup, else 64)
  int res;                   // offset (elements of the solve's precision) of the level's
                             // line-solve constants inside the solve kernel's resident LDS
                             // block, -1: staged every pass
  int facstride;             // flo, fpc, finv (and their FP32 copies) lie facstride apart;
                             // h, ih, hx, hxx lie ncol apart
  double SA_GLOBAL* f;                 // right-hand side of this level (level 0: unused, the input)
  double SA_GLOBAL* u;                 // smoothed iterate
  double SA_GLOBAL* o;                 // output of this level's cycle (level 0: unused, the output)
  // FP32 copies for the inner solve of the refinement path (null without it)
  const float SA_GLOBAL* fpc32;
  const float SA_GLOBAL* finv32;
  const float SA_GLOBAL* flo32;
  const float SA_GLOBAL* fgam32;
  float SA_GLOBAL* f32;
  float SA_GLOBAL* u32;
  float SA_GLOBAL* o32;
};

// Everything a kernel needs about one problem. Lives in device memory.
struct Problem {
  int ncol, nl, nz, n, nphys, periodic;
  int tx;                    // operator tile width: 32 where every 32-column tile has a cluster
                             // workgroup, else 64
  int res_base;              // dynamic-LDS offset (doubles) of the solve kernels' resident block
                             // of line-solve constants, -1: none
  double dx, dsig;
  const double SA_GLOBAL* wsig;        // nl x 7 first-derivative weights in sigma (1/dsig included)
  const int SA_GLOBAL* ssig;           // nl window starts in sigma
  const double SA_GLOBAL* wchi;        // 7 x 7: rows 0-2 left windows, 3 centred, 4-6 right windows
  const double SA_GLOBAL* sig;         // nl sigma values
  const double SA_GLOBAL* h;           // ncol depth (extended)
  const double SA_GLOBAL* hchi;        // ncol sixth-order dh/dchi
  double SA_GLOBAL* geo;               // 4 x ncol: 1/d_prev, d_chi prev, 1/d_cur, d_chi cur
  // preconditioner
  int pc, nu1, nu2, nlev, tail;   // tail: first level run by a single workgroup
  double omega;
  Level lev[MAXLEV];
  // ILU(0) of the still-water operator (pc == SA_PC_ILU0), per substitution (f: forward over
  // the strictly lower L, b: backward over the strictly upper U): steps of 16 independent rows
  // in level order, slot s of step t = row[16 t + s] (-1: padding), one record of 64 (column,
  // value) pairs per slot (column -1 past the row's end); 1/u_ii per backward slot
  const int SA_GLOBAL* ilu_frow;
  const int SA_GLOBAL* ilu_fcol;
  const double SA_GLOBAL* ilu_fval;
  const int SA_GLOBAL* ilu_brow;
  const int SA_GLOBAL* ilu_bcol;
  const double SA_GLOBAL* ilu_bval;
  const double SA_GLOBAL* ilu_dinv;   // per backward slot
  int ilu_nf, ilu_nb;        // steps of the two substitutions
  int ilu_lds;               // 1: z lives in the phase scratch (LDS) during the substitutions
  const double SA_GLOBAL* cinv;        // dense inverse of the coarsest operator, cn x cn (layout: cinv_rows)
  const float SA_GLOBAL* cinv32;       // its FP32 rounding (refinement path)
  int cn;
  int cinv_rows;  // 1: cinv stored row by row (a workgroup owns at most CN_ROWS rows), 0: transposed
  // solver vectors
  double SA_GLOBAL* x;
  double SA_GLOBAL* xc;
  double SA_GLOBAL* r;
  double SA_GLOBAL* rc;
  double SA_GLOBAL* t;
  double SA_GLOBAL* V;
  double SA_GLOBAL* Y[2];
  // randomized range finder: ring of the K most recent solutions (K x n, slot s at s * n) and
  // the row of Omega of each slot (K x KMAX)
  double SA_GLOBAL* Xr;
  double SA_GLOBAL* Om;
  int K;
  // inner basis and work vectors of the refinement path
  float SA_GLOBAL* V32;
  float SA_GLOBAL* t32;
  float SA_GLOBAL* r32;
  // sketch / options
  int k, m, max_restarts;
  int txg;                   // columns per tile of the block operator of the guess (16, 32, 64)
  int orth;                  // range finder: V = Q, the orthonormalised sketch (Alg. 3)
  double tau_drop;
  int precision, max_refine;
  double rtol_inner;
  // synchronisation and reports
  double SA_GLOBAL* partials;          // 2 x (G + 1) x PSTRIDE: records, then the sums
  unsigned SA_GLOBAL* bar;             // barrier counter, generation
  int SA_GLOBAL* flags;                // NFLAGS
  sa_solve_info SA_GLOBAL* log;        // LOGCAP
  int G;                     // workgroups per solve
};

struct SolveArgs {
  int push;          // store the previous solution in the sketch first
  int sketch_guess;  // x0 from the sketch (Alg. 2 with V = Y)
  int prev_guess;    // x0 = previous solution (else zero) when no sketch guess
  int ycur;          // sketch buffer holding Y before this call
  int range;         // the guess comes from the range finder (V = X Omega, kept in Y[0])
  int range_slot;    // ring slot the previous solution enters (push), else -1
  int window;        // ring slots in use after the push (slots 0 .. window - 1)
  int log_slot;
  const double SA_GLOBAL* b;      // right-hand side (n)
  const double SA_GLOBAL* eta_p;  // previous-stage surface (nphys)
  const double SA_GLOBAL* eta_c;  // current-stage surface (nphys)
  double r;          // forgetting factor
  double rtol;
  double om[KMAX];   // sketch draws of the stored solution
  unsigned long long SA_GLOBAL* prof;  // NPHASE accumulated wall-clock ticks, or nullptr
  sa_solve_info SA_GLOBAL* out;        // a second copy of the report with the problem's flags folded
                             // into its status (batched solves), or nullptr
};

// One solve of a batched launch: the workgroups [first, first + P->G) of the grid run it.
struct BatchItem {
  const Problem SA_GLOBAL* P;
  int first;
  int sketch;   // the sketch variant of the solve (EWMA guess mode)
  SolveArgs a;
};

// phase-time categories of the solve kernel (sa_get_phase_times)
enum { PH_GEOM = 0, PH_GUESS = 1, PH_SMALL = 2, PH_OPER = 3, PH_PREC = 4, PH_ORTH = 5, PH_OTHER = 6, PH_TOTAL = 7,
       NPHASE = 8 };
// detailed preconditioner timing (same buffer, after the NPHASE totals): coarse solve, then
// down / up pass of level l at PH_MG + 1 + 2 l (+1)
enum { PH_MG = NPHASE, NPROF = NPHASE + 1 + 2 * MAXLEV };

// ---- host-side setup (setup.cpp) ----------------------------------------------------
void fornberg(double z, const double* x, int n, int mmax, double* c /* n*(mmax+1) */);
int window_start(int i, int npts, int width);
void splitmix_gaussians(uint64_t seed, int64_t index, int k, double* out);
// assemble the coarsest still-water operator densely (row-major cn x cn) and invert it
int dense_still_water_inverse(int ncol, int nx, int nl, int periodic, double dx, double dsig,
                              const double* h, const double* hx, const double* hxx, double* inv);

}  // namespace sa
