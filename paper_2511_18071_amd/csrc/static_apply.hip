// sa_apply_operator_static: y = A(eta_prev, eta_cur) x without a problem object and without
// any device allocation, for callers that cannot allocate (code under stream capture, tight
// serving loops). The operator's tables, the per-column geometry of both stages, the error
// flags and the problem descriptor the kernels read live in one file-scope device array of
// a fixed size; the geometry and operator kernels are the ones sa_apply_operator launches.
#include <mutex>

#include "host.h"

using namespace sa;

namespace {

constexpr int STATIC_MAX_NCOL = 32770;  // walls: nx <= 32768; periodic: nx <= 32771
constexpr int STATIC_MAX_DEV = 64;

// bytes of the layout below for the largest grid, rounded up
constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
constexpr size_t STATIC_BYTES =
    align256(sizeof(Problem)) + align256(64) + align256((size_t)NLMAX * 7 * 8) + align256((size_t)NLMAX * 4) + align256(49 * 8) +
    align256((size_t)NLMAX * 8) + 2 * align256((size_t)STATIC_MAX_NCOL * 8) +
    align256((size_t)4 * STATIC_MAX_NCOL * 8) + align256(NFLAGS * 4) + align256((size_t)2 * STATIC_MAX_NCOL * 8);

}  // namespace

// The scratch of every call on a device: its copy of this array. In host code the name is a
// stand-in, never a device address: kernels and copies use the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) char scratch[STATIC_BYTES];

static std::mutex g_static_mu;
static void* g_static_ptr[STATIC_MAX_DEV];

// the device address of this device's copy of the scratch array (looked up once per device)
static int static_scratch(int dev, char** out) {
  if (dev < 0 || dev >= STATIC_MAX_DEV) return sa_fail(SA_EARG, "sa_apply_operator_static: device %d", dev);
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return sa_fail(SA_EDEVICE, "sa_apply_operator_static: hipGetSymbolAddress: %s", hipGetErrorString(e));
    g_static_ptr[dev] = ptr;
  }
  *out = (char*)g_static_ptr[dev];
  return SA_OK;
}

extern "C" int sa_apply_operator_static(const sa_grid* grid, const double* h, const double* eta_prev,
                                        const double* eta_cur, const double* x, double* y, void* hip_stream) {
  if (!grid || !h || !eta_prev || !eta_cur || !x || !y) return sa_fail(SA_EARG, "sa_apply_operator_static: null argument");
  const int periodic = grid->bc == SA_PERIODIC;
  if (grid->bc != SA_PERIODIC && grid->bc != SA_WALLS) return sa_fail(SA_EARG, "sa_apply_operator_static: bad bc");
  if (grid->nz < 6 || grid->nz + 1 > NLMAX) return sa_fail(SA_EARG, "sa_apply_operator_static: nz must be in [6, %d]", NLMAX - 1);
  const int ncol = periodic ? grid->nx - 1 : grid->nx + 2;
  if ((periodic && ncol < 8) || (!periodic && grid->nx < 7))
    return sa_fail(SA_EARG, "sa_apply_operator_static: nx too small for seven-point stencils");
  if (ncol > STATIC_MAX_NCOL)
    return sa_fail(SA_EARG, "sa_apply_operator_static: %d columns exceed the static scratch (at most %d)", ncol,
                   STATIC_MAX_NCOL);
  if (!(grid->length > 0.0) || !isfinite(grid->length)) return sa_fail(SA_EARG, "sa_apply_operator_static: length");
  const int nphys = periodic ? grid->nx - 1 : grid->nx;
  for (int i = 0; i < nphys; ++i) {
    if (!(h[i] > 0.0) || !isfinite(h[i])) return sa_fail(SA_EGEOM, "sa_apply_operator_static: depth must be positive");
    if (!isfinite(eta_prev[i]) || !isfinite(eta_cur[i])) return sa_fail(SA_EGEOM, "sa_apply_operator_static: non-finite surface");
  }
  const int nl = grid->nz + 1, n = ncol * nl;
  const double dx = grid->length / (grid->nx - 1), dsig = 1.0 / (grid->nz - 1);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  char* base = nullptr;
  int rc = static_scratch(dev, &base);
  if (rc) return rc;
  hipStream_t stream = (hipStream_t)hip_stream;

  OperatorTables tb;
  operator_tables(ncol, nl, nphys, periodic, dx, dsig, h, tb);
  // layout inside the scratch (offsets relative to its start)
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += align256(bytes); return o; };
  // o_bar: the cluster barrier word every kernel's workgroup-cluster view reads at start
  // (make_cl, whenever a launch has more than one workgroup): zeroed, never waited on here
  const size_t o_prob = take(sizeof(Problem)), o_bar = take(64), o_wsig = take((size_t)nl * 7 * 8), o_ssig = take((size_t)nl * 4),
               o_wchi = take(49 * 8), o_sig = take((size_t)nl * 8), o_h = take((size_t)ncol * 8),
               o_hchi = take((size_t)ncol * 8), o_geo = take((size_t)4 * ncol * 8), o_flags = take(NFLAGS * 4),
               o_eta = take((size_t)2 * nphys * 8);
  const size_t used = off;
  Problem P{};
  P.ncol = ncol; P.nl = nl; P.nz = grid->nz; P.n = n; P.nphys = nphys; P.periodic = periodic;
  P.tx = TX;
  P.dx = dx; P.dsig = dsig;
  P.wsig = (decltype(P.wsig))(base + o_wsig); P.ssig = (decltype(P.ssig))(base + o_ssig);
  P.wchi = (decltype(P.wchi))(base + o_wchi); P.sig = (decltype(P.sig))(base + o_sig);
  P.h = (decltype(P.h))(base + o_h); P.hchi = (decltype(P.hchi))(base + o_hchi);
  P.geo = (decltype(P.geo))(base + o_geo);
  P.flags = (decltype(P.flags))(base + o_flags);
  P.bar = (decltype(P.bar))(base + o_bar);
  P.G = 1;
  // one host image of everything the kernels read, flags cleared, copied in one transfer
  std::vector<char> img(used, 0);
  memcpy(img.data() + o_prob, &P, sizeof P);
  memcpy(img.data() + o_wsig, tb.wsig.data(), tb.wsig.size() * 8);
  memcpy(img.data() + o_ssig, tb.ssig.data(), tb.ssig.size() * 4);
  memcpy(img.data() + o_wchi, tb.wchi.data(), 49 * 8);
  memcpy(img.data() + o_sig, tb.sig.data(), (size_t)nl * 8);
  memcpy(img.data() + o_h, tb.hext.data(), (size_t)ncol * 8);
  memcpy(img.data() + o_hchi, tb.hchi.data(), (size_t)ncol * 8);
  memcpy(img.data() + o_eta, eta_prev, (size_t)nphys * 8);
  memcpy(img.data() + o_eta + (size_t)nphys * 8, eta_cur, (size_t)nphys * 8);
  HIPCHK(hipMemcpyAsync(base, img.data(), used, hipMemcpyHostToDevice, stream));
  // the operator's dynamic LDS: input tile with halo, two gradient tiles, coefficient block
  const int W = TX + 3;
  const size_t lds = ((size_t)(W + 12 + 2 * (W + 6)) * nl + (49 + 9 * nl + 5 * (W + 6)) + NWAVE) * sizeof(double);
  HIPCHK(hipFuncSetAttribute((const void*)sa_operator_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const Problem* dp = (const Problem*)(base + o_prob);
  const double* ep = (const double*)(base + o_eta);
  const double* ec = ep + nphys;
  const int gb = (ncol + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL(sa_geometry_kernel, dim3(gb), dim3(BLOCK), 0, stream, dp, ep, ec);
  HIPCHK(hipGetLastError());
  int nt = (ncol + TX - 1) / TX;
  if (!periodic && nt > 1 && ncol - (nt - 1) * TX < 4) --nt;  // the last wall tile absorbs up to 3 columns
  hipLaunchKernelGGL(sa_operator_kernel, dim3(nt), dim3(BLOCK), lds, stream, dp, x, y);
  HIPCHK(hipGetLastError());
  int flags[NFLAGS];
  HIPCHK(hipMemcpyAsync(flags, base + o_flags, sizeof flags, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (flags[FLAG_GEOM]) return sa_fail(SA_EGEOM, "sa_apply_operator_static: h + eta <= 0 or non-finite surface");
  return SA_OK;
}
