// Device code of the subspace-accelerated sigma-transformed Poisson solver for gfx950, shared
// by the kernel translation units (solve64.hip: FP64 path, solve32.hip: FP32 refinement path).
//
// One solve (guess + restarted GMRES) is one persistent launch: a cluster of G workgroups
// owns the problem, walks through the phases below in order, and meets at a cluster barrier
// between phases (G = 1: a workgroup barrier only). Reductions are deterministic: every
// workgroup writes its partial sums, and after the barrier every workgroup adds the G
// partials in the same order, so all workgroups take bit-identical decisions without a
// broadcast.
//
// Phases and what they compute:
//   geometry   per-column 1/d and d_chi of both stages (Sec. 2.1, surface-subgrid D_chi)
//   operator   y = A x, the mixed-stage grad^(i) . grad^(i-1) with ghost-node boundary rows
//              (Sec. 3), LDS-staged tiles of 32 or TX columns x all levels, 7-point stencils
//   guess      Y <- r Y + x omega^T fused with W = A Y, Gram W^T W and W^T b over LDS tiles,
//              then the k x k least-squares solve and x0 = Y z (Alg. 2 with Alg. 4's V = Y)
//   precond    fixed still-water V-cycle: column (line) solves, x-semicoarsening, dense
//              coarsest inverse (thread per column, coalesced level-major rows)
//   arnoldi    classical Gram-Schmidt twice, wavefront-shuffle reductions, Givens in LDS
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#pragma once
#include "internal.h"

namespace sa {

#define DEV __device__ __forceinline__

// dynamic LDS of every kernel (size given at launch)
extern __shared__ double dyn_lds[];

constexpr long SPIN_LIMIT = 1L << 24;
constexpr long POLL_FAST = 64;
static_assert(NWAVE * (MMAX + 2) >= BLOCK, "the cluster-sum scratch (wsum) holds one double per thread");

// ------------------------------------------------------------------------------------------
// cluster of workgroups cooperating on one problem
struct Cl {
  int rank, G;
  unsigned* bar;
  int* flags;
  double* partials;
  int pbuf;
  unsigned gen;  // barrier generation this workgroup last saw complete (thread 0 only)
  double* scr;   // BLOCK doubles of LDS for the cluster sums (nullptr: sums read serially)
  unsigned* sgen;  // LDS, MAXLEV: generation of each level's sub-cluster barrier word seen by
                   // this workgroup (thread 0), nullptr: every barrier spans the cluster
};

// LDS word (in the sub-cluster generation table, after the levels' entries) through which
// the thread that arrives at a cluster sum's barrier tells its workgroup it arrived last
constexpr int SGEN_LAST = 31;
static_assert(MAXLEV < SGEN_LAST, "the generation table holds the levels and the last-arrival word");

// The barrier word of the sub-cluster barrier of V-cycle level l (64 bytes apart, after the
// cluster's own word).
DEV unsigned long long* sub_word(unsigned* bar, int l) {
  return reinterpret_cast<unsigned long long*>(bar + 16 * (1 + l));
}

// The barrier word of a cluster: one 64-bit atomic, arrivals in the low half, the generation
// (completed barriers) in the high half.
DEV unsigned long long* bar_word(unsigned* bar) { return reinterpret_cast<unsigned long long*>(bar); }

// Workgroup `rank` of a cluster of G on problem P. Thread 0 reads the barrier generation once:
// it advances only after all G workgroups have arrived at a barrier, and each reads it before
// its first arrival, so all start from the same value; the barrier then tracks it locally.
DEV Cl make_cl(const Problem& P, int rank, int G) {
  Cl cl{rank, G, P.bar, P.flags, P.partials, 0, 0u, nullptr, nullptr};
  if (threadIdx.x == 0 && G > 1)
    cl.gen = (unsigned)(__hip_atomic_load(bar_word(P.bar), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32);
  return cl;
}

DEV bool aborted(const Cl& cl) {
  return __hip_atomic_load(cl.flags + FLAG_ABORT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Barrier across the workgroups of the cluster. Arrival is one release fetch-add of 1 on the
// barrier word; the barrier is complete once the arrivals of this generation reach G. The
// arrival that completes it (it reads G - 1 arrivals) then subtracts G arrivals and adds one
// generation in a single atomic; until then early arrivals at the next barrier count on top,
// which the test below allows for. Waiters poll the word with relaxed loads and take one
// acquire fence once the barrier is complete. A wait that outlasts POLL_FAST polls backs off
// (a longer sleep between polls, the abort flag read every 64th poll): many workgroups left
// waiting while a few run the coarse V-cycle passes would otherwise keep the memory system
// busy with reads of the same two words. Every wait is bounded: after SPIN_LIMIT polls the
// abort flag is raised and all waiters leave.
// One arrival of thread 0 at the barrier on `word` among G workgroups, whose generation this
// workgroup last saw complete is gen (advanced here).
DEV void bar_arrive_wait(Cl& cl, unsigned long long* word, unsigned& gen, unsigned G) {
  const unsigned g0 = gen;
  gen = g0 + 1u;
  const unsigned long long old = __hip_atomic_fetch_add(word, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  if ((unsigned)(old >> 32) == g0 && (unsigned)old == G - 1u) {
    __hip_atomic_fetch_add(word, (1ull << 32) - G, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    long spins = 0;
    for (;;) {
      const unsigned long long v = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned gv = (unsigned)(v >> 32);
      if ((gv == g0 && (unsigned)v >= G) || (int)(gv - g0) > 0) break;
      if (spins < POLL_FAST) __builtin_amdgcn_s_sleep(1);
      else __builtin_amdgcn_s_sleep(8);
      ++spins;
      if (spins > SPIN_LIMIT || ((spins & 63) == 0 && aborted(cl))) {
        __hip_atomic_store(cl.flags + FLAG_ABORT, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

DEV void csync(Cl& cl) {
  __syncthreads();
  if (cl.G == 1) return;
  if (threadIdx.x == 0) bar_arrive_wait(cl, bar_word(cl.bar), cl.gen, (unsigned)cl.G);
  __syncthreads();
}

// Barrier among the workgroups of rank < parts only (the V-cycle passes of a level with fewer
// tiles than workgroups, and the pass that consumes their output), on level l's own word;
// the other workgroups do not take part and go on to their next barrier, which every
// workgroup of rank < parts reaches only after this one. parts >= G (or no generation
// table): a barrier of the whole cluster.
DEV void lsync(Cl& cl, int parts, int l) {
  if (!cl.sgen || parts >= cl.G) {
    csync(cl);
    return;
  }
  __syncthreads();
  if (cl.rank >= parts) return;
  if (threadIdx.x == 0) bar_arrive_wait(cl, sub_word(cl.bar, l), cl.sgen[l], (unsigned)parts);
  __syncthreads();
}

DEV double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// the G partial records of value 0 .. nv-1 at part (PSTRIDE apart) added into red, in one
// fixed order (the same on whichever workgroup runs it). With an LDS scratch the G x nv loads
// are spread over the whole workgroup: thread (q, i) adds the partials g = q, q + Q, ... of
// value i (Q = BLOCK / nv threads per value, all loads issued before the adds), then the Q
// sums of each value are added in q order.
DEV void combine_partials(const Cl& cl, const double* part, double* red, int nv) {
  const int Q = nv <= BLOCK ? BLOCK / nv : 1;
  if (!cl.scr || Q < 2) {
    for (int i = threadIdx.x; i < nv; i += BLOCK) {
      double s = 0.0;
      for (int g = 0; g < cl.G; ++g) s += part[g * PSTRIDE + i];
      red[i] = s;
    }
    __syncthreads();
    return;
  }
  const int q = threadIdx.x / nv, i = threadIdx.x - q * nv;
  if (q < Q) {
    constexpr int U = 8;
    double s = 0.0;
    for (int g0 = q; g0 < cl.G; g0 += U * Q) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int g = g0 + u * Q;
        v[u] = g < cl.G ? part[g * PSTRIDE + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) s += v[u];
    }
    cl.scr[q * nv + i] = s;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nv; t += BLOCK) {
    double s = 0.0;
    for (int qq = 0; qq < Q; ++qq) s += cl.scr[qq * nv + t];
    red[t] = s;
  }
  __syncthreads();
}

// Wait (thread 0) until the generation of `word` moves past g0, then acquire. Bounded and
// backing off like the barrier's own wait.
DEV void bar_wait_generation(Cl& cl, unsigned long long* word, unsigned g0) {
  long spins = 0;
  for (;;) {
    const unsigned long long v = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((int)((unsigned)(v >> 32) - g0) > 0) break;
    if (spins < POLL_FAST) __builtin_amdgcn_s_sleep(1);
    else __builtin_amdgcn_s_sleep(8);
    ++spins;
    if (spins > SPIN_LIMIT || ((spins & 63) == 0 && aborted(cl))) {
      __hip_atomic_store(cl.flags + FLAG_ABORT, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// red[0..nv) holds this workgroup's sums; afterwards it holds the cluster sums, the same bits
// on every workgroup. Each workgroup writes its record of partials and arrives at the cluster
// barrier; the arrival that completes it (its workgroup has then seen every record) adds the
// G records in the fixed order of combine_partials, writes the sums after the records and
// only then releases the barrier, so the other workgroups read nv values instead of G x nv.
// The records alternate between two buffers of G + 1 records (the next sum writes the other
// one, and the one after it starts only once every workgroup has read this one).
DEV void cluster_sum(Cl& cl, double* red, int nv) {
  __syncthreads();
  if (cl.G == 1) return;
  double* part = cl.partials + (size_t)cl.pbuf * (cl.G + 1) * PSTRIDE;
  double* total = part + (size_t)cl.G * PSTRIDE;
  for (int i = threadIdx.x; i < nv; i += BLOCK) part[cl.rank * PSTRIDE + i] = red[i];
  cl.pbuf ^= 1;
  if (!cl.sgen) {  // no LDS flag word: every workgroup adds the records itself
    csync(cl);
    combine_partials(cl, part, red, nv);
    return;
  }
  __syncthreads();
  unsigned* last = cl.sgen + SGEN_LAST;
  unsigned long long* word = bar_word(cl.bar);
  const unsigned g0 = cl.gen;
  if (threadIdx.x == 0) {
    cl.gen = g0 + 1u;
    const unsigned long long old = __hip_atomic_fetch_add(word, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const bool done = (unsigned)(old >> 32) == g0 && (unsigned)old == (unsigned)cl.G - 1u;
    if (done) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *last = done ? 1u : 0u;
  }
  __syncthreads();
  if (*last) {
    combine_partials(cl, part, red, nv);
    for (int i = threadIdx.x; i < nv; i += BLOCK) total[i] = red[i];
    __syncthreads();
    // one atomic: the arrivals back to 0 and the generation advanced, after the sums
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(word, (1ull << 32) - (unsigned long long)cl.G, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    if (threadIdx.x == 0) bar_wait_generation(cl, word, g0);
    __syncthreads();
    for (int i = threadIdx.x; i < nv; i += BLOCK) red[i] = total[i];
  }
  __syncthreads();
}

// sum of the NWAVE per-wave values w[0..NWAVE) in a fixed pairwise order
DEV double waves_sum(const double* w) {
  double s[NWAVE];
#pragma unroll
  for (int i = 0; i < NWAVE; ++i) s[i] = w[i];
#pragma unroll
  for (int h = NWAVE / 2; h > 0; h >>= 1)
#pragma unroll
    for (int i = 0; i < h; ++i) s[i] = s[2 * i] + s[2 * i + 1];
  return s[0];
}

// per-thread value v -> red[slot] = workgroup sum (fixed tree), all threads must call
DEV void block_sum_to(double v, double* wsum /*LDS NWAVE*/, double* red, int slot) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) wsum[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) red[slot] = waves_sum(wsum);
  __syncthreads();
}

// ------------------------------------------------------------------------------------------
// geometry of both stages, per column
DEV double eta_ext(const Problem& P, const double* eta, int c) {
  if (P.periodic) return eta[c];
  if (c == 0) return eta[1];
  if (c == P.ncol - 1) return eta[P.nphys - 2];
  return eta[c - 1];
}

// window of the seven-point x derivative at column c: weight row and first column (unwrapped)
DEV void chi_window(const Problem& P, int c, int& row, int& start) {
  if (P.periodic) { row = 3; start = c - HW; return; }
  if (c < HW) { row = c; start = 0; return; }
  if (c > P.ncol - 1 - HW) { row = 4 + c - (P.ncol - HW); start = P.ncol - 7; return; }
  row = 3; start = c - HW;
}

DEV int wrapc(int c, int nc) { return c < 0 ? c + nc : (c >= nc ? c - nc : c); }

DEV void phase_geometry(const Problem& P, Cl& cl, const double* __restrict__ eta_p, const double* __restrict__ eta_c) {
  const int nc = P.ncol;
  for (int c = cl.rank * BLOCK + threadIdx.x; c < nc; c += cl.G * BLOCK) {
    int row, start;
    chi_window(P, c, row, start);
    double dp = 0.0, dc = 0.0;
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      int cc = start + m;
      if (P.periodic) cc = ((cc % nc) + nc) % nc;
      const double w = P.wchi[row * 7 + m];
      dp += w * (P.h[cc] + eta_ext(P, eta_p, cc));
      dc += w * (P.h[cc] + eta_ext(P, eta_c, cc));
    }
    const double d_p = P.h[c] + eta_ext(P, eta_p, c);
    const double d_c = P.h[c] + eta_ext(P, eta_c, c);
    if (!(d_p > 0.0) || !(d_c > 0.0) || !isfinite(d_p) || !isfinite(d_c) || !isfinite(dp) || !isfinite(dc))
      atomicOr(P.flags + FLAG_GEOM, 1);
    P.geo[c] = 1.0 / d_p;
    P.geo[nc + c] = dp;
    P.geo[2 * nc + c] = 1.0 / d_c;
    P.geo[3 * nc + c] = dc;
  }
}

// i in [0, count) split over the workgroup; the loads of U consecutive strides are issued
// before any of them is used.
template <int U, class Ld, class St>
DEV void staged(int count, Ld ld, St st) {
  using T = std::decay_t<decltype(ld(0))>;
  for (int base = threadIdx.x; base < count; base += U * BLOCK) {
    T v[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int i = base + q * BLOCK;
      v[q] = i < count ? ld(i) : T(0);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int i = base + q * BLOCK;
      if (i < count) st(i, v[q]);
    }
  }
}

// Several staging segments in one batch: segment q has cnt[q] elements; ld(q, k) loads
// element k of segment q, st(q, k, v) stores it.
template <int U, int NS, class Ld, class St>
DEV void staged_segments(const int (&cnt)[NS], Ld ld, St st) {
  using T = std::decay_t<decltype(ld(0, 0))>;
  int total = 0;
#pragma unroll
  for (int q = 0; q < NS; ++q) total += cnt[q];
  auto locate = [&](int i, int& q, int& k) {
    q = 0;
    k = i;
#pragma unroll
    for (int r = 0; r < NS - 1; ++r)
      if (q == r && k >= cnt[r]) { k -= cnt[r]; q = r + 1; }
  };
  staged<U>(total, [&](int i) -> T {
    int q, k;
    locate(i, q, k);
    return ld(q, k);
  }, [&](int i, T v) {
    int q, k;
    locate(i, q, k);
    st(q, k, v);
  });
}

// Rows of one width: R rows of `width` (<= BLOCK) elements, row r element lc loaded by
// ld(r, lc) and stored by st(r, lc, v). Threads form BLOCK / width row lanes of `width`
// threads (lc = thread % width, no division per element); each thread issues the loads of U
// rows before any of its stores.
template <int U, class Ld, class St>
DEV void staged_rows(int R, int width, Ld ld, St st) {
  using T = std::decay_t<decltype(ld(0, 0))>;
  const int RP = BLOCK / width;
  const int lc = threadIdx.x % width, r0 = threadIdx.x / width;
  if (r0 >= RP) return;
  for (int base = r0; base < R; base += U * RP) {
    T v[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int r = base + q * RP;
      v[q] = r < R ? ld(r, lc) : T(0);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int r = base + q * RP;
      if (r < R) st(r, lc, v[q]);
    }
  }
}

// fn(r, lc) over R rows of `width` (<= BLOCK) elements, same thread layout as staged_rows
template <class Fn>
DEV void for_rows(int R, int width, Fn fn) {
  const int RP = BLOCK / width;
  const int lc = threadIdx.x % width, r0 = threadIdx.x / width;
  if (r0 >= RP) return;
  for (int r = r0; r < R; r += RP) fn(r, lc);
}

// ------------------------------------------------------------------------------------------
// operator tiles
struct Tiles {
  int nt, tw;
};

DEV Tiles tiles_of(const Problem& P, int tw) {
  int nt = (P.ncol + tw - 1) / tw;
  if (!P.periodic && nt > 1 && P.ncol - (nt - 1) * tw < 4) --nt;  // last wall tile >= 4 wide
  return Tiles{nt, tw};
}

// LDS doubles of the coefficient block of an operator tile of width W
DEV constexpr int opcoef_size(int W, int nl) { return 49 + 9 * nl + 5 * (W + 6); }

// A x on the columns [c0, c0 + w) of one tile, all levels. LDS: sx (W+12) x nl input with a
// 6-column halo, sgx/sgz (W+6) x nl gradient of the previous stage, sc the coefficient block
// (x and sigma weights, sigma windows and values, per-column geometry of both stages). Every
// operand of the stencil loops is in LDS. load(level, column, tile column) returns the input;
// out(level, tile column, column, value) receives A x. coef = false keeps the coefficient
// block of the previous call on the same tile (several inputs on one tile).
template <class S, int W, class Load, class Out>
DEV void tile_operator(const Problem& P, int c0, int w, Load load, S* sx, S* sgx, S* sgz, S* sc, Out out,
                       bool coef = true) {
  const int nc = P.ncol, nl = P.nl, nz = P.nz;
  constexpr int LX = W + 12, LG = W + 6;
  S* swchi = sc;                       // 49
  S* swsig = swchi + 49;               // nl x 7
  S* ssig = swsig + 7 * nl;            // nl sigma values
  int* sstart = (int*)(ssig + nl);     // nl window starts (stored in nl slots)
  S* gip = ssig + 2 * nl;              // LG: 1/d prev
  S* gdp = gip + LG;                   // LG: d_chi prev
  S* ghc = gdp + LG;                   // LG: h_chi
  S* gic = ghc + LG;                   // LG: 1/d cur
  S* gdc = gic + LG;                   // LG: d_chi cur
  // stage the input with a 6-column halo, load(level, column, tile-local column), and (coef)
  // the coefficient block, in one batch of loads
  const int nin = LX * nl;
  const int ncoef = 49 + 8 * nl;
  staged<8>(nin + (coef ? ncoef + 5 * LG : 0), [&](int i) -> S {
    if (i < nin) {
      const int lj = i / LX, lc = i - lj * LX;
      int c = c0 - 6 + lc;
      S v = S(0);
      if (lc < w + 12) {
        if (P.periodic) {
          c = ((c % nc) + nc) % nc;
          v = load(lj, c, lc);
        } else if (c >= 0 && c < nc) {
          v = load(lj, c, lc);
        }
      }
      return v;
    }
    i -= nin;
    if (i < 49) return S(P.wchi[i]);
    if (i < 49 + 7 * nl) return S(P.wsig[i - 49]);
    if (i < 49 + 8 * nl) return S(P.sig[i - 49 - 7 * nl]);
    const int q = (i - ncoef) / LG, lc = i - ncoef - q * LG;
    int c = c0 - 3 + lc;
    if (P.periodic) c = ((c % nc) + nc) % nc;
    else if (c < 0 || c >= nc) return S(0);
    if (q == 2) return S(P.hchi[c]);
    return S(P.geo[(q < 2 ? q : q - 1) * nc + c]);
  }, [&](int i, S v) {
    if (i < nin) sx[i] = v;
    else if (i - nin < ncoef) swchi[i - nin] = v;
    else gip[i - nin - ncoef] = v;
  });
  if (coef)
    for (int j = threadIdx.x; j < nl; j += BLOCK) sstart[j] = P.ssig[j];
  __syncthreads();
  // gradient of the previous stage: G_x = D_x p + sigma_x D_sigma p, G_z = D_sigma p / d
  for (int i = threadIdx.x; i < LG * nl; i += BLOCK) {
    const int lj = i / LG, lc = i - lj * LG;
    const int c = c0 - 3 + lc;
    if (lc >= w + 6) continue;
    if (!P.periodic && (c < 0 || c >= nc)) continue;
    int row, start;
    chi_window(P, c, row, start);
    const int sidx = start - c0 + 6;
    S dxv = S(0);
#pragma unroll
    for (int m = 0; m < 7; ++m) dxv += swchi[row * 7 + m] * sx[lj * LX + sidx + m];
    const int s0 = sstart[lj];
    S dsv = S(0);
#pragma unroll
    for (int m = 0; m < 7; ++m) dsv += swsig[lj * 7 + m] * sx[(s0 + m) * LX + lc + 3];
    const S invd = gip[lc];
    const S sxp = (ghc[lc] - ssig[lj] * gdp[lc]) * invd;
    sgx[i] = dxv + sxp * dsv;
    sgz[i] = invd * dsv;
  }
  __syncthreads();
  // divergence of the current stage, boundary rows, identity rows
  for (int i = threadIdx.x; i < W * nl; i += BLOCK) {
    const int lj = i / W, lc = i - lj * W;
    if (lc >= w) continue;
    const int c = c0 + lc;
    const bool ghostcol = !P.periodic && (c == 0 || c == nc - 1);
    S v;
    if (lj == nz || (ghostcol && lj == 0)) {
      v = sx[lj * LX + lc + 6];
    } else if (ghostcol) {
      v = (c == 0) ? -sgx[lj * LG + (1 - c0) + 3] : sgx[lj * LG + (nc - 2 - c0) + 3];
    } else if (lj == 0) {
      v = -ghc[lc + 3] * sgx[LG + lc + 3] - sgz[LG + lc + 3];
    } else {
      int row, start;
      chi_window(P, c, row, start);
      const int gidx = start - c0 + 3;
      S dxg = S(0);
#pragma unroll
      for (int m = 0; m < 7; ++m) dxg += swchi[row * 7 + m] * sgx[lj * LG + gidx + m];
      const int s0 = sstart[lj];
      S dsg = S(0), dsz = S(0);
#pragma unroll
      for (int m = 0; m < 7; ++m) {
        const S ws = swsig[lj * 7 + m];
        dsg += ws * sgx[(s0 + m) * LG + lc + 3];
        dsz += ws * sgz[(s0 + m) * LG + lc + 3];
      }
      const S invd = gic[lc + 3];
      const S sxc = (ghc[lc + 3] - ssig[lj] * gdc[lc + 3]) * invd;
      v = dxg + sxc * dsg + invd * dsz;
    }
    out(lj, lc, c, v);
  }
  __syncthreads();
}

// y = A x (b == nullptr) or y = b - A x with ||y||^2 and ||b||^2 into red[slot], red[slot+1]
template <int OTX>
DEV void phase_operator_t(const Problem& P, Cl& cl, const double* __restrict__ x, double xs, double* y,
                          const double* __restrict__ b, double* lds, double* red, int slot) {
  constexpr int W = OTX + 3;  // widest tile (a last wall tile absorbs up to 3 columns)
  const bool resid = b != nullptr;
  const Tiles T = tiles_of(P, OTX);
  double* sx = lds;
  double* sgx = sx + (W + 12) * P.nl;
  double* sgz = sgx + (W + 6) * P.nl;
  double* sc = sgz + (W + 6) * P.nl;
  double* wsum = sc + opcoef_size(W, P.nl);
  const int nc = P.ncol;
  double acc = 0.0, accb = 0.0;
  for (int t = cl.rank; t < T.nt; t += cl.G) {
    const int c0 = t * OTX;
    const int w = (t == T.nt - 1) ? nc - c0 : OTX;
    auto load = [&](int lj, int c, int) { return x[(size_t)lj * nc + c] * xs; };
    tile_operator<double, W>(P, c0, w, load, sx, sgx, sgz, sc, [&](int lj, int lc, int c, double v) {
      const size_t e = (size_t)lj * nc + c;
      if (resid) {
        const double bb = b[e];
        const double rr = bb - v;
        y[e] = rr;
        acc += rr * rr;
        accb += bb * bb;
      } else {
        y[e] = v;
      }
    });
  }
  if (resid) {
    block_sum_to(acc, wsum, red, slot);
    block_sum_to(accb, wsum, red, slot + 1);
  }
}

// on the operator tile width of the problem (32 columns where every such tile has a cluster
// workgroup, else TX); the partial sums of the residual form go to red[slot], red[slot + 1]
DEV void phase_operator(const Problem& P, Cl& cl, const double* __restrict__ x, double xs, double* y,
                        const double* __restrict__ b, double* lds, double* red, int slot) {
  if (P.tx == 32) phase_operator_t<32>(P, cl, x, xs, y, b, lds, red, slot);
  else phase_operator_t<TX>(P, cl, x, xs, y, b, lds, red, slot);
}

// y = A (xs x) in the inner precision S (FP32 refinement path): same tiles, no residual form
template <class S, int OTX>
DEV void phase_operator_st(const Problem& P, Cl& cl, const S* __restrict__ x, S xs, S* y, S* lds) {
  constexpr int W = OTX + 3;
  const Tiles T = tiles_of(P, OTX);
  S* sx = lds;
  S* sgx = sx + (W + 12) * P.nl;
  S* sgz = sgx + (W + 6) * P.nl;
  S* sc = sgz + (W + 6) * P.nl;
  const int nc = P.ncol;
  for (int t = cl.rank; t < T.nt; t += cl.G) {
    const int c0 = t * OTX;
    const int w = (t == T.nt - 1) ? nc - c0 : OTX;
    auto load = [&](int lj, int c, int) { return x[(size_t)lj * nc + c] * xs; };
    tile_operator<S, W>(P, c0, w, load, sx, sgx, sgz, sc, [&](int lj, int lc, int c, S v) {
      y[(size_t)lj * nc + c] = v;
    });
  }
}

template <class S>
DEV void phase_operator_s(const Problem& P, Cl& cl, const S* __restrict__ x, S xs, S* y, S* lds) {
  if (P.tx == 32) phase_operator_st<S, 32>(P, cl, x, xs, y, lds);
  else phase_operator_st<S, TX>(P, cl, x, xs, y, lds);
}

// ------------------------------------------------------------------------------------------
// still-water preconditioner (second-order direct form at eta = 0), LDS-staged tiles of TM
// columns x all levels. A tile's fields, column data (h, 1/h, h_x, h_xx) and line-solve
// factors are staged with batched coalesced loads; residuals are formed from LDS; the
// vertical line solves run one thread per column from LDS with precomputed elimination
// factors (M is fixed), so the recurrences carry no division.
constexpr int TM = 64;
constexpr int TMS = TM + 4;  // stride of the per-thread line-solve scratch

// A level of the hierarchy seen in precision S: line-solve factors and work vectors of that
// precision (column data h, 1/h, h_x, h_xx stay FP64 and are rounded when staged).
template <class S>
struct Lv {
  int nc, nx, fstride, facstride;
  S rdx, rds;  // 1/dx of the level, 1/dsigma
  const double *h, *ih, *hx, *hxx;
  const S *fpc, *finv, *flo, *fgam;
  S *f, *u, *o;
};

template <class S>
DEV Lv<S> level_view(const Problem& P, int l) {
  const Level& L = P.lev[l];
  if constexpr (std::is_same_v<S, float>)
    return Lv<S>{L.ncol, L.nx, L.fstride, L.facstride, S(1.0 / L.dx), S(1.0 / P.dsig), L.h, L.ih, L.hx, L.hxx,
                 L.fpc32, L.finv32, L.flo32, L.fgam32, L.f32, L.u32, L.o32};
  else
    return Lv<S>{L.ncol, L.nx, L.fstride, L.facstride, 1.0 / L.dx, 1.0 / P.dsig, L.h, L.ih, L.hx, L.hxx, L.fpc, L.finv,
                 L.flo, L.fgam,
                 L.f, L.u, L.o};
}

template <class S>
DEV const S* coarse_inverse(const Problem& P) {
  if constexpr (std::is_same_v<S, float>) return P.cinv32;
  else return P.cinv;
}

// tile-local staging: column c (unwrapped) <-> slot c - base
struct Stage {
  int base, width, nc, periodic;
  DEV int slot(int c) const { return c - base; }
  DEV int col(int c) const { return periodic ? wrapc(c, nc) : c; }
  DEV bool has(int c) const { return periodic || (c >= 0 && c < nc); }
};

// (M u)(c, j): U(cc, jj) returns the staged field at unwrapped column cc; CD(cc, q) the
// staged column data q = 0 h, 1 1/h, 2 h_x, 3 h_xx of unwrapped column cc.
template <class S, class U, class CD>
DEV S m_apply(const Problem& P, int nc, S rdx, S rds, S oms, int c, int j, U u, CD cd) {
  const int nz = P.nz;
  const S half = S(0.5), two = S(2), quarter = S(0.25);
  if (j == nz) return u(c, j);
  if (!P.periodic && (c == 0 || c == nc - 1)) {
    if (j == 0) return u(c, j);
    const int w = (c == 0) ? 1 : nc - 2;
    const S s = cd(w, 2) * oms * cd(w, 1);
    const S gx = (u(w + 1, j) - u(w - 1, j)) * half * rdx + s * (u(w, j + 1) - u(w, j - 1)) * half * rds;
    return c == 0 ? -gx : gx;
  }
  const S ih = cd(c, 1), hx = cd(c, 2);
  if (j == 0) {
    const S s1 = hx * ih;
    const S dz = (u(c, 2) - u(c, 0)) * half * rds;
    const S gx = (u(c + 1, 1) - u(c - 1, 1)) * half * rdx + s1 * dz;
    return -hx * gx - dz * ih;
  }
  const S s = hx * oms * ih;
  const S sxx = oms * cd(c, 3) * ih - two * oms * hx * hx * ih * ih;
  const S uc = u(c, j);
  const S dxx = (u(c + 1, j) - two * uc + u(c - 1, j)) * rdx * rdx;
  const S dxz = (u(c + 1, j + 1) - u(c + 1, j - 1) - u(c - 1, j + 1) + u(c - 1, j - 1)) * quarter * rdx * rds;
  const S dzz = (u(c, j + 1) - two * uc + u(c, j - 1)) * rds * rds;
  const S dz = (u(c, j + 1) - u(c, j - 1)) * half * rds;
  return dxx + two * s * dxz + (s * s + ih * ih) * dzz + sxx * dz;
}

// Line solve of one column in place: r <- L^-1 r with L the same-column part of M. The bed
// row (coupling levels 0 and 2) is combined with row 1 (factor gam) so the system is
// tridiagonal; lo, pc, inv are the precomputed sub-diagonal, elimination ratios and inverse
// pivots (free-surface row: identity). Level stride rs for r, fs for the factors.
// The recurrences run in blocks of LSB levels: the operands of the next block are read from
// LDS before the current block's results are written back, so the dependent chain is the
// arithmetic alone, not an LDS round trip per level (same operations in the same order as
// the plain level-by-level loop, which finishes the levels left over).
constexpr int LSB = 4;
template <class S>
DEV void line_solve(int nz, S gam, S* __restrict__ r, int rs, const S* __restrict__ lo, const S* __restrict__ pc,
                    const S* __restrict__ inv, int fs) {
  S pd = (r[0] - gam * r[rs]) * inv[0];
  r[0] = pd;
  // forward elimination, levels 1 .. nz - 1
  int j = 1;
  if (nz - 1 >= LSB) {
    S ra[LSB], la[LSB], ia[LSB];
#pragma unroll
    for (int q = 0; q < LSB; ++q) {
      ra[q] = r[(1 + q) * rs];
      la[q] = lo[(1 + q) * fs];
      ia[q] = inv[(1 + q) * fs];
    }
    for (; j + 2 * LSB <= nz; j += LSB) {  // levels j .. j+3 now, j+4 .. j+7 (< nz) read ahead
      S rb[LSB], lb[LSB], ib[LSB];
#pragma unroll
      for (int q = 0; q < LSB; ++q) {
        rb[q] = r[(j + LSB + q) * rs];
        lb[q] = lo[(j + LSB + q) * fs];
        ib[q] = inv[(j + LSB + q) * fs];
      }
#pragma unroll
      for (int q = 0; q < LSB; ++q) {
        pd = (ra[q] - la[q] * pd) * ia[q];
        r[(j + q) * rs] = pd;
      }
#pragma unroll
      for (int q = 0; q < LSB; ++q) { ra[q] = rb[q]; la[q] = lb[q]; ia[q] = ib[q]; }
    }
#pragma unroll
    for (int q = 0; q < LSB; ++q) {
      pd = (ra[q] - la[q] * pd) * ia[q];
      r[(j + q) * rs] = pd;
    }
    j += LSB;
  }
  for (; j < nz; ++j) {
    pd = (r[j * rs] - lo[j * fs] * pd) * inv[j * fs];
    r[j * rs] = pd;
  }
  // back substitution, levels nz - 1 .. 0 (the free-surface row nz is the identity)
  S d = r[nz * rs];
  j = nz - 1;
  if (nz >= LSB) {
    S rv[LSB], pv[LSB];
#pragma unroll
    for (int q = 0; q < LSB; ++q) {
      rv[q] = r[(j - q) * rs];
      pv[q] = pc[(j - q) * fs];
    }
    for (; j >= 2 * LSB - 1; j -= LSB) {  // levels j .. j-3 now, j-4 .. j-7 (>= 0) read ahead
      S rw[LSB], pw[LSB];
#pragma unroll
      for (int q = 0; q < LSB; ++q) {
        rw[q] = r[(j - LSB - q) * rs];
        pw[q] = pc[(j - LSB - q) * fs];
      }
#pragma unroll
      for (int q = 0; q < LSB; ++q) {
        d = rv[q] - pv[q] * d;
        r[(j - q) * rs] = d;
      }
#pragma unroll
      for (int q = 0; q < LSB; ++q) { rv[q] = rw[q]; pv[q] = pw[q]; }
    }
#pragma unroll
    for (int q = 0; q < LSB; ++q) {
      d = rv[q] - pv[q] * d;
      r[(j - q) * rs] = d;
    }
    j -= LSB;
  }
  for (; j >= 0; --j) {
    d = r[j * rs] - pc[j * fs] * d;
    r[j * rs] = d;
  }
}

// coarse value interpolated to fine column c (linear in x), level j
template <class S>
DEV S prolong_at(const Problem& P, int ncf, int ncc, const S* e, int c, int j) {
  const S* ec = e + (size_t)j * ncc;
  const S half = S(0.5);
  if (P.periodic) return (c & 1) ? half * (ec[(c - 1) >> 1] + ec[wrapc((c + 1) >> 1, ncc)]) : ec[c >> 1];
  if (c == 0 || c == ncf - 1) return ec[c == 0 ? 0 : ncc - 1];
  const int p = c - 1;
  return (p & 1) ? half * (ec[((p - 1) >> 1) + 1] + ec[((p + 1) >> 1) + 1]) : ec[(p >> 1) + 1];
}

// the coarse columns (and whether two are averaged) prolong_at reads for fine column c
DEV void prolong_cols(const Problem& P, int ncf, int ncc, int c, int& i0, int& i1, bool& odd) {
  odd = false;
  i1 = 0;
  if (P.periodic) {
    if (c & 1) { odd = true; i0 = (c - 1) >> 1; i1 = wrapc((c + 1) >> 1, ncc); }
    else i0 = c >> 1;
    return;
  }
  if (c == 0 || c == ncf - 1) { i0 = c == 0 ? 0 : ncc - 1; return; }
  const int p = c - 1;
  if (p & 1) { odd = true; i0 = ((p - 1) >> 1) + 1; i1 = ((p + 1) >> 1) + 1; }
  else i0 = (p >> 1) + 1;
}

DEV int ptiles(int nc) { return (nc + TM - 1) / TM; }
DEV int coarse_centre(const Problem& P, int C, int ncc, int ncf) {
  if (P.periodic) return 2 * C;
  if (C == 0) return 0;
  if (C == ncc - 1) return ncf - 1;
  return 2 * C - 1;
}

// column data q (0 h, 1 1/h, 2 h_x, 3 h_xx) of global column cg, rounded to S
template <class S>
DEV S coldata(const Lv<S>& L, int q, int cg) {
  return S(L.h[q * L.nc + cg]);  // h | 1/h | h_x | h_xx, ncol apart
}

// line-solve factor qq (0 lo, 1 pc, 2 inv) at level j of global column cg
template <class S>
DEV S factor(const Lv<S>& L, int qq, int j, int cg) {
  // lo | pc | inv, facstride apart
  return L.flo[qq * L.facstride + j * (L.fstride ? L.fstride : 1) + (L.fstride ? cg : 0)];
}

// value i of a uniform level's one set of line-solve constants: the factors lo | pc | inv
// (nl levels each, i < 3 nl), then gamma
template <class S>
DEV S uniform_factor(const Lv<S>& L, int nl, int i) {
  return i < 3 * nl ? L.flo[i] : L.fgam[0];
}

// o = u + omega L^-1 (f - M u) on level l, u = (uin or 0) + (e ? P e : 0) formed on load.
// Residuals are formed by all threads in LDS, then one thread per column eliminates.
template <class S, int TW = TM>
DEV void phase_sweep(const Problem& P, Cl& cl, int l, const S* f, const S* uin, const S* e, S* o, S* lds,
                      const S* rc = nullptr) {
  const Lv<S> L = level_view<S>(P, l);
  const int nc = L.nc, nl = P.nl, nz = P.nz;
  const int ncc = e ? P.lev[l + 1].ncol : 0;
  constexpr int LW = TW + 2;
  S* su = lds;                 // LW x nl
  S* sr = su + LW * nl;        // TW x nl: f, then the residual, then the correction
  S* scd = sr + TW * nl;       // 4 x LW
  S* sfac = scd + 4 * LW;      // 3 x TW x nl
  S* sgam = sfac + 3 * TW * nl;  // TW
  // or the workgroup's resident block rc of this level: the layout of the down pass (columns
  // c0 - 2 .. c0 + w + 1, stride TW + 4), read at the offsets of this pass's columns
  constexpr int LR = TW + 4;
  const S* ccd = rc ? rc + 1 : scd;            // column c0 - 1 + lc at [lc]
  const int cds = rc ? LR : LW;
  // factors of column c0 + lc at [lc * cst], level stride fst, gamma after the 3 nl factor
  // rows; on a uniform level every column shares one set (cst = 0, level stride 1)
  const bool uni = L.fstride == 0;
  const int cst = uni ? 0 : 1;
  const S* cfac = rc ? rc + 4 * LR + 2 * cst : sfac;
  const int fst = uni ? 1 : (rc ? LR : TW);
  const S* cgam = cfac + 3 * fst * nl;
  const bool zero = !uin && !e;
  for (int t = cl.rank; t < (nc + TW - 1) / TW; t += cl.G) {
    const int c0 = t * TW, w = min(TW, nc - c0);
    const Stage st{c0 - 1, w + 2, nc, P.periodic};
    // rows of width w + 2 (column c0 - 1 + lc): u (with the prolongated correction) and column
    // data over the halo, f, factors and gamma over the tile's own columns
    const int ww = w + 2;
    const int nu = zero ? 0 : nl, ncd = zero ? 0 : 4;
    const int rf = nu, rcd = rf + nl, rfac = rcd + ncd, rgam = rfac + 3 * nl;
    const int fsm = L.fstride ? L.fstride : 1;
    // u and f: each thread owns one column of the rows it stages (the column's wrap, halo
    // and prolongation stencil worked out once), so the loads of all its rows are issued
    // together with no per-element branching
    {
      const int RP = BLOCK / ww;
      const int lc = threadIdx.x % ww, r0 = threadIdx.x / ww;
      if (r0 < RP) {
        const int c = c0 - 1 + lc;
        const bool has = st.has(c), own = lc >= 1 && lc <= w;
        const int cg = has ? st.col(c) : 0;
        int i0 = 0, i1 = 0;
        bool odd = false;
        if (e && has) prolong_cols(P, nc, ncc, cg, i0, i1, odd);
        // u (with the prolongated correction) and f of each row in one batch of loads
        constexpr int U = 3;
        for (int rb = r0; rb < nl; rb += U * RP) {
          S v[U], g[U];
#pragma unroll
          for (int q = 0; q < U; ++q) {
            const int r = rb + q * RP;
            S t = S(0);
            if (!zero && r < nl && has) {
              t = uin ? uin[(size_t)r * nc + cg] : S(0);
              if (e) {
                const S* er = e + (size_t)r * ncc;
                t += odd ? S(0.5) * (er[i0] + er[i1]) : er[i0];
              }
            }
            v[q] = t;
            g[q] = (own && r < nl) ? f[(size_t)r * nc + c] : S(0);
          }
#pragma unroll
          for (int q = 0; q < U; ++q) {
            const int r = rb + q * RP;
            if (r < nl) {
              if (!zero) su[r * LW + lc] = v[q];
              if (own) sr[r * TW + lc - 1] = g[q];
            }
          }
        }
      }
    }
    // column data over the halo, factors and gamma over the own columns (unless resident;
    // a uniform level's one set of factors and gamma: one value per thread, in the same batch)
    if (!rc) {
      const int nf = uni ? 3 * nl + 1 : 0;
      const S fv = (int)threadIdx.x < nf ? uniform_factor(L, nl, threadIdx.x) : S(0);
      staged_rows<16>((uni ? rfac : rgam + 1) - rcd, ww, [&](int rr, int lc) -> S {
        const int r = rr + rcd;
        const int c = c0 - 1 + lc;
        const bool own = lc >= 1 && lc <= w;
        if (r < rfac) return st.has(c) ? coldata(L, r - rcd, st.col(c)) : S(1);
        if (r < rgam) return own ? L.flo[(r - rfac) * fsm + (L.fstride ? c : 0)] : S(0);
        return own ? L.fgam[L.fstride ? c : 0] : S(0);
      }, [&](int rr, int lc, S v) {
        const int r = rr + rcd;
        if (!(lc >= 1 && lc <= w) && r >= rfac) return;
        if (r < rfac) scd[(r - rcd) * LW + lc] = v;
        else if (r < rgam) sfac[(r - rfac) * TW + lc - 1] = v;
        else sgam[lc - 1] = v;
      });
      if ((int)threadIdx.x < nf) sfac[threadIdx.x] = fv;
    }
    __syncthreads();
    if (!zero) {
      auto U = [&](int cc, int jj) { return su[jj * LW + st.slot(cc)]; };
      auto CD = [&](int cc, int q) { return ccd[q * cds + st.slot(cc)]; };
      for (int i = threadIdx.x; i < TW * nl; i += BLOCK) {
        const int j = i / TW, lc = i - j * TW;
        if (lc < w) sr[i] -= m_apply<S>(P, nc, L.rdx, L.rds, S(1.0 - P.sig[j]), c0 + lc, j, U, CD);
      }
      __syncthreads();
    }
    if (threadIdx.x < w) {
      const int lc = threadIdx.x, lf = lc * cst;
      line_solve<S>(nz, cgam[lf], sr + lc, TW, cfac + lf, cfac + fst * nl + lf, cfac + 2 * fst * nl + lf, fst);
    }
    __syncthreads();
    const S om = S(P.omega);
    for (int i = threadIdx.x; i < TW * nl; i += BLOCK) {
      const int j = i / TW, lc = i - j * TW;
      if (lc < w) o[(size_t)j * nc + c0 + lc] = (zero ? S(0) : su[j * LW + lc + 1]) + om * sr[i];
    }
    __syncthreads();
  }
}

// Two sweeps o = u1 + omega L^-1 (f - M u1), u1 = u + omega L^-1 (f - M u) in one pass, on a
// periodic level whose columns share one set of line-solve constants: u (uin plus the
// prolongated correction e) is staged with two columns each side, the first sweep runs on the
// tile and one column each side, the second on the tile. The first sweep's halo columns repeat
// the arithmetic of the neighbouring tiles' own first sweep, so o is the two-pass result bit for
// bit, one pass and one barrier sooner. rc: the workgroup's resident block of this level (the
// down pass's layout: columns c0 - 2 .. c0 + w + 1, the shared factors and gamma after them).
template <class S, int TW = TM>
DEV void phase_sweep2(const Problem& P, Cl& cl, int l, const S* f, const S* uin, const S* e, S* o, S* lds,
                      const S* rc = nullptr) {
  const Lv<S> L = level_view<S>(P, l);
  const int nc = L.nc, nl = P.nl, nz = P.nz;
  const int ncc = e ? P.lev[l + 1].ncol : 0;
  constexpr int LW = TW + 4;   // u and column data: columns c0 - 2 .. c0 + w + 1
  constexpr int LF = TW + 2;   // f and the residual: columns c0 - 1 .. c0 + w
  S* su = lds;                 // LW x nl
  S* sf = su + LW * nl;        // LF x nl
  S* sr = sf + LF * nl;        // LF x nl
  S* scd = sr + LF * nl;       // 4 x LW
  S* sfac = scd + 4 * LW;      // 3 nl + 1: lo | pc | inv, gamma
  const S* ccd = rc ? rc : scd;
  const S* cfac = rc ? rc + 4 * LW : sfac;
  const S om = S(P.omega);
  for (int t = cl.rank; t < (nc + TW - 1) / TW; t += cl.G) {
    const int c0 = t * TW, w = min(TW, nc - c0);
    const int ww = w + 4;
    // u (with the prolongated correction) over the two-column halo, f over the one-column
    // halo: each thread owns one column of the rows it stages
    {
      const int RP = BLOCK / ww;
      const int lc = threadIdx.x % ww, r0 = threadIdx.x / ww;
      if (r0 < RP) {
        const int cg = wrapc(c0 - 2 + lc, nc);
        const bool fo = lc >= 1 && lc <= w + 2;
        int i0 = 0, i1 = 0;
        bool odd = false;
        if (e) prolong_cols(P, nc, ncc, cg, i0, i1, odd);
        constexpr int U = 3;
        for (int rb = r0; rb < nl; rb += U * RP) {
          S v[U], g[U];
#pragma unroll
          for (int q = 0; q < U; ++q) {
            const int r = rb + q * RP;
            S tv = S(0);
            if (r < nl) {
              tv = uin ? uin[(size_t)r * nc + cg] : S(0);
              if (e) {
                const S* er = e + (size_t)r * ncc;
                tv += odd ? S(0.5) * (er[i0] + er[i1]) : er[i0];
              }
            }
            v[q] = tv;
            g[q] = (fo && r < nl) ? f[(size_t)r * nc + cg] : S(0);
          }
#pragma unroll
          for (int q = 0; q < U; ++q) {
            const int r = rb + q * RP;
            if (r < nl) {
              su[r * LW + lc] = v[q];
              if (fo) sf[r * LF + lc - 1] = g[q];
            }
          }
        }
      }
    }
    if (!rc) {
      // column data over the two-column halo and the one set of factors and gamma
      const int nf = 3 * nl + 1;
      const S fv = (int)threadIdx.x < nf ? uniform_factor(L, nl, threadIdx.x) : S(0);
      staged_rows<16>(4, ww, [&](int q, int lc) -> S { return coldata(L, q, wrapc(c0 - 2 + lc, nc)); },
                      [&](int q, int lc, S v) { scd[q * LW + lc] = v; });
      if ((int)threadIdx.x < nf) sfac[threadIdx.x] = fv;
    }
    __syncthreads();
    // first sweep on columns c0 - 1 .. c0 + w (unwrapped column cc sits at slot cc - c0 + 2)
    {
      auto U = [&](int cc, int jj) { return su[jj * LW + cc - c0 + 2]; };
      auto CD = [&](int cc, int q) { return ccd[q * LW + cc - c0 + 2]; };
      for (int i = threadIdx.x; i < LF * nl; i += BLOCK) {
        const int j = i / LF, lf = i - j * LF;
        if (lf < w + 2) sr[i] = sf[i] - m_apply<S>(P, nc, L.rdx, L.rds, S(1.0 - P.sig[j]), c0 - 1 + lf, j, U, CD);
      }
    }
    __syncthreads();
    const S gam = cfac[3 * nl];  // staged above (or resident)
    if ((int)threadIdx.x < w + 2)
      line_solve<S>(nz, gam, sr + threadIdx.x, LF, cfac, cfac + nl, cfac + 2 * nl, 1);
    __syncthreads();
    for (int i = threadIdx.x; i < LF * nl; i += BLOCK) {
      const int j = i / LF, lf = i - j * LF;
      if (lf < w + 2) su[j * LW + lf + 1] = su[j * LW + lf + 1] + om * sr[i];
    }
    __syncthreads();
    // second sweep on the tile
    {
      auto U = [&](int cc, int jj) { return su[jj * LW + cc - c0 + 2]; };
      auto CD = [&](int cc, int q) { return ccd[q * LW + cc - c0 + 2]; };
      for (int i = threadIdx.x; i < LF * nl; i += BLOCK) {
        const int j = i / LF, lf = i - j * LF;
        if (lf >= 1 && lf <= w) sr[i] = sf[i] - m_apply<S>(P, nc, L.rdx, L.rds, S(1.0 - P.sig[j]), c0 - 1 + lf, j, U, CD);
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < w)
      line_solve<S>(nz, gam, sr + threadIdx.x + 1, LF, cfac, cfac + nl, cfac + 2 * nl, 1);
    __syncthreads();
    for (int i = threadIdx.x; i < TW * nl; i += BLOCK) {
      const int j = i / TW, lc = i - j * TW;
      if (lc < w) o[(size_t)j * nc + c0 + lc] = su[j * LW + lc + 2] + om * sr[j * LF + lc + 1];
    }
    __syncthreads();
  }
}

DEV void coarse_range(const Problem& P, int c0, int w, int nc, int ncc, int& Cfirst, int& Clast) {
  if (P.periodic) { Cfirst = (c0 + 1) / 2; Clast = (c0 + w - 1) / 2; return; }
  Cfirst = (c0 == 0) ? 0 : (c0 + 2) / 2;
  Clast = (c0 + w >= nc) ? ncc - 1 : (c0 + w) / 2;
}

// full weighting of the residual R(cc) around the centre of coarse column C
template <class S, class RR>
DEV S restrict_at(const Problem& P, int C, int ncc, int nxc, int nc, RR Rr) {
  const int cf = coarse_centre(P, C, ncc, nc);
  const S half = S(0.5), quarter = S(0.25);
  if (P.periodic) return quarter * Rr(cf - 1) + half * Rr(cf) + quarter * Rr(cf + 1);
  if (C == 0 || C == ncc - 1) return Rr(cf);
  if (C == 1) return half * Rr(1) + half * Rr(2);
  if (C == nxc) return half * Rr(cf) + half * Rr(cf - 1);
  return quarter * Rr(cf - 1) + half * Rr(cf) + quarter * Rr(cf + 1);
}

// Pre-smoothing from zero, residual and restriction in one pass (nu1 = 1):
// u = omega L^-1 f on the tile plus a 2-column halo, u written for the tile's columns,
// fc(C) = full weighting of f - M u at the fine columns around C's centre.
template <class S, int TW = TM>
DEV void phase_down(const Problem& P, Cl& cl, int l, const S* f, S* u, S* fc, S* lds, const S* rc = nullptr) {
  const Lv<S> L = level_view<S>(P, l);
  const int nc = L.nc, nl = P.nl, nz = P.nz;
  const int ncc = P.lev[l + 1].ncol, nxc = P.lev[l + 1].nx;
  constexpr int LW = TW + 4;
  S* sf = lds;                 // LW x nl
  S* su = sf + LW * nl;        // LW x nl
  // column data (4 x LW), factors (3 x LW x nl) and gamma (LW): staged below, or the
  // workgroup's resident block rc of the same layout (its one tile of this level)
  S* scd = su + LW * nl;
  S* sfac = scd + 4 * LW;
  S* sgam = sfac + 3 * LW * nl;
  const S* ccd = rc ? rc : scd;
  // factors of column c0 - 2 + lc at [lc * cst], level stride fst, gamma after them (one
  // shared set on a uniform level: cst = 0, level stride 1)
  const bool uni = L.fstride == 0;
  const int cst = uni ? 0 : 1, fst = uni ? 1 : LW;
  const S* cfac = rc ? rc + 4 * LW : sfac;
  const S* cgam = cfac + 3 * fst * nl;
  for (int t = cl.rank; t < (nc + TW - 1) / TW; t += cl.G) {
    const int c0 = t * TW, w = min(TW, nc - c0);
    const Stage st{c0 - 2, w + 4, nc, P.periodic};
    // rows of width w + 4 (column c0 - 2 + lc): f, column data, factors lo | pc | inv, gamma
    const int ww = w + 4;
    const int rcd = nl, rfac = nl + 4, rgam = rfac + 3 * nl;
    const int fsm = L.fstride ? L.fstride : 1;
    // f: each thread owns one column of the rows it stages (wrap and halo worked out once)
    {
      const int RP = BLOCK / ww;
      const int lc = threadIdx.x % ww, r0 = threadIdx.x / ww;
      if (r0 < RP) {
        const int c = c0 - 2 + lc;
        const bool has = st.has(c);
        const int cg = has ? st.col(c) : 0;
        constexpr int U = 8;
        for (int rb = r0; rb < nl; rb += U * RP) {
          S v[U];
#pragma unroll
          for (int q = 0; q < U; ++q) {
            const int r = rb + q * RP;
            v[q] = (r < nl && has) ? f[(size_t)r * nc + cg] : S(0);
          }
#pragma unroll
          for (int q = 0; q < U; ++q) {
            const int r = rb + q * RP;
            if (r < nl) { sf[r * LW + lc] = v[q]; su[r * LW + lc] = v[q]; }
          }
        }
      }
    }
    // column data, factors lo | pc | inv and gamma (unless resident; a uniform level's one
    // set: one value per thread, in the same batch)
    if (!rc) {
      const int nf = uni ? 3 * nl + 1 : 0;
      const S fv = (int)threadIdx.x < nf ? uniform_factor(L, nl, threadIdx.x) : S(0);
      staged_rows<16>((uni ? rfac : rgam + 1) - rcd, ww, [&](int rr, int lc) -> S {
        const int r = rr + rcd;
        const int c = c0 - 2 + lc;
        if (!st.has(c)) return (r < rfac) || (r >= rfac + 2 * nl && r < rgam) ? S(1) : S(0);
        const int cg = st.col(c);
        if (r < rfac) return coldata(L, r - rcd, cg);
        if (r < rgam) return L.flo[(r - rfac) * fsm + (L.fstride ? cg : 0)];
        return L.fgam[L.fstride ? cg : 0];
      }, [&](int rr, int lc, S v) {
        const int r = rr + rcd;
        if (r < rfac) scd[(r - rcd) * LW + lc] = v;
        else if (r < rgam) sfac[(r - rfac) * LW + lc] = v;
        else sgam[lc] = v;
      });
      if ((int)threadIdx.x < nf) sfac[threadIdx.x] = fv;
    }
    __syncthreads();
    if (threadIdx.x < w + 4 && st.has(c0 - 2 + (int)threadIdx.x)) {
      const int lc = threadIdx.x, lf = lc * cst;
      line_solve<S>(nz, cgam[lf], su + lc, LW, cfac + lf, cfac + fst * nl + lf, cfac + 2 * fst * nl + lf, fst);
    }
    __syncthreads();
    const S om = S(P.omega);
    for (int i = threadIdx.x; i < ww * nl; i += BLOCK) {
      const int j = i / ww, lc = i - j * ww;
      su[j * LW + lc] *= om;
    }
    __syncthreads();
    for_rows(nl, w, [&](int j, int lc) { u[(size_t)j * nc + c0 + lc] = su[j * LW + lc + 2]; });
    auto U = [&](int cc, int jj) { return su[jj * LW + st.slot(cc)]; };
    auto F = [&](int cc, int jj) { return sf[jj * LW + st.slot(cc)]; };
    auto CD = [&](int cc, int q) { return ccd[q * LW + st.slot(cc)]; };
    int Cfirst, Clast;
    coarse_range(P, c0, w, nc, ncc, Cfirst, Clast);
    const int ncw = Clast - Cfirst + 1;
    // the residual f - M u, once per fine node, on the columns the restriction reads
    // ([c0 - 1, c0 + w]), in place of f; then the full weighting from it
    for_rows(nl, w + 2, [&](int j, int k) {
      const int cc = c0 - 1 + k;
      if (!st.has(cc)) return;
      const S oms = S(1.0 - P.sig[j]);
      sf[j * LW + st.slot(cc)] = F(cc, j) - m_apply<S>(P, nc, L.rdx, L.rds, oms, cc, j, U, CD);
    });
    __syncthreads();
    if (ncw > 0)
      for_rows(nl, ncw, [&](int j, int k) {
        auto Rr = [&](int cc) { return F(cc, j); };
        fc[(size_t)j * ncc + Cfirst + k] = restrict_at<S>(P, Cfirst + k, ncc, nxc, nc, Rr);
      });
    __syncthreads();
  }
}

// The line-solve constants (column data, factors, gamma) of this workgroup's tile of level l
// (tile = rank), in the layout of the down pass's staging (a uniform level: the column data
// rows, then its one set of factors and gamma), into dst: kept in LDS through a whole solve
// where the level has at most one tile per workgroup.
template <class S, int TW>
DEV void stage_resident(const Problem& P, const Cl& cl, int l, S* dst) {
  const Lv<S> L = level_view<S>(P, l);
  const int nc = L.nc, nl = P.nl;
  constexpr int LW = TW + 4;
  if (cl.rank >= (nc + TW - 1) / TW) return;
  const int c0 = cl.rank * TW, w = min(TW, nc - c0);
  const Stage st{c0 - 2, w + 4, nc, P.periodic};
  const int fsm = L.fstride ? L.fstride : 1;
  // a uniform level: column data over the window, then its one set of factors and gamma
  const int nf = L.fstride == 0 ? 3 * nl + 1 : 0;
  const S fv = (int)threadIdx.x < nf ? uniform_factor(L, nl, threadIdx.x) : S(0);
  staged_rows<16>(nf ? 4 : 5 + 3 * nl, w + 4, [&](int r, int lc) -> S {
    const int c = c0 - 2 + lc;
    // outside the grid: column data and inverse pivots 1, the rest 0 (as the down pass)
    if (!st.has(c)) return (r < 4 || (r >= 4 + 2 * nl && r < 4 + 3 * nl)) ? S(1) : S(0);
    const int cg = st.col(c);
    if (r < 4) return coldata(L, r, cg);
    if (r < 4 + 3 * nl) return L.flo[(r - 4) * fsm + (L.fstride ? cg : 0)];
    return L.fgam[L.fstride ? cg : 0];
  }, [&](int r, int lc, S v) { dst[r * LW + lc] = v; });
  if ((int)threadIdx.x < nf) dst[4 * LW + threadIdx.x] = fv;
}

// fc = full weighting of f - M u (used when nu1 != 1)
template <class S>
DEV void phase_restrict(const Problem& P, Cl& cl, int l, const S* f, const S* u, S* fc, S* lds) {
  const Lv<S> L = level_view<S>(P, l);
  const int nc = L.nc, nl = P.nl;
  const int ncc = P.lev[l + 1].ncol, nxc = P.lev[l + 1].nx;
  constexpr int LW = TM + 4;
  S* sf = lds;
  S* su = sf + LW * nl;
  S* scd = su + LW * nl;
  for (int t = cl.rank; t < ptiles(nc); t += cl.G) {
    const int c0 = t * TM, w = min(TM, nc - c0);
    const Stage st{c0 - 2, w + 4, nc, P.periodic};
    const int cnt[3] = {LW * nl, LW * nl, 4 * LW};
    staged_segments<8>(cnt, [&](int q, int k) -> S {
      if (q == 2) {
        const int qq = k / LW, lc = k - qq * LW;
        const int c = c0 - 2 + lc;
        return st.has(c) ? coldata(L, qq, st.col(c)) : S(1);
      }
      const int j = k / LW, lc = k - j * LW;
      const int c = c0 - 2 + lc;
      const S* src = q == 0 ? f : u;
      return (lc < w + 4 && st.has(c)) ? src[(size_t)j * nc + st.col(c)] : S(0);
    }, [&](int q, int k, S v) { (q == 0 ? sf : (q == 1 ? su : scd))[k] = v; });
    __syncthreads();
    auto U = [&](int cc, int jj) { return su[jj * LW + st.slot(cc)]; };
    auto F = [&](int cc, int jj) { return sf[jj * LW + st.slot(cc)]; };
    auto CD = [&](int cc, int q) { return scd[q * LW + st.slot(cc)]; };
    int Cfirst, Clast;
    coarse_range(P, c0, w, nc, ncc, Cfirst, Clast);
    const int ncw = Clast - Cfirst + 1;
    for (int i = threadIdx.x; i < ncw * nl; i += BLOCK) {
      const int j = i / ncw, C = Cfirst + i - j * ncw;
      const S oms = S(1.0 - P.sig[j]);
      auto Rr = [&](int cc) { return F(cc, j) - m_apply<S>(P, nc, L.rdx, L.rds, oms, cc, j, U, CD); };
      fc[(size_t)j * ncc + C] = restrict_at<S>(P, C, ncc, nxc, nc, Rr);
    }
    __syncthreads();
  }
}

// u += P e on level l
template <class S>
DEV void phase_prolong(const Problem& P, Cl& cl, int l, const S* e, S* u) {
  const int nc = P.lev[l].ncol, ncc = P.lev[l + 1].ncol;
  const int total = nc * P.nl;
  for (int i = cl.rank * BLOCK + threadIdx.x; i < total; i += cl.G * BLOCK) {
    const int j = i / nc, c = i - j * nc;
    u[i] += prolong_at(P, nc, ncc, e, c, j);
  }
}

// o = M_c^-1 f on the coarsest grid with the stored (transposed) inverse. Each workgroup of
// the cluster takes a contiguous slice of R rows; when R < BLOCK the slice's dot products are
// split over Q = BLOCK / R threads per row (thread (q, r) takes j = q, q + Q, ...; consecutive
// threads read consecutive rows of one column, coalesced), eight loads in flight per thread,
// and the Q partial sums are added in LDS in a fixed order. f is staged in LDS first.
template <class S>
DEV void phase_coarse(const Problem& P, Cl& cl, const S* f, S* o, S* lds) {
  const int cn = P.cn;
  const S* ci = coarse_inverse<S>(P);
  S* sf = lds;             // cn
  S* part = lds + cn;      // BLOCK partial sums
  for (int j = threadIdx.x; j < cn; j += BLOCK) sf[j] = f[j];
  __syncthreads();
  const int R = (cn + cl.G - 1) / cl.G;
  const int r0 = cl.rank * R;
  const int r1 = min(cn, r0 + R);
  if (r0 >= r1) return;
  const int rows = r1 - r0;
  if (P.cinv_rows) {
    // the inverse row by row (at most CN_ROWS rows here): the workgroup streams its rows in
    // groups of RB, every thread adding the entries j = t, t + BLOCK, ... of each row, then a
    // fixed-order reduction over the waves
    constexpr int RB = 8;
    for (int rb = 0; rb < rows; rb += RB) {
      const int nr = min(RB, rows - rb);
      S acc[RB];
#pragma unroll
      for (int u = 0; u < RB; ++u) acc[u] = S(0);
      for (int j = threadIdx.x; j < cn; j += BLOCK) {
        const S x = sf[j];
#pragma unroll
        for (int u = 0; u < RB; ++u)
          if (u < nr) acc[u] += ci[(size_t)(r0 + rb + u) * cn + j] * x;
      }
      const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        S v = acc[u];
#pragma unroll
        for (int o2 = 32; o2 > 0; o2 >>= 1) v += __shfl_xor(v, o2, 64);
        if (lane == 0) part[wave * RB + u] = v;
      }
      __syncthreads();
      if (threadIdx.x < nr) {
        S sum = S(0);
        for (int wv = 0; wv < NWAVE; ++wv) sum += part[wv * RB + threadIdx.x];
        o[r0 + rb + threadIdx.x] = sum;
      }
      __syncthreads();
    }
    return;
  }
  const int Q = rows < BLOCK ? BLOCK / rows : 1;
  const int t = threadIdx.x;
  const int q = t / rows, rl = t - q * rows;
  for (int rb = 0; rb < rows; rb += BLOCK) {  // one pass unless the slice exceeds BLOCK rows
    const int r = Q > 1 ? rl : rb + t;
    const bool active = Q > 1 ? q < Q : r < rows;
    S acc = S(0);
    if (active) {
      const size_t i = (size_t)(r0 + r);
      S a[8];
      int j = q;
      for (; j + 7 * Q < cn; j += 8 * Q) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = ci[(size_t)(j + u * Q) * cn + i];
        S s0 = S(0), s1 = S(0);
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
          s0 += a[u] * sf[j + u * Q];
          s1 += a[u + 1] * sf[j + (u + 1) * Q];
        }
        acc += s0 + s1;
      }
      for (; j < cn; j += Q) acc += ci[(size_t)j * cn + i] * sf[j];
    }
    if (Q == 1) {
      if (active) o[r0 + r] = acc;
      continue;
    }
    part[t] = active ? acc : S(0);
    __syncthreads();
    if (t < rows) {
      S sum = S(0);
      for (int qq = 0; qq < Q; ++qq) sum += part[qq * rows + t];
      o[r0 + t] = sum;
    }
    __syncthreads();
  }
}

template <class S>
DEV void phase_zero(const Problem& P, Cl& cl, S* v, int len) {
  for (int i = cl.rank * BLOCK + threadIdx.x; i < len; i += cl.G * BLOCK) v[i] = S(0);
}

template <class S, class D>
DEV void phase_copy(const Problem& P, Cl& cl, const S* src, D* dst, int len) {
  for (int i = cl.rank * BLOCK + threadIdx.x; i < len; i += cl.G * BLOCK) dst[i] = D(src[i]);
}

// per-phase wall-clock accounting (rank-0 workgroup, thread 0), enabled with a profile buffer:
// each tick adds the time since the previous one to its category in the buffer directly, so
// that no per-category state stays live through the solve
struct PhaseClock {
  unsigned long long* out;     // NPHASE totals, then the detail counters; nullptr: off
  unsigned long long last, start;
  DEV void begin(bool enable, int rank, unsigned long long* buf = nullptr) {
    out = (enable && rank == 0 && threadIdx.x == 0) ? buf : nullptr;
    last = start = out ? wall_clock64() : 0;
  }
  DEV void tick(int cat) {
    if (!out) return;
    const unsigned long long now = wall_clock64();
    atomicAdd(out + cat, now - last);
    last = now;
  }
  // detailed tick: charged to the detail slot and to the preconditioner total
  DEV void dtick(int slot) {
    if (!out) return;
    const unsigned long long now = wall_clock64();
    atomicAdd(out + PH_MG + slot, now - last);
    atomicAdd(out + PH_PREC, now - last);
    last = now;
  }
  DEV void flush(unsigned long long*) {
    if (!out) return;
    atomicAdd(out + PH_TOTAL, wall_clock64() - start);
  }
};

// tiles of level l at its V-cycle tile width: the workgroups of rank < this have work there
DEV int level_tiles(const Problem& P, int l) {
  const int tw = P.lev[l].tm;
  return (P.lev[l].ncol + tw - 1) / tw;
}

// Workgroups that take part in the sub-cluster barriers of cluster level l (levels < lt):
// the most tiles any cluster level from l on has, so that the participants never grow on the
// way down (a workgroup that skips a level's barrier has no tile on any coarser level) and
// every pass's producers and consumers are inside the barriers around it.
DEV int sub_parts(const Problem& P, int l, int lt) {
  int q = 0;
  for (int i = l; i < lt; ++i) q = max(q, level_tiles(P, i));
  return q;
}

// one V-cycle level pair on the way down / up (cluster or single-workgroup view). parts > 0:
// the next pass reads only what the workgroups of rank < parts wrote, so the barrier after
// the down pass spans those workgroups only (on level l's word).
template <class S>
DEV void mg_down(const Problem& P, Cl& cl, int l, const S* v, S* lds, const S* rc = nullptr, int parts = 0) {
  const Lv<S> L = level_view<S>(P, l);
  const Lv<S> Lc = level_view<S>(P, l + 1);
  const S* f = l == 0 ? v : L.f;
  S* A = L.u;
  S* B = L.o;
  if (P.nu1 == 1) {
    if (P.lev[l].tm == 32) phase_down<S, 32>(P, cl, l, f, A, Lc.f, lds, rc);
    else phase_down<S, TM>(P, cl, l, f, A, Lc.f, lds, rc);
    if (parts > 0) lsync(cl, parts, l);
    else csync(cl);
    return;
  }
  const S* prev = nullptr;
  S* dst = A;
  if (P.nu1 == 0) {
    phase_zero<S>(P, cl, A, L.nc * P.nl);
    csync(cl);
  }
  for (int s = 0; s < P.nu1; ++s) {
    dst = (prev == A) ? B : A;
    phase_sweep<S>(P, cl, l, f, prev, nullptr, dst, lds);
    csync(cl);
    prev = dst;
  }
  if (dst != A) {
    phase_copy(P, cl, (const S*)dst, A, L.nc * P.nl);
    csync(cl);
  }
  phase_restrict<S>(P, cl, l, f, A, Lc.f, lds);
  csync(cl);
}

// the buffer that holds level l's output after its up pass (l > 0): the post-sweeps alternate
// between the level's two work vectors, starting from u, so an odd count ends in o
template <class S>
DEV const S* level_output(const Problem& P, int l) {
  const Lv<S> L = level_view<S>(P, l);
  return (P.nu2 % 2 == 1) ? (const S*)L.o : (const S*)L.u;
}

// returns the buffer holding level l's output; z is level 0's destination. Post-sweeps never
// run in place (a sweep reads one halo column of its neighbour tiles, which other workgroups
// write in the same phase): they alternate between the level's two work vectors, the first
// adding the prolongated coarse correction on load, and at level 0 the last one writes z.
template <class S>
DEV const S* mg_up(const Problem& P, Cl& cl, int l, const S* v, const S* e, S* z, S* lds,
                   const S* rc = nullptr, int parts = 0, int parts_up = 0) {
  const Lv<S> L = level_view<S>(P, l);
  const S* f = l == 0 ? v : L.f;
  S* A = L.u;
  S* B = L.o;
  if (P.nu2 == 0) {
    phase_prolong<S>(P, cl, l, e, A);
    csync(cl);
    if (l == 0) {
      phase_copy(P, cl, (const S*)A, z, P.n);
      csync(cl);
      return z;
    }
    return A;
  }
  const S* prev = A;
  const S* corr = e;
  int s0 = 0;
  // the first two post-sweeps in one pass on the cluster levels of a periodic problem whose
  // columns share one set of factors (the output leaves A, which its neighbours still read)
  if (P.nu2 >= 2 && P.periodic && L.fstride == 0 && parts >= 0 && cl.G > 1) {
    S* nd = (l == 0 && P.nu2 == 2) ? z : B;
    if (P.lev[l].tm == 32) phase_sweep2<S, 32>(P, cl, l, f, prev, corr, nd, lds, rc);
    else phase_sweep2<S, TM>(P, cl, l, f, prev, corr, nd, lds, rc);
    if (parts <= 0 || l == 0) csync(cl);
    else if (P.nu2 > 2) lsync(cl, parts, l);
    else lsync(cl, parts_up, l - 1);
    prev = nd;
    corr = nullptr;
    s0 = 2;
  }
  for (int s = s0; s < P.nu2; ++s) {
    S* nd = (l == 0 && s == P.nu2 - 1) ? z : (prev == B ? A : B);
    if (P.lev[l].tm == 32) phase_sweep<S, 32>(P, cl, l, f, prev, corr, nd, lds, rc);
    else phase_sweep<S, TM>(P, cl, l, f, prev, corr, nd, lds, rc);
    // the next pass: this level's next sweep (parts, level l's word), else the up pass of
    // level l - 1 (parts_up >= parts, level l - 1's word), else (level 0) the whole cluster
    if (parts <= 0 || l == 0) csync(cl);
    else if (s < P.nu2 - 1) lsync(cl, parts, l);
    else lsync(cl, parts_up, l - 1);
    prev = nd;
    corr = nullptr;
  }
  return prev;
}

// z = U^-1 L^-1 v of the ILU(0) factors by level-scheduled substitution, on the rank-0
// workgroup. A substitution is a sequence of steps of 16 independent rows (a level of the
// schedule, or part of one); wave w takes slots w and w + 8 of a step, its lanes the row's
// entries (one record of 64), and a wave reduction in a fixed order gives the row's sum.
// Workgroup barriers separate the steps. A step's own work is short against a load's latency,
// so each wave keeps the records of its two slots of the next three steps in registers, loaded
// three steps before they are used; every address follows from the step number, and only the
// reads of z wait on the step before. Arithmetic in FP64 whatever S is.

template <class S>
DEV void ilu_sweep(int nstep, const int SA_GLOBAL* row, const int SA_GLOBAL* col, const double SA_GLOBAL* val,
                   const double SA_GLOBAL* dinv, const S* v, S* z, double* zl) {
  // zl: z in LDS (all n values), else z in global memory
  auto zget = [&](int c) { return zl ? zl[c] : (double)z[c]; };
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  struct Rec { int r, c; double a, g; };  // row, this lane's column and value, the row's 1/u_ii
  auto fetch = [&](int t, int k) {
    Rec q{-1, -1, 0.0, 0.0};
    if (t < nstep) {
      const long s = (long)t * (2 * NWAVE) + wave + k * NWAVE;
      q.r = row[s];
      q.c = col[s * 64 + lane];
      q.a = val[s * 64 + lane];
      if (dinv) q.g = dinv[s];
    }
    return q;
  };
  // forward: z_r = v_r - sum (v already copied into zl when z lives in LDS); backward:
  // z_r = (z_r - sum) / u_rr
  auto store = [&](const Rec& q, double sum) {
    const double base = (dinv || zl) ? zget(q.r) : (double)v[q.r];
    const double zr = dinv ? (base - sum) * q.g : base - sum;
    if (zl) zl[q.r] = zr; else z[q.r] = (S)zr;
  };
  // the two rows of a step: both sums reduced side by side (one latency chain, not two);
  // padding slots (row -1) are uniform over the wave and contribute zeros
  auto finish2 = [&](const Rec& q0, const Rec& q1) {
    double s0 = (q0.r >= 0 && q0.c >= 0) ? q0.a * zget(q0.c) : 0.0;
    double s1 = (q1.r >= 0 && q1.c >= 0) ? q1.a * zget(q1.c) : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      s0 += __shfl_xor(s0, o, 64);
      s1 += __shfl_xor(s1, o, 64);
    }
    if (lane == 0) {
      if (q0.r >= 0) store(q0, s0);
      if (q1.r >= 0) store(q1, s1);
    }
  };
  // three register sets, step t in set t mod 3, refilled (by loads, never by copies: a copy
  // would wait for the load) with step t + 3 right after step t is done
  Rec a0 = fetch(0, 0), a1 = fetch(0, 1), b0 = fetch(1, 0), b1 = fetch(1, 1), c0 = fetch(2, 0), c1 = fetch(2, 1);
  for (int t = 0; t < nstep; t += 3) {
    finish2(a0, a1);
    a0 = fetch(t + 3, 0);
    a1 = fetch(t + 3, 1);
    __syncthreads();
    if (t + 1 < nstep) {
      finish2(b0, b1);
      b0 = fetch(t + 4, 0);
      b1 = fetch(t + 4, 1);
      __syncthreads();
    }
    if (t + 2 < nstep) {
      finish2(c0, c1);
      c0 = fetch(t + 5, 0);
      c1 = fetch(t + 5, 1);
      __syncthreads();
    }
  }
}

// lds: the phase scratch, at least n doubles when P.ilu_lds (z is then formed there and copied
// out at the end). Not inlined: the solve kernels' register allocation for the V-cycle path
// stays as without it.
template <class S>
__device__ __attribute__((noinline)) void ilu_apply(const Problem& P, Cl& cl, const S* v, S* z, S* lds) {
  if (cl.rank != 0) return;
  double* zl = P.ilu_lds ? reinterpret_cast<double*>(lds) : nullptr;
  if (zl) {
    for (int i = threadIdx.x; i < P.n; i += BLOCK) zl[i] = (double)v[i];
    __syncthreads();
  }
  ilu_sweep<S>(P.ilu_nf, P.ilu_frow, P.ilu_fcol, P.ilu_fval, nullptr, v, z, zl);
  ilu_sweep<S>(P.ilu_nb, P.ilu_brow, P.ilu_bcol, P.ilu_bval, P.ilu_dinv, v, z, zl);
  if (zl)
    for (int i = threadIdx.x; i < P.n; i += BLOCK) z[i] = (S)zl[i];
}

// z = M^-1 v in precision S. v and z are level-0 vectors distinct from each other and from
// the level-0 scratch (u, o of level 0). Levels from P.tail on (at most one tile wide) are
// run by the rank-0 workgroup alone with workgroup barriers only. Ends with a cluster barrier.
template <class S>
DEV void precond(const Problem& P, Cl& cl, const S* v, S* z, S* lds, PhaseClock* ck = nullptr,
                 const S* res = nullptr) {
  const int n = P.n;
  if (P.pc == SA_PC_NONE) {
    phase_copy(P, cl, v, z, n);
    csync(cl);
    return;
  }
  if (P.pc == SA_PC_ILU0) {
    ilu_apply<S>(P, cl, v, z, lds);
    csync(cl);
    return;
  }
  const Lv<S> L0 = level_view<S>(P, 0);
  S* A0 = L0.u;
  S* B0 = L0.o;
  if (P.pc == SA_PC_LINE) {  // nu1 sweeps from zero, the last one writes z
    const S* prev = nullptr;
    for (int s = 0; s < P.nu1; ++s) {
      S* dst = (s == P.nu1 - 1) ? z : ((prev == A0) ? B0 : A0);
      phase_sweep<S>(P, cl, 0, v, prev, nullptr, dst, lds);
      csync(cl);
      prev = dst;
    }
    return;
  }
  const int L = P.nlev;
  if (L == 1) {
    phase_coarse<S>(P, cl, v, z, lds);
    csync(cl);
    return;
  }
  // levels [lt, L-1) are one tile wide: the rank-0 workgroup runs their passes alone
  // (workgroup barriers only); the coarsest dense solve is shared by the whole cluster
  const int lt = (cl.G > 1 && P.tail < L - 1) ? P.tail : L - 1;
  auto tk = [&](int slot) { if (ck) ck->dtick(slot); };
  // the resident constants of cluster level l (res: the solve's resident block, or none)
  auto rc = [&](int l) -> const S* { return (res && P.lev[l].res >= 0) ? res + P.lev[l].res : nullptr; };
  // sub-cluster barriers between the passes of the cluster levels; the last cluster level
  // before the coarsest solve (no single-workgroup levels between) ends with a cluster barrier
  for (int l = 0; l < lt; ++l) {
    mg_down<S>(P, cl, l, v, lds, rc(l), (l + 1 < lt || lt < L - 1) ? sub_parts(P, l, lt) : 0);
    tk(1 + 2 * l);
  }
  Cl solo{0, 1, cl.bar, cl.flags, cl.partials, cl.pbuf, 0u, nullptr, nullptr};
  if (lt < L - 1) {
    if (cl.rank == 0)
      for (int l = lt; l < L - 1; ++l) { mg_down<S>(P, solo, l, v, lds); tk(1 + 2 * l); }
    csync(cl);
    tk(2 * MAXLEV);
  }
  const Lv<S> Lc = level_view<S>(P, L - 1);
  phase_coarse<S>(P, cl, Lc.f, Lc.o, lds);
  csync(cl);
  tk(0);
  const S* e = Lc.o;
  if (lt < L - 1) {
    if (cl.rank == 0)
      for (int l = L - 2; l >= lt; --l) { e = mg_up<S>(P, solo, l, v, e, z, lds); tk(2 + 2 * l); }
    csync(cl);
    tk(2 * MAXLEV);
    // every workgroup knows which buffer holds the tail's output
    e = (lt == 0) ? z : level_output<S>(P, lt);
    if (lt == 0) return;
  }
  for (int l = lt - 1; l >= 0; --l) {
    e = mg_up<S>(P, cl, l, v, e, z, lds, rc(l), sub_parts(P, l, lt), l > 0 ? sub_parts(P, l - 1, lt) : 0);
    tk(2 + 2 * l);
  }
}

// ------------------------------------------------------------------------------------------
// Arnoldi pieces. V holds raw (unnormalised) basis vectors; vs[i] scales V_i to unit norm.

// Per-wave partial dot products of w with the vectors V_0..V_{nv-1} (and with itself when
// with_norm) over this workgroup's elements, into wsum[i * NWAVE + wave]. Vectors go in groups
// of four and every thread takes two of its elements per step, so ten loads are in flight per
// step; products and sums are FP64, in a fixed order.
template <class S>
DEV void dot_groups(const Problem& P, Cl& cl, const S* V, int nv, const S* w, bool with_norm, double* wsum) {
  const int n = P.n;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int stride = cl.G * BLOCK, e0 = cl.rank * BLOCK + threadIdx.x;
  const int nred = nv + (with_norm ? 1 : 0);
  for (int g0 = 0; g0 < nred; g0 += 4) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int e = e0; e < n; e += 2 * stride) {
      const bool ok2 = e + stride < n;
      const double w0 = w[e], w1 = ok2 ? double(w[e + stride]) : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = g0 + q;
        if (i < nred) {
          const S* a = i < nv ? V + (size_t)i * n : w;
          const double a0 = a[e], a1 = ok2 ? double(a[e + stride]) : 0.0;
          acc[q] += a0 * w0 + a1 * w1;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double sum = wave_sum(acc[q]);
      if (lane == 0 && g0 + q < nred) wsum[(g0 + q) * NWAVE + wave] = sum;
    }
  }
}

// red[i] = vs[i] * (V_i . w), i < nv; red[nv] = ||w||^2 if with_norm. V and w are stored in S.
template <class S>
DEV void phase_dots(const Problem& P, Cl& cl, const S* V, const double* vs, int nv, const S* w,
                    bool with_norm, double* wsum, double* red) {
  const int nred = nv + (with_norm ? 1 : 0);
  dot_groups<S>(P, cl, V, nv, w, with_norm, wsum);
  __syncthreads();
  for (int i = threadIdx.x; i < nred; i += BLOCK) {
    const double sm = waves_sum(wsum + i * NWAVE);
    red[i] = (i < nv) ? vs[i] * sm : sm;
  }
  __syncthreads();
}

// w -= sum_i h[i] vs[i] V_i (in place, this workgroup's elements; groups of four vectors, two
// elements per step); then red[i] = vs[i] (V_i . w) for i < nv when dots, or red[0] = ||w||^2
// when !dots. The dots read back the stored (rounded) w.
template <class S>
DEV void phase_update(const Problem& P, Cl& cl, const S* V, const double* vs, const double* h, int nv,
                      S* w, bool dots, double* wsum, double* red) {
  const int n = P.n;
  const int stride = cl.G * BLOCK, e0 = cl.rank * BLOCK + threadIdx.x;
  double nrm = 0.0;
  for (int e = e0; e < n; e += 2 * stride) {
    const bool ok2 = e + stride < n;
    double w0 = w[e], w1 = ok2 ? double(w[e + stride]) : 0.0;
    for (int i = 0; i < nv; i += 4) {
      double a0[4], a1[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const S* v = V + (size_t)(i + q < nv ? i + q : i) * n;
        a0[q] = v[e];
        a1[q] = ok2 ? double(v[e + stride]) : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (i + q < nv) {
          const double c = h[i + q] * vs[i + q];
          w0 -= a0[q] * c;
          w1 -= a1[q] * c;
        }
      }
    }
    const S s0 = S(w0), s1 = S(w1);
    w[e] = s0;
    if (ok2) w[e + stride] = s1;
    nrm += double(s0) * double(s0) + (ok2 ? double(s1) * double(s1) : 0.0);
  }
  if (dots) {
    dot_groups<S>(P, cl, V, nv, w, false, wsum);
    __syncthreads();
    for (int i = threadIdx.x; i < nv; i += BLOCK) red[i] = vs[i] * waves_sum(wsum + i * NWAVE);
    __syncthreads();
  } else {
    block_sum_to(nrm, wsum, red, 0);
  }
}

// dst = src + sum_i y[i] vs[i] V_i (FP64 result, basis stored in S)
template <class S>
DEV void phase_combine(const Problem& P, Cl& cl, const S* V, const double* vs, const double* y, int nv,
                       const double* src, double* dst) {
  const int n = P.n;
  for (int e = cl.rank * BLOCK + threadIdx.x; e < n; e += cl.G * BLOCK) {
    double v = src[e];
    int i = 0;
    for (; i + 3 < nv; i += 4) {
      const double v0 = V[(size_t)i * n + e], v1 = V[(size_t)(i + 1) * n + e];
      const double v2 = V[(size_t)(i + 2) * n + e], v3 = V[(size_t)(i + 3) * n + e];
      v += v0 * (y[i] * vs[i]) + v1 * (y[i + 1] * vs[i + 1]) + v2 * (y[i + 2] * vs[i + 2]) + v3 * (y[i + 3] * vs[i + 3]);
    }
    for (; i < nv; ++i) v += double(V[(size_t)i * n + e]) * (y[i] * vs[i]);
    dst[e] = v;
  }
}

// ------------------------------------------------------------------------------------------
// sketch guess (Alg. 2 with V = Y of Alg. 4)

// Y_new = r Y_old + x omega^T (all k columns, elementwise)
DEV void phase_push(const Problem& P, Cl& cl, const SolveArgs& a, const double* Yo, double* Yn) {
  const size_t n = P.n;
  for (size_t e = (size_t)cl.rank * BLOCK + threadIdx.x; e < n; e += (size_t)cl.G * BLOCK) {
    const double xe = P.x[e];
    int c = 0;
    for (; c + 3 < P.k; c += 4) {
      const double y0 = Yo[c * n + e], y1 = Yo[(c + 1) * n + e], y2 = Yo[(c + 2) * n + e], y3 = Yo[(c + 3) * n + e];
      Yn[c * n + e] = a.r * y0 + a.om[c] * xe;
      Yn[(c + 1) * n + e] = a.r * y1 + a.om[c + 1] * xe;
      Yn[(c + 2) * n + e] = a.r * y2 + a.om[c + 2] * xe;
      Yn[(c + 3) * n + e] = a.r * y3 + a.om[c + 3] * xe;
    }
    for (; c < P.k; ++c) Yn[c * n + e] = a.r * Yo[c * n + e] + a.om[c] * xe;
  }
}

// Randomized range finder (Alg. 3): the previous solution enters ring slot a.range_slot
// (replacing the oldest one once the window is full) and V = X Omega over the a.window slots
// in use, column c of V = sum_s Omega[s][c] x_s, elementwise (no halo), slots in ring order.
// The rows of Omega of the slots are staged in LDS (lds: KWIN * KMAX doubles); the new slot's
// row comes with the solve's draws a.om and is stored for the later solves by the first
// workgroup (the other workgroups never read that row from memory in this phase).
DEV void phase_range_form(const Problem& P, Cl& cl, const SolveArgs& a, double* V, double* lds) {
  const size_t n = P.n;
  const int k = P.k, win = a.window, slot = a.range_slot;
  for (int i = threadIdx.x; i < win * KMAX; i += BLOCK) {
    const int sl = i / KMAX, c = i - sl * KMAX;
    lds[i] = (sl == slot) ? (c < k ? a.om[c] : 0.0) : P.Om[i];
  }
  __syncthreads();
  if (cl.rank == 0 && slot >= 0)
    for (int c = threadIdx.x; c < KMAX; c += BLOCK) P.Om[(size_t)slot * KMAX + c] = c < k ? a.om[c] : 0.0;
  for (size_t e = (size_t)cl.rank * BLOCK + threadIdx.x; e < n; e += (size_t)cl.G * BLOCK) {
    double acc[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) acc[c] = 0.0;
    for (int sl = 0; sl < win; ++sl) {
      double xs;
      if (sl == slot) {
        xs = P.x[e];
        P.Xr[(size_t)sl * n + e] = xs;
      } else {
        xs = P.Xr[(size_t)sl * n + e];
      }
      const double* om = lds + sl * KMAX;
#pragma unroll
      for (int c = 0; c < KMAX; ++c)
        if (c < k) acc[c] += om[c] * xs;
    }
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      if (c < k) V[(size_t)c * n + e] = acc[c];
  }
}

// ---- double-double helpers (error-free transformations, Dekker / Knuth / Bailey) -------
struct dd {
  double hi, lo;
};

DEV dd two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  return dd{s, (a - (s - bb)) + (b - bb)};
}

DEV dd quick_two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  return dd{s, b - (s - a)};
}

DEV dd two_prod(double a, double b) {
  const double p = a * b;
  return dd{p, fma(a, b, -p)};
}

DEV dd dd_add(dd a, dd b) {
#pragma clang fp contract(off)
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}

DEV dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }
DEV dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

DEV dd dd_mul(dd a, dd b) {
#pragma clang fp contract(off)
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return quick_two_sum(p.hi, p.lo);
}

DEV dd dd_mul_d(dd a, double b) {
#pragma clang fp contract(off)
  dd p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return quick_two_sum(p.hi, p.lo);
}

DEV dd dd_div(dd a, dd b) {
  const double q1 = a.hi / b.hi;
  dd r = dd_sub(a, dd_mul_d(b, q1));
  const double q2 = r.hi / b.hi;
  r = dd_sub(r, dd_mul_d(b, q2));
  const double q3 = r.hi / b.hi;
  dd q = quick_two_sum(q1, q2);
  return dd_add(q, dd{q3, 0.0});
}

DEV dd dd_sqrt(dd a) {
  if (!(a.hi > 0.0)) return dd{0.0, 0.0};
  const double x = sqrt(a.hi);
  const dd r = dd_sub(a, two_prod(x, x));
  return quick_two_sum(x, r.hi / (2.0 * x));
}

// For every tile: Y_new (fused push), W_a = A Y_new_a into LDS, then the products
// G_ab = W_a . W_b (a <= b) and c_a = W_a . b. Products are exact (FMA TwoProduct) and
// sums compensated (TwoSum), so the Gram carries the accuracy a QR of W would: its
// condition number is the square of W's, and the sketch's columns are nearly dependent.
// Output: red[2 i], red[2 i + 1] = hi, lo of item i (pairs in row order, then c).
template <int TG>
DEV void phase_block_gram(const Problem& P, Cl& cl, const SolveArgs& a, const double* Yo, double* Yn,
                          double* lds, double* red) {
  const int nc = P.ncol, nl = P.nl, k = P.k;
  const size_t n = P.n;
  const Tiles T = tiles_of(P, TG);
  constexpr int W = TG + 3;  // widest tile (a last wall tile absorbs up to 3 columns)
  double* sW = lds;                         // k x W x nl
  double* sb = sW + (size_t)k * W * nl;     // W x nl
  double* sx = sb + W * nl;                 // (W+12) x nl
  double* sgx = sx + (W + 12) * nl;         // (W+6) x nl
  double* sgz = sgx + (W + 6) * nl;         // (W+6) x nl
  double* sc = sgz + (W + 6) * nl;          // coefficient block
  const int npair = k * (k + 1) / 2;
  const int nitem = npair + k;
  const int Q = BLOCK / nitem > 0 ? BLOCK / nitem : 1;  // threads per item
  const int item = threadIdx.x % nitem, qq = threadIdx.x / nitem;
  const bool active = qq < Q;
  int pa = 0, pb = -1;
  if (item < npair) {
    int t = item, rowlen = k;
    while (t >= rowlen) { t -= rowlen; ++pa; --rowlen; }
    pb = pa + t;
  } else {
    pa = item - npair;
  }
  double accS = 0.0, accC = 0.0;
  for (int t = cl.rank; t < T.nt; t += cl.G) {
    const int c0 = t * TG;
    const int w = (t == T.nt - 1) ? nc - c0 : TG;
    for (int i = threadIdx.x; i < W * nl; i += BLOCK) {
      const int lj = i / W, lc = i - lj * W;
      sb[i] = (lc < w) ? a.b[(size_t)lj * nc + c0 + lc] : 0.0;
    }
    for (int col = 0; col < k; ++col) {
      const double* yo = Yo + (size_t)col * n;
      double* yn = Yn + (size_t)col * n;
      const double om = a.om[col];
      // Y_new = r Y_old + omega x, recomputed on the halo (no race with other tiles); the
      // tile's own columns are written back
      auto load = [&](int lj, int c, int lc) {
        const size_t e = (size_t)lj * nc + c;
        if (!a.push) return yo[e];
        const double v = a.r * yo[e] + om * P.x[e];
        if (lc >= 6 && lc < w + 6) yn[e] = v;
        return v;
      };
      double* wcol = sW + (size_t)col * W * nl;
      tile_operator<double, W>(P, c0, w, load, sx, sgx, sgz, sc, [&](int lj, int lc, int, double v) {
        wcol[lj * W + lc] = v;
      }, col == 0);
    }
    // zero the unused tile columns so that the products can run over the full W x nl
    for (int i = threadIdx.x; i < k * W * nl; i += BLOCK) {
      const int lc = i % W;
      if (lc >= w) sW[i] = 0.0;
    }
    __syncthreads();
    if (active) {
      const double* wa = sW + (size_t)pa * W * nl;
      const double* wb = (pb >= 0) ? sW + (size_t)pb * W * nl : sb;
      for (int p = qq; p < W * nl; p += Q) {
        const dd pr = two_prod(wa[p], wb[p]);
        const dd s = two_sum(accS, pr.hi);
        accS = s.hi;
        accC += s.lo + pr.lo;
      }
    }
    __syncthreads();
  }
  // combine the Q partials of each item in a fixed order
  double* sS = lds;
  double* sC = lds + BLOCK;
  sS[threadIdx.x] = active ? accS : 0.0;
  sC[threadIdx.x] = active ? accC : 0.0;
  __syncthreads();
  if (threadIdx.x < nitem) {
    dd acc{0.0, 0.0};
    for (int q = 0; q < Q; ++q) acc = dd_add(acc, quick_two_sum(sS[q * nitem + threadIdx.x], sC[q * nitem + threadIdx.x]));
    red[2 * threadIdx.x] = acc.hi;
    red[2 * threadIdx.x + 1] = acc.lo;
  }
  __syncthreads();
}

// red holds nv double-double values (hi, lo interleaved) of this workgroup; afterwards the
// cluster sums, added in rank order with double-double arithmetic.
DEV void cluster_sum_dd(Cl& cl, double* red, int nv) {
  __syncthreads();
  if (cl.G == 1) return;
  double* part = cl.partials + (size_t)cl.pbuf * (cl.G + 1) * PSTRIDE;
  for (int i = threadIdx.x; i < 2 * nv; i += BLOCK) part[cl.rank * PSTRIDE + i] = red[i];
  cl.pbuf ^= 1;
  csync(cl);
  for (int i = threadIdx.x; i < nv; i += BLOCK) {
    dd s{0.0, 0.0};
    for (int g = 0; g < cl.G; ++g) s = dd_add(s, dd{part[g * PSTRIDE + 2 * i], part[g * PSTRIDE + 2 * i + 1]});
    red[2 * i] = s.hi;
    red[2 * i + 1] = s.lo;
  }
  __syncthreads();
}

// k x k least squares from the Gram: column scaling D = diag(G_aa)^-1/2, right-looking
// double-double Cholesky of D G D taking columns in order and dropping a column whose pivot
// falls below tau^2 (the projected norm of the unit column below tau, as in a QR with the
// same drop rule), then z = D (L L^T)^-1 D c over the kept columns. The whole workgroup
// runs it on identical inputs in every workgroup of the cluster. Returns the rank.
DEV int small_solve(const Problem& P, const double* red, double tau, double* z, double* scr) {
  const int k = P.k, tid = threadIdx.x;
  double* gh = scr;               // k x k hi (lower part becomes L)
  double* gl = gh + k * k;        // k x k lo
  double* dsc = gl + k * k;       // k
  double* vh = dsc + k;           // k rhs / solution hi
  double* vl = vh + k;            // k lo
  int* kept = (int*)(vl + k);     // k
  auto item = [&](int i, int j) {
    const int a = i < j ? i : j, b = i < j ? j : i;
    return a * k - a * (a - 1) / 2 + (b - a);
  };
  const int npair = k * (k + 1) / 2;
  if (tid < k) {
    const double gii = red[2 * item(tid, tid)];
    dsc[tid] = gii > 0.0 ? 1.0 / sqrt(gii) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += BLOCK) {
    const int i = e / k, j = e - i * k;
    const int it = item(i, j);
    const dd g = dd_mul_d(dd_mul_d(dd{red[2 * it], red[2 * it + 1]}, dsc[i]), dsc[j]);
    gh[e] = g.hi;
    gl[e] = g.lo;
  }
  if (tid < k) {
    const dd c = dd_mul_d(dd{red[2 * (npair + tid)], red[2 * (npair + tid) + 1]}, dsc[tid]);
    vh[tid] = c.hi;
    vl[tid] = c.lo;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (tid == 0) {
      const dd d{gh[j * k + j], gl[j * k + j]};
      const bool keep = dsc[j] > 0.0 && d.hi >= tau * tau;
      kept[j] = keep;
      const dd ljj = keep ? dd_sqrt(d) : dd{0.0, 0.0};
      gh[j * k + j] = ljj.hi;
      gl[j * k + j] = ljj.lo;
    }
    __syncthreads();
    if (!kept[j]) continue;
    const dd ljj{gh[j * k + j], gl[j * k + j]};
    if (tid > j && tid < k) {
      const dd lij = dd_div(dd{gh[tid * k + j], gl[tid * k + j]}, ljj);
      gh[tid * k + j] = lij.hi;
      gl[tid * k + j] = lij.lo;
    }
    __syncthreads();
    for (int e = tid; e < k * k; e += BLOCK) {
      const int i = e / k, l = e - i * k;
      if (l > j && i >= l) {
        const dd upd = dd_mul(dd{gh[i * k + j], gl[i * k + j]}, dd{gh[l * k + j], gl[l * k + j]});
        const dd g = dd_sub(dd{gh[e], gl[e]}, upd);
        gh[e] = g.hi;
        gl[e] = g.lo;
      }
    }
    __syncthreads();
  }
  // forward substitution L y = D c, then L^T z = y (kept columns only)
  for (int j = 0; j < k; ++j) {
    if (kept[j]) {
      if (tid == 0) {
        const dd y = dd_div(dd{vh[j], vl[j]}, dd{gh[j * k + j], gl[j * k + j]});
        vh[j] = y.hi;
        vl[j] = y.lo;
      }
      __syncthreads();
      if (tid > j && tid < k && kept[tid]) {
        const dd v = dd_sub(dd{vh[tid], vl[tid]}, dd_mul(dd{gh[tid * k + j], gl[tid * k + j]}, dd{vh[j], vl[j]}));
        vh[tid] = v.hi;
        vl[tid] = v.lo;
      }
    }
    __syncthreads();
  }
  for (int j = k - 1; j >= 0; --j) {
    if (kept[j]) {
      if (tid == 0) {
        const dd y = dd_div(dd{vh[j], vl[j]}, dd{gh[j * k + j], gl[j * k + j]});
        vh[j] = y.hi;
        vl[j] = y.lo;
      }
      __syncthreads();
      if (tid < j && kept[tid]) {
        const dd v = dd_sub(dd{vh[tid], vl[tid]}, dd_mul(dd{gh[j * k + tid], gl[j * k + tid]}, dd{vh[j], vl[j]}));
        vh[tid] = v.hi;
        vl[tid] = v.lo;
      }
    }
    __syncthreads();
  }
  int rank = 0;
  for (int j = 0; j < k; ++j) rank += kept[j];
  if (tid < k) z[tid] = kept[tid] ? (vh[tid] + vl[tid]) * dsc[tid] : 0.0;
  __syncthreads();
  return rank;
}

// Gram V^T V of the range finder's sketch (V = X Omega, k columns of n) for its QR (V = Q):
// chunks of CH elements of the k columns staged in LDS, the products exact and the sums
// compensated as in phase_block_gram, items (pairs in row order) in red as hi, lo.
DEV void phase_sketch_gram(const Problem& P, Cl& cl, const double* V, double* lds, double* red) {
  constexpr int CH = 512;
  const int k = P.k;
  const size_t n = P.n;
  const int npair = k * (k + 1) / 2;
  const int Q = BLOCK / npair > 0 ? BLOCK / npair : 1;  // threads per item
  const int item = threadIdx.x % npair, qq = threadIdx.x / npair;
  const bool active = qq < Q;
  int pa = 0, pb = 0;
  {
    int t = item, rowlen = k;
    while (t >= rowlen) { t -= rowlen; ++pa; --rowlen; }
    pb = pa + t;
  }
  double accS = 0.0, accC = 0.0;
  for (size_t e0 = (size_t)cl.rank * CH; e0 < n; e0 += (size_t)cl.G * CH) {
    const int cnt = (int)min((size_t)CH, n - e0);
    for (int i = threadIdx.x; i < k * CH; i += BLOCK) {
      const int c = i / CH, j = i - c * CH;
      lds[i] = j < cnt ? V[(size_t)c * n + e0 + j] : 0.0;
    }
    __syncthreads();
    if (active) {
      const double* va = lds + pa * CH;
      const double* vb = lds + pb * CH;
      for (int p = qq; p < cnt; p += Q) {
        const dd pr = two_prod(va[p], vb[p]);
        const dd s = two_sum(accS, pr.hi);
        accS = s.hi;
        accC += s.lo + pr.lo;
      }
    }
    __syncthreads();
  }
  double* sS = lds;
  double* sC = lds + BLOCK;
  sS[threadIdx.x] = active ? accS : 0.0;
  sC[threadIdx.x] = active ? accC : 0.0;
  __syncthreads();
  if (threadIdx.x < npair) {
    dd acc{0.0, 0.0};
    for (int q = 0; q < Q; ++q) acc = dd_add(acc, quick_two_sum(sS[q * npair + threadIdx.x], sC[q * npair + threadIdx.x]));
    red[2 * threadIdx.x] = acc.hi;
    red[2 * threadIdx.x + 1] = acc.lo;
  }
  __syncthreads();
}

// The QR of the sketch from its Gram G: column scaling D = diag(G_aa)^-1/2, double-double
// Cholesky L L^T = D G D taking columns in order and dropping a column whose pivot falls below
// tau^2 (its projected unit norm below tau, the least squares' rule), then T = D L^-T over the
// kept columns (zero columns for dropped ones), so that Q = V T has orthonormal columns. T
// column-major (T[i + j k]) in t; every workgroup computes it from identical inputs.
DEV void small_qr_factor(const Problem& P, const double* red, double tau, double* t, double* scr) {
  const int k = P.k, tid = threadIdx.x;
  double* gh = scr;            // k x k hi (lower part becomes L)
  double* gl = gh + k * k;     // k x k lo
  double* dsc = gl + k * k;    // k
  int* kept = (int*)(dsc + k); // k
  auto item = [&](int i, int j) {
    const int a = i < j ? i : j, b = i < j ? j : i;
    return a * k - a * (a - 1) / 2 + (b - a);
  };
  if (tid < k) {
    const double gii = red[2 * item(tid, tid)];
    dsc[tid] = gii > 0.0 ? 1.0 / sqrt(gii) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += BLOCK) {
    const int i = e / k, j = e - i * k;
    const int it = item(i, j);
    const dd g = dd_mul_d(dd_mul_d(dd{red[2 * it], red[2 * it + 1]}, dsc[i]), dsc[j]);
    gh[e] = g.hi;
    gl[e] = g.lo;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (tid == 0) {
      const dd d{gh[j * k + j], gl[j * k + j]};
      const bool keep = dsc[j] > 0.0 && d.hi >= tau * tau;
      kept[j] = keep;
      const dd ljj = keep ? dd_sqrt(d) : dd{0.0, 0.0};
      gh[j * k + j] = ljj.hi;
      gl[j * k + j] = ljj.lo;
    }
    __syncthreads();
    if (!kept[j]) continue;
    const dd ljj{gh[j * k + j], gl[j * k + j]};
    if (tid > j && tid < k) {
      const dd lij = dd_div(dd{gh[tid * k + j], gl[tid * k + j]}, ljj);
      gh[tid * k + j] = lij.hi;
      gl[tid * k + j] = lij.lo;
    }
    __syncthreads();
    for (int e = tid; e < k * k; e += BLOCK) {
      const int i = e / k, l = e - i * k;
      if (l > j && i >= l) {
        const dd upd = dd_mul(dd{gh[i * k + j], gl[i * k + j]}, dd{gh[l * k + j], gl[l * k + j]});
        const dd g = dd_sub(dd{gh[e], gl[e]}, upd);
        gh[e] = g.hi;
        gl[e] = g.lo;
      }
    }
    __syncthreads();
  }
  // column j of L^-T (kept j): solve L^T y = e_j over the kept indices, y_i = 0 for i > j;
  // one thread per column, back substitution from i = j down
  if (tid < k) {
    const int j = tid;
    for (int i = 0; i < k; ++i) t[i + j * k] = 0.0;
    if (kept[j]) {
      dd y[KMAX];
      for (int i = j; i >= 0; --i) {
        if (!kept[i]) { y[i] = dd{0.0, 0.0}; continue; }
        dd r = (i == j) ? dd{1.0, 0.0} : dd{0.0, 0.0};
        for (int m = i + 1; m <= j; ++m)
          if (kept[m]) r = dd_sub(r, dd_mul(dd{gh[m * k + i], gl[m * k + i]}, y[m]));
        y[i] = dd_div(r, dd{gh[i * k + i], gl[i * k + i]});
      }
      for (int i = 0; i <= j; ++i) t[i + j * k] = kept[i] ? (y[i].hi + y[i].lo) * dsc[i] : 0.0;
    }
  }
  __syncthreads();
}

// V <- V T in place, elementwise (T upper triangular, k x k column-major, in LDS)
DEV void phase_apply_qr(const Problem& P, Cl& cl, double* V, const double* t) {
  const int k = P.k;
  const size_t n = P.n;
  for (size_t e = (size_t)cl.rank * BLOCK + threadIdx.x; e < n; e += (size_t)cl.G * BLOCK) {
    double v[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) v[c] = c < k ? V[(size_t)c * n + e] : 0.0;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      if (j < k) {
        double q = 0.0;
#pragma unroll
        for (int i = 0; i <= j; ++i) q += v[i] * t[i + j * k];
        V[(size_t)j * n + e] = q;
      }
    }
  }
}

// x = Y z
DEV void phase_sketch_combine(const Problem& P, Cl& cl, const double* Yn, const double* z) {
  const size_t n = P.n;
  for (size_t e = (size_t)cl.rank * BLOCK + threadIdx.x; e < n; e += (size_t)cl.G * BLOCK) {
    double v = 0.0;
    int c = 0;
    for (; c + 3 < P.k; c += 4) {
      const double y0 = Yn[c * n + e], y1 = Yn[(c + 1) * n + e], y2 = Yn[(c + 2) * n + e], y3 = Yn[(c + 3) * n + e];
      v += y0 * z[c] + y1 * z[c + 1] + y2 * z[c + 2] + y3 * z[c + 3];
    }
    for (; c < P.k; ++c) v += Yn[c * n + e] * z[c];
    P.x[e] = v;
  }
}

// ------------------------------------------------------------------------------------------
// LDS layout of the solve kernel
struct Smem {
  double* red;    // PSTRIDE
  double* wsum;   // NWAVE * (MMAX + 2)
  double* H;      // (m+1) x m, column j at j*(m+1)
  double* cs;     // m
  double* sn;     // m
  double* g;      // m+1
  double* vs;     // m+1
  double* y;      // m
  double* z;      // KMAX
  double* scr;    // 4 KMAX^2 + 8
  unsigned* sgen; // 32 unsigned (16 doubles): sub-cluster barrier generations
  double* big;    // phase scratch
};

DEV Smem carve(double* s, int m) {
  Smem S;
  S.red = s;
  S.wsum = S.red + PSTRIDE;
  S.H = S.wsum + NWAVE * (MMAX + 2);
  S.cs = S.H + (m + 1) * m;
  S.sn = S.cs + m;
  S.g = S.sn + m;
  S.vs = S.g + m + 1;
  S.y = S.vs + m + 1;
  S.z = S.y + m;
  S.scr = S.z + KMAX;
  S.sgen = (unsigned*)(S.scr + 4 * KMAX * KMAX + 8);
  S.big = S.scr + 4 * KMAX * KMAX + 8 + 16;
  return S;
}

// back substitution R y = g on the leading jj x jj block of H (thread 0), y in LDS
DEV void back_substitute(const Smem& S, int m, int jj) {
  if (threadIdx.x == 0) {
    for (int i = jj - 1; i >= 0; --i) {
      double s = S.g[i];
      for (int q = i + 1; q < jj; ++q) s -= S.H[q * (m + 1) + i] * S.y[q];
      S.y[i] = s / S.H[i * (m + 1) + i];
    }
  }
  __syncthreads();
}

// Geometry of both stages, the initial guess and r0 = b - A x0 (shared by both precisions).
// Fills info (rank, relres0) and returns whether the solve is already finished.
DEV bool solve_start(const Problem& P, Cl& cl, const SolveArgs& a, const Smem& S, PhaseClock& clk,
                     sa_solve_info& info, double& nb, double& rn) {
  const int tid = threadIdx.x;
  const size_t n = P.n;
  phase_geometry(P, cl, a.eta_p, a.eta_c);
  csync(cl);
  clk.tick(PH_GEOM);

  const double* Yo = P.Y[a.ycur];
  double* Yn = P.Y[a.ycur ^ 1];
  int rank = 0;
  if (a.range) {
    // range finder: the ring takes the previous solution and V = X Omega goes to Y[0]; the
    // block pass below then reads V as it is (no fused update)
    if (a.push || a.sketch_guess) {
      phase_range_form(P, cl, a, P.Y[0], S.big);
      csync(cl);
    }
    if (P.orth && a.sketch_guess) {
      // V = Q (Alg. 3's orthonormalised sketch): Gram, Cholesky with drop, V <- V D L^-T
      phase_sketch_gram(P, cl, P.Y[0], S.big, S.red);
      cluster_sum_dd(cl, S.red, P.k * (P.k + 1) / 2);
      small_qr_factor(P, S.red, P.tau_drop, S.big, S.scr);
      phase_apply_qr(P, cl, P.Y[0], S.big);
      csync(cl);
    }
    Yo = P.Y[0];
    Yn = P.Y[0];
  }
  if (a.sketch_guess) {
    SolveArgs ab = a;
    if (a.range) ab.push = 0;
    // the widest tiles (64, 32 or 16 columns) whose block operator fits the LDS
    if (P.txg == 64) phase_block_gram<64>(P, cl, ab, Yo, Yn, S.big, S.red);
    else if (P.txg == 32) phase_block_gram<32>(P, cl, ab, Yo, Yn, S.big, S.red);
    else phase_block_gram<16>(P, cl, ab, Yo, Yn, S.big, S.red);
    const int nv = P.k * (P.k + 1) / 2 + P.k;
    cluster_sum_dd(cl, S.red, nv);
    clk.tick(PH_GUESS);
    rank = small_solve(P, S.red, P.tau_drop, S.z, S.scr);
    csync(cl);  // every tile has read x (the previous solution) before it is overwritten
    clk.tick(PH_SMALL);
    phase_sketch_combine(P, cl, ab.push ? Yn : Yo, S.z);
  } else {
    if (a.push && !a.range) phase_push(P, cl, a, Yo, Yn);
    if (!a.prev_guess) {
      csync(cl);
      for (size_t e = (size_t)cl.rank * BLOCK + tid; e < n; e += (size_t)cl.G * BLOCK) P.x[e] = 0.0;
    }
  }
  csync(cl);
  clk.tick(PH_GUESS);

  phase_operator(P, cl, P.x, 1.0, P.r, a.b, S.big, S.red, 0);
  cluster_sum(cl, S.red, 2);
  clk.tick(PH_OPER);
  nb = sqrt(S.red[1]);
  rn = sqrt(S.red[0]);
  info.iters = 0; info.restarts = 0; info.refinements = 0; info.status = SA_OK; info.rank = rank; info.checks = 0;
  info.relres0 = nb > 0.0 ? rn / nb : 0.0;
  info.relres = info.relres0;
  if (!(nb > 0.0)) {
    if (!(nb == 0.0)) atomicOr(P.flags + FLAG_NONFINITE, 1);
    for (size_t e = (size_t)cl.rank * BLOCK + tid; e < n; e += (size_t)cl.G * BLOCK) P.x[e] = 0.0;
    info.relres0 = info.relres = 0.0;
    return true;
  }
  if (!isfinite(rn)) {
    atomicOr(P.flags + FLAG_NONFINITE, 1);
    return true;
  }
  return rn <= a.rtol * nb;
}

// Givens rotation of Hessenberg column j (h2 = second CGS pass added here), new g, basis scale
DEV void givens_step(const Smem& S, int m, int j, double hn) {
  if (threadIdx.x == 0) {
    double* col = S.H + j * (m + 1);
    for (int i = 0; i <= j; ++i) col[i] += S.y[i];
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const double t0 = S.cs[i] * col[i] + S.sn[i] * col[i + 1];
      col[i + 1] = -S.sn[i] * col[i] + S.cs[i] * col[i + 1];
      col[i] = t0;
    }
    const double den = hypot(col[j], col[j + 1]);
    S.cs[j] = col[j] / den;
    S.sn[j] = col[j + 1] / den;
    col[j] = den;
    col[j + 1] = 0.0;
    S.g[j + 1] = -S.sn[j] * S.g[j];
    S.g[j] = S.cs[j] * S.g[j];
    S.vs[j + 1] = 1.0 / hn;
  }
  __syncthreads();
}

// CGS2 of the new Arnoldi vector w = V_{j+1} against V_0..V_j (h1 = V^T w with ||w||, w -= V h1,
// h2 = V^T w, w -= V h2), then the Givens rotation of Hessenberg column j. Returns ||w|| after
// orthogonalisation; w0 receives ||w|| before it.
template <class T>
DEV double cgs2_givens(const Problem& P, Cl& cl, const Smem& S, PhaseClock& clk, T* V, int j, double& w0) {
  const size_t n = P.n;
  const int m = P.m, tid = threadIdx.x;
  T* wv = V + (size_t)(j + 1) * n;
  phase_dots<T>(P, cl, V, S.vs, j + 1, wv, true, S.wsum, S.red);
  cluster_sum(cl, S.red, j + 2);
  w0 = sqrt(S.red[j + 1]);
  if (tid < j + 1) S.H[j * (m + 1) + tid] = S.red[tid];
  __syncthreads();
  phase_update<T>(P, cl, V, S.vs, S.H + j * (m + 1), j + 1, wv, true, S.wsum, S.red);
  cluster_sum(cl, S.red, j + 1);
  if (tid < j + 1) S.y[tid] = S.red[tid];  // h2 (y is free here)
  __syncthreads();
  phase_update<T>(P, cl, V, S.vs, S.y, j + 1, wv, false, S.wsum, S.red);
  cluster_sum(cl, S.red, 1);
  clk.tick(PH_ORTH);
  const double hn = sqrt(S.red[0]);
  givens_step(S, m, j, hn);
  return hn;
}

// ||v||^2 summed over the cluster into red[0]
template <class T>
DEV double cluster_norm(const Problem& P, Cl& cl, const Smem& S, const T* v) {
  const size_t n = P.n;
  block_sum_to([&] {
    double s = 0.0;
    for (size_t e = (size_t)cl.rank * BLOCK + threadIdx.x; e < n; e += (size_t)cl.G * BLOCK) s += double(v[e]) * double(v[e]);
    return s;
  }(), S.wsum, S.red, 0);
  cluster_sum(cl, S.red, 1);
  return sqrt(S.red[0]);
}

// Stages of a Krylov solve. Every preconditioner application of a solve goes through one call
// site (the V-cycle is by far the largest piece of code): the stage says what it is applied to.
enum { ST_START = 1, ST_STEP = 2 };

// FP64 restarted GMRES from P.x with residual P.r (left-preconditioned, CGS2, decisions on the
// true residual): the check trigger starts at rtol ||b|| ||M^-1 r0|| / ||r0|| (the first
// cycle's preconditioned residual norm in the true residual's scale, no preconditioner
// application of b); a candidate x + V y is checked on b - A x when the Arnoldi estimate
// reaches it, the trigger is rescaled with the candidate's residual after a failed check;
// lucky breakdown restarts from the checked candidate.
DEV void gmres64(const Problem& P, Cl& cl, const SolveArgs& a, const Smem& S, PhaseClock& clk,
                 sa_solve_info& info, double nb, double rn) {
  const int m = P.m, tid = threadIdx.x;
  const size_t n = P.n;
  const double rtol = a.rtol;
  double* x = P.x;
  double* xc = P.xc;
  double* r = P.r;
  double* rc = P.rc;
  double* V = P.V;
  double trigger = -1.0;  // set at the first cycle start
  int stage = ST_START, j = 0;
  // line-solve constants kept in LDS for the whole solve (levels with one tile per workgroup)
  double* res = P.res_base >= 0 ? dyn_lds + P.res_base : nullptr;
  if (res) {
    for (int l = 0; l < P.nlev; ++l)
      if (P.lev[l].res >= 0) {
        if (P.lev[l].tm == 32) stage_resident<double, 32>(P, cl, l, res + P.lev[l].res);
        else stage_resident<double, TM>(P, cl, l, res + P.lev[l].res);
      }
    __syncthreads();
  }
  while (!aborted(cl)) {
    const double* src = r;
    double* dst = V;
    clk.tick(PH_OTHER);
    if (stage == ST_STEP) {
      info.iters += 1;
      phase_operator(P, cl, V + (size_t)j * n, S.vs[j], P.t, nullptr, S.big, S.red, 0);
      csync(cl);
      clk.tick(PH_OPER);
      src = P.t;
      dst = V + (size_t)(j + 1) * n;
    }
    precond<double>(P, cl, src, dst, S.big, &clk, res);
    clk.tick(PH_PREC);
    if (stage == ST_START) {
      const double beta = cluster_norm(P, cl, S, (const double*)V);
      if (trigger < 0.0) trigger = rtol * beta * nb / rn;
      if (tid == 0) {
        S.vs[0] = 1.0 / beta;
        S.g[0] = beta;
      }
      __syncthreads();
      j = 0;
      stage = ST_STEP;
      continue;
    }
    double w0;
    const double hn = cgs2_givens<double>(P, cl, S, clk, V, j, w0);
    const bool breakdown = hn <= 1e-14 * w0;
    bool end_cycle = false;
    if (breakdown || fabs(S.g[j + 1]) <= trigger) {
      back_substitute(S, m, j + 1);
      phase_combine<double>(P, cl, V, S.vs, S.y, j + 1, x, xc);
      csync(cl);
      clk.tick(PH_OTHER);
      phase_operator(P, cl, xc, 1.0, rc, a.b, S.big, S.red, 0);
      cluster_sum(cl, S.red, 2);
      clk.tick(PH_OPER);
      const double rcn = sqrt(S.red[0]);
      info.checks += 1;
      if (rcn <= rtol * nb) {
        double* t = x; x = xc; xc = t;
        info.relres = rcn / nb;
        break;
      }
      if (breakdown || !isfinite(rcn)) {
        double* t = x; x = xc; xc = t;
        t = r; r = rc; rc = t;
        rn = rcn;
        if (!isfinite(rcn)) { atomicOr(P.flags + FLAG_NONFINITE, 1); break; }
        end_cycle = true;
      } else {
        trigger = fabs(S.g[j + 1]) * rtol * nb / rcn;
      }
    }
    if (!end_cycle && j + 1 == m) {  // cycle complete: x += V y, true residual
      back_substitute(S, m, m);
      phase_combine<double>(P, cl, V, S.vs, S.y, m, x, x);
      csync(cl);
      clk.tick(PH_OTHER);
      phase_operator(P, cl, x, 1.0, r, a.b, S.big, S.red, 0);
      cluster_sum(cl, S.red, 2);
      clk.tick(PH_OPER);
      rn = sqrt(S.red[0]);
      info.relres = rn / nb;
      if (rn <= rtol * nb) break;
      if (!isfinite(rn)) { atomicOr(P.flags + FLAG_NONFINITE, 1); break; }
      end_cycle = true;
    }
    if (end_cycle) {  // restart from (x, r)
      info.relres = rn / nb;
      info.restarts += 1;
      if (info.restarts > P.max_restarts) {
        info.status = SA_NOCONV;
        break;
      }
      stage = ST_START;
      continue;
    }
    j += 1;
  }
  // the solution must end in P.x (the next solve's previous solution)
  if (x != P.x) {
    csync(cl);
    phase_copy(P, cl, (const double*)x, P.x, P.n);
  }
}

// Mixed precision: FP64 iterative refinement around FP32 GMRES cycles on A d = r / ||r||.
// Operator, V-cycle and basis are FP32; Gram-Schmidt sums, Hessenberg and Givens are FP64.
// Candidates x + ||r|| V y are checked on the FP64 residual b - A x with the trigger rule of
// the FP64 path (first at rtol ||b|| ||M^-1 fl32(r0 / ||r0||)||, rescaled after a failed check);
// when the cycle reaches FP32 resolution (estimate down by rtol_inner, or h_{j+1,j} <=
// 1e-7 ||w||) the checked candidate becomes the new x and the next correction starts from its
// residual; a complete cycle adds its correction and starts the next one.
DEV void refine32(const Problem& P, Cl& cl, const SolveArgs& a, const Smem& S, PhaseClock& clk,
                  sa_solve_info& info, double nb, double rn) {
  const int m = P.m, tid = threadIdx.x;
  const size_t n = P.n;
  const double rtol = a.rtol;
  float* V = P.V32;
  float* r32 = P.r32;
  float* lds = (float*)S.big;
  double* x = P.x;
  double* xc = P.xc;
  double* r = P.r;
  double* rc = P.rc;
  double trigger = -1.0, beta = 0.0;  // trigger: set at the first cycle start
  int stage = ST_START, j = 0;
  // FP32 line-solve constants kept in LDS for the whole solve (levels with one tile per
  // workgroup)
  float* res = P.res_base >= 0 ? (float*)(dyn_lds + P.res_base) : nullptr;
  if (res) {
    for (int l = 0; l < P.nlev; ++l)
      if (P.lev[l].res >= 0) {
        if (P.lev[l].tm == 32) stage_resident<float, 32>(P, cl, l, res + P.lev[l].res);
        else stage_resident<float, TM>(P, cl, l, res + P.lev[l].res);
      }
    __syncthreads();
  }
  while (!aborted(cl)) {
    const float* src = r32;
    float* dst = P.t32;
    clk.tick(PH_OTHER);
    if (stage == ST_START) {  // fl32(r / ||r||)
      if (info.refinements >= P.max_refine) {
        info.status = SA_NOCONV;
        break;
      }
      info.refinements += 1;
      dst = V;
      const double sc = 1.0 / rn;
      for (size_t e = (size_t)cl.rank * BLOCK + tid; e < n; e += (size_t)cl.G * BLOCK) r32[e] = float(r[e] * sc);
      csync(cl);
    } else {
      info.iters += 1;
      phase_operator_s<float>(P, cl, V + (size_t)j * n, float(S.vs[j]), P.t32, lds);
      csync(cl);
      clk.tick(PH_OPER);
      src = P.t32;
      dst = V + (size_t)(j + 1) * n;
    }
    precond<float>(P, cl, src, dst, lds, &clk, res);
    clk.tick(PH_PREC);
    if (stage == ST_START) {
      beta = cluster_norm(P, cl, S, (const float*)V);
      if (trigger < 0.0) trigger = rtol * nb * beta;
      if (tid == 0) {
        S.vs[0] = 1.0 / beta;
        S.g[0] = beta;
      }
      __syncthreads();
      j = 0;
      stage = ST_STEP;
      continue;
    }
    double w0;
    const double hn = cgs2_givens<float>(P, cl, S, clk, V, j, w0);
    const double est = rn * fabs(S.g[j + 1]);
    const bool floor = hn <= 1e-7 * w0 || fabs(S.g[j + 1]) <= P.rtol_inner * beta;
    bool next = false;
    if (floor || est <= trigger) {
      back_substitute(S, m, j + 1);
      if (tid <= j) S.y[tid] *= rn;
      __syncthreads();
      phase_combine<float>(P, cl, V, S.vs, S.y, j + 1, x, xc);
      csync(cl);
      clk.tick(PH_OTHER);
      phase_operator(P, cl, xc, 1.0, rc, a.b, S.big, S.red, 0);
      cluster_sum(cl, S.red, 2);
      clk.tick(PH_OPER);
      const double rcn = sqrt(S.red[0]);
      info.checks += 1;
      if (!isfinite(rcn)) {
        atomicOr(P.flags + FLAG_NONFINITE, 1);
        break;
      }
      if (rcn <= rtol * nb || floor) {
        double* t = x; x = xc; xc = t;
        t = r; r = rc; rc = t;
        rn = rcn;
        info.relres = rn / nb;
        if (rcn <= rtol * nb) break;
        next = true;
      } else {
        trigger = est * rtol * nb / rcn;
      }
    }
    if (!next && j + 1 == m) {  // cycle complete: x += ||r|| V y, true residual
      back_substitute(S, m, m);
      if (tid < m) S.y[tid] *= rn;
      __syncthreads();
      phase_combine<float>(P, cl, V, S.vs, S.y, m, x, x);
      csync(cl);
      clk.tick(PH_OTHER);
      phase_operator(P, cl, x, 1.0, r, a.b, S.big, S.red, 0);
      cluster_sum(cl, S.red, 2);
      clk.tick(PH_OPER);
      rn = sqrt(S.red[0]);
      info.relres = rn / nb;
      if (!isfinite(rn)) { atomicOr(P.flags + FLAG_NONFINITE, 1); break; }
      if (rn <= rtol * nb) break;
      next = true;
    }
    if (next) {
      stage = ST_START;
      continue;
    }
    j += 1;
  }
  if (x != P.x) {
    csync(cl);
    phase_copy(P, cl, (const double*)x, P.x, P.n);
  }
}

// One solve of the problem by the cluster workgroup `rank`: guess, then FP64 GMRES (PREC =
// SA_FP64) or FP32 refinement (PREC = SA_FP32_IR), then the report into the log.
template <int PREC>
DEV void solve_body(const Problem* __restrict__ PP, const SolveArgs& a, int rank) {
  const Problem& P = *PP;
  double* smem = dyn_lds;
  Smem S = carve(smem, P.m);
  Cl cl = make_cl(P, rank, P.G);
  cl.scr = S.wsum;  // NWAVE * (MMAX + 2) >= BLOCK doubles, free whenever a cluster sum runs
  // sub-cluster barriers of the V-cycle levels: every workgroup starts from the generations
  // the words hold (no barrier is in flight between launches)
  if (P.G > 1) {
    if (threadIdx.x < MAXLEV)
      S.sgen[threadIdx.x] = (unsigned)(__hip_atomic_load(sub_word(P.bar, threadIdx.x), __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT) >> 32);
    __syncthreads();
    cl.sgen = S.sgen;
  }
  PhaseClock clk;
  clk.begin(a.prof != nullptr, rank, a.prof);
  sa_solve_info info;
  double nb = 0.0, rn = 0.0;
  const bool done = solve_start(P, cl, a, S, clk, info, nb, rn);
  if (!done) {
    if constexpr (PREC == SA_FP32_IR) refine32(P, cl, a, S, clk, info, nb, rn);
    else gmres64(P, cl, a, S, clk, info, nb, rn);
  }
  clk.tick(PH_OTHER);
  if (cl.rank == 0 && threadIdx.x == 0) {
    if (aborted(cl)) info.status = SA_EDEVICE;
    P.log[a.log_slot] = info;
    if (a.out) {  // batched solve: fold and clear the problem's error flags
      if (info.status == SA_OK || info.status == SA_NOCONV) {
        if (atomicExch(P.flags + FLAG_GEOM, 0)) info.status = SA_EGEOM;
        if (atomicExch(P.flags + FLAG_NONFINITE, 0) && info.status != SA_EGEOM) info.status = SA_ENONFINITE;
      }
      *a.out = info;
    }
  }
  clk.flush(a.prof);
}

// Entry of the solve kernels. With nitems = 0 the grid solves the single problem of `one`
// (sa_solve); otherwise its workgroups are split into consecutive clusters, item i owning
// [first_i, first_i + G_i), and every cluster solves its own problem (the server's batched
// launch). Each problem has its own barrier words, partial sums and log, so clusters never
// interact. One entry serves every guess mode: without a sketch no push or sketch guess is
// requested.
template <int PREC>
DEV void solve_entry(const BatchItem* __restrict__ items, int nitems, const BatchItem& one) {
  const Problem SA_GLOBAL* P = one.P;
  const SolveArgs* a = &one.a;
  int rank = (int)blockIdx.x;
  if (nitems > 0) {
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].first <= (int)blockIdx.x) lo = mid;
      else hi = mid - 1;
    }
    P = items[lo].P;
    a = &items[lo].a;
    rank = (int)blockIdx.x - items[lo].first;
    if (rank < 0 || rank >= P->G) return;  // padding workgroups of the launch
  }
  solve_body<PREC>(P, *a, rank);  // one call site: one inlined copy of the solve
}

}  // namespace sa
