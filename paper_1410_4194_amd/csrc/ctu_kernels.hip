// ctu_kernels.hip -- HIP kernels (gfx950) of one CTU timestep, Sec. 2.1 of Schneider &
// Robertson 2015: ghost fill, per-direction PPMC trace and first Riemann solve, transverse
// correction and second Riemann solve, conservative update fused with the CFL reduction.
//
// Data layout: structure of arrays over the allocated box, x fastest, three ghost layers
// (see ctu.h).  Interface arrays store face c+1/2 at the index of cell c.  Threads run along
// x, so every global access of a wavefront is a contiguous run along x.  Each launch serves a
// table of grids (ctu_kernels.hpp); a block finds its grid and local block index first.
#include "ctu_kernels.hpp"

namespace ctu {

// Rotation of momentum slots for a sweep along D (cyclic): rotated slot s <- global rot(D,s).
template <int D>
__device__ __forceinline__ int rot(int s) {
  if (s == 0 || s == 4) return s;
  return 1 + ((s - 1 + D) % 3);
}

// Grid owning block b of a launch: start[g] <= b < start[g+1].
__device__ __forceinline__ int find_grid(const int* __restrict__ start, int ngrids, int b) {
  int lo = 0, hi = ngrids;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Pointers read from a descriptor are generic; holding them in global-address-space pointer
// types lets the compiler emit global (not flat) loads and stores through them.
#define GLOBAL __attribute__((address_space(1)))

struct BlockRef {
  const GridDesc* G;
  long long lb;  // block index within the grid's range
  long long nb;  // padded block count of the grid's range
};

__device__ __forceinline__ BlockRef block_ref(const LaunchTab& tab) {
  const int b = blockIdx.x;
  const int g = find_grid(tab.start, tab.ngrids, b);
  BlockRef r;
  r.G = tab.grids + g;
  r.lb = b - tab.start[g];
  r.nb = tab.start[g + 1] - tab.start[g];
  return r;
}

// ---- reductions --------------------------------------------------------------------------
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block minimum of v written to part[lb] (no atomics); every thread must call it.
__device__ __forceinline__ void block_min_store(double v, GLOBAL double* part, long long lb) {
  __shared__ double smin[32];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  v = wave_min(v);
  if (lane == 0) smin[wave] = v;
  __syncthreads();
  if (wave == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    double m = lane < nw ? smin[lane] : INFINITY;
    m = wave_min(m);
    if (lane == 0) part[lb] = m;
  }
}

// Per-cell CFL bound min(dx/(|u|+a), dy/(|v|+a), dz/(|w|+a)) (eq. calc_dt_3D without C0).
template <typename T>
__device__ __forceinline__ double cell_dt_bound(const T U[5], const GridParams& P) {
  T W[5];
  cons_to_prim(U, T(P.gm1), T(P.p_floor), W);
  double a = sqrt(P.gamma * (double)W[4] / (double)W[0]);
  double tx = P.dx[0] / (fabs((double)W[1]) + a);
  double ty = P.dx[1] / (fabs((double)W[2]) + a);
  double tz = P.dx[2] / (fabs((double)W[3]) + a);
  return fmin(tx, fmin(ty, tz));
}

// Workgroups are dealt to the 8 XCDs round robin; within a grid's block range (which starts
// at a multiple of 8) this gives each XCD a contiguous run of logical blocks.
__device__ __forceinline__ long long xcd_local(long long lb, long long nb) {
  const long long per = nb / 8;
  return (lb % 8) * per + lb / 8;
}

// ---- step bookkeeping ----------------------------------------------------------------------
__global__ void k_set_dt(DevScalars* s, double dt) { s->dt = dt; }

__global__ void k_set_end(DevScalars* s, double t_end, long long steps_left) {
  s->t_end = t_end;
  s->steps_left = steps_left;
}

// Device-side time step of every grid: C0 * (min CFL bound), clipped to t_end - t; a grid
// whose step budget is used up, or whose state was flagged non-physical, takes dt = 0 (its
// passes become no-ops).
__global__ void k_begin_step(const GridDesc* __restrict__ grids, int ngrids) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < ngrids; g += gridDim.x * blockDim.x) {
    DevScalars* s = grids[g].s;
    const double bound = __longlong_as_double((long long)s->dt_next_bits);
    double dt = fmin(grids[g].P.cfl * bound, s->t_end - s->t);
    if (s->steps_left <= 0 || (s->flags & 3u)) dt = 0.0;  // budget used up, or non-physical
    s->dt = dt;
  }
}

__global__ void k_end_step(const GridDesc* __restrict__ grids, int ngrids) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < ngrids; g += gridDim.x * blockDim.x) {
    DevScalars* s = grids[g].s;
    if (s->dt > 0.0) {
      s->t += s->dt;
      s->steps += 1;
      s->steps_left -= 1;
    }
  }
}

// Copies of the scalars of n grids into one array (one read-back for a whole batch).
__global__ void k_gather_scalars(DevScalars* const* __restrict__ src, int n, DevScalars* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = *src[i];
}

// ---- a1: ghost fill (Sec. 3.1) ------------------------------------------------------------
// Axis AXIS ghosts over the full extent of the other two axes (ghosts included), so
// running x, then y, then z fills edges and corners consistently.
template <typename T, int AXIS>
__global__ __launch_bounds__(256) void k_bc_fill(LaunchTab tab) {
  const BlockRef r = block_ref(tab);
  const GridParams P = r.G->P;
  if (!(r.G->s->dt > 0.0)) return;
  GLOBAL T* __restrict__ u = (GLOBAL T*)r.G->u;
  const int n = P.n[AXIS];
  const long long tid = r.lb * blockDim.x + threadIdx.x;
  int i, j, k, layer;
  if (AXIS == 0) {
    const long long total = 2LL * NG * P.N[1] * P.N[2];
    if (tid >= total) return;
    layer = (int)(tid % (2 * NG));
    const long long q = tid / (2 * NG);
    j = (int)(q % P.N[1]) - NG;
    k = (int)(q / P.N[1]) - NG;
    i = 0;
  } else if (AXIS == 1) {
    const long long total = 2LL * NG * P.N[0] * P.N[2];
    if (tid >= total) return;
    i = (int)(tid % P.N[0]) - NG;
    const long long q = tid / P.N[0];
    layer = (int)(q % (2 * NG));
    k = (int)(q / (2 * NG)) - NG;
    j = 0;
  } else {
    const long long total = 2LL * NG * P.N[0] * P.N[1];
    if (tid >= total) return;
    i = (int)(tid % P.N[0]) - NG;
    const long long q = tid / P.N[0];
    j = (int)(q % P.N[1]) - NG;
    layer = (int)(q / P.N[1]);
    k = 0;
  }
  const int q = layer < NG ? layer - NG : n + (layer - NG);
  const int bc = layer < NG ? r.G->bc[2 * AXIS] : r.G->bc[2 * AXIS + 1];
  int src;
  if (bc == 0) {
    src = q % n;
    if (src < 0) src += n;
  } else {
    src = q < 0 ? 0 : n - 1;
  }
  const long long d = cell_index(P, AXIS == 0 ? q : i, AXIS == 1 ? q : j, AXIS == 2 ? q : k);
  const long long sidx =
      cell_index(P, AXIS == 0 ? src : i, AXIS == 1 ? src : j, AXIS == 2 ? src : k);
#pragma unroll
  for (int f = 0; f < 5; ++f) u[f * P.stride + d] = u[f * P.stride + sidx];
}

// ---- fused sweeps --------------------------------------------------------------------------
// Stage 1 (a2-a5) and stage 2 (a2-a4 re-traced, a6-a7) of one direction D each run as one
// kernel.  Along y and z a thread owns one column and marches along D over a segment of
// P.seg[D] faces, keeping a register window of primitives (cells c-1..c+2) and limited
// slopes (c-1..c+1): every primitive, slope and trace is computed once per cell (plus a
// short warm-up per segment) and each face's Riemann problem once.  Along x a wavefront covers 64
// consecutive cells of one row and exchanges neighbours with lane shuffles; it yields XW
// faces.

template <typename T, int D>
__device__ __forceinline__ void load_prim(const GLOBAL T* __restrict__ u, long long stride, long long id,
                                          const GridParams& P, Prim<T>& c) {
  T Ur[5];
#pragma unroll
  for (int sl = 0; sl < 5; ++sl) Ur[sl] = u[rot<D>(sl) * stride + id];
  make_prim(Ur, T(P.gamma), T(P.gm1), T(P.p_floor), c);
}

template <typename T>
__device__ __forceinline__ void safe_prim(Prim<T>& c) {
  c.w[0] = T(1);
  c.w[1] = c.w[2] = c.w[3] = T(0);
  c.w[4] = T(1);
  c.a = T(1);
  c.ia = T(1);
  c.irho = T(1);
}

template <typename T>
__device__ __forceinline__ Prim<T> shfl_prim(const Prim<T>& p, int src) {
  Prim<T> r;
#pragma unroll
  for (int q = 0; q < 5; ++q) r.w[q] = __shfl(p.w[q], src, 64);
  r.a = __shfl(p.a, src, 64);
  r.ia = __shfl(p.ia, src, 64);
  r.irho = __shfl(p.irho, src, 64);
  return r;
}

// Transverse flux difference of a cell (eq. transverse_evolution), rotated to the sweep
// frame: dT = h1 (F_t1(c - e_t1) - F_t1(c)) + h2 (F_t2(c - e_t2) - F_t2(c)).
template <typename T, int D>
__device__ __forceinline__ void transverse_delta(const GLOBAL T* __restrict__ fstar_all, long long fds,
                                                 long long stride, long long c, long long st1,
                                                 long long st2, T h1, T h2, T dT[5]) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const GLOBAL T* F1 = fstar_all + T1 * fds;
  const GLOBAL T* F2 = fstar_all + T2 * fds;
#pragma unroll
  for (int sl = 0; sl < 5; ++sl) {
    const long long o = rot<D>(sl) * stride + c;
    dT[sl] = h1 * (F1[o - st1] - F1[o]) + h2 * (F2[o - st2] - F2[o]);
  }
}

// Primitive -> conserved with E = p/(g-1) + rho V^2/2, multiplying by 1/(g-1).
template <typename T>
__device__ __forceinline__ void to_cons(const T W[5], T inv_gm1, T U[5]) {
  const T rho = W[0];
  U[0] = rho;
  U[1] = rho * W[1];
  U[2] = rho * W[2];
  U[3] = rho * W[3];
  U[4] = W[4] * inv_gm1 + T(0.5) * rho * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
}

__device__ __forceinline__ void flush_counts(const RiemannCounts& cnt, DevScalars* s) {
  if (cnt.floors) {
    atomicAdd(&s->counters[0], (unsigned long long)cnt.floors);
    atomicOr(&s->flags, 4u);
  }
  if (cnt.caps) {
    atomicAdd(&s->counters[1], (unsigned long long)cnt.caps);
    atomicOr(&s->flags, 8u);
  }
}

// Newton-iteration histogram of the solves of one wavefront (instrumented sweeps only):
// each solve's bin is counted over the active lanes with a ballot, so lanes that left the
// kernel early are simply not counted.
struct NewtonHist {
  unsigned long long n[8];
  __device__ void add(int iters) {
    const int b = iters == 0 ? 7
                  : iters <= 4 ? iters - 1 : (iters <= 8 ? 4 : (iters <= 16 ? 5 : 6));
#pragma unroll
    for (int k = 0; k < 8; ++k) n[k] += __popcll(__ballot(b == k));
  }
  // The first active lane adds the wave's counts to the grid's histogram.
  __device__ void flush(DevScalars* s) const {
    const unsigned long long act = __ballot(1);
    if ((int)__lane_id() == __ffsll((long long)act) - 1) {
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (n[k]) atomicAdd(&s->newton_hist[k], n[k]);
    }
  }
};

// STAGE = 1: first-stage fluxes F*_D on faces c-1/2, c in [0, n_D], transverse range
//            [-1, n] on both other axes; written at cell c-1.
// STAGE = 2: CTU fluxes F^{n+1/2}_D on the same faces over the real transverse range, from
//            the re-traced states plus the transverse flux differences of stage 1.
// Block layout per grid: (plane block of kBlock columns, segment), plane blocks fastest.
template <typename T, int D, int STAGE, bool HIST>
__global__ __launch_bounds__(256, 2) void k_sweep_march(LaunchTab tab) {
  static_assert(D == 1 || D == 2, "marching sweeps run along y or z");
  const BlockRef r = block_ref(tab);
  const GridParams P = r.G->P;
  DevScalars* __restrict__ s = r.G->s;
  const double dt = s->dt;
  if (!(dt > 0.0)) return;
  const GLOBAL T* __restrict__ u = (const GLOBAL T*)r.G->u;
  const GLOBAL T* __restrict__ fstar_all = (const GLOBAL T*)r.G->flux;
  const long long fds = 5 * P.stride;
  GLOBAL T* __restrict__ out = (GLOBAL T*)r.G->flux + (STAGE == 1 ? D : 3 + D) * fds;
  constexpr int B = (D == 1) ? 2 : 1;  // the transverse axis other than x
  const int lo = STAGE == 1 ? -1 : 0;
  const int ea = P.n[0] + (STAGE == 1 ? 2 : 0);
  const int eb = P.n[B] + (STAGE == 1 ? 2 : 0);
  const int nd = P.n[D];
  const long long nbx = ((long long)ea * eb + kBlock - 1) / kBlock;
  const int seg = P.seg[D];
  const long long nseg = (nd + 1 + seg - 1) / seg;
  if (r.lb >= nbx * nseg) return;
  const long long tid = (r.lb % nbx) * kBlock + threadIdx.x;
  if (tid >= (long long)ea * eb) return;
  const int i = (int)(tid % ea) + lo;
  const int o = (int)(tid / ea) + lo;
  const int f0 = (int)(r.lb / nbx) * seg;
  const int f1 = min(f0 + seg, nd + 1);
  const long long stx = 1, sty = P.N[0], stz = (long long)P.N[0] * P.N[1];
  const long long sd = D == 1 ? sty : stz;
  const long long c0 = D == 1 ? cell_index(P, i, 0, o) : cell_index(P, i, o, 0);
  const T dtodx = T(dt / P.dx[D]);
  const T igm1 = T(P.inv_gm1);
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const long long st1 = T1 == 0 ? stx : (T1 == 1 ? sty : stz);
  const long long st2 = T2 == 0 ? stx : (T2 == 1 ? sty : stz);
  const T h1 = T(0.5 * dt / P.dx[T1]);
  const T h2 = T(0.5 * dt / P.dx[T2]);

  Prim<T> q0, q1, q2, q3;  // cells c-1, c, c+1, c+2 around the traced cell c
  T s0[5], s1[5], s2[5];   // limited slopes of c-1, c, c+1
  {
    Prim<T> qm;
    load_prim<T, D>(u, P.stride, c0 + (long long)(f0 - 3) * sd, P, qm);
    load_prim<T, D>(u, P.stride, c0 + (long long)(f0 - 2) * sd, P, q0);
    load_prim<T, D>(u, P.stride, c0 + (long long)(f0 - 1) * sd, P, q1);
    load_prim<T, D>(u, P.stride, c0 + (long long)(f0)*sd, P, q2);
    load_prim<T, D>(u, P.stride, c0 + (long long)(f0 + 1) * sd, P, q3);
    slope_fast(qm, q0, q1, s0);
    slope_fast(q0, q1, q2, s1);
    slope_fast(q1, q2, q3, s2);
  }
  // warm-up: trace cell f0-1 (window: q0 = f0-2, q1 = f0-1, q2 = f0, q3 = f0+1)
  T prevR[5];
  {
    T WL[5], WR[5];
    trace_fast(q0, q1, q2, s0, s1, s2, dtodx, WL, WR);
    to_cons(WR, igm1, prevR);
    if (STAGE == 2) {
      T dT[5];
      transverse_delta<T, D>(fstar_all, fds, P.stride, c0 + (long long)(f0 - 1) * sd, st1, st2, h1,
                             h2, dT);
#pragma unroll
      for (int q = 0; q < 5; ++q) prevR[q] += dT[q];
    }
  }
  // shift so that the window is centred on f0 at the top of the loop
  q0 = q1;
  q1 = q2;
  q2 = q3;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    s0[q] = s1[q];
    s1[q] = s2[q];
  }
  // the conserved values of cell c+2 are loaded one iteration ahead (software pipelining)
  T raw[5];
#pragma unroll
  for (int sl = 0; sl < 5; ++sl) raw[sl] = u[rot<D>(sl) * P.stride + c0 + (long long)(f0 + 2) * sd];
  RiemannCounts cnt{0u, 0u, 0};
  NewtonHist hist{};
  for (int c = f0; c < f1; ++c) {
    // window: q0 = c-1, q1 = c, q2 = c+1, slopes s0 = c-1, s1 = c
    make_prim(raw, T(P.gamma), T(P.gm1), T(P.p_floor), q3);  // cell c+2
    if (c + 1 < f1) {
      const long long nid = c0 + (long long)(c + 3) * sd;
#pragma unroll
      for (int sl = 0; sl < 5; ++sl) raw[sl] = u[rot<D>(sl) * P.stride + nid];
    }
    slope_fast(q1, q2, q3, s2);  // slope of c+1
    T WL[5], WR[5], UL[5], UR[5], F[5];
    trace_fast(q0, q1, q2, s0, s1, s2, dtodx, WL, WR);
    to_cons(WL, igm1, UL);
    to_cons(WR, igm1, UR);
    if (STAGE == 2) {
      T dT[5];
      transverse_delta<T, D>(fstar_all, fds, P.stride, c0 + (long long)c * sd, st1, st2, h1, h2,
                             dT);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        UL[q] += dT[q];
        UR[q] += dT[q];
      }
    }
    exact_flux_fast(prevR, UL, P, F, cnt);
    if (HIST) hist.add(cnt.iters);
    const long long fo = c0 + (long long)(c - 1) * sd;
#pragma unroll
    for (int sl = 0; sl < 5; ++sl) out[rot<D>(sl) * P.stride + fo] = F[sl];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      prevR[q] = UR[q];
      s0[q] = s1[q];
      s1[q] = s2[q];
    }
    q0 = q1;
    q1 = q2;
    q2 = q3;
  }
  flush_counts(cnt, s);
  if (HIST) hist.flush(s);
}

// x-direction sweep: one wavefront per (row, segment of XW faces).  Lane l holds cell
// cw - 3 + l; slopes are valid on lanes 1..62, traces on 2..61, faces c-1/2 on 3..61.
template <typename T, int STAGE, bool HIST>
__global__ __launch_bounds__(256) void k_sweep_x(LaunchTab tab) {
  const BlockRef r = block_ref(tab);
  const GridParams P = r.G->P;
  DevScalars* __restrict__ s = r.G->s;
  const double dt = s->dt;
  if (!(dt > 0.0)) return;
  const GLOBAL T* __restrict__ u = (const GLOBAL T*)r.G->u;
  const GLOBAL T* __restrict__ fstar_all = (const GLOBAL T*)r.G->flux;
  const long long fds = 5 * P.stride;
  GLOBAL T* __restrict__ out = (GLOBAL T*)r.G->flux + (STAGE == 1 ? 0 : 3) * fds;
  const int lane = threadIdx.x & 63;
  const long long task = r.lb * (kBlock / 64) + (threadIdx.x >> 6);
  const int lo = STAGE == 1 ? -1 : 0;
  const int ey = P.n[1] + (STAGE == 1 ? 2 : 0);
  const int ez = P.n[2] + (STAGE == 1 ? 2 : 0);
  const int nseg = (P.n[0] + 1 + XW - 1) / XW;
  if (task >= (long long)nseg * ey * ez) return;  // whole wavefront exits together
  const int sx = (int)(task % nseg);
  const long long row = task / nseg;
  const int j = (int)(row % ey) + lo;
  const int k = (int)(row / ey) + lo;
  const int cw = sx * XW;
  const int c = cw - 3 + lane;  // this lane's cell along x
  const long long id = cell_index(P, c, j, k);
  const bool in_alloc = c >= -NG && c < P.n[0] + NG;
  const T dtodx = T(dt / P.dx[0]);
  const T igm1 = T(P.inv_gm1);

  Prim<T> me;
  if (in_alloc)
    load_prim<T, 0>(u, P.stride, id, P, me);
  else
    safe_prim(me);
  const int lm1 = lane > 0 ? lane - 1 : 0;
  const int lp1 = lane < 63 ? lane + 1 : 63;
  const Prim<T> left = shfl_prim(me, lm1);
  const Prim<T> right = shfl_prim(me, lp1);
  T sl[5];
  slope_fast(left, me, right, sl);
  T slm[5], slp[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    slm[q] = __shfl(sl[q], lm1, 64);
    slp[q] = __shfl(sl[q], lp1, 64);
  }
  T WL[5], WR[5], UL[5], UR[5];
  trace_fast(left, me, right, slm, sl, slp, dtodx, WL, WR);
  to_cons(WL, igm1, UL);
  to_cons(WR, igm1, UR);
  const bool traced = lane >= 2 && lane <= 61 && c >= -1 && c <= P.n[0];
  if (STAGE == 2 && traced) {
    T dT[5];
    transverse_delta<T, 0>(fstar_all, fds, P.stride, id, (long long)P.N[0],
                           (long long)P.N[0] * P.N[1], T(0.5 * dt / P.dx[1]),
                           T(0.5 * dt / P.dx[2]), dT);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      UL[q] += dT[q];
      UR[q] += dT[q];
    }
  }
  T prevR[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) prevR[q] = __shfl(UR[q], lm1, 64);
  if (lane >= 3 && lane <= 61 && c >= 0 && c <= P.n[0]) {
    RiemannCounts cnt{0u, 0u, 0};
    T F[5];
    exact_flux_fast(prevR, UL, P, F, cnt);
#pragma unroll
    for (int q = 0; q < 5; ++q) out[q * P.stride + id - 1] = F[q];
    flush_counts(cnt, s);
    if (HIST) {
      NewtonHist hist{};
      hist.add(cnt.iters);
      hist.flush(s);
    }
  }
}

// ---- a8-a9: conservative update and CFL reduction ------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_update(LaunchTab tab) {
  const BlockRef r = block_ref(tab);
  const GridParams P = r.G->P;
  DevScalars* __restrict__ s = r.G->s;
  const double dt = s->dt;
  if (!(dt > 0.0)) return;  // a no-op step keeps the previous partials (state unchanged)
  const long long total = (long long)P.n[0] * P.n[1] * P.n[2];
  const long long nblocks = (total + kBlock - 1) / kBlock;
  const long long lb = xcd_local(r.lb, r.nb);
  if (lb >= nblocks) return;  // whole block idle
  GLOBAL T* __restrict__ u = (GLOBAL T*)r.G->u;
  const long long fds = 5 * P.stride;
  const GLOBAL T* __restrict__ Fx = (const GLOBAL T*)r.G->flux + 3 * fds;
  const GLOBAL T* __restrict__ Fy = Fx + fds;
  const GLOBAL T* __restrict__ Fz = Fy + fds;
  const long long tid = lb * kBlock + threadIdx.x;
  double bound = INFINITY;
  if (tid < total) {
    const int i = (int)(tid % P.n[0]);
    const int j = (int)((tid / P.n[0]) % P.n[1]);
    const int k = (int)(tid / ((long long)P.n[0] * P.n[1]));
    const long long c = cell_index(P, i, j, k);
    const long long st[3] = {1, (long long)P.N[0], (long long)P.N[0] * P.N[1]};
    const T dtdx = T(dt / P.dx[0]), dtdy = T(dt / P.dx[1]), dtdz = T(dt / P.dx[2]);
    T U[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      const long long o = f * P.stride + c;
      T v = u[o];
      v = v + dtdx * (Fx[o - st[0]] - Fx[o]);
      v = v + dtdy * (Fy[o - st[1]] - Fy[o]);
      v = v + dtdz * (Fz[o - st[2]] - Fz[o]);
      U[f] = v;
      u[o] = v;
    }
    bool finite = true;
#pragma unroll
    for (int f = 0; f < 5; ++f) finite = finite && isfinite((double)U[f]);
    if (!finite || !(U[0] > T(0))) {
      atomicOr(&s->flags, finite ? 2u : 1u);
      atomicAdd(&s->counters[2], 1ull);
    } else {
      bound = cell_dt_bound(U, P);
    }
  }
  block_min_store(bound, (GLOBAL double*)r.G->part, lb);
}

template <typename T>
__global__ __launch_bounds__(256) void k_dt(LaunchTab tab) {
  const BlockRef r = block_ref(tab);
  const GridParams P = r.G->P;
  const long long total = (long long)P.n[0] * P.n[1] * P.n[2];
  const long long nblocks = (total + kBlock - 1) / kBlock;
  const long long lb = xcd_local(r.lb, r.nb);
  if (lb >= nblocks) return;
  const GLOBAL T* __restrict__ u = (const GLOBAL T*)r.G->u;
  const long long tid = lb * kBlock + threadIdx.x;
  double bound = INFINITY;
  if (tid < total) {
    const int i = (int)(tid % P.n[0]);
    const int j = (int)((tid / P.n[0]) % P.n[1]);
    const int k = (int)(tid / ((long long)P.n[0] * P.n[1]));
    const long long c = cell_index(P, i, j, k);
    T U[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) U[f] = u[f * P.stride + c];
    bound = cell_dt_bound(U, P);
  }
  block_min_store(bound, (GLOBAL double*)r.G->part, lb);
}

// Minimum of each grid's block partials into its dt_next_bits: block g reduces grid g.
__global__ __launch_bounds__(1024) void k_dt_final(const GridDesc* __restrict__ grids) {
  const GridDesc& G = grids[blockIdx.x];
  const long long total = (long long)G.P.n[0] * G.P.n[1] * G.P.n[2];
  const long long nblocks = (total + kBlock - 1) / kBlock;
  const GLOBAL double* __restrict__ part = (const GLOBAL double*)G.part;
  double m = INFINITY;
  for (long long b = threadIdx.x; b < nblocks; b += blockDim.x) m = fmin(m, part[b]);
  __shared__ double smin[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  m = wave_min(m);
  if (lane == 0) smin[wave] = m;
  __syncthreads();
  if (wave == 0) {
    double v = lane < (int)(blockDim.x >> 6) ? smin[lane] : INFINITY;
    v = wave_min(v);
    if (lane == 0)
      G.s->dt_next_bits = (unsigned long long)__double_as_longlong(v);
  }
}

// ---- conservation totals (fixed-order, deterministic) -------------------------------------
template <typename T>
__global__ void k_totals_partial(const T* __restrict__ u, GridParams P, double* __restrict__ part) {
  const long long total = (long long)P.n[0] * P.n[1] * P.n[2];
  double acc[5] = {0, 0, 0, 0, 0};
  for (long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x; tid < total;
       tid += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(tid % P.n[0]);
    const int j = (int)((tid / P.n[0]) % P.n[1]);
    const int k = (int)(tid / ((long long)P.n[0] * P.n[1]));
    const long long c = cell_index(P, i, j, k);
#pragma unroll
    for (int f = 0; f < 5; ++f) acc[f] += (double)u[f * P.stride + c];
  }
  __shared__ double sh[5][32];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    double v = wave_sum(acc[f]);
    if (lane == 0) sh[f][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    const int nw = blockDim.x >> 6;
    double v = 0.0;
    for (int w = 0; w < nw; ++w) v += sh[threadIdx.x][w];
    part[blockIdx.x * 5 + threadIdx.x] = v;
  }
}

__global__ void k_totals_final(const double* __restrict__ part, int nblocks, double* __restrict__ out) {
  if (threadIdx.x < 5) {
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) v += part[b * 5 + threadIdx.x];
    out[threadIdx.x] = v;
  }
}

// ---- host-facing data movement -------------------------------------------------------------
// Packed real cells (field-major, x fastest) <-> allocated layout.
template <typename T>
__global__ void k_scatter(const T* __restrict__ packed, T* __restrict__ u, GridParams P) {
  const long long total = (long long)P.n[0] * P.n[1] * P.n[2];
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= total) return;
  const int i = (int)(tid % P.n[0]);
  const int j = (int)((tid / P.n[0]) % P.n[1]);
  const int k = (int)(tid / ((long long)P.n[0] * P.n[1]));
  const long long c = cell_index(P, i, j, k);
#pragma unroll
  for (int f = 0; f < 5; ++f) u[f * P.stride + c] = packed[f * total + tid];
}

template <typename T>
__global__ void k_gather(const T* __restrict__ u, T* __restrict__ packed, GridParams P) {
  const long long total = (long long)P.n[0] * P.n[1] * P.n[2];
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= total) return;
  const int i = (int)(tid % P.n[0]);
  const int j = (int)((tid / P.n[0]) % P.n[1]);
  const int k = (int)(tid / ((long long)P.n[0] * P.n[1]));
  const long long c = cell_index(P, i, j, k);
#pragma unroll
  for (int f = 0; f < 5; ++f) packed[f * total + tid] = u[f * P.stride + c];
}

// Primitive (double, packed) -> conserved (T, allocated layout) with the ideal-gas EOS.
template <typename T>
__global__ void k_prim_to_cons(const double* __restrict__ packed, T* __restrict__ u, GridParams P) {
  const long long total = (long long)P.n[0] * P.n[1] * P.n[2];
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= total) return;
  const int i = (int)(tid % P.n[0]);
  const int j = (int)((tid / P.n[0]) % P.n[1]);
  const int k = (int)(tid / ((long long)P.n[0] * P.n[1]));
  const long long c = cell_index(P, i, j, k);
  double W[5], U[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) W[f] = packed[f * total + tid];
  prim_to_cons(W, P.gm1, U);
#pragma unroll
  for (int f = 0; f < 5; ++f) u[f * P.stride + c] = T(U[f]);
}

// ---- per-kernel timing ----------------------------------------------------------------------
const char* kernel_class_name(int k) {
  static const char* names[K_NUM_CLASSES] = {
      "bc_fill_x", "bc_fill_y", "bc_fill_z", "sweep1_x", "sweep1_y", "sweep1_z",
      "sweep2_x", "sweep2_y", "sweep2_z", "update", "dt_final"};
  return (k >= 0 && k < K_NUM_CLASSES) ? names[k] : "";
}

hipEvent_t Profiler::take() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void Profiler::begin(int cls, hipStream_t s) {
  Pair p{cls, take(), take()};
  if (p.start) (void)hipEventRecord(p.start, s);
  pending.push_back(p);
}

void Profiler::end(hipStream_t s) {
  if (!pending.empty() && pending.back().stop) (void)hipEventRecord(pending.back().stop, s);
}

hipError_t Profiler::collect() {
  hipError_t err = hipSuccess;
  for (auto& p : pending) {
    float t = 0.f;
    if (p.start && p.stop) {
      hipError_t e = hipEventSynchronize(p.stop);
      if (e == hipSuccess) e = hipEventElapsedTime(&t, p.start, p.stop);
      if (e != hipSuccess) err = e;
    }
    ms[p.cls] += t;
    launches[p.cls] += 1;
    if (p.start) pool.push_back(p.start);
    if (p.stop) pool.push_back(p.stop);
  }
  pending.clear();
  return err;
}

void Profiler::reset() {
  for (auto& p : pending) {
    if (p.start) pool.push_back(p.start);
    if (p.stop) pool.push_back(p.stop);
  }
  pending.clear();
  for (int k = 0; k < K_NUM_CLASSES; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
}

Profiler::~Profiler() {
  reset();
  for (auto e : pool) (void)hipEventDestroy(e);
}

// ---- launch sizes and sequence ----------------------------------------------------------------
static inline long long cdiv(long long a, long long b) { return (a + b - 1) / b; }

long long pass_blocks(const GridParams& P, int pass) {
  const long long n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  const long long N0 = P.N[0], N1 = P.N[1], N2 = P.N[2];
  const long long nseg_x = cdiv(n0 + 1, XW);
  switch (pass) {
    case P_BC_X: return cdiv(2LL * NG * N1 * N2, kBlock);
    case P_BC_Y: return cdiv(2LL * NG * N0 * N2, kBlock);
    case P_BC_Z: return cdiv(2LL * NG * N0 * N1, kBlock);
    case P_S1_X: return cdiv(nseg_x * (n1 + 2) * (n2 + 2), kBlock / 64);
    case P_S1_Y: return cdiv((n0 + 2) * (n2 + 2), kBlock) * cdiv(n1 + 1, P.seg[1]);
    case P_S1_Z: return cdiv((n0 + 2) * (n1 + 2), kBlock) * cdiv(n2 + 1, P.seg[2]);
    case P_S2_X: return cdiv(nseg_x * n1 * n2, kBlock / 64);
    case P_S2_Y: return cdiv(n0 * n2, kBlock) * cdiv(n1 + 1, P.seg[1]);
    case P_S2_Z: return cdiv(n0 * n1, kBlock) * cdiv(n2 + 1, P.seg[2]);
    case P_UPDATE:
    case P_DT: return cdiv(n0 * n1 * n2, kBlock);
  }
  return 0;
}

#define TIMED(cls, launch)                            \
  do {                                                \
    if (prof && prof->timing) prof->begin(cls, stream); \
    launch;                                           \
    if (prof && prof->timing) prof->end(stream);        \
  } while (0)

template <typename T, bool HIST>
static void enqueue_step(const PlanView& v, bool device_dt, hipStream_t stream, Profiler* prof) {
  const int stride = v.ngrids + 1;
  auto tab = [&](int pass) { return LaunchTab{v.d_grids, v.d_start + pass * stride, v.ngrids}; };
  auto nblocks = [&](int pass) { return dim3((unsigned)v.h_start[pass * stride + v.ngrids]); };
  const dim3 B(kBlock);
  const dim3 gsmall((unsigned)cdiv(v.ngrids, kBlock));
  if (device_dt) hipLaunchKernelGGL(k_begin_step, gsmall, B, 0, stream, v.d_grids, v.ngrids);
  // a1: ghost fill x, then y, then z
  TIMED(K_BC_X,
        hipLaunchKernelGGL((k_bc_fill<T, 0>), nblocks(P_BC_X), B, 0, stream, tab(P_BC_X)));
  TIMED(K_BC_Y,
        hipLaunchKernelGGL((k_bc_fill<T, 1>), nblocks(P_BC_Y), B, 0, stream, tab(P_BC_Y)));
  TIMED(K_BC_Z,
        hipLaunchKernelGGL((k_bc_fill<T, 2>), nblocks(P_BC_Z), B, 0, stream, tab(P_BC_Z)));
  // stage 1 (a2-a5): F*, G*, H* on the extended transverse range
  TIMED(K_SWEEP1_X,
        hipLaunchKernelGGL((k_sweep_x<T, 1, HIST>), nblocks(P_S1_X), B, 0, stream, tab(P_S1_X)));
  TIMED(K_SWEEP1_Y,
        hipLaunchKernelGGL((k_sweep_march<T, 1, 1, HIST>), nblocks(P_S1_Y), B, 0, stream, tab(P_S1_Y)));
  TIMED(K_SWEEP1_Z,
        hipLaunchKernelGGL((k_sweep_march<T, 2, 1, HIST>), nblocks(P_S1_Z), B, 0, stream, tab(P_S1_Z)));
  // stage 2 (a2-a4 re-traced, a6-a7): F^{n+1/2}, G^{n+1/2}, H^{n+1/2} on the real faces
  TIMED(K_SWEEP2_X,
        hipLaunchKernelGGL((k_sweep_x<T, 2, HIST>), nblocks(P_S2_X), B, 0, stream, tab(P_S2_X)));
  TIMED(K_SWEEP2_Y,
        hipLaunchKernelGGL((k_sweep_march<T, 1, 2, HIST>), nblocks(P_S2_Y), B, 0, stream, tab(P_S2_Y)));
  TIMED(K_SWEEP2_Z,
        hipLaunchKernelGGL((k_sweep_march<T, 2, 2, HIST>), nblocks(P_S2_Z), B, 0, stream, tab(P_S2_Z)));
  // a8-a9
  TIMED(K_UPDATE, hipLaunchKernelGGL(k_update<T>, nblocks(P_UPDATE), B, 0, stream, tab(P_UPDATE)));
  TIMED(K_DT_FINAL,
        hipLaunchKernelGGL(k_dt_final, dim3(v.ngrids), dim3(1024), 0, stream, v.d_grids));
  hipLaunchKernelGGL(k_end_step, gsmall, B, 0, stream, v.d_grids, v.ngrids);
}

hipError_t launch_step(const PlanView& v, bool device_dt, hipStream_t stream, Profiler* prof) {
  const bool hist = prof && prof->hist;
  if (v.prec == 0) {
    if (hist)
      enqueue_step<double, true>(v, device_dt, stream, prof);
    else
      enqueue_step<double, false>(v, device_dt, stream, prof);
  } else {
    if (hist)
      enqueue_step<float, true>(v, device_dt, stream, prof);
    else
      enqueue_step<float, false>(v, device_dt, stream, prof);
  }
  return hipGetLastError();
}

template <typename T>
static void enqueue_dt(const PlanView& v, hipStream_t stream) {
  const int stride = v.ngrids + 1;
  const LaunchTab tab{v.d_grids, v.d_start + P_DT * stride, v.ngrids};
  hipLaunchKernelGGL(k_dt<T>, dim3((unsigned)v.h_start[P_DT * stride + v.ngrids]), dim3(kBlock), 0,
                     stream, tab);
  hipLaunchKernelGGL(k_dt_final, dim3(v.ngrids), dim3(1024), 0, stream, v.d_grids);
}

hipError_t launch_dt(const PlanView& v, hipStream_t stream) {
  if (v.prec == 0)
    enqueue_dt<double>(v, stream);
  else
    enqueue_dt<float>(v, stream);
  return hipGetLastError();
}

hipError_t launch_set_dt(DevScalars* s, double dt, hipStream_t stream) {
  hipLaunchKernelGGL(k_set_dt, dim3(1), dim3(1), 0, stream, s, dt);
  return hipGetLastError();
}

hipError_t launch_set_end(DevScalars* s, double t_end, long long steps_left, hipStream_t stream) {
  hipLaunchKernelGGL(k_set_end, dim3(1), dim3(1), 0, stream, s, t_end, steps_left);
  return hipGetLastError();
}

hipError_t launch_gather_scalars(DevScalars* const* src, int n, DevScalars* out,
                                 hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_scalars, dim3((unsigned)cdiv(n, 64)), dim3(64), 0, stream, src, n,
                     out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_totals(const T* u, const GridParams& P, double* part, int nblocks, double* out,
                         hipStream_t stream) {
  hipLaunchKernelGGL(k_totals_partial<T>, dim3(nblocks), dim3(256), 0, stream, u, P, part);
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(64), 0, stream, part, nblocks, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scatter(const T* packed, T* u, const GridParams& P, hipStream_t stream) {
  const long long real = (long long)P.n[0] * P.n[1] * P.n[2];
  hipLaunchKernelGGL(k_scatter<T>, dim3((unsigned)cdiv(real, 256)), dim3(256), 0, stream, packed,
                     u, P);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const T* u, T* packed, const GridParams& P, hipStream_t stream) {
  const long long real = (long long)P.n[0] * P.n[1] * P.n[2];
  hipLaunchKernelGGL(k_gather<T>, dim3((unsigned)cdiv(real, 256)), dim3(256), 0, stream, u,
                     packed, P);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prim_to_cons(const double* packed, T* u, const GridParams& P, hipStream_t stream) {
  const long long real = (long long)P.n[0] * P.n[1] * P.n[2];
  hipLaunchKernelGGL(k_prim_to_cons<T>, dim3((unsigned)cdiv(real, 256)), dim3(256), 0, stream,
                     packed, u, P);
  return hipGetLastError();
}

#define CTU_INSTANTIATE(T)                                                                        \
  template hipError_t launch_totals<T>(const T*, const GridParams&, double*, int, double*,      \
                                       hipStream_t);                                             \
  template hipError_t launch_scatter<T>(const T*, T*, const GridParams&, hipStream_t);          \
  template hipError_t launch_gather<T>(const T*, T*, const GridParams&, hipStream_t);           \
  template hipError_t launch_prim_to_cons<T>(const double*, T*, const GridParams&, hipStream_t);

CTU_INSTANTIATE(double)
CTU_INSTANTIATE(float)

}  // namespace ctu
