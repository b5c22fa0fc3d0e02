// ctu_kernels.hip -- HIP kernels (gfx950) of one CTU timestep, Sec. 2.1 of Schneider &
// Robertson 2015: ghost fill, per-direction PPMC trace and first Riemann solve, transverse
// correction and second Riemann solve, conservative update fused with the CFL reduction.
//
// Data layout: structure of arrays over the allocated box, x fastest, three ghost layers
// (see ctu.h).  Interface arrays store face c+1/2 at the index of cell c.  Threads run along
// x, so every global access of a wavefront is a contiguous run along x.  Each launch serves a
// table of grids (ctu_kernels.hpp); a block finds its grid and local block index first.
#include "ctu_common.hpp"

namespace ctu {

// ---- step bookkeeping ----------------------------------------------------------------------
__global__ void k_set_dt(DevScalars* s, double dt) { s->dt = dt; }

__global__ void k_set_end(DevScalars* s, double t_end, long long steps_left) {
  s->t_end = t_end;
  s->steps_left = steps_left;
}

// Device-side time step of every grid: C0 * (min CFL bound), clipped to t_end - t; a grid
// whose step budget is used up, or whose state was flagged non-physical, takes dt = 0 (its
// passes become no-ops).
// Device-side time step of a grid (Sec. 3.5): dt = min(C0 x bound, t_end - t) from the CFL
// bound of the current state, or 0 once the step budget is used or the state was flagged
// non-physical (the grid then takes no-op steps).
__device__ __forceinline__ double device_step_dt(const GridDesc& G) {
  const DevScalars* s = G.s;
  const double bound = __longlong_as_double((long long)s->dt_next_bits);
  double dt = fmin(G.P.cfl * bound, s->t_end - s->t);
  if (s->steps_left <= 0 || (s->flags & 3u)) dt = 0.0;
  return dt;
}

// Copies of the scalars of n grids into one array (one read-back for a whole batch).
__global__ void k_gather_scalars(DevScalars* const* __restrict__ src, int n, DevScalars* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = *src[i];
}

// ---- a1: ghost fill (Sec. 3.1) ------------------------------------------------------------
// Source index along one axis of a cell index q of the allocated box (q itself for a real
// cell): periodic one period away, outflow the edge cell, reflect the mirror image across the
// wall (n >= ng is validated); *flip is set for a reflected ghost.
__device__ __forceinline__ int ghost_source(int q, int n, int bc_lo, int bc_hi, bool* flip) {
  if (q >= 0 && q < n) return q;
  const int bc = q < 0 ? bc_lo : bc_hi;
  if (bc == 0) {
    int s = q % n;
    return s < 0 ? s + n : s;
  }
  if (bc == 1) return q < 0 ? 0 : n - 1;
  *flip = true;
  return q < 0 ? -1 - q : 2 * n - 1 - q;
}

// Every ghost cell in one pass, copied from its source real cell with the momentum component
// of every reflecting axis negated: the composition of the three one-axis fills (x over the
// whole extent of y and z, then y, then z), which is what they leave in edges and corners, so
// one pass gives the same values.  The ghost cells are taken as three disjoint slabs: x ghosts
// over all (j, k); y ghosts over real i and all k; z ghosts over real i and j.
// The pass is the first of a step: with begin != 0 it also takes the device-side time step.
// Every block computes it from the grid's scalars and the grid's first block stores it for the
// passes after this one (nothing in this launch reads it back).
template <typename T>
__global__ __launch_bounds__(256) void k_bc_fill(LaunchTab tab, int begin) {
  const BlockRef r = block_ref(tab);
  const GridParams P = r.G->P;
  double dt;
  if (begin) {
    dt = device_step_dt(*r.G);
    if (r.lb == 0 && threadIdx.x == 0) r.G->s->dt = dt;
  } else {
    dt = r.G->s->dt;
  }
  if (!(dt > 0.0)) return;
  GLOBAL T* __restrict__ u = (GLOBAL T*)r.G->u;
  const int ng = P.ng;  // ghost layers of this grid
  const long long tid = r.lb * blockDim.x + threadIdx.x;
  const long long sx = 2LL * ng * P.N[1] * P.N[2];
  const long long sy = (long long)P.n[0] * 2 * ng * P.N[2];
  const long long sz = (long long)P.n[0] * P.n[1] * 2 * ng;
  int i, j, k;
  if (tid < sx) {  // x ghosts, ghost layer fastest
    const int layer = (int)(tid % (2 * ng));
    const long long q = tid / (2 * ng);
    i = layer < ng ? layer - ng : P.n[0] + (layer - ng);
    j = (int)(q % P.N[1]) - ng;
    k = (int)(q / P.N[1]) - ng;
  } else if (tid < sx + sy) {  // y ghosts of real i, i fastest
    const long long t = tid - sx;
    i = (int)(t % P.n[0]);
    const long long q = t / P.n[0];
    const int layer = (int)(q % (2 * ng));
    j = layer < ng ? layer - ng : P.n[1] + (layer - ng);
    k = (int)(q / (2 * ng)) - ng;
  } else if (tid < sx + sy + sz) {  // z ghosts of real i and j, i fastest
    const long long t = tid - sx - sy;
    i = (int)(t % P.n[0]);
    const long long q = t / P.n[0];
    j = (int)(q % P.n[1]);
    const int layer = (int)(q / P.n[1]);
    k = layer < ng ? layer - ng : P.n[2] + (layer - ng);
  } else {
    return;
  }
  bool fx = false, fy = false, fz = false;
  const int si = ghost_source(i, P.n[0], r.G->bc[0], r.G->bc[1], &fx);
  const int sj = ghost_source(j, P.n[1], r.G->bc[2], r.G->bc[3], &fy);
  const int sk = ghost_source(k, P.n[2], r.G->bc[4], r.G->bc[5], &fz);
  const long long d = cell_index(P, i, j, k);
  const long long sidx = cell_index(P, si, sj, sk);
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const T v = u[f * P.stride + sidx];
    const bool neg = (f == 1 && fx) || (f == 2 && fy) || (f == 3 && fz);
    u[f * P.stride + d] = neg ? -v : v;
  }
}


// ---- PPMP flattening and steepening coefficients (App. A.4) ----------------------------------
// For each cell of the box [-1 - ext, n + ext]^3 (every cell the sweeps trace) and each axis
// d: the shock-flattening coefficient F_d and the contact-steepening coefficient eta_d, from
// the densities, pressures and normal velocities of the cells within three along d.  Both
// depend on u^n only, so one pass per axis before the first stage serves both stages.  The
// steepening test reads an inflection of the density (second differences of opposite sign on
// the two sides of the cell, as in CW84); the 1/(6 dx^2) of the second differences cancels in
// eta~ and does not change the sign test, so it is left out.
template <typename T>
__device__ __forceinline__ T flat_tilde(T pm, T pmm, T pp, T ppp, T um, T up) {
  const T dp = pp - pm;  // p_{i+1} - p_{i-1}
  if (tfabs(dp) < tmin(pp, pm) * (T(1) / T(3))) return T(0);  // weak jump
  if (up - um > T(0)) return T(0);                               // expansion
  const T S = dp / (ppp - pmm);  // over p_{i+2} - p_{i-2}
  return tmax(T(0), tmin(T(1), T(10) * (S - T(0.75))));
}

// Steepening coefficient of cell i from rho_{i-2..i+2} and p_{i-1}, p_{i+1}.
template <typename T>
__device__ __forceinline__ T steep_eta(T rmm, T rm, T r0, T rp, T rpp, T pm, T pp, T gamma) {
  const T dr = tfabs(rp - rm) / tmin(rp, rm);
  const T dpr = tfabs(pp - pm) / tmin(pp, pm);
  if (!(dr > T(0.01) && dpr < T(0.1) * gamma * dr)) return T(0);
  const T d2m = r0 - T(2) * rm + rmm;
  const T d2p = rpp - T(2) * rp + r0;
  if (!(d2m * d2p < T(0))) return T(0);
  const T et = -(d2p - d2m) / (T(6) * (rp - rm));
  return tmax(T(0), tmin(T(20) * et - T(1), T(1)));
}

// Density, pressure (floored) and the velocity along axis d of one cell.
template <typename T, int DIR>
__device__ __forceinline__ void coef_prim(const GLOBAL T* __restrict__ u, long long stride,
                                          long long id, T gm1, T pf, T& rho, T& p, T& un) {
  const T r0 = u[id], m1 = u[stride + id], m2 = u[2 * stride + id];
  const T m3 = u[3 * stride + id], E = u[4 * stride + id];
  const T ir = rcp_nr(r0);
  T pr = gm1 * (E - T(0.5) * (m1 * m1 + m2 * m2 + m3 * m3) * ir);
  if (!(pr >= pf)) pr = pf;
  rho = r0;
  p = pr;
  un = (DIR == 0 ? m1 : (DIR == 1 ? m2 : m3)) * ir;
}

// Coefficients of the centre cell of a seven-cell window (cells c-3..c+3).
template <typename T>
__device__ __forceinline__ void ppmp_coefs(const T r[7], const T p[7], const T un[7], T gamma,
                                           T& flat, T& eta) {
  const T Fm = flat_tilde(p[1], p[0], p[3], p[4], un[1], un[3]);  // cell c-1
  const T F0 = flat_tilde(p[2], p[1], p[4], p[5], un[2], un[4]);  // cell c
  const T Fp = flat_tilde(p[3], p[2], p[5], p[6], un[3], un[5]);  // cell c+1
  flat = (p[4] - p[2] < T(0)) ? tmax(F0, Fp) : tmax(F0, Fm);
  eta = steep_eta(r[1], r[2], r[3], r[4], r[5], p[2], p[4], gamma);
}

// Axis x: the rows of one z-plane (over [-1 - ext, n_y + ext]) lie back to back and are
// treated as one flattened line; lane l holds position XW w - 3 + l and reads its neighbours
// within three by lane shuffles; lanes 3..60 store their cell's coefficients.  The stencil of
// every cell that needs coefficients lies in its own row.
template <typename T>
__global__ __launch_bounds__(256) void k_ppmp_coef_x(LaunchTab tab) {
  const BlockRef r = block_ref(tab);
  const GridParams P = r.G->P;
  if (!(r.G->s->dt > 0.0)) return;
  const int e = 1 + P.ext;  // cells [-e, n + e - 1] per axis
  const int lane = threadIdx.x & 63;
  const long long task = r.lb * (kBlock / 64) + wave_in_block();
  const long long plen = (long long)(P.n[1] + 2 * e) * P.N[0];
  const long long nw = (plen + XW - 1) / XW;
  if (task >= nw * (P.n[2] + 2 * e)) return;  // whole wavefront exits together
  const int k = (int)(task / nw) - e;
  const long long pos0 = (task % nw) * XW - 3;  // position of lane 0
  const long long pos = pos0 + lane;
  const bool in_line = pos >= 0 && pos < plen;
  const int c = in_line ? wave_row_pos(pos0, lane, P.N[0]) - P.ng : -P.ng - 1;
  const long long id = cell_index(P, -P.ng, -e, k) + pos;
  const GLOBAL T* __restrict__ u = (const GLOBAL T*)r.G->u;
  T rho = T(1), p = T(1), un = T(0);
  if (in_line) coef_prim<T, 0>(u, P.stride, id, T(P.gm1), T(P.p_floor), rho, p, un);
  T rw[7], pw[7], uw[7];
#pragma unroll
  for (int s = 0; s < 7; ++s) {
    const int src = min(max(lane + s - 3, 0), 63);
    rw[s] = __shfl(rho, src, 64);
    pw[s] = __shfl(p, src, 64);
    uw[s] = __shfl(un, src, 64);
  }
  if (lane >= 3 && lane <= 60 && in_line && c >= -e && c < P.n[0] + e) {
    T flat, eta;
    ppmp_coefs(rw, pw, uw, T(P.gamma), flat, eta);
    GLOBAL T* __restrict__ coef = (GLOBAL T*)r.G->coef;
    coef[id] = flat;
    coef[P.stride + id] = eta;
  }
}

// Axes y and z: each thread marches one column along D over a segment of kCoefSeg cells with a
// seven-cell window, reading each cell once.  Block layout per grid: (plane block, segment).
constexpr int kCoefSeg = 8;

template <typename T, int D>
__global__ __launch_bounds__(256) void k_ppmp_coef_march(LaunchTab tab) {
  const BlockRef r = block_ref(tab);
  const GridParams P = r.G->P;
  if (!(r.G->s->dt > 0.0)) return;
  constexpr int B = (D == 1) ? 2 : 1;  // the transverse axis other than x
  const int e = 1 + P.ext;
  const int ea = P.n[0] + 2 * e, eb = P.n[B] + 2 * e, nd = P.n[D] + 2 * e;
  const long long nbx = ((long long)ea * eb + kBlock - 1) / kBlock;
  const long long nseg = (nd + kCoefSeg - 1) / kCoefSeg;
  if (r.lb >= nbx * nseg) return;
  const long long tid = (r.lb % nbx) * kBlock + threadIdx.x;
  if (tid >= (long long)ea * eb) return;
  const int i = (int)(tid % ea) - e;
  const int o = (int)(tid / ea) - e;
  const int f0 = (int)(r.lb / nbx) * kCoefSeg - e;
  const int f1 = min(f0 + kCoefSeg, nd - e);
  const long long sd = D == 1 ? (long long)P.N[0] : (long long)P.N[0] * P.N[1];
  const long long c0 = D == 1 ? cell_index(P, i, 0, o) : cell_index(P, i, o, 0);
  const GLOBAL T* __restrict__ u = (const GLOBAL T*)r.G->u;
  GLOBAL T* __restrict__ coef = (GLOBAL T*)r.G->coef + 2 * D * P.stride;
  const T gm1 = T(P.gm1), pf = T(P.p_floor), gamma = T(P.gamma);
  T rw[7], pw[7], uw[7];
#pragma unroll
  for (int s = 1; s < 7; ++s)  // cells f0-3 .. f0+2 into slots 0..5 (shifted below)
    coef_prim<T, D>(u, P.stride, c0 + (long long)(f0 + s - 4) * sd, gm1, pf, rw[s], pw[s], uw[s]);
  for (int c = f0; c < f1; ++c) {
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      rw[s] = rw[s + 1];
      pw[s] = pw[s + 1];
      uw[s] = uw[s + 1];
    }
    coef_prim<T, D>(u, P.stride, c0 + (long long)(c + 3) * sd, gm1, pf, rw[6], pw[6], uw[6]);
    T flat, eta;
    ppmp_coefs(rw, pw, uw, gamma, flat, eta);
    const long long id = c0 + (long long)c * sd;
    coef[id] = flat;
    coef[P.stride + id] = eta;
  }
}


// ---- a8-a9: conservative update and CFL reduction ------------------------------------------
// CFL bound of the current state with the partial layout of the fused update: one wavefront
// per x-row of real cells, kBlock/64 rows per block.
template <typename T>
__global__ __launch_bounds__(256) void k_dt(LaunchTab tab) {
  const BlockRef r = block_ref(tab);
  const GridParams P = r.G->P;
  constexpr int kWaves = kBlock / 64;
  const long long ngy = (P.n[1] + P.xrows - 1) / P.xrows;
  const long long ngroups = ngy * P.n[2];
  if (r.lb * kWaves >= ngroups) return;  // whole block idle
  const GLOBAL T* __restrict__ u = (const GLOBAL T*)r.G->u;
  const long long grp = r.lb * kWaves + wave_in_block();
  double bound = INFINITY;
  if (grp < ngroups) {
    const int j0 = (int)(grp % ngy) * P.xrows;
    const int k = (int)(grp / ngy);
    for (int j = j0; j < min(j0 + P.xrows, P.n[1]); ++j) {
      const long long base = cell_index(P, 0, j, k);
      for (int i = threadIdx.x & 63; i < P.n[0]; i += 64) {
        T U[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) U[f] = u[f * P.stride + base + i];
        bound = fmin(bound, cell_dt_bound(U, P));
      }
    }
  }
  block_min_store(bound, (GLOBAL double*)r.G->part, r.lb);
}

// Minimum of each grid's block partials into its dt_next_bits: block g reduces grid g.
// end_step != 0 (the last pass of a step): also account the step taken, t += dt, one step more
// and one less in the budget, unless it was a no-op step.
__global__ __launch_bounds__(1024) void k_dt_final(const GridDesc* __restrict__ grids,
                                                   int end_step) {
  const GridDesc& G = grids[blockIdx.x];
  const long long nblocks = update_blocks(G.P);
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
    if (lane == 0) {
      DevScalars* s = G.s;
      if (end_step && s->dt > 0.0) {
        s->t += s->dt;
        s->steps += 1;
        s->steps_left -= 1;
      }
      s->dt_next_bits = (unsigned long long)__double_as_longlong(v);
    }
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
      "bc_fill", "ppmp_coef", "sweep1_x", "sweep1_y", "sweep1_z",
      "hcorr_eta", "sweep2_y", "sweep2_z", "sweep2_x_update", "dt_final"};
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
  switch (pass) {
    case P_BC: return cdiv(2LL * P.ng * (N1 * N2 + n0 * N2 + n0 * n1), kBlock);
    case P_COEF_X: {
      const long long e = 2 + 2 * P.ext;  // cells [-1 - ext, n + ext] per axis
      return P.recon == 1 ? cdiv(cdiv((n1 + e) * N0, XW) * (n2 + e), kBlock / 64) : 0;
    }
    case P_COEF_Y: {
      const long long e = 2 + 2 * P.ext;
      return P.recon == 1 ? cdiv((n0 + e) * (n2 + e), kBlock) * cdiv(n1 + e, kCoefSeg) : 0;
    }
    case P_COEF_Z: {
      const long long e = 2 + 2 * P.ext;
      return P.recon == 1 ? cdiv((n0 + e) * (n1 + e), kBlock) * cdiv(n2 + e, kCoefSeg) : 0;
    }
    case P_S1_X: return cdiv(cdiv((n1 + 2) * N0, XW) * (n2 + 2), P.xchunks * (kBlock / 64));
    case P_S1_Y: return cdiv((n0 + 2) * (n2 + 2), kBlock) * cdiv(n1 + 2 * P.ext, P.seg[1]);
    case P_S1_Z: return cdiv((n0 + 2) * (n1 + 2), kBlock) * cdiv(n2 + 2 * P.ext, P.seg[2]);
    case P_ETA_X: return P.ext ? cdiv(cdiv((n1 + 2) * N0, XW) * (n2 + 2), kBlock / 64) : 0;
    case P_S2_Y:  // with the H correction over the first stage's transverse range (eta)
      return P.ext ? cdiv((n0 + 2) * (n2 + 2), kBlock) * cdiv(n1, P.seg[1])
                   : cdiv(n0 * n2, kBlock) * cdiv(n1, P.seg[1]);
    case P_ETA_Z: return P.ext ? cdiv((n0 + 2) * (n1 + 2), kBlock) * cdiv(n2, P.seg[2]) : 0;
    case P_S2_Z: return cdiv(n0 * n1, kBlock) * cdiv(n2, P.seg[2]);
    case P_S2_X:
    case P_DT: return update_blocks(P);
  }
  return 0;
}

template <typename T, int D>
void launch_ppmp_coef(const PlanView& v, hipStream_t stream) {
  const int stride = v.ngrids + 1;
  const int pass = D == 0 ? P_COEF_X : (D == 1 ? P_COEF_Y : P_COEF_Z);
  const LaunchTab tab{v.d_grids, v.d_start + pass * stride, v.ngrids};
  const dim3 nb((unsigned)v.h_start[pass * stride + v.ngrids]);
  if constexpr (D == 0)
    hipLaunchKernelGGL((k_ppmp_coef_x<T>), nb, dim3(kBlock), 0, stream, tab);
  else
    hipLaunchKernelGGL((k_ppmp_coef_march<T, D>), nb, dim3(kBlock), 0, stream, tab);
}
template void launch_ppmp_coef<double, 0>(const PlanView&, hipStream_t);
template void launch_ppmp_coef<double, 1>(const PlanView&, hipStream_t);
template void launch_ppmp_coef<double, 2>(const PlanView&, hipStream_t);
template void launch_ppmp_coef<float, 0>(const PlanView&, hipStream_t);
template void launch_ppmp_coef<float, 1>(const PlanView&, hipStream_t);
template void launch_ppmp_coef<float, 2>(const PlanView&, hipStream_t);

template <typename T, int R>
static hipError_t sweeps_r(const PlanView& v, int stage, hipStream_t stream, Profiler* prof) {
  switch (v.gclass) {
    case 3: return launch_sweeps<T, 3, R>(v, stage, stream, prof);
    case 5: return launch_sweeps<T, 5, R>(v, stage, stream, prof);
    case kRoe: return launch_sweeps<T, kRoe, R>(v, stage, stream, prof);
    case kRoeH: return launch_sweeps<T, kRoeH, R>(v, stage, stream, prof);
    default: return launch_sweeps<T, 0, R>(v, stage, stream, prof);
  }
}

template <typename T>
static hipError_t sweeps(const PlanView& v, int stage, hipStream_t stream, Profiler* prof) {
  return v.recon == 1 ? sweeps_r<T, 1>(v, stage, stream, prof)
                      : sweeps_r<T, 0>(v, stage, stream, prof);
}

template <typename T>
static hipError_t enqueue_step(const PlanView& v, bool device_dt, hipStream_t stream,
                               Profiler* prof) {
  const int stride = v.ngrids + 1;
  auto tab = [&](int pass) { return LaunchTab{v.d_grids, v.d_start + pass * stride, v.ngrids}; };
  auto nblocks = [&](int pass) { return dim3((unsigned)v.h_start[pass * stride + v.ngrids]); };
  const dim3 B(kBlock);
  // a1: ghost fill (which takes the device-side time step when asked)
  CTU_TIMED(K_BC, hipLaunchKernelGGL((k_bc_fill<T>), nblocks(P_BC), B, 0, stream, tab(P_BC),
                                     device_dt ? 1 : 0));
  // (in the overlapped schedule the first-stage sweeps launch the PPMP coefficient passes,
  // each beside other work)
  if (v.recon == 1 && !overlapped(v, prof)) {
    CTU_TIMED(K_PPMP_COEF, (launch_ppmp_coef<T, 0>(v, stream)));
    CTU_TIMED(K_PPMP_COEF, (launch_ppmp_coef<T, 1>(v, stream)));
    CTU_TIMED(K_PPMP_COEF, (launch_ppmp_coef<T, 2>(v, stream)));
  }
  // stage 1 (a2-a5), then stage 2 (a2-a4 re-traced, a6-a7) with the update (a8) fused into
  // its last sweep
  hipError_t e = sweeps<T>(v, 1, stream, prof);
  if (e == hipSuccess) e = sweeps<T>(v, 2, stream, prof);
  if (e != hipSuccess) return e;
  // a9: minimum of the CFL partials that the fused update wrote, and the step's accounting
  CTU_TIMED(K_DT_FINAL,
            hipLaunchKernelGGL(k_dt_final, dim3(v.ngrids), dim3(1024), 0, stream, v.d_grids, 1));
  return hipGetLastError();
}

hipError_t launch_step(const PlanView& v, bool device_dt, hipStream_t stream, Profiler* prof) {
  return v.prec == 0 ? enqueue_step<double>(v, device_dt, stream, prof)
                     : enqueue_step<float>(v, device_dt, stream, prof);
}

template <typename T>
static void enqueue_dt(const PlanView& v, hipStream_t stream) {
  const int stride = v.ngrids + 1;
  const LaunchTab tab{v.d_grids, v.d_start + P_DT * stride, v.ngrids};
  hipLaunchKernelGGL(k_dt<T>, dim3((unsigned)v.h_start[P_DT * stride + v.ngrids]), dim3(kBlock), 0,
                     stream, tab);
  hipLaunchKernelGGL(k_dt_final, dim3(v.ngrids), dim3(1024), 0, stream, v.d_grids, 0);
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
