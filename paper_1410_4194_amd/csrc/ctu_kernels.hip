// ctu_kernels.hip -- HIP kernels (gfx950) of one CTU timestep, Sec. 2.1 of Schneider &
// Robertson 2015: ghost fill, per-direction PPMC trace and first Riemann solve, transverse
// correction and second Riemann solve, conservative update fused with the CFL reduction.
//
// Data layout: structure of arrays over the allocated box, x fastest, three ghost layers
// (see ctu.h).  Interface arrays store face c+1/2 at the index of cell c.  All kernels are
// one thread per cell or face with x as the fastest thread index, so every global access
// of a wavefront is a contiguous run along x.
#include "ctu_kernels.hpp"

namespace ctu {

// Rotation of momentum slots for a sweep along D (cyclic): rotated slot s <- global rot(D,s).
template <int D>
__device__ __forceinline__ int rot(int s) {
  if (s == 0 || s == 4) return s;
  return 1 + ((s - 1 + D) % 3);
}

__device__ __forceinline__ double ordered_min_to_double(unsigned long long b) {
  return __longlong_as_double((long long)b);
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

// Block-wide minimum folded into *bits with an exact, order-free atomicMin on the IEEE bit
// pattern (monotone for non-negative doubles).  Every thread of the block must call it.
__device__ void block_min_atomic(double v, unsigned long long* bits) {
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
    if (lane == 0 && m < INFINITY) atomicMin(bits, (unsigned long long)__double_as_longlong(m));
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

// ---- step bookkeeping ----------------------------------------------------------------------
__global__ void k_set_dt(DevScalars* s, double dt) {
  s->dt = dt;
  s->dt_next_bits = 0x7ff0000000000000ull;  // +inf
}

// Device-side time step for ctu_advance: C0 * (min CFL bound), clipped to t_end - t.
__global__ void k_begin_step(DevScalars* s, double cfl, double t_end) {
  double bound = ordered_min_to_double(s->dt_next_bits);
  double dt = fmin(cfl * bound, t_end - s->t);
  s->dt = dt;
  if (dt > 0.0) s->dt_next_bits = 0x7ff0000000000000ull;
}

__global__ void k_end_step(DevScalars* s) {
  if (s->dt > 0.0) {
    s->t += s->dt;
    s->steps += 1;
  }
}

__global__ void k_reset_dt_bits(DevScalars* s) { s->dt_next_bits = 0x7ff0000000000000ull; }

// ---- a1: ghost fill (Sec. 3.1) ------------------------------------------------------------
// Axis `axis` ghosts over the full extent of the other two axes (ghosts included), so
// running x, then y, then z fills edges and corners consistently.
template <typename T>
__global__ void k_bc_fill(T* __restrict__ u, GridParams P, int axis, int bc_lo, int bc_hi) {
  const int n = P.n[axis];
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k, layer;
  if (axis == 0) {
    long long total = 2LL * NG * P.N[1] * P.N[2];
    if (tid >= total) return;
    layer = (int)(tid % (2 * NG));
    long long r = tid / (2 * NG);
    j = (int)(r % P.N[1]) - NG;
    k = (int)(r / P.N[1]) - NG;
    i = 0;
  } else if (axis == 1) {
    long long total = 2LL * NG * P.N[0] * P.N[2];
    if (tid >= total) return;
    i = (int)(tid % P.N[0]) - NG;
    long long r = tid / P.N[0];
    layer = (int)(r % (2 * NG));
    k = (int)(r / (2 * NG)) - NG;
    j = 0;
  } else {
    long long total = 2LL * NG * P.N[0] * P.N[1];
    if (tid >= total) return;
    i = (int)(tid % P.N[0]) - NG;
    long long r = tid / P.N[0];
    j = (int)(r % P.N[1]) - NG;
    layer = (int)(r / P.N[1]);
    k = 0;
  }
  const int q = layer < NG ? layer - NG : n + (layer - NG);
  const int bc = layer < NG ? bc_lo : bc_hi;
  int src;
  if (bc == 0) {
    src = q % n;
    if (src < 0) src += n;
  } else {
    src = q < 0 ? 0 : n - 1;
  }
  int dst_pos[3] = {i, j, k};
  int src_pos[3] = {i, j, k};
  dst_pos[axis] = q;
  src_pos[axis] = src;
  const long long d = cell_index(P, dst_pos[0], dst_pos[1], dst_pos[2]);
  const long long s = cell_index(P, src_pos[0], src_pos[1], src_pos[2]);
#pragma unroll
  for (int f = 0; f < 5; ++f) u[f * P.stride + d] = u[f * P.stride + s];
}

// ---- a2-a4: primitives, PPMC and tracing per cell, along D -------------------------------
// One thread per cell of the extended box [-1, n+1)^3.  Writes the conserved traced states
// of the cell's two faces (global component order): ustar[0..4] = U*_L (left face),
// ustar[5..9] = U*_R (right face).
template <typename T, int D>
__global__ void k_trace(const T* __restrict__ u, T* __restrict__ ustar, GridParams P,
                        const DevScalars* __restrict__ s) {
  const double dt = s->dt;
  if (!(dt > 0.0)) return;
  const int ex = P.n[0] + 2, ey = P.n[1] + 2, ez = P.n[2] + 2;
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (long long)ex * ey * ez) return;
  const int i = (int)(tid % ex) - 1;
  const int j = (int)((tid / ex) % ey) - 1;
  const int k = (int)(tid / ((long long)ex * ey)) - 1;
  const long long c = cell_index(P, i, j, k);
  long long step = D == 0 ? 1 : (D == 1 ? (long long)P.N[0] : (long long)P.N[0] * P.N[1]);
  const T gm1 = T(P.gm1), pf = T(P.p_floor);
  T w[5][5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const long long id = c + (m - 2) * step;
    T U[5], Ur[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) U[f] = u[f * P.stride + id];
#pragma unroll
    for (int sl = 0; sl < 5; ++sl) Ur[sl] = U[rot<D>(sl)];
    cons_to_prim(Ur, gm1, pf, w[m]);
  }
  T WsL[5], WsR[5], UsL[5], UsR[5];
  ppmc(w, T(dt / P.dx[D]), T(P.gamma), WsL, WsR);
  prim_to_cons(WsL, gm1, UsL);
  prim_to_cons(WsR, gm1, UsR);
#pragma unroll
  for (int sl = 0; sl < 5; ++sl) {
    ustar[rot<D>(sl) * P.stride + c] = UsL[sl];
    ustar[(5 + rot<D>(sl)) * P.stride + c] = UsR[sl];
  }
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

// ---- a5: first Riemann solve on D-faces ----------------------------------------------------
// Faces c+1/2 for c in [-1, n_D - 1] along D and [-1, n_t] across.  The left input is the
// right-face state of cell c, the right input the left-face state of cell c+1.
template <typename T, int D>
__global__ void k_riemann1(const T* __restrict__ ustar, T* __restrict__ fstar, GridParams P,
                           DevScalars* __restrict__ s) {
  if (!(s->dt > 0.0)) return;
  const int e0 = P.n[0] + (D == 0 ? 1 : 2);
  const int e1 = P.n[1] + (D == 1 ? 1 : 2);
  const int e2 = P.n[2] + (D == 2 ? 1 : 2);
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (long long)e0 * e1 * e2) return;
  const int i = (int)(tid % e0) - 1;
  const int j = (int)((tid / e0) % e1) - 1;
  const int k = (int)(tid / ((long long)e0 * e1)) - 1;
  const long long c = cell_index(P, i, j, k);
  const long long step = D == 0 ? 1 : (D == 1 ? (long long)P.N[0] : (long long)P.N[0] * P.N[1]);
  T UL[5], UR[5], F[5];
#pragma unroll
  for (int sl = 0; sl < 5; ++sl) {
    UL[sl] = ustar[(5 + rot<D>(sl)) * P.stride + c];
    UR[sl] = ustar[rot<D>(sl) * P.stride + c + step];
  }
  RiemannCounts cnt{0u, 0u};
  exact_flux(UL, UR, P, F, cnt);
  flush_counts(cnt, s);
#pragma unroll
  for (int sl = 0; sl < 5; ++sl) fstar[rot<D>(sl) * P.stride + c] = F[sl];
}

// ---- a6-a7: transverse correction and second Riemann solve on D-faces --------------------
// Faces c+1/2 for c in [-1, n_D - 1] along D and the real range across (eq.
// transverse_evolution, cyclic order: x uses y then z, y uses z then x, z uses x then y).
template <typename T, int D>
__global__ void k_riemann2(const T* __restrict__ ustar, const T* __restrict__ fstar_all,
                           T* __restrict__ fhalf, GridParams P, DevScalars* __restrict__ s,
                           long long fstar_dir_stride) {
  const double dt = s->dt;
  if (!(dt > 0.0)) return;
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const int e0 = P.n[0] + (D == 0 ? 1 : 0);
  const int e1 = P.n[1] + (D == 1 ? 1 : 0);
  const int e2 = P.n[2] + (D == 2 ? 1 : 0);
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (long long)e0 * e1 * e2) return;
  const int i = (int)(tid % e0) - (D == 0 ? 1 : 0);
  const int j = (int)((tid / e0) % e1) - (D == 1 ? 1 : 0);
  const int k = (int)(tid / ((long long)e0 * e1)) - (D == 2 ? 1 : 0);
  const long long st[3] = {1, (long long)P.N[0], (long long)P.N[0] * P.N[1]};
  const long long cl = cell_index(P, i, j, k);
  const long long cr = cl + st[D];
  const T* F1 = fstar_all + T1 * fstar_dir_stride;
  const T* F2 = fstar_all + T2 * fstar_dir_stride;
  const T h1 = T(0.5 * dt / P.dx[T1]);
  const T h2 = T(0.5 * dt / P.dx[T2]);
  T Uh[2][5];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const long long cc = side == 0 ? cl : cr;
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      T us = side == 0 ? ustar[(5 + f) * P.stride + cc] : ustar[f * P.stride + cc];
      T d1 = F1[f * P.stride + cc - st[T1]] - F1[f * P.stride + cc];
      T d2 = F2[f * P.stride + cc - st[T2]] - F2[f * P.stride + cc];
      Uh[side][f] = us + h1 * d1 + h2 * d2;
    }
  }
  T UL[5], UR[5], F[5];
#pragma unroll
  for (int sl = 0; sl < 5; ++sl) {
    UL[sl] = Uh[0][rot<D>(sl)];
    UR[sl] = Uh[1][rot<D>(sl)];
  }
  RiemannCounts cnt{0u, 0u};
  exact_flux(UL, UR, P, F, cnt);
  flush_counts(cnt, s);
#pragma unroll
  for (int sl = 0; sl < 5; ++sl) fhalf[rot<D>(sl) * P.stride + cl] = F[sl];
}

// ---- a8-a9: conservative update and CFL reduction ------------------------------------------
template <typename T>
__global__ void k_update(T* __restrict__ u, const T* __restrict__ fhalf_all, GridParams P,
                         DevScalars* __restrict__ s, long long fdir_stride) {
  const double dt = s->dt;
  if (!(dt > 0.0)) return;
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)P.n[0] * P.n[1] * P.n[2];
  double bound = INFINITY;
  if (tid < total) {
    const int i = (int)(tid % P.n[0]);
    const int j = (int)((tid / P.n[0]) % P.n[1]);
    const int k = (int)(tid / ((long long)P.n[0] * P.n[1]));
    const long long c = cell_index(P, i, j, k);
    const long long st[3] = {1, (long long)P.N[0], (long long)P.N[0] * P.N[1]};
    const T dtdx = T(dt / P.dx[0]), dtdy = T(dt / P.dx[1]), dtdz = T(dt / P.dx[2]);
    const T* Fx = fhalf_all;
    const T* Fy = fhalf_all + fdir_stride;
    const T* Fz = fhalf_all + 2 * fdir_stride;
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
  block_min_atomic(bound, &s->dt_next_bits);
}

template <typename T>
__global__ void k_dt(const T* __restrict__ u, GridParams P, DevScalars* __restrict__ s) {
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)P.n[0] * P.n[1] * P.n[2];
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
  block_min_atomic(bound, &s->dt_next_bits);
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
      "bc_fill_x", "bc_fill_y", "bc_fill_z", "trace_x", "trace_y", "trace_z",
      "riemann1_x", "riemann1_y", "riemann1_z", "riemann2_x", "riemann2_y", "riemann2_z",
      "update_dt"};
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

// ---- launch wrappers ------------------------------------------------------------------------
static inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

#define TIMED(cls, launch)              \
  do {                                  \
    if (prof) prof->begin(cls, stream); \
    launch;                             \
    if (prof) prof->end(stream);        \
  } while (0)

template <typename T>
hipError_t launch_step(const StepBuffers<T>& b, const GridParams& P, const int bc[6],
                       hipStream_t stream, Profiler* prof) {
  constexpr int BS = 256;
  // a1: ghost fill x, then y, then z
  for (int axis = 0; axis < 3; ++axis) {
    const int o1 = axis == 0 ? 1 : 0, o2 = axis == 2 ? 1 : 2;
    long long total = 2LL * NG * P.N[o1] * P.N[o2];
    TIMED(K_BC_X + axis,
          hipLaunchKernelGGL(k_bc_fill<T>, dim3(blocks_for(total, BS)), dim3(BS), 0, stream, b.u,
                             P, axis, bc[2 * axis], bc[2 * axis + 1]));
  }
  const long long ext = (long long)(P.n[0] + 2) * (P.n[1] + 2) * (P.n[2] + 2);
  // a2-a5 per direction
  TIMED(K_TRACE_X, hipLaunchKernelGGL((k_trace<T, 0>), dim3(blocks_for(ext, BS)), dim3(BS), 0,
                                      stream, b.u, b.ustar[0], P, b.scalars));
  {
    long long nf = (long long)(P.n[0] + 1) * (P.n[1] + 2) * (P.n[2] + 2);
    TIMED(K_RIEMANN1_X, hipLaunchKernelGGL((k_riemann1<T, 0>), dim3(blocks_for(nf, BS)), dim3(BS),
                                           0, stream, b.ustar[0], b.fstar[0], P, b.scalars));
  }
  TIMED(K_TRACE_Y, hipLaunchKernelGGL((k_trace<T, 1>), dim3(blocks_for(ext, BS)), dim3(BS), 0,
                                      stream, b.u, b.ustar[1], P, b.scalars));
  {
    long long nf = (long long)(P.n[0] + 2) * (P.n[1] + 1) * (P.n[2] + 2);
    TIMED(K_RIEMANN1_Y, hipLaunchKernelGGL((k_riemann1<T, 1>), dim3(blocks_for(nf, BS)), dim3(BS),
                                           0, stream, b.ustar[1], b.fstar[1], P, b.scalars));
  }
  TIMED(K_TRACE_Z, hipLaunchKernelGGL((k_trace<T, 2>), dim3(blocks_for(ext, BS)), dim3(BS), 0,
                                      stream, b.u, b.ustar[2], P, b.scalars));
  {
    long long nf = (long long)(P.n[0] + 2) * (P.n[1] + 2) * (P.n[2] + 1);
    TIMED(K_RIEMANN1_Z, hipLaunchKernelGGL((k_riemann1<T, 2>), dim3(blocks_for(nf, BS)), dim3(BS),
                                           0, stream, b.ustar[2], b.fstar[2], P, b.scalars));
  }
  // a6-a7 per direction
  const long long fds = b.fstar[1] - b.fstar[0];
  {
    long long nf = (long long)(P.n[0] + 1) * P.n[1] * P.n[2];
    TIMED(K_RIEMANN2_X, hipLaunchKernelGGL((k_riemann2<T, 0>), dim3(blocks_for(nf, BS)), dim3(BS),
                                           0, stream, b.ustar[0], b.fstar[0], b.fhalf[0], P,
                                           b.scalars, fds));
  }
  {
    long long nf = (long long)P.n[0] * (P.n[1] + 1) * P.n[2];
    TIMED(K_RIEMANN2_Y, hipLaunchKernelGGL((k_riemann2<T, 1>), dim3(blocks_for(nf, BS)), dim3(BS),
                                           0, stream, b.ustar[1], b.fstar[0], b.fhalf[1], P,
                                           b.scalars, fds));
  }
  {
    long long nf = (long long)P.n[0] * P.n[1] * (P.n[2] + 1);
    TIMED(K_RIEMANN2_Z, hipLaunchKernelGGL((k_riemann2<T, 2>), dim3(blocks_for(nf, BS)), dim3(BS),
                                           0, stream, b.ustar[2], b.fstar[0], b.fhalf[2], P,
                                           b.scalars, fds));
  }
  // a8-a9
  const long long real = (long long)P.n[0] * P.n[1] * P.n[2];
  const long long hds = b.fhalf[1] - b.fhalf[0];
  TIMED(K_UPDATE, hipLaunchKernelGGL(k_update<T>, dim3(blocks_for(real, BS)), dim3(BS), 0, stream,
                                     b.u, b.fhalf[0], P, b.scalars, hds));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dt(T* u, const GridParams& P, DevScalars* s, hipStream_t stream) {
  constexpr int BS = 256;
  hipLaunchKernelGGL(k_reset_dt_bits, dim3(1), dim3(1), 0, stream, s);
  const long long real = (long long)P.n[0] * P.n[1] * P.n[2];
  hipLaunchKernelGGL(k_dt<T>, dim3(blocks_for(real, BS)), dim3(BS), 0, stream, u, P, s);
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
  hipLaunchKernelGGL(k_scatter<T>, dim3(blocks_for(real, 256)), dim3(256), 0, stream, packed, u, P);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const T* u, T* packed, const GridParams& P, hipStream_t stream) {
  const long long real = (long long)P.n[0] * P.n[1] * P.n[2];
  hipLaunchKernelGGL(k_gather<T>, dim3(blocks_for(real, 256)), dim3(256), 0, stream, u, packed, P);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prim_to_cons(const double* packed, T* u, const GridParams& P, hipStream_t stream) {
  const long long real = (long long)P.n[0] * P.n[1] * P.n[2];
  hipLaunchKernelGGL(k_prim_to_cons<T>, dim3(blocks_for(real, 256)), dim3(256), 0, stream, packed,
                     u, P);
  return hipGetLastError();
}

hipError_t launch_set_dt(DevScalars* s, double dt, hipStream_t stream) {
  hipLaunchKernelGGL(k_set_dt, dim3(1), dim3(1), 0, stream, s, dt);
  return hipGetLastError();
}
hipError_t launch_begin_step(DevScalars* s, double cfl, double t_end, hipStream_t stream) {
  hipLaunchKernelGGL(k_begin_step, dim3(1), dim3(1), 0, stream, s, cfl, t_end);
  return hipGetLastError();
}
hipError_t launch_end_step(DevScalars* s, hipStream_t stream) {
  hipLaunchKernelGGL(k_end_step, dim3(1), dim3(1), 0, stream, s);
  return hipGetLastError();
}

#define CTU_INSTANTIATE(T)                                                                        \
  template hipError_t launch_step<T>(const StepBuffers<T>&, const GridParams&, const int*,       \
                                     hipStream_t, Profiler*);                                    \
  template hipError_t launch_dt<T>(T*, const GridParams&, DevScalars*, hipStream_t);            \
  template hipError_t launch_totals<T>(const T*, const GridParams&, double*, int, double*,      \
                                       hipStream_t);                                             \
  template hipError_t launch_scatter<T>(const T*, T*, const GridParams&, hipStream_t);          \
  template hipError_t launch_gather<T>(const T*, T*, const GridParams&, hipStream_t);           \
  template hipError_t launch_prim_to_cons<T>(const double*, T*, const GridParams&, hipStream_t);

CTU_INSTANTIATE(double)
CTU_INSTANTIATE(float)

}  // namespace ctu
