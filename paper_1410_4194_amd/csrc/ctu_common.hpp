// ctu_common.hpp -- device helpers shared by the CTU kernels: grid lookup in a launch table,
// momentum-slot rotation, reductions and the CFL bound of a cell.
#pragma once

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

// Index of this wavefront within its block as a wave-uniform value, so that the arithmetic
// that derives a wavefront's task from it runs on the scalar unit, not the vector ALU.
__device__ __forceinline__ int wave_in_block() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// (base + lane) mod n for base + lane >= 0, with base wave-uniform, lane in [0, 64) and
// n >= 1: one scalar remainder, then no vector division when a row is at least a wavefront
// long.  (The value for base + lane < 0 is unspecified; callers mask those lanes.)
__device__ __forceinline__ int wave_row_pos(long long base, int lane, int n) {
  const long long bm = base % n;
  const int b = (int)(bm < 0 ? bm + n : bm);
  const int q = b + lane;
  if (n >= 64) return q >= n ? q - n : q;
  return q % n;
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

}  // namespace ctu
