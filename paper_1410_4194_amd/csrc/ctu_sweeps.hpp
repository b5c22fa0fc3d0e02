// ctu_sweeps.hpp -- the fused sweep kernels of the CTU step (gfx950): per direction, PPMC
// reconstruction with characteristic tracing and the exact Riemann solve, for the first stage
// and, re-traced with the transverse correction, for the second (Sec. 2.1, App. A.3, B.1).
#pragma once

#include "ctu_common.hpp"

namespace ctu {

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

// Transverse correction of a cell (eq. transverse_evolution), rotated to the sweep frame:
// dT = h1 dF_t1(c) + h2 dF_t2(c), where dF(c) = F(c - 1/2) - F(c + 1/2) is the per-cell
// difference of the first-stage fluxes that the first-stage sweeps store.
template <typename T, int D>
__device__ __forceinline__ void transverse_delta(const GLOBAL T* __restrict__ dstar_all,
                                                 long long fds, long long stride, long long c,
                                                 T h1, T h2, T dT[5]) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const GLOBAL T* D1 = dstar_all + T1 * fds;
  const GLOBAL T* D2 = dstar_all + T2 * fds;
#pragma unroll
  for (int sl = 0; sl < 5; ++sl) {
    const long long o = rot<D>(sl) * stride + c;
    dT[sl] = h1 * D1[o] + h2 * D2[o];
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
  if (cnt.hlle) atomicAdd(&s->counters[3], (unsigned long long)cnt.hlle);
}

// PPMP coefficients of a cell along axis D (zero, unused, for PPMC).
template <int R, int D, typename T>
__device__ __forceinline__ PpmpCoef<T> load_coef(const GridDesc* G, long long stride,
                                                  long long id) {
  PpmpCoef<T> k{T(0), T(0)};
  if constexpr (R == 1) {
    const GLOBAL T* __restrict__ cf = (const GLOBAL T*)G->coef;
    k.flat = cf[(2 * D) * stride + id];
    k.eta = cf[(2 * D + 1) * stride + id];
  }
  return k;
}

// Newton-iteration histogram of the solves of one wavefront (instrumented sweeps only):
// each solve's bin is counted over the active lanes with a ballot, so lanes that left the
// kernel early are simply not counted.  The wave counts sit in vector registers, so add and
// flush must run with the same set of active lanes (or add with all lanes active).
struct NewtonHist {
  unsigned long long n[8];
  __device__ void add(int iters, bool counted = true) {
    const int b = iters >= kItersCapped ? 7
                  : iters <= 1 ? 0 : (iters <= 4 ? iters - 1 : (iters <= 8 ? 4 : (iters <= 16 ? 5 : 6)));
#pragma unroll
    for (int k = 0; k < 8; ++k) n[k] += __popcll(__ballot(counted && b == k));
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

// H correction (App. C): eta^H of the D-face between cells cm and cp = cm + e_D, the largest
// eta of the face itself and of the faces on both sides of cm and cp along the other two
// axes (the nine-point stencil).  eta holds one field per axis, face c-1/2 at cell c.
template <int D, typename T>
__device__ __forceinline__ T eta_h_at(const GLOBAL T* __restrict__ eta, const GridParams& P,
                                      long long cm, long long cp) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const long long st[3] = {1, P.N[0], (long long)P.N[0] * P.N[1]};
  const GLOBAL T* __restrict__ e1 = eta + T1 * P.stride;
  const GLOBAL T* __restrict__ e2 = eta + T2 * P.stride;
  T e = eta[D * P.stride + cp];
  e = tmax(e, tmax(tmax(e1[cm], e1[cm + st[T1]]), tmax(e1[cp], e1[cp + st[T1]])));
  e = tmax(e, tmax(tmax(e2[cm], e2[cm + st[T2]]), tmax(e2[cp], e2[cp + st[T2]])));
  return e;
}

// The same with the face's own eta given (computed by the caller from the face's states).
template <int D, typename T>
__device__ __forceinline__ T eta_h_own(const GLOBAL T* __restrict__ eta, const GridParams& P,
                                       long long cm, long long cp, T own) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const long long st[3] = {1, P.N[0], (long long)P.N[0] * P.N[1]};
  const GLOBAL T* __restrict__ e1 = eta + T1 * P.stride;
  const GLOBAL T* __restrict__ e2 = eta + T2 * P.stride;
  T e = own;
  e = tmax(e, tmax(tmax(e1[cm], e1[cm + st[T1]]), tmax(e1[cp], e1[cp + st[T1]])));
  e = tmax(e, tmax(tmax(e2[cm], e2[cm + st[T2]]), tmax(e2[cp], e2[cp + st[T2]])));
  return e;
}

// K is the gas class of the exact solver (see pfun_fast).
// STAGE = 1: first-stage fluxes F*_D on the faces c-1/2, c in [0, n_D], transverse range
//            [-1, n] on both other axes.
// STAGE = 2: CTU fluxes F^{n+1/2}_D on the same faces over the real transverse range, from
//            the re-traced states plus the transverse correction of stage 1.
// Each stores the per-cell difference dF(c) = F(c - 1/2) - F(c + 1/2) of the real cells
// c in [0, n_D): the consumers (transverse correction, update) need only that, and read it
// once per cell instead of two faces.  A thread's segment covers the cells [f0, f1) and
// solves the f1 - f0 + 1 faces around them.
// Block layout per grid: (plane block of kBlock columns, segment), plane blocks fastest.
template <typename T, int D, int STAGE, bool HIST, int K, int R>
__global__ __launch_bounds__(256, 2) void k_sweep_march(LaunchTab tab) {
  static_assert(D == 1 || D == 2, "marching sweeps run along y or z");
  // STAGE 3 (H correction): the second-stage states of the faces over the first stage's
  // transverse range, reduced to eta = |(u+a)_R - (u+a)_L|/2 instead of solved
  constexpr bool ETA = STAGE == 3;
  constexpr bool S2 = STAGE >= 2;  // second-stage states (re-traced + transverse correction)
  // With the H correction the second-stage y sweep takes the eta pass along y over: it runs
  // over the first stage's transverse range, stores eta of every face it sees (the z and x
  // sweeps after it read them) and solves only the faces of real columns, whose eta^H takes
  // the face's own eta from registers.  The eta passes along x and z run before it.
  constexpr bool FUSE_ETA = STAGE == 2 && D == 1 && K == kRoeH;
  const BlockRef r = block_ref(tab);
  const GridParams P = r.G->P;
  DevScalars* __restrict__ s = r.G->s;
  const double dt = s->dt;
  if (!(dt > 0.0)) return;
  const GLOBAL T* __restrict__ u = (const GLOBAL T*)r.G->u;
  const GLOBAL T* __restrict__ dstar_all = (const GLOBAL T*)r.G->flux;
  const long long fds = 5 * P.stride;
  GLOBAL T* __restrict__ out = (GLOBAL T*)r.G->flux + (STAGE == 1 ? D : 3 + D) * fds;
  constexpr int B = (D == 1) ? 2 : 1;  // the transverse axis other than x
  constexpr bool EXT_T = STAGE != 2 || FUSE_ETA;  // transverse range [-1, n]
  const int lo = EXT_T ? -1 : 0;
  const int ea = P.n[0] + (EXT_T ? 2 : 0);
  const int eb = P.n[B] + (EXT_T ? 2 : 0);
  // cells along D: the real ones, one more on each side in the first stage with the H
  // correction (its eta pass needs second-stage states one cell beyond the real box)
  const int dlo = STAGE == 1 ? -P.ext : 0;
  const int nd = P.n[D] - dlo;  // end of the range
  const long long nbx = ((long long)ea * eb + kBlock - 1) / kBlock;
  const int seg = P.seg[D];
  const long long nseg = (nd - dlo + seg - 1) / seg;
  if (r.lb >= nbx * nseg) return;
  const long long tid = (r.lb % nbx) * kBlock + threadIdx.x;
  if (tid >= (long long)ea * eb) return;
  const int i = (int)(tid % ea) + lo;
  const int o = (int)(tid / ea) + lo;
  const int f0 = dlo + (int)(r.lb / nbx) * seg;
  const int f1 = min(f0 + seg, nd);
  // a column outside the real box along x or the other transverse axis: eta only
  const bool ring = FUSE_ETA && (i < 0 || i >= P.n[0] || o < 0 || o >= P.n[B]);
  const long long stx = 1, sty = P.N[0], stz = (long long)P.N[0] * P.N[1];
  const long long sd = D == 1 ? sty : stz;
  const long long c0 = D == 1 ? cell_index(P, i, 0, o) : cell_index(P, i, o, 0);
  const T dtodx = T(dt / P.dx[D]);
  const T igm1 = T(P.inv_gm1);
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const T h1 = T(0.5 * dt / P.dx[T1]);
  const T h2 = T(0.5 * dt / P.dx[T2]);
  (void)stx;

  Prim<T> q0, q1, q2, q3;  // cells c-1, c, c+1, c+2 around the traced cell c
  T s0[5], s1[5], s2[5];   // limited slopes of c-1, c, c+1
  {
    Prim<T> qm;
    load_prim<T, D>(u, P.stride, c0 + (long long)(f0 - 3) * sd, P, qm);
    load_prim<T, D>(u, P.stride, c0 + (long long)(f0 - 2) * sd, P, q0);
    load_prim<T, D>(u, P.stride, c0 + (long long)(f0 - 1) * sd, P, q1);
    load_prim<T, D>(u, P.stride, c0 + (long long)(f0)*sd, P, q2);
    load_prim<T, D>(u, P.stride, c0 + (long long)(f0 + 1) * sd, P, q3);
    slope_sel<R>(qm, q0, q1, s0);
    slope_sel<R>(q0, q1, q2, s1);
    slope_sel<R>(q1, q2, q3, s2);
  }
  // warm-up: trace cell f0-1 (window: q0 = f0-2, q1 = f0-1, q2 = f0, q3 = f0+1)
  T prevR[5];  // right-face state of the previous cell: primitive in stage 1, conserved in 2
  {
    T WL[5], WR[5];
    trace_sel<R>(q0, q1, q2, s0, s1, s2,
                 load_coef<R, D, T>(r.G, P.stride, c0 + (long long)(f0 - 1) * sd),
                 T(P.gamma), dtodx, WL, WR);
    if (STAGE == 1) {
#pragma unroll
      for (int q = 0; q < 5; ++q) prevR[q] = WR[q];
    } else {
      to_cons(WR, igm1, prevR);
    }
    if (S2) {
      T dT[5];
      transverse_delta<T, D>(dstar_all, fds, P.stride, c0 + (long long)(f0 - 1) * sd, h1, h2,
                             dT);
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
  // flux at face c-3/2, kept in LDS (each thread its own slot): registers would cost the
  // first-stage sweeps a wave per SIMD
  __shared__ T prevF[5][kBlock];
  for (int c = f0; c <= f1; ++c) {
    // window: q0 = c-1, q1 = c, q2 = c+1, slopes s0 = c-1, s1 = c; face c-1/2
    make_prim(raw, T(P.gamma), T(P.gm1), T(P.p_floor), q3);  // cell c+2
    if (c + 1 <= f1) {
      const long long nid = c0 + (long long)(c + 3) * sd;
#pragma unroll
      for (int sl = 0; sl < 5; ++sl) raw[sl] = u[rot<D>(sl) * P.stride + nid];
    }
    slope_sel<R>(q1, q2, q3, s2);  // slope of c+1
    T WL[5], WR[5], UL[5], UR[5], F[5];
    trace_sel<R>(q0, q1, q2, s0, s1, s2, load_coef<R, D, T>(r.G, P.stride, c0 + (long long)c * sd),
                 T(P.gamma), dtodx, WL, WR);
    // the segment's last face is solved again as the next segment's first: count it there
    const bool dupface = c == f1 && f1 < nd;
    RiemannCounts dup{0u, 0u, 0};
    if (STAGE == 1) {
      face_flux_w<T, K>(prevR, WL, P, F, dupface ? dup : cnt);
#pragma unroll
      for (int q = 0; q < 5; ++q) UR[q] = WR[q];
    } else {
      to_cons(WL, igm1, UL);
      to_cons(WR, igm1, UR);
      T dT[5];
      transverse_delta<T, D>(dstar_all, fds, P.stride, c0 + (long long)c * sd, h1, h2, dT);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        UL[q] += dT[q];
        UR[q] += dT[q];
      }
      T eta_h = T(0);
      if constexpr (ETA || FUSE_ETA) {
        Prim<T> Lq, Rq;
        make_prim(prevR, T(P.gamma), T(P.gm1), T(P.p_floor), Lq);
        make_prim(UL, T(P.gamma), T(P.gm1), T(P.p_floor), Rq);
        const T e = T(0.5) * tfabs((Rq.w[1] + Rq.a) - (Lq.w[1] + Lq.a));
        // the face is written by the segment that owns it (not the duplicate)
        if (!dupface) ((GLOBAL T*)r.G->eta + D * P.stride)[c0 + (long long)c * sd] = e;
        if constexpr (FUSE_ETA) {
          if (!ring)
            eta_h = eta_h_own<D>((const GLOBAL T*)r.G->eta, P, c0 + (long long)(c - 1) * sd,
                                 c0 + (long long)c * sd, e);
        }
      } else if constexpr (K == kRoeH) {  // (the eta passes wrote these)
        eta_h = eta_h_at<D>((const GLOBAL T*)r.G->eta, P, c0 + (long long)(c - 1) * sd,
                            c0 + (long long)c * sd);
      }
      if constexpr (!ETA) {
        if (!ring) face_flux_u<T, K>(prevR, UL, P, F, dupface ? dup : cnt, eta_h);
      }
    }
    if (HIST) hist.add(dupface ? dup.iters : cnt.iters, !dupface);
    // keep the LDS read of the previous flux below the solve (hoisted above it, the five
    // values would stay live through the solve and cost the first stage a wave per SIMD)
    asm volatile("" ::: "memory");
    if (!ETA && !ring && c > f0) {  // cell c-1 now has both faces
      const long long co = c0 + (long long)(c - 1) * sd;
#pragma unroll
      for (int sl = 0; sl < 5; ++sl)
        out[rot<D>(sl) * P.stride + co] = prevF[sl][threadIdx.x] - F[sl];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      if (!ETA) prevF[q][threadIdx.x] = F[q];
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

// H correction along x: eta of the x-faces of the real cells (c in [0, n_x]) over rows and
// planes [-1, n], from the second-stage states (re-traced, plus the transverse correction),
// on the flattened plane lines of the first-stage x sweep; lanes 3..60 write the face of
// their own cell, so every face is written once.
template <typename T, int R>
__global__ __launch_bounds__(256) void k_eta_x(LaunchTab tab) {
  const BlockRef r = block_ref(tab);
  const GridParams P = r.G->P;
  const double dt = r.G->s->dt;
  if (!(dt > 0.0)) return;
  const GLOBAL T* __restrict__ u = (const GLOBAL T*)r.G->u;
  const GLOBAL T* __restrict__ dstar_all = (const GLOBAL T*)r.G->flux;
  const long long fds = 5 * P.stride;
  const int lane = threadIdx.x & 63;
  const long long task = r.lb * (kBlock / 64) + wave_in_block();
  const long long plen = (long long)(P.n[1] + 2) * P.N[0];
  const long long nw = (plen + XW - 1) / XW;
  if (task >= nw * (P.n[2] + 2)) return;  // whole wavefront exits together
  const int k = (int)(task / nw) - 1;
  const long long p0 = (task % nw) * XW - 3;  // position of lane 0
  const long long p = p0 + lane;
  const bool in_line = p >= 0 && p < plen;
  const int c = in_line ? wave_row_pos(p0, lane, P.N[0]) - P.ng : -P.ng - 1;
  const long long id = cell_index(P, -P.ng, -1, k) + p;
  const T dtodx = T(dt / P.dx[0]);
  const T h1 = T(0.5 * dt / P.dx[1]), h2 = T(0.5 * dt / P.dx[2]);
  const T igm1 = T(P.inv_gm1), g = T(P.gamma);
  Prim<T> me;
  if (in_line)
    load_prim<T, 0>(u, P.stride, id, P, me);
  else
    safe_prim(me);
  const int lm1 = lane > 0 ? lane - 1 : 0;
  const int lp1 = lane < 63 ? lane + 1 : 63;
  const Prim<T> left = shfl_prim(me, lm1);
  const Prim<T> right = shfl_prim(me, lp1);
  T sl[5];
  slope_sel<R>(left, me, right, sl);
  T slm[5], slp[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    slm[q] = __shfl(sl[q], lm1, 64);
    slp[q] = __shfl(sl[q], lp1, 64);
  }
  T WL[5], WR[5], UL[5], UR[5];
  PpmpCoef<T> kc{T(0), T(0)};
  if (R == 1 && in_line && c >= -1 && c <= P.n[0]) kc = load_coef<R, 0, T>(r.G, P.stride, id);
  trace_sel<R>(left, me, right, slm, sl, slp, kc, g, dtodx, WL, WR);
  to_cons(WL, igm1, UL);
  to_cons(WR, igm1, UR);
  if (lane >= 2 && lane <= 61 && in_line && c >= -1 && c <= P.n[0]) {
    T dT[5];
    transverse_delta<T, 0>(dstar_all, fds, P.stride, id, h1, h2, dT);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      UL[q] += dT[q];
      UR[q] += dT[q];
    }
  }
  T prevR[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) prevR[q] = __shfl(UR[q], lm1, 64);
  if (lane >= 3 && lane <= 60 && in_line && c >= 0 && c <= P.n[0]) {
    Prim<T> Lq, Rq;
    make_prim(prevR, g, T(P.gm1), T(P.p_floor), Lq);
    make_prim(UL, g, T(P.gm1), T(P.p_floor), Rq);
    GLOBAL T* __restrict__ eta = (GLOBAL T*)r.G->eta;
    eta[id] = T(0.5) * tfabs((Rq.w[1] + Rq.a) - (Lq.w[1] + Lq.a));
  }
}

// First-stage x sweep.  The x-rows of one z-plane (j over the extended range [-1, n_y], each
// row with its three ghost cells per side) lie back to back in memory, so they are treated
// as one flattened line of positions p = (j + 1) N_x + (c + 3).  A chunk covers 64
// consecutive positions: lane l holds position XW w - 3 + l, slopes are valid on lanes
// 1..62, traces on 2..61, lanes 3..61 solve the face c-1/2 of their cell when
// 0 <= c <= n_x, and lanes 3..60 store the difference dF(c) = F(c-1/2) - F(c+1/2) of their
// real cell (F(c+1/2) from the next lane).  Every stencil of such a face lies in its own
// row, so short rows share a chunk instead of leaving most of its lanes idle.  A wavefront
// takes P.xchunks consecutive chunks, paying its set-up once for them.
template <typename T, int STAGE, bool HIST, int K, int R>
__global__ __launch_bounds__(256) void k_sweep_x(LaunchTab tab) {
  static_assert(STAGE == 1, "the second-stage x sweep is fused with the update");
  const BlockRef r = block_ref(tab);
  const GridParams P = r.G->P;
  DevScalars* __restrict__ s = r.G->s;
  const double dt = s->dt;
  if (!(dt > 0.0)) return;
  const GLOBAL T* __restrict__ u = (const GLOBAL T*)r.G->u;
  GLOBAL T* __restrict__ out = (GLOBAL T*)r.G->flux;
  const int lane = threadIdx.x & 63;
  const int nchunks = P.xchunks;
  const long long task0 = (r.lb * (kBlock / 64) + wave_in_block()) * nchunks;
  const long long plen = (long long)(P.n[1] + 2) * P.N[0];  // positions of one plane
  const long long nw = (plen + XW - 1) / XW;                   // chunks per plane
  const long long ntask = nw * (P.n[2] + 2);
  if (task0 >= ntask) return;  // whole wavefront exits together
  const T dtodx = T(dt / P.dx[0]);
  const int lm1 = lane > 0 ? lane - 1 : 0;
  const int lp1 = lane < 63 ? lane + 1 : 63;
  const int e = P.ext;  // one more cell on each side with the H correction
  NewtonHist hist{};
  for (int qc = 0; qc < nchunks; ++qc) {
    const long long task = task0 + qc;
    if (task >= ntask) break;  // wave-uniform
    const int k = (int)(task / nw) - 1;
    const long long p0 = (task % nw) * XW - 3;  // position of lane 0
    const long long p = p0 + lane;
    const bool in_line = p >= 0 && p < plen;
    const int c = in_line ? wave_row_pos(p0, lane, P.N[0]) - P.ng : -P.ng - 1;
    const long long id = cell_index(P, -P.ng, -1, k) + p;

    Prim<T> me;
    if (in_line)
      load_prim<T, 0>(u, P.stride, id, P, me);
    else
      safe_prim(me);
    const Prim<T> left = shfl_prim(me, lm1);
    const Prim<T> right = shfl_prim(me, lp1);
    T sl[5];
    slope_sel<R>(left, me, right, sl);
    T slm[5], slp[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      slm[q] = __shfl(sl[q], lm1, 64);
      slp[q] = __shfl(sl[q], lp1, 64);
    }
    // traced primitive face states enter the solver directly
    T WL[5], WR[5];
    PpmpCoef<T> kc{T(0), T(0)};
    if (R == 1 && in_line && c >= -1 - P.ext && c <= P.n[0] + P.ext)
      kc = load_coef<R, 0, T>(r.G, P.stride, id);
    trace_sel<R>(left, me, right, slm, sl, slp, kc, T(P.gamma), dtodx, WL, WR);
    T prevR[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) prevR[q] = __shfl(WR[q], lm1, 64);
    T F[5] = {T(0), T(0), T(0), T(0), T(0)};  // flux at face c-1/2
    int iters = -1;  // Newton iterations of this lane's counted solve
    if (lane >= 3 && lane <= 61 && c >= -e && c <= P.n[0] + e) {
      // lane 61's face is solved again as the next chunk's first face: count it there
      const bool counted = lane <= 60 || task % nw == nw - 1;
      RiemannCounts cnt{0u, 0u, 0};
      face_flux_w<T, K>(prevR, WL, P, F, cnt);
      if (counted) {
        flush_counts(cnt, s);
        iters = cnt.iters;
      }
    }
    T Fr[5];  // flux at face c+1/2
#pragma unroll
    for (int q = 0; q < 5; ++q) Fr[q] = __shfl(F[q], lp1, 64);
    if (lane >= 3 && lane <= 60 && c >= -e && c < P.n[0] + e) {
#pragma unroll
      for (int q = 0; q < 5; ++q) out[q * P.stride + id] = F[q] - Fr[q];
    }
    if (HIST) hist.add(iters, iters >= 0);  // every lane takes the add
  }
  if (HIST) hist.flush(s);
}

// Second-stage x sweep fused with the conservative update (a8) and the CFL bound (a9).
// One wavefront owns P.xrows consecutive x-rows of real cells of one z-plane; with their
// ghost cells they lie back to back in memory and are marched as one flattened line of
// positions p = (row - first row) N_x + (c + 3), in chunks of XU positions: lane l holds
// position cw - 3 + l, computes the face flux F(c-1/2) as the first-stage sweep does
// (re-traced, plus the transverse correction from the y and z first-stage flux
// differences), takes F(c+1/2) from lane l+1, and updates the real cells among positions
// cw..cw+XU-1 (lanes 3..60) with the y and z second-stage flux differences, which the two
// earlier second-stage sweeps stored.  The new state is written in place, but only after the next chunk has read its
// stencil (the cells up to three behind it), so every stencil sees u^n; stencils of real
// faces stay within their row and no other wavefront reads these rows.
template <typename T, bool HIST, int K, int R>
__global__ __launch_bounds__(256) void k_sweep_x_update(LaunchTab tab) {
  const BlockRef r = block_ref(tab);
  const GridParams P = r.G->P;
  DevScalars* __restrict__ s = r.G->s;
  const double dt = s->dt;
  if (!(dt > 0.0)) return;  // a no-op step keeps the previous partials (state unchanged)
  constexpr int kWaves = kBlock / 64;
  const long long ngy = (P.n[1] + P.xrows - 1) / P.xrows;  // row groups per plane
  const long long ngroups = ngy * P.n[2];
  if (r.lb * kWaves >= ngroups) return;  // whole block idle
  GLOBAL T* __restrict__ u = (GLOBAL T*)r.G->u;
  const GLOBAL T* __restrict__ dstar_all = (const GLOBAL T*)r.G->flux;
  const long long fds = 5 * P.stride;
  GLOBAL T* __restrict__ out = (GLOBAL T*)r.G->flux + 3 * fds;  // dF^{n+1/2}_x (debug only)
  const bool keep = (r.G->flags & GRID_KEEP_X_FLUXES) != 0;
  const GLOBAL T* __restrict__ dG = (const GLOBAL T*)r.G->flux + 4 * fds;  // dG^{n+1/2}
  const GLOBAL T* __restrict__ dH = dG + fds;                              // dH^{n+1/2}
  const int lane = threadIdx.x & 63;
  const long long grp = r.lb * kWaves + wave_in_block();
  double bound = INFINITY;
  if (grp < ngroups) {  // wave-uniform
    const int j0 = (int)(grp % ngy) * P.xrows;
    const int k = (int)(grp / ngy);
    const int plen = min(P.xrows, P.n[1] - j0) * P.N[0];  // at most 8 rows: fits 32 bits
    const int ng = P.ng;
    const long long linebase = cell_index(P, -ng, j0, k);  // position 0
    const T dtodx = T(dt / P.dx[0]);
    const T dtdx = T(dt / P.dx[0]), dtdy = T(dt / P.dx[1]), dtdz = T(dt / P.dx[2]);
    const T igm1 = T(P.inv_gm1);
    const T h1 = T(0.5 * dt / P.dx[1]), h2 = T(0.5 * dt / P.dx[2]);
    const int lm1 = lane > 0 ? lane - 1 : 0;
    const int lp1 = lane < 63 ? lane + 1 : 63;
    RiemannCounts cnt{0u, 0u, 0};
    NewtonHist hist{};
    unsigned bad = 0;
    T Udef[5] = {T(0), T(0), T(0), T(0), T(0)};
    long long def_id = -1;  // cell whose new state waits for the next chunk's loads
    for (int cw = ng; cw < plen - ng; cw += XU) {
      const int p = cw - 3 + lane;
      const bool in_line = p >= 0 && p < plen;
      const int c = in_line ? wave_row_pos(cw - 3, lane, P.N[0]) - ng : -ng - 1;
      const long long id = linebase + p;
      T U0[5];
      Prim<T> me;
      if (in_line) {
#pragma unroll
        for (int f = 0; f < 5; ++f) U0[f] = u[f * P.stride + id];
        make_prim(U0, T(P.gamma), T(P.gm1), T(P.p_floor), me);
      } else {
#pragma unroll
        for (int f = 0; f < 5; ++f) U0[f] = T(0);
        safe_prim(me);
      }
      // the y and z second-stage differences of the cell this lane updates, loaded now so
      // that their latency hides behind the trace and the Riemann solve
      const bool upd = lane >= 3 && lane <= 60 && c >= 0 && c < P.n[0];
      T dGc[5], dHc[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        dGc[f] = upd ? dG[f * P.stride + id] : T(0);
        dHc[f] = upd ? dH[f * P.stride + id] : T(0);
      }
      // this chunk's stencil has been read (make_prim consumed it): the previous chunk's
      // new states can go out
      if (def_id >= 0) {
#pragma unroll
        for (int f = 0; f < 5; ++f) u[f * P.stride + def_id] = Udef[f];
      }
      def_id = -1;
      const Prim<T> left = shfl_prim(me, lm1);
      const Prim<T> right = shfl_prim(me, lp1);
      T sl[5];
      slope_sel<R>(left, me, right, sl);
      T slm[5], slp[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        slm[q] = __shfl(sl[q], lm1, 64);
        slp[q] = __shfl(sl[q], lp1, 64);
      }
      T WL[5], WR[5], UL[5], UR[5];
      PpmpCoef<T> kc{T(0), T(0)};
      if (R == 1 && in_line && c >= -1 && c <= P.n[0]) kc = load_coef<R, 0, T>(r.G, P.stride, id);
      trace_sel<R>(left, me, right, slm, sl, slp, kc, T(P.gamma), dtodx, WL, WR);
      to_cons(WL, igm1, UL);
      to_cons(WR, igm1, UR);
      if (lane >= 2 && lane <= 61 && c >= -1 && c <= P.n[0]) {
        T dT[5];
        transverse_delta<T, 0>(dstar_all, fds, P.stride, id, h1, h2, dT);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          UL[q] += dT[q];
          UR[q] += dT[q];
        }
      }
      T prevR[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) prevR[q] = __shfl(UR[q], lm1, 64);
      T F[5] = {T(0), T(0), T(0), T(0), T(0)};  // flux at face c-1/2
      int iters = -1;  // Newton iterations of this lane's counted solve
      if (lane >= 3 && lane <= 61 && c >= 0 && c <= P.n[0]) {
        // lane 61's face is solved again as the next chunk's first face: count it there
        const bool counted = lane <= 60 || cw + XU >= plen - ng;
        RiemannCounts dup{0u, 0u, 0};
        T eta_h = T(0);
        if constexpr (K == kRoeH) eta_h = eta_h_at<0>((const GLOBAL T*)r.G->eta, P, id - 1, id);
        face_flux_u<T, K>(prevR, UL, P, F, counted ? cnt : dup, eta_h);
        if (counted) iters = cnt.iters;
      }
      // the histogram keeps its wave counts in vector registers: every lane takes the add
      if (HIST) hist.add(iters, iters >= 0);
      T Fr[5];  // flux at face c+1/2
#pragma unroll
      for (int q = 0; q < 5; ++q) Fr[q] = __shfl(F[q], lp1, 64);
      if (upd) {
        // u^{n+1} = u^n + dt/dx (F_{-1/2} - F_{+1/2}) + dt/dy (...) + dt/dz (...), in this order
        T Un[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          const T dFx = F[f] - Fr[f];
          if (keep) out[f * P.stride + id] = dFx;  // consumed in registers: debugging only
          T v = U0[f];
          v = v + dtdx * dFx;
          v = v + dtdy * dGc[f];
          v = v + dtdz * dHc[f];
          Un[f] = v;
        }
        bool finite = true;
#pragma unroll
        for (int f = 0; f < 5; ++f) finite = finite && isfinite((double)Un[f]);
        if (!finite || !(Un[0] > T(0))) {
          atomicOr(&s->flags, finite ? 2u : 1u);
          ++bad;
        } else {
          bound = fmin(bound, cell_dt_bound(Un, P));
        }
#pragma unroll
        for (int f = 0; f < 5; ++f) Udef[f] = Un[f];
        def_id = id;
      }
    }
    if (def_id >= 0) {
#pragma unroll
      for (int f = 0; f < 5; ++f) u[f * P.stride + def_id] = Udef[f];
    }
    flush_counts(cnt, s);
    if (bad) atomicAdd(&s->counters[2], (unsigned long long)bad);
    if (HIST) hist.flush(s);
  }
  block_min_store(bound, (GLOBAL double*)r.G->part, r.lb);
}

// First- and second-stage z sweeps in one march (the fused-z schedule; not with the H
// correction, whose eta pass along z needs the second-stage states of the ring columns).  The
// second-stage z sweep needs only the x and y first-stage differences, so once those are done
// both z stages can share one march: the column's primitives, slopes and traces are computed
// once per cell, and each face is solved twice, from the traced primitive states (stage 1,
// H*) and from the same states in conserved form plus the transverse correction (stage 2,
// H^{n+1/2}).  u^n is read once for both.  Stage 1 covers the extended transverse range
// [-1, n] (its differences feed the y and x corrections there), stage 2 the real columns.
// Same block layout and segments as the first-stage z sweep.
template <typename T, bool HIST, int K, int R>
__global__ __launch_bounds__(256, 2) void k_sweep_z_both(LaunchTab tab) {
  constexpr int D = 2;
  const BlockRef r = block_ref(tab);
  const GridParams P = r.G->P;
  DevScalars* __restrict__ s = r.G->s;
  const double dt = s->dt;
  if (!(dt > 0.0)) return;
  const GLOBAL T* __restrict__ u = (const GLOBAL T*)r.G->u;
  const GLOBAL T* __restrict__ dstar_all = (const GLOBAL T*)r.G->flux;
  const long long fds = 5 * P.stride;
  GLOBAL T* __restrict__ out1 = (GLOBAL T*)r.G->flux + D * fds;
  GLOBAL T* __restrict__ out2 = (GLOBAL T*)r.G->flux + (3 + D) * fds;
  const int ea = P.n[0] + 2;
  const int eb = P.n[1] + 2;
  const int nd = P.n[D];
  const long long nbx = ((long long)ea * eb + kBlock - 1) / kBlock;
  const int seg = P.seg[D];
  const long long nseg = (nd + seg - 1) / seg;
  if (r.lb >= nbx * nseg) return;
  const long long tid = (r.lb % nbx) * kBlock + threadIdx.x;
  if (tid >= (long long)ea * eb) return;
  const int i = (int)(tid % ea) - 1;
  const int o = (int)(tid / ea) - 1;
  const int f0 = (int)(r.lb / nbx) * seg;
  const int f1 = min(f0 + seg, nd);
  const bool real = i >= 0 && i < P.n[0] && o >= 0 && o < P.n[1];
  const long long sd = (long long)P.N[0] * P.N[1];
  const long long c0 = cell_index(P, i, o, 0);
  const T dtodx = T(dt / P.dx[D]);
  const T igm1 = T(P.inv_gm1);
  const T h1 = T(0.5 * dt / P.dx[0]);
  const T h2 = T(0.5 * dt / P.dx[1]);

  Prim<T> q0, q1, q2, q3;
  T s0[5], s1[5], s2[5];
  {
    Prim<T> qm;
    load_prim<T, D>(u, P.stride, c0 + (long long)(f0 - 3) * sd, P, qm);
    load_prim<T, D>(u, P.stride, c0 + (long long)(f0 - 2) * sd, P, q0);
    load_prim<T, D>(u, P.stride, c0 + (long long)(f0 - 1) * sd, P, q1);
    load_prim<T, D>(u, P.stride, c0 + (long long)(f0)*sd, P, q2);
    load_prim<T, D>(u, P.stride, c0 + (long long)(f0 + 1) * sd, P, q3);
    slope_sel<R>(qm, q0, q1, s0);
    slope_sel<R>(q0, q1, q2, s1);
    slope_sel<R>(q1, q2, q3, s2);
  }
  T prevR1[5], prevR2[5];  // right-face state of the previous cell: primitive / conserved
  {
    T WL[5], WR[5];
    trace_sel<R>(q0, q1, q2, s0, s1, s2,
                 load_coef<R, D, T>(r.G, P.stride, c0 + (long long)(f0 - 1) * sd),
                 T(P.gamma), dtodx, WL, WR);
#pragma unroll
    for (int q = 0; q < 5; ++q) prevR1[q] = WR[q];
    to_cons(WR, igm1, prevR2);
    if (real) {
      T dT[5];
      transverse_delta<T, D>(dstar_all, fds, P.stride, c0 + (long long)(f0 - 1) * sd, h1, h2, dT);
#pragma unroll
      for (int q = 0; q < 5; ++q) prevR2[q] += dT[q];
    }
  }
  q0 = q1;
  q1 = q2;
  q2 = q3;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    s0[q] = s1[q];
    s1[q] = s2[q];
  }
  T raw[5];
#pragma unroll
  for (int sl = 0; sl < 5; ++sl) raw[sl] = u[rot<D>(sl) * P.stride + c0 + (long long)(f0 + 2) * sd];
  RiemannCounts cnt{0u, 0u, 0};
  NewtonHist hist{};
  __shared__ T prevF1[5][kBlock];
  __shared__ T prevF2[5][kBlock];
  for (int c = f0; c <= f1; ++c) {
    make_prim(raw, T(P.gamma), T(P.gm1), T(P.p_floor), q3);
    if (c + 1 <= f1) {
      const long long nid = c0 + (long long)(c + 3) * sd;
#pragma unroll
      for (int sl = 0; sl < 5; ++sl) raw[sl] = u[rot<D>(sl) * P.stride + nid];
    }
    slope_sel<R>(q1, q2, q3, s2);
    T WL[5], WR[5], F1[5], F2[5];
    trace_sel<R>(q0, q1, q2, s0, s1, s2, load_coef<R, D, T>(r.G, P.stride, c0 + (long long)c * sd),
                 T(P.gamma), dtodx, WL, WR);
    const bool dupface = c == f1 && f1 < nd;
    RiemannCounts dup{0u, 0u, 0};
    face_flux_w<T, K>(prevR1, WL, P, F1, dupface ? dup : cnt);
    if (HIST) hist.add(dupface ? dup.iters : cnt.iters, !dupface);
    T UL[5], UR[5];
    to_cons(WL, igm1, UL);
    to_cons(WR, igm1, UR);
#pragma unroll
    for (int q = 0; q < 5; ++q) F2[q] = T(0);
    int it2 = -1;
    if (real) {
      T dT[5];
      transverse_delta<T, D>(dstar_all, fds, P.stride, c0 + (long long)c * sd, h1, h2, dT);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        UL[q] += dT[q];
        UR[q] += dT[q];
      }
      RiemannCounts dup2{0u, 0u, 0};
      face_flux_u<T, K>(prevR2, UL, P, F2, dupface ? dup2 : cnt, T(0));
      it2 = dupface ? dup2.iters : cnt.iters;
    }
    if (HIST) hist.add(it2 < 0 ? 0 : it2, real && !dupface);
    asm volatile("" ::: "memory");
    if (c > f0) {
      const long long co = c0 + (long long)(c - 1) * sd;
#pragma unroll
      for (int sl = 0; sl < 5; ++sl) out1[rot<D>(sl) * P.stride + co] = prevF1[sl][threadIdx.x] - F1[sl];
      if (real) {
#pragma unroll
        for (int sl = 0; sl < 5; ++sl)
          out2[rot<D>(sl) * P.stride + co] = prevF2[sl][threadIdx.x] - F2[sl];
      }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      prevF1[q][threadIdx.x] = F1[q];
      prevF2[q][threadIdx.x] = F2[q];
      prevR1[q] = WR[q];
      prevR2[q] = UR[q];
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

// The three sweeps of one stage for every grid of a plan (one launch per direction).
// With a side stream in the plan the passes overlap where the data allow it (x1 = first-stage
// x sweep, y2 = second-stage y sweep, z12 = both z stages in one march, ...; PPMP coefficient
// passes in parentheses).  Fused z (large grids, where two concurrent memory-bound sweeps no
// longer fit the last-level cache):
//   launch stream: [fork] (coef x) x1 (coef z) [y done] z12 y2 update
//   side stream:   [fork] (coef y) y1 [y done]
// Overlapped:
//   launch stream: [fork] (coef x) x1 (coef z) [x done] z1 [y done] y2 [side done] update
//   side stream:   [fork] (coef y) y1 [y done] [x done] z2 [side done]
// The first-stage y sweep needs only u^n and its own coefficients, so it runs beside the x
// sweep; the second-stage z sweep needs only the first-stage x and y differences and the z
// coefficients, so it follows on the side as soon as those are done, beside the first-stage
// z sweep (bound by FP64 issue) and the second-stage y sweep (bound by memory); the
// memory-bound coefficient passes run beside the first-stage sweeps.
// With the H correction the second-stage z sweep reads the eta along y that the second-stage
// y sweep writes, so those two stay in order; the eta pass along z (which needs the x and y
// first-stage differences) moves to the side instead:
//   launch stream: [fork] (coef x) x1 (coef z) [x done] z1 [y done] eta_x [side done] y2 z2 update
//   side stream:   [fork] (coef y) y1 [y done] [x done] eta_z [side done]
// A pass still starts only after everything it reads is complete, so the overlapped results
// are bitwise those of the serial order; the fused z march agrees with them to rounding (a
// separately compiled copy of the same formulas).  Not while kernels are timed one by one.
template <typename T, int K, bool HIST, int R>
hipError_t enqueue_sweeps(const PlanView& v, int stage, hipStream_t stream, Profiler* prof) {
  const int stride = v.ngrids + 1;
  auto tab = [&](int pass) { return LaunchTab{v.d_grids, v.d_start + pass * stride, v.ngrids}; };
  auto nblocks = [&](int pass) { return dim3((unsigned)v.h_start[pass * stride + v.ngrids]); };
  const dim3 B(kBlock);
  const bool overlap = overlapped(v, prof);
  const bool fz = fused_z(v, prof);
  hipError_t e = hipSuccess;
  if (stage == 1) {
    // a2-a5: F*, G*, H* on the extended transverse range
    if (overlap) {
      e = hipEventRecord(v.fork, stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(v.side, v.fork, 0);
      if (e != hipSuccess) return e;
      if constexpr (R == 1) launch_ppmp_coef<T, 1>(v, v.side);
      hipLaunchKernelGGL((k_sweep_march<T, 1, 1, HIST, K, R>), nblocks(P_S1_Y), B, 0, v.side,
                         tab(P_S1_Y));
      e = hipEventRecord(v.ydone, v.side);
      if (e != hipSuccess) return e;
      if constexpr (R == 1) launch_ppmp_coef<T, 0>(v, stream);
      hipLaunchKernelGGL((k_sweep_x<T, 1, HIST, K, R>), nblocks(P_S1_X), B, 0, stream,
                         tab(P_S1_X));
      if constexpr (R == 1) launch_ppmp_coef<T, 2>(v, stream);
      if constexpr (K != kRoeH) {
        if (fz) {  // both z stages, once the side's y differences are done
          e = hipStreamWaitEvent(stream, v.ydone, 0);
          if (e != hipSuccess) return e;
          hipLaunchKernelGGL((k_sweep_z_both<T, HIST, K, R>), nblocks(P_S1_Z), B, 0, stream,
                             tab(P_S1_Z));
          return hipGetLastError();
        }
      }
      e = hipEventRecord(v.xdone, stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(v.side, v.xdone, 0);
      if (e != hipSuccess) return e;
      if constexpr (K == kRoeH)  // eta along z
        hipLaunchKernelGGL((k_sweep_march<T, 2, 3, false, K, R>), nblocks(P_ETA_Z), B, 0, v.side,
                           tab(P_ETA_Z));
      else
        hipLaunchKernelGGL((k_sweep_march<T, 2, 2, HIST, K, R>), nblocks(P_S2_Z), B, 0, v.side,
                           tab(P_S2_Z));
      e = hipEventRecord(v.join, v.side);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_sweep_march<T, 2, 1, HIST, K, R>), nblocks(P_S1_Z), B, 0, stream,
                         tab(P_S1_Z));
    } else {
      CTU_TIMED(K_SWEEP1_X, hipLaunchKernelGGL((k_sweep_x<T, 1, HIST, K, R>), nblocks(P_S1_X), B,
                                               0, stream, tab(P_S1_X)));
      CTU_TIMED(K_SWEEP1_Y, hipLaunchKernelGGL((k_sweep_march<T, 1, 1, HIST, K, R>),
                                               nblocks(P_S1_Y), B, 0, stream, tab(P_S1_Y)));
      CTU_TIMED(K_SWEEP1_Z, hipLaunchKernelGGL((k_sweep_march<T, 2, 1, HIST, K, R>),
                                               nblocks(P_S1_Z), B, 0, stream, tab(P_S1_Z)));
    }
  } else {
    // the side's PPMP y coefficients (read by the second-stage y sweep) and first-stage y
    // differences (read by the eta pass along x)
    if (overlap && (R == 1 || K == kRoeH)) {
      e = hipStreamWaitEvent(stream, v.ydone, 0);
      if (e != hipSuccess) return e;
    }
    if constexpr (K == kRoeH) {
      // eta of every face the H stencils of the second stage read
      // (along y the second-stage y sweep computes them itself)
      CTU_TIMED(K_HCORR_ETA, hipLaunchKernelGGL((k_eta_x<T, R>), nblocks(P_ETA_X), B, 0, stream,
                                                tab(P_ETA_X)));
      if (overlap) {  // eta along z came from the side stream
        e = hipStreamWaitEvent(stream, v.join, 0);
        if (e != hipSuccess) return e;
      } else {
        CTU_TIMED(K_HCORR_ETA, hipLaunchKernelGGL((k_sweep_march<T, 2, 3, false, K, R>),
                                                  nblocks(P_ETA_Z), B, 0, stream, tab(P_ETA_Z)));
      }
    }
    // a2-a4 re-traced, a6-a7: G^{n+1/2}, H^{n+1/2} on the real faces, then F^{n+1/2} with the
    // update (a8) and the CFL bound of the new state (a9)
    CTU_TIMED(K_SWEEP2_Y, hipLaunchKernelGGL((k_sweep_march<T, 1, 2, HIST, K, R>), nblocks(P_S2_Y),
                                             B, 0, stream, tab(P_S2_Y)));
    if (fz) {
      // the second-stage z differences came from the fused z march
    } else if (overlap && K != kRoeH) {  // the second-stage z sweep ran on the side stream
      e = hipStreamWaitEvent(stream, v.join, 0);
      if (e != hipSuccess) return e;
    } else {
      CTU_TIMED(K_SWEEP2_Z, hipLaunchKernelGGL((k_sweep_march<T, 2, 2, HIST, K, R>),
                                               nblocks(P_S2_Z), B, 0, stream, tab(P_S2_Z)));
    }
    CTU_TIMED(K_SWEEP2_X_UPDATE,
              hipLaunchKernelGGL((k_sweep_x_update<T, HIST, K, R>), nblocks(P_S2_X), B, 0, stream,
                                 tab(P_S2_X)));
  }
  return hipGetLastError();
}

}  // namespace ctu
