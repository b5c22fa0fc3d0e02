// ctu_device.hpp -- device-side arithmetic of the CTU step for gfx950: equation of state,
// PPMC reconstruction with characteristic tracing (App. A.3 of Schneider & Robertson 2015,
// reusing the PLMC slope step of App. A.2) and the exact Riemann solver (App. B.1).
//
// Storage type T is double or float.  The star-pressure Newton iteration always runs in
// double (the FP32 form keeps FP64 there).  Readings of garbled equations follow the same
// corrections the paper's own consistency demands: projection xi_0 = (dp/a^2 - rho du/a)/2,
// w6 = 6w - 3(W_L + W_R), B and D as differences of the alpha^m/alpha^p and beta^p/beta^0
// integrals, right-fan speed 2/(g+1)(a_R - (g-1)/2 u_R).
#pragma once

#include <hip/hip_runtime.h>

namespace ctu {

// Per-grid constants passed by value to every kernel.
struct GridParams {
  int n[3];             // real cells per axis
  int ng;               // ghost layers per side: 3 (PPMC), 4 (PPMP), plus ext
  int N[3];             // allocated cells per axis (n + 2 ng)
  long long stride;     // elements between consecutive fields
  double dx[3];         // cell widths
  double gamma;
  double newton_tol;
  int newton_max_iter;
  double p_floor;
  double cfl;
  // derived gamma constants
  double gm1;           // gamma - 1
  double z_exp;         // (gamma - 1) / (2 gamma)
  double inv_gamma;     // 1 / gamma
  double two_over_gm1;  // 2 / (gamma - 1)
  double two_over_gp1;  // 2 / (gamma + 1)
  double gm1_over_gp1;  // (gamma - 1) / (gamma + 1)
  double shock_a;       // (gamma + 1) / (2 gamma)
  double shock_b;       // (gamma - 1) / (2 gamma)
  int fan_int_exp;      // 2/(gamma-1) when it is an integer (3 for 5/3, 5 for 7/5), else 0
  int root_m;           // 2 gamma/(gamma-1) when it is an integer (5 for 5/3, 7 for 7/5), else 0
  double inv_root_m;    // (gamma - 1) / (2 gamma)
  double inv_gm1;       // 1 / (gamma - 1)
  int seg[3];           // faces per thread segment of the marching sweeps along y and z
  int xrows;            // x-rows of real cells per wavefront in the fused x update
  int xchunks;          // chunks of the flattened line per wavefront of the first-stage x sweep
  int riemann;          // 0 exact, 1 Roe with the HLLE failsafe
  int recon;            // 0 PPMC, 1 PPMP
  int ext;              // 1 with the H correction: the first stage covers one more cell
                        // along its axis, whose second-stage states the eta pass needs
};

// Device scalars of one grid (in the workspace).
struct DevScalars {
  double dt;                        // time step of the step being taken
  double t;                         // accumulated simulation time
  unsigned long long dt_next_bits;  // min over real cells of the CFL bound (before C0), as bits
  unsigned int flags;               // CTU_FLAG_* bits
  unsigned int pad0;
  unsigned long long counters[4];   // p-floor hits, Newton caps, non-physical cells, reserved
  long long steps;
  double t_end;                     // end time of the device-side time step
  long long steps_left;             // step budget of the device-side time step
  unsigned long long newton_hist[8];  // Newton iterations per solve: 1, 2, 3, 4, 5-8, 9-16,
                                      // >16, cap (instrumented steps only)
};

__device__ __forceinline__ long long cell_index(const GridParams& P, int i, int j, int k) {
  const int g = P.ng;
  return (long long)(i + g) + (long long)P.N[0] * ((long long)(j + g) + (long long)P.N[1] * (k + g));
}

// ---- type-generic math -----------------------------------------------------------------
__device__ __forceinline__ double tsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float tsqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double tpow(double x, double y) { return pow(x, y); }
__device__ __forceinline__ float tpow(float x, float y) { return powf(x, y); }
__device__ __forceinline__ double tfabs(double x) { return fabs(x); }
__device__ __forceinline__ float tfabs(float x) { return fabsf(x); }
__device__ __forceinline__ double tmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float tmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double tmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float tmax(float a, float b) { return fmaxf(a, b); }

// Integer power for the fan exponents when 2/(gamma-1) is an integer.
template <typename T>
__device__ __forceinline__ T ipow(T x, int n) {
  T r = T(1);
  for (int i = 0; i < n; ++i) r *= x;
  return r;
}

// ---- equation of state (Sec. 2) --------------------------------------------------------
// Conserved (rho, m_n, m_t1, m_t2, E) -> primitive (rho, v_n, v_t1, v_t2, p >= p_floor).
template <typename T>
__device__ __forceinline__ bool cons_to_prim(const T U[5], T gm1, T p_floor, T W[5]) {
  T rho = U[0];
  T u = U[1] / rho, v = U[2] / rho, w = U[3] / rho;
  T p = gm1 * (U[4] - T(0.5) * rho * (u * u + v * v + w * w));
  bool floored = !(p >= p_floor);
  if (floored) p = p_floor;
  W[0] = rho;
  W[1] = u;
  W[2] = v;
  W[3] = w;
  W[4] = p;
  return floored;
}

template <typename T>
__device__ __forceinline__ void prim_to_cons(const T W[5], T gm1, T U[5]) {
  T rho = W[0];
  U[0] = rho;
  U[1] = rho * W[1];
  U[2] = rho * W[2];
  U[3] = rho * W[3];
  U[4] = W[4] / gm1 + T(0.5) * rho * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
}

// ---- PPMC (App. A.3) -------------------------------------------------------------------
// Monotonized-central limiter, sgn(0) = +1.
template <typename T>
__device__ __forceinline__ T mc_limit(T dl, T dr, T dc) {
  if (dl * dr > T(0)) {
    T m = tmin(tfabs(dc), tmin(T(2) * tfabs(dl), T(2) * tfabs(dr)));
    return dc < T(0) ? -m : m;
  }
  return T(0);
}

template <typename T>
__device__ __forceinline__ T ppm_IL(T alpha, T dw, T w6) {
  return T(0.5) * alpha * (dw + w6 * (T(1) + (T(2) / T(3)) * alpha));
}
template <typename T>
__device__ __forceinline__ T ppm_IR(T beta, T dw, T w6) {
  return T(0.5) * beta * (dw - w6 * (T(1) - (T(2) / T(3)) * beta));
}

// ---- exact Riemann solver (App. B.1) -----------------------------------------------------
// Newton iterations recorded for a solve that hit the iteration cap.
constexpr int kItersCapped = 1 << 30;

struct RiemannCounts {
  unsigned floors;
  unsigned caps;
  int iters;      // Newton iterations of the last solve (0 for equal states, kItersCapped
                  // when it hit the cap)
  unsigned hlle;  // Roe solves that substituted the HLLE flux
};

// ======================================================================================
// Forms used by the fused sweep kernels, arranged for the gfx950 VALU: one reciprocal per
// cell instead of repeated divisions, and the power (p/p_k)^((g-1)/(2g)) of the Riemann
// solver taken as an integer root when 2g/(g-1) is an integer.  They differ from the
// textbook formulas only by rounding.
// ======================================================================================

// Reciprocal, quotient and square root for positive normal operands from the hardware
// estimates (v_rcp_f64, v_rsq_f64) refined by Newton-Raphson steps in fused multiply-adds:
// within about an ulp of the correctly rounded result, in roughly half the instructions of
// the IEEE expansions (which also handle zero, denormal and overflowing operands).
__device__ __forceinline__ double rcp_nr(double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  return fma(r, fma(-b, r, 1.0), r);
}
__device__ __forceinline__ float rcp_nr(float b) {
  const float r = __builtin_amdgcn_rcpf(b);
  return fmaf(r, fmaf(-b, r, 1.0f), r);
}
template <typename T>
__device__ __forceinline__ T div_nr(T a, T b) {
  const T r = rcp_nr(b);
  const T q = a * r;
  return fma(r, fma(-b, q, a), q);
}
// s = sqrt(x) and rs = 1/sqrt(x) (coupled Newton iteration on g ~ sqrt(x), h ~ 1/(2 sqrt(x))).
__device__ __forceinline__ void sqrt_rsqrt_nr(double x, double& s, double& rs) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  s = fma(fma(-g, g, x), h, g);
  rs = 2.0 * h;
}
__device__ __forceinline__ void sqrt_rsqrt_nr(float x, float& s, float& rs) {
  s = sqrtf(x);
  rs = rcp_nr(s);
}
__device__ __forceinline__ double sqrt_nr(double x) {
  double s, rs;
  sqrt_rsqrt_nr(x, s, rs);
  return s;
}

// Inverse integer root y = r^(-1/m) for r > 0 and integer m >= 2: a float estimate from
// the hardware log2/exp2 units, then two Newton steps y <- y + y (1 - r y^m) / m in double,
// which need no division and converge quadratically from ~1e-6 relative error to full
// double precision.  Returns y and y^(m-1); then r^(1/m) = r y^(m-1).  Outside the float
// range r is first scaled by 2^(-m j) (an exact power of two), so y scales by 2^j.
// M > 0 fixes m at compile time; M = 0 takes the runtime m.
template <int M>
__device__ __forceinline__ void inv_root_int(double r, int m_rt, double inv_m_rt, double& y,
                                             double& ym1) {
  const int m = M > 0 ? M : m_rt;
  const double inv_m = M > 0 ? 1.0 / M : inv_m_rt;
  float rf = (float)r;
  int j = 0;
  if (!(rf > 1.0e-30f && rf < 1.0e30f)) {
    int e;
    (void)frexp(r, &e);
    j = e / m;
    r = ldexp(r, -m * j);
    rf = (float)r;
  }
  y = (double)__builtin_amdgcn_exp2f(-__builtin_amdgcn_logf(rf) * (float)inv_m);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    double yp = y;
#pragma unroll
    for (int i = 1; i < (M > 0 ? M : 16); ++i) {
      if (M == 0 && i >= m) break;
      yp *= y;  // y^m
    }
    y = fma(y * inv_m, fma(-r, yp, 1.0), y);
  }
  ym1 = y;
#pragma unroll
  for (int i = 2; i < (M > 0 ? M : 16); ++i) {
    if (M == 0 && i >= m) break;
    ym1 *= y;
  }
  if (j) {
    y = ldexp(y, -j);
    ym1 = ldexp(ym1, -j * (m - 1));
  }
}

// x^N for a compile-time N >= 1, or the runtime n when N = 0.
template <int N, typename T>
__device__ __forceinline__ T ipow_n(T x, int n) {
  if (N > 0) {
    T r = x;
#pragma unroll
    for (int i = 1; i < N; ++i) r *= x;
    return r;
  }
  return ipow(x, n);
}

// Primitive variables of one cell in the rotated frame of a sweep, with its sound speed
// and 1/rho.
template <typename T>
struct Prim {
  T w[5];
  T a;
  T ia;    // 1 / a
  T irho;  // 1 / rho
};

template <typename T>
__device__ __forceinline__ void make_prim(const T Ur[5], T gamma, T gm1, T p_floor, Prim<T>& c) {
  const T rho = Ur[0];
  const T ir = rcp_nr(rho);
  const T u = Ur[1] * ir, v = Ur[2] * ir, w = Ur[3] * ir;
  T p = gm1 * (Ur[4] - T(0.5) * rho * (u * u + v * v + w * w));
  if (!(p >= p_floor)) p = p_floor;
  c.w[0] = rho;
  c.w[1] = u;
  c.w[2] = v;
  c.w[3] = w;
  c.w[4] = p;
  c.irho = ir;
  sqrt_rsqrt_nr(gamma * p * ir, c.a, c.ia);
}

// PLMC slope step of cell c (App. A.2) with the cell's own rho and a.
template <typename T>
__device__ __forceinline__ void slope_fast(const Prim<T>& m, const Prim<T>& c, const Prim<T>& p,
                                           T dw[5]) {
  const T rho = c.w[0];
  const T ia = c.ia;
  const T ia2 = ia * ia;
  const T ra = rho * ia;
  T d[3][5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    d[0][q] = c.w[q] - m.w[q];
    d[1][q] = p.w[q] - c.w[q];
    d[2][q] = T(0.5) * (p.w[q] - m.w[q]);
  }
  T x0[3], x1[3], x4[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T dp = d[k][4] * ia2;
    const T du = ra * d[k][1];
    x0[k] = T(0.5) * (dp - du);
    x1[k] = d[k][0] - dp;
    x4[k] = T(0.5) * (dp + du);
  }
  const T xi0 = mc_limit(x0[0], x0[1], x0[2]);
  const T xi1 = mc_limit(x1[0], x1[1], x1[2]);
  const T xi4 = mc_limit(x4[0], x4[1], x4[2]);
  dw[0] = xi0 + xi1 + xi4;
  dw[1] = (c.a * c.irho) * (xi4 - xi0);
  dw[2] = mc_limit(d[0][2], d[1][2], d[2][2]);
  dw[3] = mc_limit(d[0][3], d[1][3], d[2][3]);
  dw[4] = (c.a * c.a) * (xi0 + xi4);
}

// PPMC parabola, monotonicity and characteristic tracing (App. A.3) of cell c from the
// primitives of c-1, c, c+1 and the limited slopes of the same three cells.
template <typename T>
__device__ __forceinline__ void trace_fast(const Prim<T>& m, const Prim<T>& c, const Prim<T>& p,
                                           const T dwm[5], const T dwc[5], const T dwp[5],
                                           T dtodx, T WsL[5], T WsR[5]) {
  const T sixth = T(1) / T(6);
  const T rho = c.w[0];
  const T a = c.a;
  const T ia = c.ia;
  const T ia2 = ia * ia;
  const T lm = c.w[1] - a, l0 = c.w[1], lp = c.w[1] + a;
  const T am = dtodx * tmin(lm, T(0)), bm = dtodx * tmax(lm, T(0));
  const T a0 = dtodx * tmin(l0, T(0)), b0 = dtodx * tmax(l0, T(0));
  const T ap = dtodx * tmin(lp, T(0)), bp = dtodx * tmax(lp, T(0));
  T dwv[5], w6v[5], ILm[5], IRp[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const T cq = c.w[q];
    T wl = T(0.5) * (cq + m.w[q]) - (dwc[q] - dwm[q]) * sixth;
    T wr = T(0.5) * (p.w[q] + cq) - (dwp[q] - dwc[q]) * sixth;
    if ((wr - cq) * (cq - wl) <= T(0)) {
      wl = cq;
      wr = cq;
    }
    if ((wr - wl) * (wl - (T(3) * cq - T(2) * wr)) < T(0)) wl = T(3) * cq - T(2) * wr;
    if ((wr - wl) * ((T(3) * cq - T(2) * wl) - wr) < T(0)) wr = T(3) * cq - T(2) * wl;
    wl = tmin(tmax(cq, m.w[q]), tmax(tmin(cq, m.w[q]), wl));
    wr = tmin(tmax(cq, p.w[q]), tmax(tmin(cq, p.w[q]), wr));
    dwv[q] = wr - wl;
    w6v[q] = T(6) * cq - T(3) * (wl + wr);
    ILm[q] = ppm_IL(am, dwv[q], w6v[q]);
    IRp[q] = ppm_IR(bp, dwv[q], w6v[q]);
    WsL[q] = wl - ILm[q];
    WsR[q] = wr - IRp[q];
  }
  // Corrections for the other waves moving toward each face; each integral difference is
  // formed only for the components its correction uses.
  if (l0 < T(0)) {
    T E[5];
#pragma unroll
    for (int q = 0; q < 5; ++q)
      if (q != 1) E[q] = ILm[q] - ppm_IL(a0, dwv[q], w6v[q]);
    WsL[0] += E[0] - E[4] * ia2;
    WsL[2] += E[2];
    WsL[3] += E[3];
  }
  if (lp < T(0)) {
    const T B1 = ILm[1] - ppm_IL(ap, dwv[1], w6v[1]);
    const T B4 = ILm[4] - ppm_IL(ap, dwv[4], w6v[4]);
    WsL[0] += T(0.5) * (rho * B1 * ia + B4 * ia2);
    WsL[1] += T(0.5) * (B1 + B4 * ia * c.irho);
    WsL[4] += T(0.5) * (rho * B1 * a + B4);
  }
  if (lm > T(0)) {
    const T C1 = IRp[1] - ppm_IR(bm, dwv[1], w6v[1]);
    const T C4 = IRp[4] - ppm_IR(bm, dwv[4], w6v[4]);
    WsR[0] += T(0.5) * (-rho * C1 * ia + C4 * ia2);
    WsR[1] += T(0.5) * (C1 - C4 * ia * c.irho);
    WsR[4] += T(0.5) * (-rho * C1 * a + C4);
  }
  if (l0 > T(0)) {
    T D[5];
#pragma unroll
    for (int q = 0; q < 5; ++q)
      if (q != 1) D[q] = IRp[q] - ppm_IR(b0, dwv[q], w6v[q]);
    WsR[0] += D[0] - D[4] * ia2;
    WsR[2] += D[2];
    WsR[3] += D[3];
  }
}

// ---- PPMP (App. A.4) -------------------------------------------------------------------
// Van Leer's monotonized central slopes of the primitive variables (App. A.1).
template <typename T>
__device__ __forceinline__ void slope_vl(const Prim<T>& m, const Prim<T>& c, const Prim<T>& p,
                                         T dw[5]) {
#pragma unroll
  for (int q = 0; q < 5; ++q)
    dw[q] = mc_limit(c.w[q] - m.w[q], p.w[q] - c.w[q], T(0.5) * (p.w[q] - m.w[q]));
}

// Per-cell PPMP coefficients along the sweep axis: shock flattening and contact steepening.
template <typename T>
struct PpmpCoef {
  T flat, eta;
};

// PPMP interface values of cell c from the primitives and van Leer slopes of c-1, c, c+1,
// density steepening (eta) and flattening (flat), the monotonicity fixes, then the
// integration under the parabola along each characteristic and the CW84 tracing with the
// chi corrections.  Readings: steepened rho_R uses rho_{c+1}; the third monotonicity rule
// sets W_R; chi^p_L takes (p^m - p^p)/C and chi^m_R takes rho^p_R.
template <typename T>
__device__ __forceinline__ void trace_ppmp(const Prim<T>& m, const Prim<T>& c, const Prim<T>& p,
                                           const T dwm[5], const T dwc[5], const T dwp[5],
                                           PpmpCoef<T> k, T gamma, T dtodx, T WsL[5],
                                           T WsR[5]) {
  const T sixth = T(1) / T(6);
  const T a = c.a;
  const T lm = c.w[1] - a, l0 = c.w[1], lp = c.w[1] + a;
  const T am = dtodx * tmin(lm, T(0)), bm = dtodx * tmax(lm, T(0));
  const T a0 = dtodx * tmin(l0, T(0)), b0 = dtodx * tmax(l0, T(0));
  const T ap = dtodx * tmin(lp, T(0)), bp = dtodx * tmax(lp, T(0));
  // time-evolved face values: L_m, L_0, L_p at the left face, R_m, R_0, R_p at the right
  T Lm[5], L0[5], Lp[5], Rm[5], R0[5], Rp[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const T cq = c.w[q];
    T wl = T(0.5) * (cq + m.w[q]) - (dwc[q] - dwm[q]) * sixth;
    T wr = T(0.5) * (p.w[q] + cq) - (dwp[q] - dwc[q]) * sixth;
    if (q == 0) {
      wl = wl * (T(1) - k.eta) + (m.w[0] + T(0.5) * dwm[0]) * k.eta;
      wr = wr * (T(1) - k.eta) + (p.w[0] - T(0.5) * dwp[0]) * k.eta;
    }
    wl = k.flat * cq + (T(1) - k.flat) * wl;
    wr = k.flat * cq + (T(1) - k.flat) * wr;
    if ((wr - cq) * (cq - wl) <= T(0)) {
      wl = cq;
      wr = cq;
    }
    if ((wr - wl) * (wl - (T(3) * cq - T(2) * wr)) < T(0)) wl = T(3) * cq - T(2) * wr;
    if ((wr - wl) * ((T(3) * cq - T(2) * wl) - wr) < T(0)) wr = T(3) * cq - T(2) * wl;
    const T dw = wr - wl;
    const T w6 = T(6) * (cq - T(0.5) * (wl + wr));
    Lm[q] = wl - ppm_IL(am, dw, w6);
    L0[q] = wl - ppm_IL(a0, dw, w6);
    Lp[q] = wl - ppm_IL(ap, dw, w6);
    Rm[q] = wr - ppm_IR(bm, dw, w6);
    R0[q] = wr - ppm_IR(b0, dw, w6);
    Rp[q] = wr - ppm_IR(bp, dw, w6);
  }
  // reference states: the fastest wave toward each face (rho, u, p); the advection wave for
  // the transverse velocities
  T aL, iaL, aR, iaR;
  const T irL = rcp_nr(Lm[0]), irR = rcp_nr(Rp[0]);
  sqrt_rsqrt_nr(gamma * Lm[4] * irL, aL, iaL);
  sqrt_rsqrt_nr(gamma * Rp[4] * irR, aR, iaR);
  const T CL = Lm[0] * aL, iCL = irL * iaL;
  const T CR = Rp[0] * aR, iCR = irR * iaR;
  T chipL = -(T(0.5) * iCL) * ((Lm[1] - Lp[1]) + (Lm[4] - Lp[4]) * iCL);
  T chimR = (T(0.5) * iCR) * ((Rp[1] - Rm[1]) - (Rp[4] - Rm[4]) * iCR);
  T chi0L = (Lm[4] - L0[4]) * (iCL * iCL) + irL - rcp_nr(L0[0]);
  T chi0R = (Rp[4] - R0[4]) * (iCR * iCR) + irR - rcp_nr(R0[0]);
  if (l0 > T(0)) chi0L = T(0);
  if (lp > T(0)) chipL = T(0);
  if (lm < T(0)) chimR = T(0);
  if (l0 < T(0)) chi0R = T(0);
  WsL[0] = rcp_nr(irL - chi0L - chipL);
  WsL[1] = Lm[1] + CL * chipL;
  WsL[2] = L0[2];
  WsL[3] = L0[3];
  WsL[4] = Lm[4] + CL * CL * chipL;
  WsR[0] = rcp_nr(irR - chimR - chi0R);
  WsR[1] = Rp[1] - CR * chimR;
  WsR[2] = R0[2];
  WsR[3] = R0[3];
  WsR[4] = Rp[4] + CR * CR * chimR;
}

// The reconstruction of the sweep kernels: R = 0 PPMC, R = 1 PPMP.
template <int R, typename T>
__device__ __forceinline__ void slope_sel(const Prim<T>& m, const Prim<T>& c, const Prim<T>& p,
                                          T dw[5]) {
  if constexpr (R == 1)
    slope_vl(m, c, p, dw);
  else
    slope_fast(m, c, p, dw);
}

template <int R, typename T>
__device__ __forceinline__ void trace_sel(const Prim<T>& m, const Prim<T>& c, const Prim<T>& p,
                                          const T dwm[5], const T dwc[5], const T dwp[5],
                                          PpmpCoef<T> k, T gamma, T dtodx, T WsL[5], T WsR[5]) {
  if constexpr (R == 1)
    trace_ppmp(m, c, p, dwm, dwc, dwp, k, gamma, dtodx, WsL, WsR);
  else
    trace_fast(m, c, p, dwm, dwc, dwp, dtodx, WsL, WsR);
}

// Pressure function and derivative at p for one side, given 1/p and the side's constants.
struct SideK {
  double rho, u, p, a;
  double ip;     // 1 / p_k
  double irhoa;  // 1 / (rho_k a_k)
  double A, B;   // 2/((g+1) rho_k), (g-1)/(g+1) p_k
};

// K is the gas class: K > 0 when 2/(g-1) = K and 2g/(g-1) = K + 2 are integers (K = 3 for
// g = 5/3, K = 5 for g = 7/5), fixed at compile time; K = 0 decides from the runtime constants.
template <int K>
__device__ __forceinline__ void pfun_fast(double p, const SideK& k, const GridParams& P,
                                          double& f, double& df, double& z) {
  if (p <= k.p) {
    const double r = p * k.ip;
    if (K > 0 || P.root_m) {
      // z = r^((g-1)/(2g)) = r y^(m-1) with y = r^(-1/m); f' = z/(r rho a) = y^(m-1)/(rho a)
      double y, ym1;
      inv_root_int<(K > 0 ? K + 2 : 0)>(r, P.root_m, P.inv_root_m, y, ym1);
      z = r * ym1;
      df = ym1 * k.irhoa;
    } else {
      z = pow(r, P.z_exp);
      df = z / r * k.irhoa;
    }
    f = P.two_over_gm1 * k.a * (z - 1.0);
  } else {
    const double ipb = rcp_nr(p + k.B);
    const double q = sqrt_nr(k.A * ipb);
    f = (p - k.p) * q;
    df = q * (1.0 - 0.5 * (p - k.p) * ipb);
    z = 0.0;
  }
}

// Exact Riemann flux from rotated conserved states (App. B.1), fast form; K as in pfun_fast.
template <typename T, int K>
__device__ __forceinline__ void exact_flux_prim(const Prim<T>& L, const Prim<T>& R,
                                                const GridParams& P, T F[5], RiemannCounts& cnt);

template <typename T, int K>
__device__ __forceinline__ void exact_flux_fast(const T UL[5], const T UR[5], const GridParams& P,
                                                T F[5], RiemannCounts& cnt) {
  const T pf = T(P.p_floor);
  Prim<T> L, R;
  make_prim(UL, T(P.gamma), T(P.gm1), pf, L);
  make_prim(UR, T(P.gamma), T(P.gm1), pf, R);
  // floor hits: make_prim applied the floor when the pressure equals p_floor after the check
  cnt.floors += (L.w[4] == pf) + (R.w[4] == pf);
  exact_flux_prim<T, K>(L, R, P, F, cnt);
}

// The same flux from primitive states (rho, u_n, u_t1, u_t2, p): the traced states of the
// first stage enter the solver without the round trip through conserved variables, which
// returns them unchanged up to rounding.  The pressure floor applies as in make_prim.
template <typename T, int K>
__device__ __forceinline__ void exact_flux_w(const T WL[5], const T WR[5], const GridParams& P,
                                             T F[5], RiemannCounts& cnt) {
  const T pf = T(P.p_floor);
  const T g = T(P.gamma);
  Prim<T> L, R;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    L.w[q] = WL[q];
    R.w[q] = WR[q];
  }
  cnt.floors += (!(L.w[4] >= pf)) + (!(R.w[4] >= pf));
  if (!(L.w[4] >= pf)) L.w[4] = pf;
  if (!(R.w[4] >= pf)) R.w[4] = pf;
  L.irho = rcp_nr(L.w[0]);
  R.irho = rcp_nr(R.w[0]);
  sqrt_rsqrt_nr(g * L.w[4] * L.irho, L.a, L.ia);
  sqrt_rsqrt_nr(g * R.w[4] * R.irho, R.a, R.ia);
  exact_flux_prim<T, K>(L, R, P, F, cnt);
}

template <typename T, int K>
__device__ __forceinline__ void exact_flux_prim(const Prim<T>& L, const Prim<T>& R,
                                                const GridParams& P, T F[5], RiemannCounts& cnt) {
  const T gm1 = T(P.gm1);

  // Equal states: the exact solution is that state at every x/t, so the flux is the state's
  // physical flux (the Newton solve would return the same up to rounding).  Uniform regions
  // trace to equal face states, so whole wavefronts there skip the solve.
  if (L.w[0] == R.w[0] && L.w[1] == R.w[1] && L.w[2] == R.w[2] && L.w[3] == R.w[3] &&
      L.w[4] == R.w[4]) {
    const T rho = L.w[0], u = L.w[1], pres = L.w[4];
    const T mu = rho * u;
    const T E = pres * T(P.inv_gm1) + T(0.5) * rho * (u * u + L.w[2] * L.w[2] + L.w[3] * L.w[3]);
    F[0] = mu;
    F[1] = mu * u + pres;
    F[2] = mu * L.w[2];
    F[3] = mu * L.w[3];
    F[4] = (E + pres) * u;
    cnt.iters = 0;
    return;
  }

  SideK kl, kr;
  kl.rho = L.w[0];
  kl.u = L.w[1];
  kl.p = L.w[4];
  kr.rho = R.w[0];
  kr.u = R.w[1];
  kr.p = R.w[4];
  if (sizeof(T) == sizeof(double)) {
    kl.a = L.a;
    kr.a = R.a;
    kl.irhoa = (double)L.irho * (double)L.ia;
    kr.irhoa = (double)R.irho * (double)R.ia;
  } else {
    kl.a = sqrt_nr(P.gamma * kl.p * rcp_nr(kl.rho));
    kr.a = sqrt_nr(P.gamma * kr.p * rcp_nr(kr.rho));
    kl.irhoa = rcp_nr(kl.rho * kl.a);
    kr.irhoa = rcp_nr(kr.rho * kr.a);
  }
  kl.ip = rcp_nr(kl.p);
  kr.ip = rcp_nr(kr.p);
  kl.A = P.two_over_gp1 * (double)L.irho;
  kr.A = P.two_over_gp1 * (double)R.irho;
  kl.B = P.gm1_over_gp1 * kl.p;
  kr.B = P.gm1_over_gp1 * kr.p;

  double pt = 0.5 * (kl.p + kr.p) + 0.125 * (kl.u - kr.u) * (kl.rho + kr.rho) * (kl.a + kr.a);
  pt = pt < 0.0 ? 0.0 : pt;
  const double gl = sqrt_nr(kl.A * rcp_nr(pt + kl.B));
  const double gr = sqrt_nr(kr.A * rcp_nr(pt + kr.B));
  double p = div_nr(gl * kl.p + gr * kr.p - (kr.u - kl.u), gl + gr);
  p = p < 1.0e-6 ? 1.0e-6 : p;
  const double du = kr.u - kl.u;
  double fl, dfl, fr, dfr, zl, zr;
  bool conv = false;
  bool same = false;  // the last Newton step left p unchanged
  for (int it = 0; it < P.newton_max_iter; ++it) {
    pfun_fast<K>(p, kl, P, fl, dfl, zl);
    pfun_fast<K>(p, kr, P, fr, dfr, zr);
    double pn = p - div_nr(fl + fr + du, dfl + dfr);
    if (!(pn >= P.p_floor)) pn = P.p_floor;
    // relative change 2|pn - p|/|pn + p| < tol, without the division
    const bool done = 2.0 * fabs(pn - p) < P.newton_tol * fabs(pn + p);
    same = pn == p;
    p = pn;
    if (done) {
      conv = true;
      cnt.iters = it + 1;
      break;
    }
  }
  cnt.caps += conv ? 0u : 1u;
  if (!conv) cnt.iters = kItersCapped;
  // u* from f_L, f_R at the final star pressure; when the last step did not move p the
  // values just computed are already those.
  if (!same) {
    pfun_fast<K>(p, kl, P, fl, dfl, zl);
    pfun_fast<K>(p, kr, P, fr, dfr, zr);
  }
  const double ps = p;
  const double us = 0.5 * (kl.u + kr.u + fr - fl);

  T rho, u, pres;
  if (us >= 0.0) {
    if (ps <= kl.p) {
      if (kl.u - kl.a >= 0.0) {
        rho = L.w[0];
        u = L.w[1];
        pres = L.w[4];
      } else if (us - kl.a * zl < 0.0) {
        rho = T(kl.rho * ((K > 0 || P.fan_int_exp) ? ipow_n<K>(zl, P.fan_int_exp)
                                                      : pow(zl, P.two_over_gm1)));
        u = T(us);
        pres = T(ps);
      } else {
        const T c = T(P.two_over_gp1) * (T(kl.a) + T(0.5) * gm1 * L.w[1]);
        const T r = div_nr(c, T(kl.a));
        const T rr_ = (K > 0 || P.fan_int_exp) ? ipow_n<K>(r, P.fan_int_exp)
                                                 : tpow(r, T(P.two_over_gm1));
        rho = L.w[0] * rr_;
        u = c;
        pres = L.w[4] * rr_ * r * r;
      }
    } else {
      const double sl = kl.u - kl.a * sqrt_nr(P.shock_a * ps * kl.ip + P.shock_b);
      if (sl >= 0.0) {
        rho = L.w[0];
        u = L.w[1];
        pres = L.w[4];
      } else {
        const double q = ps * kl.ip;
        rho = T(kl.rho * div_nr(q + P.gm1_over_gp1, q * P.gm1_over_gp1 + 1.0));
        u = T(us);
        pres = T(ps);
      }
    }
  } else {
    if (ps <= kr.p) {
      if (kr.u + kr.a <= 0.0) {
        rho = R.w[0];
        u = R.w[1];
        pres = R.w[4];
      } else if (us + kr.a * zr >= 0.0) {
        rho = T(kr.rho * ((K > 0 || P.fan_int_exp) ? ipow_n<K>(zr, P.fan_int_exp)
                                                      : pow(zr, P.two_over_gm1)));
        u = T(us);
        pres = T(ps);
      } else {
        const T c = T(P.two_over_gp1) * (T(kr.a) - T(0.5) * gm1 * R.w[1]);
        const T r = div_nr(c, T(kr.a));
        const T rr_ = (K > 0 || P.fan_int_exp) ? ipow_n<K>(r, P.fan_int_exp)
                                                 : tpow(r, T(P.two_over_gm1));
        rho = R.w[0] * rr_;
        u = -c;
        pres = R.w[4] * rr_ * r * r;
      }
    } else {
      const double sr = kr.u + kr.a * sqrt_nr(P.shock_a * ps * kr.ip + P.shock_b);
      if (sr <= 0.0) {
        rho = R.w[0];
        u = R.w[1];
        pres = R.w[4];
      } else {
        const double q = ps * kr.ip;
        rho = T(kr.rho * div_nr(q + P.gm1_over_gp1, q * P.gm1_over_gp1 + 1.0));
        u = T(us);
        pres = T(ps);
      }
    }
  }
  const T vt = (u >= T(0)) ? L.w[2] : R.w[2];
  const T wt = (u >= T(0)) ? L.w[3] : R.w[3];
  const T mu = rho * u;
  const T E = pres * T(P.inv_gm1) + T(0.5) * rho * (u * u + vt * vt + wt * wt);
  F[0] = mu;
  F[1] = mu * u + pres;
  F[2] = mu * vt;
  F[3] = mu * wt;
  F[4] = (E + pres) * u;
}

// ======================================================================================
// Roe solver with the HLLE failsafe (App. B.2), in rotated components (slot 1 normal).
// W holds the primitives with the pressure floor applied, U the conserved state built from
// them; a, irho as in Prim.  eta_h >= 0 is the H-correction
// floor on |lambda| (App. C; 0 leaves the eigenvalues unchanged).
// ======================================================================================
template <typename T>
__device__ __forceinline__ void roe_core(const Prim<T>& L, const Prim<T>& R, const T UL[5],
                                         const T UR[5], const GridParams& P, T eta_h, T F[5],
                                         RiemannCounts& cnt) {
  const T gm1 = T(P.gm1);
  T FL[5], FR[5];
  {
    const T ml = L.w[0] * L.w[1], mr = R.w[0] * R.w[1];
    FL[0] = ml;
    FL[1] = ml * L.w[1] + L.w[4];
    FL[2] = ml * L.w[2];
    FL[3] = ml * L.w[3];
    FL[4] = (UL[4] + L.w[4]) * L.w[1];
    FR[0] = mr;
    FR[1] = mr * R.w[1] + R.w[4];
    FR[2] = mr * R.w[2];
    FR[3] = mr * R.w[3];
    FR[4] = (UR[4] + R.w[4]) * R.w[1];
  }
  // equal states: dU = 0, so every wave strength vanishes and the flux is F_L
  if (L.w[0] == R.w[0] && L.w[1] == R.w[1] && L.w[2] == R.w[2] && L.w[3] == R.w[3] &&
      L.w[4] == R.w[4]) {
#pragma unroll
    for (int q = 0; q < 5; ++q) F[q] = FL[q];
    return;
  }
  // Roe averages, weights sqrt(rho)
  T sl, isl, sr, isr;
  sqrt_rsqrt_nr(L.w[0], sl, isl);
  sqrt_rsqrt_nr(R.w[0], sr, isr);
  const T isum = rcp_nr(sl + sr);
  const T HL = (UL[4] + L.w[4]) * L.irho, HR = (UR[4] + R.w[4]) * R.irho;
  const T ut = (sl * L.w[1] + sr * R.w[1]) * isum;
  const T vt = (sl * L.w[2] + sr * R.w[2]) * isum;
  const T wt = (sl * L.w[3] + sr * R.w[3]) * isum;
  const T Ht = (sl * HL + sr * HR) * isum;
  const T V2 = ut * ut + vt * vt + wt * wt;
  // a~^2 = (g-1)(H~ - V~^2/2) through the equal form (g-1)[w_L h_L + w_R h_R +
  // w_L w_R |V_L - V_R|^2 / 2], h = a^2/(g-1): no cancellation when p/rho << V^2
  const T wl = sl * isum, wr = sr * isum;
  const T dv0 = R.w[1] - L.w[1], dv1 = R.w[2] - L.w[2], dv2 = R.w[3] - L.w[3];
  T at, iat;
  sqrt_rsqrt_nr(wl * (L.a * L.a) + wr * (R.a * R.a) +
                    T(0.5) * gm1 * wl * wr * (dv0 * dv0 + dv1 * dv1 + dv2 * dv2),
                at, iat);
  const T lm = ut - at, lp = ut + at;
  if (lm >= T(0)) {  // supersonic to the right
#pragma unroll
    for (int q = 0; q < 5; ++q) F[q] = FL[q];
    return;
  }
  if (lp <= T(0)) {  // supersonic to the left
#pragma unroll
    for (int q = 0; q < 5; ++q) F[q] = FR[q];
    return;
  }
  T dU[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) dU[q] = UR[q] - UL[q];
  const T ia2 = iat * iat;
  const T Na = T(0.5) * ia2;
  const T gv = gm1 * (vt * dU[2] + wt * dU[3]);  // shared transverse terms
  const T gE = gm1 * dU[4];
  const T xi0 = Na * (dU[0] * (T(0.5) * gm1 * V2 + ut * at) - dU[1] * (gm1 * ut + at) - gv + gE);
  const T xi1 = dU[2] - dU[0] * vt;
  const T xi2 = dU[3] - dU[0] * wt;
  const T xi3 = dU[0] * (T(1) - Na * gm1 * V2) + ia2 * (gm1 * ut * dU[1] + gv - gE);
  const T xi4 = Na * (dU[0] * (T(0.5) * gm1 * V2 - ut * at) - dU[1] * (gm1 * ut - at) - gv + gE);
  const T am = fmax(fabs(lm), eta_h), a0 = fmax(fabs(ut), eta_h), ap = fmax(fabs(lp), eta_h);
  const T C0 = xi0 * am, C1 = xi1 * a0, C2 = xi2 * a0, C3 = xi3 * a0, C4 = xi4 * ap;
  const T uat = ut * at;
  // intermediate states: crossing the left acoustic wave, then the contact and shear waves
  T Um[5];
  Um[0] = UL[0] + xi0;
  Um[1] = UL[1] + xi0 * lm;
  Um[2] = UL[2] + xi0 * vt;
  Um[3] = UL[3] + xi0 * wt;
  Um[4] = UL[4] + xi0 * (Ht - uat);
  // positive pressure <=> 2 E rho - |m|^2 > 0 once rho > 0
  bool bad = !(Um[0] > T(0)) ||
             !(T(2) * Um[4] * Um[0] - (Um[1] * Um[1] + Um[2] * Um[2] + Um[3] * Um[3]) > T(0));
  if (!bad) {
    Um[0] += xi3;
    Um[1] += xi3 * ut;
    Um[2] += xi1 + xi3 * vt;
    Um[3] += xi2 + xi3 * wt;
    Um[4] += xi1 * vt + xi2 * wt + T(0.5) * xi3 * V2;
    bad = !(Um[0] > T(0)) ||
          !(T(2) * Um[4] * Um[0] - (Um[1] * Um[1] + Um[2] * Um[2] + Um[3] * Um[3]) > T(0));
  }
  if (!bad) {
    const T s0 = C0 + C3 + C4;
    const T s1 = C0 * lm + C3 * ut + C4 * lp;
    const T s2 = (C0 + C3 + C4) * vt + C1;
    const T s3 = (C0 + C3 + C4) * wt + C2;
    const T s4 = C0 * (Ht - uat) + C1 * vt + C2 * wt + T(0.5) * C3 * V2 + C4 * (Ht + uat);
    F[0] = T(0.5) * (FL[0] + FR[0] - s0);
    F[1] = T(0.5) * (FL[1] + FR[1] - s1);
    F[2] = T(0.5) * (FL[2] + FR[2] - s2);
    F[3] = T(0.5) * (FL[3] + FR[3] - s3);
    F[4] = T(0.5) * (FL[4] + FR[4] - s4);
    return;
  }
  // HLLE: bounding speeds from the Roe eigenvalues and the input acoustic speeds
  cnt.hlle += 1;
  const T bm = fmin(fmin(lm, L.w[1] - L.a), T(0));
  const T bp = fmax(fmax(lp, R.w[1] + R.a), T(0));
  const T ratio = (bp + bm) * rcp_nr(bp - bm);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const T fl = FL[q] - bm * UL[q];
    const T fr = FR[q] - bp * UR[q];
    F[q] = T(0.5) * ((fl + fr) + (fl - fr) * ratio);
  }
}

// Roe flux from rotated conserved states (second stage).  The solver starts from the
// primitive states (App. B.2): the conserved states it uses are rebuilt from them, so a
// floored pressure also sets the total energy.
template <typename T>
__device__ __forceinline__ void roe_flux_u(const T Uin_L[5], const T Uin_R[5], const GridParams& P,
                                           T eta_h, T F[5], RiemannCounts& cnt) {
  const T pf = T(P.p_floor), igm1 = T(P.inv_gm1);
  Prim<T> L, R;
  make_prim(Uin_L, T(P.gamma), T(P.gm1), pf, L);
  make_prim(Uin_R, T(P.gamma), T(P.gm1), pf, R);
  cnt.floors += (L.w[4] == pf) + (R.w[4] == pf);
  T UL[5], UR[5];
  UL[0] = L.w[0];
  UR[0] = R.w[0];
#pragma unroll
  for (int q = 1; q < 4; ++q) {
    UL[q] = L.w[0] * L.w[q];
    UR[q] = R.w[0] * R.w[q];
  }
  UL[4] = L.w[4] * igm1 + T(0.5) * L.w[0] * (L.w[1] * L.w[1] + L.w[2] * L.w[2] + L.w[3] * L.w[3]);
  UR[4] = R.w[4] * igm1 + T(0.5) * R.w[0] * (R.w[1] * R.w[1] + R.w[2] * R.w[2] + R.w[3] * R.w[3]);
  roe_core(L, R, UL, UR, P, eta_h, F, cnt);
}

// Roe flux from rotated primitive states (the traced states of the first stage), with the
// pressure floor as in make_prim and E = p/(g-1) + rho V^2/2.
template <typename T>
__device__ __forceinline__ void roe_flux_w(const T WL[5], const T WR[5], const GridParams& P,
                                           T eta_h, T F[5], RiemannCounts& cnt) {
  const T pf = T(P.p_floor);
  const T g = T(P.gamma), igm1 = T(P.inv_gm1);
  Prim<T> L, R;
  T UL[5], UR[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    L.w[q] = WL[q];
    R.w[q] = WR[q];
  }
  cnt.floors += (!(L.w[4] >= pf)) + (!(R.w[4] >= pf));
  if (!(L.w[4] >= pf)) L.w[4] = pf;
  if (!(R.w[4] >= pf)) R.w[4] = pf;
  L.irho = rcp_nr(L.w[0]);
  R.irho = rcp_nr(R.w[0]);
  sqrt_rsqrt_nr(g * L.w[4] * L.irho, L.a, L.ia);
  sqrt_rsqrt_nr(g * R.w[4] * R.irho, R.a, R.ia);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    UL[q] = q == 0 ? L.w[0] : L.w[0] * L.w[q];
    UR[q] = q == 0 ? R.w[0] : R.w[0] * R.w[q];
  }
  UL[4] = L.w[4] * igm1 + T(0.5) * L.w[0] * (L.w[1] * L.w[1] + L.w[2] * L.w[2] + L.w[3] * L.w[3]);
  UR[4] = R.w[4] * igm1 + T(0.5) * R.w[0] * (R.w[1] * R.w[1] + R.w[2] * R.w[2] + R.w[3] * R.w[3]);
  roe_core(L, R, UL, UR, P, eta_h, F, cnt);
}

// Solver class of the sweep kernels: the exact solver specialized for its gas class K (0, 3
// or 5), the Roe solver (kRoe), or the Roe solver with the H correction of its second-stage
// fluxes (kRoeH).
constexpr int kRoe = 1;
constexpr int kRoeH = 2;

template <typename T, int K>
__device__ __forceinline__ void face_flux_w(const T WL[5], const T WR[5], const GridParams& P,
                                            T F[5], RiemannCounts& cnt) {
  if constexpr (K == kRoe || K == kRoeH)  // the first stage is not H-corrected
    roe_flux_w<T>(WL, WR, P, T(0), F, cnt);
  else
    exact_flux_w<T, K>(WL, WR, P, F, cnt);
}

// eta_h: the H-correction floor (kRoeH only).
template <typename T, int K>
__device__ __forceinline__ void face_flux_u(const T UL[5], const T UR[5], const GridParams& P,
                                            T F[5], RiemannCounts& cnt, T eta_h = T(0)) {
  if constexpr (K == kRoeH)
    roe_flux_u<T>(UL, UR, P, eta_h, F, cnt);
  else if constexpr (K == kRoe)
    roe_flux_u<T>(UL, UR, P, T(0), F, cnt);
  else
    exact_flux_fast<T, K>(UL, UR, P, F, cnt);
}

}  // namespace ctu
