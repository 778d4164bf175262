// Gas model of the hot path, shared by the edge and vertex passes and the
// adjoint: Euler fluxes in perturbation form about a reference state (zero in
// the float64 form), the Roe state with its eigenvector matrices, and the
// Riemann fluxes (Rusanov, Roe with an entropy fix, HLLC; Section 2.3).
// Templates over the arithmetic type: float, double, and the forward-mode
// dual numbers through which the adjoint differentiates the Roe and HLLC
// fluxes.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.h"

namespace hfd {

// Division, reciprocal and square root.  The float32 form uses the hardware
// reciprocal and square root (about 1 ulp, far below the rounding of its
// float32 perturbation data) instead of the much longer correctly rounded
// instruction sequences.  float64 keeps correctly rounded division and square
// root; its reciprocals 1/x take the hardware estimate (relative error about
// 2^-23) and two Newton-Raphson steps r <- r + r (1 - x r), each of which
// squares the relative error, to within about an ulp (x finite, nonzero and
// of normal magnitude: the densities, sound speeds and sums of these
// kernels).
template <class T>
__device__ inline T fdiv(T a, T b) {
  return a / b;
}
template <>
__device__ inline float fdiv<float>(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);
}
template <class T>
__device__ inline T frcp(T x) {
  return T(1) / x;
}
template <>
__device__ inline float frcp<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}
template <>
__device__ inline double frcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
template <class T>
__device__ inline T fsqrt(T x) {
  return sqrt(x);
}
template <>
__device__ inline float fsqrt<float>(float x) {
  return __builtin_amdgcn_sqrtf(x);
}

// Nonlinear weights of uniform WENO5 interpolation from the five projected
// values c of one side (order c_{-2} .. c_2): Jiang-Shu smoothness indicators
// beta, alpha_j = d_j / (eps + beta_j)^2 with d = (1/16, 10/16, 5/16), and
// omega = alpha / sum(alpha).  With t_j = (eps + beta_j)^2 the weights are
// omega_j = n_j / (n_1 + n_2 + n_3), n_j = d_j t_k t_l: the same numbers with
// one reciprocal instead of six divisions (t >= eps^2, so the products
// neither underflow nor, for any finite state of these problems, overflow).
// The switch tests omega_1 in (lo, hi) as lo S < n_1 < hi S (S > 0), with no
// division; the weights themselves are formed only where the 3-node branch
// is taken.  Shared by the edge passes and the adjoint, so that both take the
// same decisions.
template <class T>
__device__ inline void weno_beta(const T c[5], T be[3]) {
  const T t1 = c[0] - T(2) * c[1] + c[2], t2 = c[0] - T(4) * c[1] + T(3) * c[2];
  const T t3 = c[1] - T(2) * c[2] + c[3], t4 = c[1] - c[3];
  const T t5 = c[2] - T(2) * c[3] + c[4], t6 = T(3) * c[2] - T(4) * c[3] + c[4];
  be[0] = T(13.0 / 12.0) * t1 * t1 + T(0.25) * t2 * t2;
  be[1] = T(13.0 / 12.0) * t3 * t3 + T(0.25) * t4 * t4;
  be[2] = T(13.0 / 12.0) * t5 * t5 + T(0.25) * t6 * t6;
}

// Both sides' indicators from an edge's six projected node values v, side 0
// reading v[0..4] and side 1 v[5..1].  With d_k = v_{k+1} - v_k and
// D_k = d_{k+1} - d_k, the second differences of the substencils are the D_k
// and the other terms D_k +- 2 d (one-sided) or d + d' (central), so the
// 13/12 D_k^2 serve both sides.
template <class T>
__device__ inline void weno_beta_pair(const T v[6], T b0[3], T b1[3]) {
  T d[5], D[4], A[4];
#pragma unroll
  for (int k = 0; k < 5; ++k) d[k] = v[k + 1] - v[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    D[k] = d[k + 1] - d[k];
    A[k] = T(13.0 / 12.0) * D[k] * D[k];
  }
  const T s0 = D[0] + T(2) * d[1], s1 = d[1] + d[2], s2 = D[2] - T(2) * d[2];
  const T r0 = D[3] - T(2) * d[3], r1 = d[2] + d[3], r2 = D[1] + T(2) * d[2];
  b0[0] = A[0] + T(0.25) * s0 * s0;
  b0[1] = A[1] + T(0.25) * s1 * s1;
  b0[2] = A[2] + T(0.25) * s2 * s2;
  b1[0] = A[3] + T(0.25) * r0 * r0;
  b1[1] = A[2] + T(0.25) * r1 * r1;
  b1[2] = A[1] + T(0.25) * r2 * r2;
}

template <class T>
__device__ inline void weno_num(const T be[3], T eps, T n[3]) {
  const T q1 = (eps + be[0]) * (eps + be[0]), q2 = (eps + be[1]) * (eps + be[1]);
  const T q3 = (eps + be[2]) * (eps + be[2]);
  n[0] = T(1.0 / 16.0) * (q2 * q3);
  n[1] = T(10.0 / 16.0) * (q1 * q3);
  n[2] = T(5.0 / 16.0) * (q1 * q2);
}

// omega_1 in (lo, hi) (false for a non-finite indicator)
template <class T>
__device__ inline bool weno_in(const T be[3], T eps, T lo, T hi) {
  T n[3];
  weno_num<T>(be, eps, n);
  const T S = n[0] + n[1] + n[2];
  return n[0] > lo * S && n[0] < hi * S;
}

template <class T>
__device__ inline void weno_omega(const T be[3], T eps, T o[3]) {
  T n[3];
  weno_num<T>(be, eps, n);
  const T r = frcp(n[0] + n[1] + n[2]);
  o[0] = n[0] * r;
  o[1] = n[1] * r;
  o[2] = n[2] * r;
}

template <class T>
__device__ inline void weno_weights(const T c[5], T eps, T be[3], T o[3]) {
  weno_beta<T>(c, be);
  weno_omega<T>(be, eps, o);
}

// Fluxes minus the reference fluxes, from the perturbation w' and the full
// density/momenta.  With a zero reference these are the plain fluxes.
template <class T>
struct Ref {
  T w[4];   // reference state
  T u, v;   // reference velocity
  T etr;    // E + p of the reference
};

template <class T>
__device__ inline void pert_flux(const T wp[4], const Ref<T>& R, T gm1, T f[4],
                                 T g[4], T* p_full = nullptr, T* rho_full = nullptr,
                                 T* u_full = nullptr, T* v_full = nullptr,
                                 T* p_pert = nullptr) {
  const T rho = R.w[0] + wp[0];
  const T m = R.w[1] + wp[1];
  const T n = R.w[2] + wp[2];
  const T ir = frcp(rho);
  // m^2/rho - m_r u_r, m n/rho - m_r v_r, n^2/rho - n_r v_r
  const T amm = (wp[1] * (m + R.w[1]) - R.w[1] * R.u * wp[0]) * ir;
  const T amn = (wp[1] * n + R.w[1] * wp[2] - R.w[1] * R.v * wp[0]) * ir;
  const T ann = (wp[2] * (n + R.w[2]) - R.w[2] * R.v * wp[0]) * ir;
  const T pp = gm1 * (wp[3] - T(0.5) * (amm + ann));  // p - p_r
  const T du = (wp[1] - R.u * wp[0]) * ir;              // u - u_r
  const T dv = (wp[2] - R.v * wp[0]) * ir;              // v - v_r
  const T u = R.u + du, v = R.v + dv;
  const T etp = wp[3] + pp;                              // (E + p) - (E + p)_r
  f[0] = wp[1];
  f[1] = amm + pp;
  f[2] = amn;
  f[3] = etp * u + R.etr * du;
  g[0] = wp[2];
  g[1] = amn;
  g[2] = ann + pp;
  g[3] = etp * v + R.etr * dv;
  if (p_full) {
    *p_full = (R.etr - R.w[3]) + pp;
    *rho_full = rho;
    *u_full = u;
    *v_full = v;
  }
  if (p_pert) *p_pert = pp;
}

// A parameter in the kernel's precision: float32 kernels take the copy the
// host rounded once, the others convert the float64 value.
template <class T>
__device__ inline T gpar(double d, float f) {
  if constexpr (std::is_same<T, float>::value) return f;
  else return T(d);
}

template <class T>
__device__ inline Ref<T> make_ref(const GasParams& gp) {
  Ref<T> r;
  if constexpr (std::is_same<T, float>::value) {
    for (int q = 0; q < 4; ++q) r.w[q] = gp.f_wref[q];
    r.u = gp.f_uref;
    r.v = gp.f_vref;
    r.etr = gp.f_etr_ref;
  } else {
    // only the float32 kernels carry a reference state: the float64 form
    // (and the adjoint's dual-number fluxes of full states) have none
    for (int q = 0; q < 4; ++q) r.w[q] = T(0);
    r.u = r.v = r.etr = T(0);
  }
  return r;
}

// Roe average of the edge's end states (nodes i, i+1) along n.  The
// eigenvector matrices of the flux Jacobian are applied from its scalars:
// proj(w) = L w (rows of L: the left eigenvectors for u.n - c, u.n, u.n + c
// and the shear wave) and back(C) = R C (columns of R: the right ones), each
// in about 14 operations instead of the 16 multiply-adds of a 4 x 4 product,
// with 11 values to hold instead of the 32 entries of L and R.
template <class T>
struct RoeState {
  T u, v, hh, cc, un, ut, b1, b2, ic, nx, ny;
  __device__ void proj(const T w[4], T o[4]) const {
    // L w = (a + b, 2 (w0 - a), a - b) / 2 and the shear row, with
    // a = b2 w0 - b1 (u w1 + v w2 - w3), b = (un w0 - nx w1 - ny w2) / c
    const T a = b2 * w[0] - b1 * (u * w[1] + v * w[2] - w[3]);
    const T b = ic * (un * w[0] - nx * w[1] - ny * w[2]);
    o[0] = T(0.5) * (a + b);
    o[1] = w[0] - a;
    o[2] = T(0.5) * (a - b);
    o[3] = -ut * w[0] - ny * w[1] + nx * w[2];
  }
  __device__ void back(const T C[4], T o[4]) const {
    const T sum = C[0] + C[1] + C[2], d = cc * (C[2] - C[0]);
    o[0] = sum;
    o[1] = u * sum + nx * d - ny * C[3];
    o[2] = v * sum + ny * d + nx * C[3];
    o[3] = hh * (C[0] + C[2]) + T(0.5) * (u * u + v * v) * C[1] + un * d + ut * C[3];
  }
};

template <class T>
__device__ inline RoeState<T> roe_state(const V4<T>& A, const V4<T>& B, T nx, T ny,
                                        const Ref<T>& ref, T gm1) {
  const T ra = ref.w[0] + A.x, rb = ref.w[0] + B.x;
  const T ira = frcp(ra), irb = frcp(rb);
  const T ua = (ref.w[1] + A.y) * ira, ub = (ref.w[1] + B.y) * irb;
  const T va = (ref.w[2] + A.z) * ira, vb = (ref.w[2] + B.z) * irb;
  const T Ea = ref.w[3] + A.w, Eb = ref.w[3] + B.w;
  const T pa = gm1 * (Ea - T(0.5) * ra * (ua * ua + va * va));
  const T pb = gm1 * (Eb - T(0.5) * rb * (ub * ub + vb * vb));
  const T sa = fsqrt(ra), sb = fsqrt(rb);
  const T iw = frcp(sa + sb);
  const T u = (sa * ua + sb * ub) * iw;
  const T v = (sa * va + sb * vb) * iw;
  const T hh = (sa * (Ea + pa) * ira + sb * (Eb + pb) * irb) * iw;
  const T cc = fsqrt(gm1 * (hh - T(0.5) * (u * u + v * v)));
  const T q2 = u * u + v * v;
  const T un = u * nx + v * ny, ut = -u * ny + v * nx;
  const T ic = frcp(cc), b1 = gm1 * ic * ic, b2 = T(0.5) * b1 * q2;
  return RoeState<T>{u, v, hh, cc, un, ut, b1, b2, ic, nx, ny};
}

// The same with the matrices stored (Roe's flux).
template <class T>
struct Frame {
  T L[4][4], R[4][4];
  T un, c;  // normal velocity and sound speed of the Roe state
};

template <class T>
__device__ inline Frame<T> roe_frame(const V4<T>& A, const V4<T>& B, T nx, T ny,
                                     const Ref<T>& ref, T gm1) {
  const RoeState<T> S = roe_state<T>(A, B, nx, ny, ref, gm1);
  const T u = S.u, v = S.v, hh = S.hh, cc = S.cc, un = S.un, ut = S.ut;
  const T b1 = S.b1, b2 = S.b2, ic = S.ic, q2 = u * u + v * v;
  return Frame<T>{
      {{T(0.5) * (b2 + un * ic), T(-0.5) * (b1 * u + nx * ic), T(-0.5) * (b1 * v + ny * ic), T(0.5) * b1},
       {T(1) - b2, b1 * u, b1 * v, -b1},
       {T(0.5) * (b2 - un * ic), T(-0.5) * (b1 * u - nx * ic), T(-0.5) * (b1 * v - ny * ic), T(0.5) * b1},
       {-ut, -ny, nx, T(0)}},
      {{T(1), T(1), T(1), T(0)},
       {u - cc * nx, u, u + cc * nx, -ny},
       {v - cc * ny, v, v + cc * ny, nx},
       {hh - un * cc, T(0.5) * q2, hh + un * cc, ut}},
      un, cc};
}

// Rusanov flux along n of the two interface states (perturbation form),
// h = (F_L.n + F_R.n)/2 - lam (w_R - w_L)/2 with lam the larger of the two
// sides' |u.n| + c.  One side's part: its normal flux fn and speed sp.
template <class T>
__device__ inline void rusanov_side(const T w[4], T nx, T ny, const Ref<T>& ref, T gam, T gm1,
                                    T fn[4], T& sp) {
  T f[4], g[4], p, r, u, v;
  pert_flux<T>(w, ref, gm1, f, g, &p, &r, &u, &v);
  sp = fabs(u * nx + v * ny) + fsqrt(gam * p * frcp(r));
#pragma unroll
  for (int q = 0; q < 4; ++q) fn[q] = f[q] * nx + g[q] * ny;
}

template <class T>
__device__ inline void rusanov_join(const T wl[4], const T wr[4], const T fnl[4],
                                    const T fnr[4], T sl, T sr, T h[4]) {
  // NaN-propagating maximum: a non-physical state must not be hidden
  const T lam = (isnan(sl) || isnan(sr)) ? sl + sr : (sl > sr ? sl : sr);
#pragma unroll
  for (int q = 0; q < 4; ++q) h[q] = T(0.5) * (fnl[q] + fnr[q]) - T(0.5) * lam * (wr[q] - wl[q]);
}

template <class T>
__device__ inline void rusanov(const T wl[4], const T wr[4], T nx, T ny, const Ref<T>& ref,
                               T gam, T gm1, T h[4]) {
  T fnl[4], fnr[4], sl, sr;
  rusanov_side<T>(wl, nx, ny, ref, gam, gm1, fnl, sl);
  rusanov_side<T>(wr, nx, ny, ref, gam, gm1, fnr, sr);
  rusanov_join<T>(wl, wr, fnl, fnr, sl, sr, h);
}

// Roe's flux at the Roe average of the two interface states, with Harten's
// entropy fix on the acoustic waves (|lambda| < d -> (lambda^2 + d^2)/(2 d),
// d = 0.1 (|u.n| + c)); the dissipation acts on w_R - w_L, which the
// perturbation form gives exactly.
template <class T>
__device__ inline void roe_flux(const T wl[4], const T wr[4], T nx, T ny, const Ref<T>& ref,
                                T gm1, T h[4]) {
  T fl[4], gl[4], fr[4], gr[4];
  pert_flux<T>(wl, ref, gm1, fl, gl);
  pert_flux<T>(wr, ref, gm1, fr, gr);
  const Frame<T> F = roe_frame<T>(V4<T>{wl[0], wl[1], wl[2], wl[3]},
                                  V4<T>{wr[0], wr[1], wr[2], wr[3]}, nx, ny, ref, gm1);
  const T d = T(0.1) * (fabs(F.un) + F.c);
  const T lam[4] = {F.un - F.c, F.un, F.un + F.c, F.un};
  T al[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    al[k] = fabs(lam[k]);
    if ((k == 0 || k == 2) && al[k] < d) al[k] = fdiv(lam[k] * lam[k] + d * d, T(2) * d);
  }
  const T dw[4] = {wr[0] - wl[0], wr[1] - wl[1], wr[2] - wl[2], wr[3] - wl[3]};
  T a[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    a[k] = al[k] * (F.L[k][0] * dw[0] + F.L[k][1] * dw[1] + F.L[k][2] * dw[2] + F.L[k][3] * dw[3]);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    h[q] = T(0.5) * ((fl[q] + fr[q]) * nx + (gl[q] + gr[q]) * ny) -
           T(0.5) * (F.R[q][0] * a[0] + F.R[q][1] * a[1] + F.R[q][2] * a[2] + F.R[q][3] * a[3]);
}

// Toro's HLLC flux with the Davis-Einfeldt wave speeds (Roe state).  In the
// perturbation form the star-state jumps U*_K - U_K are written so that no
// large terms cancel: with g = (S_M - u_nK)/(S_K - S_M) and f = 1 + g,
//   rho* - rho = g rho,  m* - m = g m + f rho (S_M - u_nK) n,
//   E* - E = g E + f rho (S_M - u_nK)(S_M + p/(rho (S_K - u_nK))),
// and pressure differences are taken from the perturbations.
template <class T>
__device__ inline void hllc_flux(const T wl[4], const T wr[4], T nx, T ny, const Ref<T>& ref,
                                 T gam, T gm1, T h[4]) {
  T fl[4], gl[4], fr[4], gr[4], pl, rl, ul, vl, pr, rr, ur, vr, ppl, ppr;
  pert_flux<T>(wl, ref, gm1, fl, gl, &pl, &rl, &ul, &vl, &ppl);
  pert_flux<T>(wr, ref, gm1, fr, gr, &pr, &rr, &ur, &vr, &ppr);
  const Frame<T> F = roe_frame<T>(V4<T>{wl[0], wl[1], wl[2], wl[3]},
                                  V4<T>{wr[0], wr[1], wr[2], wr[3]}, nx, ny, ref, gm1);
  const T unl = ul * nx + vl * ny, unr = ur * nx + vr * ny;
  const T cl = fsqrt(fdiv(gam * pl, rl)), cr = fsqrt(fdiv(gam * pr, rr));
  const T sl = fmin(unl - cl, F.un - F.c), sr = fmax(unr + cr, F.un + F.c);
  const T sm = fdiv((ppr - ppl) + rl * unl * (sl - unl) - rr * unr * (sr - unr),
                    rl * (sl - unl) - rr * (sr - unr));
  T Fn[4];
  const T* w;
  T rho, u, v, p, un, sk;
  // regions in the order: left of S_L, S_L..S_M, S_M..S_R, right of S_R
  if (sl >= T(0)) {
#pragma unroll
    for (int q = 0; q < 4; ++q) h[q] = fl[q] * nx + gl[q] * ny;
    return;
  }
  if (sm < T(0) && sr < T(0)) {
#pragma unroll
    for (int q = 0; q < 4; ++q) h[q] = fr[q] * nx + gr[q] * ny;
    return;
  }
  if (sm >= T(0)) {
#pragma unroll
    for (int q = 0; q < 4; ++q) Fn[q] = fl[q] * nx + gl[q] * ny;
    w = wl, rho = rl, u = ul, v = vl, p = pl, un = unl, sk = sl;
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) Fn[q] = fr[q] * nx + gr[q] * ny;
    w = wr, rho = rr, u = ur, v = vr, p = pr, un = unr, sk = sr;
  }
  const T dm = sm - un;
  const T g = fdiv(dm, sk - sm), f = T(1) + g;
  const T E = ref.w[3] + w[3];
  const T dU[4] = {g * rho, g * rho * u + f * rho * dm * nx, g * rho * v + f * rho * dm * ny,
                   g * E + f * rho * dm * (sm + fdiv(p, rho * (sk - un)))};
#pragma unroll
  for (int q = 0; q < 4; ++q) h[q] = Fn[q] + sk * dU[q];
}

// The configured Riemann flux (hfd_flux; uniform across the launch).
template <class T>
__device__ inline void riemann(int kind, const T wl[4], const T wr[4], T nx, T ny,
                               const Ref<T>& ref, T gam, T gm1, T h[4]) {
  if (kind == HFD_FLUX_ROE) roe_flux<T>(wl, wr, nx, ny, ref, gm1, h);
  else if (kind == HFD_FLUX_HLLC) hllc_flux<T>(wl, wr, nx, ny, ref, gam, gm1, h);
  else rusanov<T>(wl, wr, nx, ny, ref, gam, gm1, h);
}

// Viscous fluxes (f_vis, g_vis) at a vertex from the full state w and the
// gradients of the conservative variables: Newtonian stress with the Stokes
// hypothesis, constant mu, Fourier heat flux kappa grad T with
// kappa = mu c_p / Pr and T = p / (rho R) (Section 2.3, "Computing Viscous
// Flux").
template <class T>
__device__ inline void viscous_flux(const T w[4], const T wx[4], const T wy[4],
                                    const GasParams& gp, T fv[4], T gv[4]) {
  const T gm1 = T(gp.gamma - 1.0);
  const T rho = w[0], ir = frcp(rho);
  const T u = w[1] * ir, v = w[2] * ir;
  const T p = gm1 * (w[3] - T(0.5) * rho * (u * u + v * v));
  const T iR = T(1.0 / gp.gas_R);
  auto grads = [&](const T* d, T& du, T& dv, T& dT) {
    du = (d[1] - u * d[0]) * ir;
    dv = (d[2] - v * d[0]) * ir;
    T dp = gm1 * (d[3] - (u * d[1] + v * d[2]) + T(0.5) * (u * u + v * v) * d[0]);
    dT = (dp - p * ir * d[0]) * ir * iR;
  };
  T ux, vx, Tx, uy, vy, Ty;
  grads(wx, ux, vx, Tx);
  grads(wy, uy, vy, Ty);
  const T mu = T(gp.mu);
  const T kap = T(gp.mu * gp.gamma * gp.gas_R / ((gp.gamma - 1.0) * gp.prandtl));
  const T dv3 = T(2.0 / 3.0) * mu * (ux + vy);
  const T txx = T(2) * mu * ux - dv3, tyy = T(2) * mu * vy - dv3;
  const T txy = mu * (uy + vx);
  fv[0] = T(0);
  fv[1] = txx;
  fv[2] = txy;
  fv[3] = u * txx + v * txy + kap * Tx;
  gv[0] = T(0);
  gv[1] = txy;
  gv[2] = tyy;
  gv[3] = u * txy + v * tyy + kap * Ty;
}

}  // namespace hfd
