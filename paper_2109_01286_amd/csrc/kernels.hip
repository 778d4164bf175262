// Hot-path kernels of the Hermite finite-difference method (gfx950).
//
// Edge pass (Section 2.2 / 2.3, Algorithm 1, eq. 2d_hweno_intp): one thread
// per active edge.  Roe average of the edge's end states, characteristic
// projection of values and gradients at the six stencil nodes, per side and
// characteristic component the uniform WENO5 weights and the switch, the
// 5-node Hermite value (15-term dot product with the stored row) or the
// omega-weighted 3-node values, back-projection, Rusanov flux along the edge.
//
// Vertex pass (eq. flux_polynomials and the rows d0, dx, dy; viscous
// vertex-only rows; three-stage TVD Runge-Kutta): 16 lanes per owned vertex
// stride over the vertex slots (analytic fluxes recomputed from the
// gathered state, dotted with the coefficient record of the slot) and the
// edge slots (gathered edge flux); a xor-shuffle reduction gives the twelve
// right-hand sides, lane k < 12 applies the Runge-Kutta combination to
// component k.  No atomics: every output has exactly one writer.
//
// Two precisions share the code: float64 throughout, or float32 arithmetic
// on a float32 perturbation state w' = w - w_ref (gradients unchanged) with
// fluxes in perturbation form F(w) - F(w_ref), written so that nothing large
// cancels, and float64 accumulation of the Runge-Kutta state.
#include <hip/hip_runtime.h>

#include "kernels.h"

// Tuning parameters (compile-time).
#ifndef HFD_VERTEX_LANES
#define HFD_VERTEX_LANES 16   // lanes per vertex in the vertex pass
#endif
#ifndef HFD_NT_COEF
#define HFD_NT_COEF 0         // 1: non-temporal loads for single-use coefficient streams
#endif
#ifndef HFD_XCD_REMAP
#define HFD_XCD_REMAP 1       // 1: contiguous block ranges per XCD
#endif

namespace hfd {
namespace {

// Load of a value that is used once per launch (coefficients, indices):
// optionally marked non-temporal so it does not displace gathered data.
template <class T>
__device__ inline T ldc(const T* p) {
#if HFD_NT_COEF
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
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
                                 T* u_full = nullptr, T* v_full = nullptr) {
  const T rho = R.w[0] + wp[0];
  const T m = R.w[1] + wp[1];
  const T n = R.w[2] + wp[2];
  const T ir = T(1) / rho;
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
}

template <class T>
__device__ inline Ref<T> make_ref(const GasParams& gp) {
  Ref<T> r;
  for (int q = 0; q < 4; ++q) r.w[q] = T(gp.wref[q]);
  double rho = gp.wref[0];
  double u = rho > 0 ? gp.wref[1] / rho : 0.0, v = rho > 0 ? gp.wref[2] / rho : 0.0;
  double p = (gp.gamma - 1.0) * (gp.wref[3] - 0.5 * rho * (u * u + v * v));
  r.u = T(u);
  r.v = T(v);
  r.etr = T(gp.wref[3] + p);
  return r;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Renumber them so that XCD x runs one contiguous range of logical
// blocks: neighbouring vertices / edges then share an L2 for their gathers.
constexpr int kXcd = 8;
__device__ inline int64_t xcd_block() {
#if !HFD_XCD_REMAP
  return blockIdx.x;
#endif
  const int64_t b = blockIdx.x, nb = gridDim.x;
  const int64_t x = b % kXcd, k = b / kXcd;
  const int64_t q = nb / kXcd, r = nb % kXcd;
  return x * q + (x < r ? x : r) + k;
}

// ---------------------------------------------------------------------------
// Edge pass
// ---------------------------------------------------------------------------
// LPE lanes per edge.  LPE = 2: lane side s = 0 interpolates the left state
// from nodes (i-2 .. i+2), s = 1 the right state from (i+3 .. i-1); the pair
// swaps states and both evaluate the flux (lane 0 stores it).  LPE = 1: one
// lane does both sides in turn.
// Waves per SIMD the edge pass is compiled for (register budget 512/waves).
template <class T> struct EdgeWaves { static constexpr int value = 3; };
template <> struct EdgeWaves<double> { static constexpr int value = 2; };

template <class T, int LPE>
__global__ void __launch_bounds__(256, EdgeWaves<T>::value)
k_edge(int64_t ne, EdgeCoef<T> c, GasParams gp, const V4<T>* __restrict__ Gv,
       const V4<T>* __restrict__ Gg, const uint8_t* __restrict__ force,
       V4<T>* __restrict__ H, double* __restrict__ hsoa, double* __restrict__ wlr,
       uint8_t* __restrict__ mask) {
  const int64_t tid = xcd_block() * blockDim.x + threadIdx.x;
  const int s0 = LPE == 2 ? int(tid & 1) : 0;
  const int64_t e = tid / LPE;
  if (e >= ne) return;
  const Ref<T> ref = make_ref<T>(gp);
  const T gam = T(gp.gamma), gm1 = T(gp.gamma - 1.0);
  const int ia = c.stg[2 * ne + e], ib = c.stg[3 * ne + e];
  const T nx = c.n[e], ny = c.n[ne + e];

  // Roe average of the two end states (nodes i, i+1)
  T u, v, hh, cc;
  {
    const V4<T> A = Gv[ia], B = Gv[ib];
    T ra = ref.w[0] + A.x, rb = ref.w[0] + B.x;
    T ua = (ref.w[1] + A.y) / ra, ub = (ref.w[1] + B.y) / rb;
    T va = (ref.w[2] + A.z) / ra, vb = (ref.w[2] + B.z) / rb;
    T Ea = ref.w[3] + A.w, Eb = ref.w[3] + B.w;
    T pa = gm1 * (Ea - T(0.5) * ra * (ua * ua + va * va));
    T pb = gm1 * (Eb - T(0.5) * rb * (ub * ub + vb * vb));
    T sa = sqrt(ra), sb = sqrt(rb);
    T iw = T(1) / (sa + sb);
    u = (sa * ua + sb * ub) * iw;
    v = (sa * va + sb * vb) * iw;
    hh = (sa * (Ea + pa) / ra + sb * (Eb + pb) / rb) * iw;
    cc = sqrt(gm1 * (hh - T(0.5) * (u * u + v * v)));
  }
  const T q2 = u * u + v * v;
  const T un = u * nx + v * ny, ut = -u * ny + v * nx;
  const T b1 = gm1 / (cc * cc), b2 = T(0.5) * b1 * q2, ic = T(1) / cc;
  // left eigenvectors (rows), inverse of the right eigenvector matrix below
  const T L[4][4] = {
      {T(0.5) * (b2 + un * ic), T(-0.5) * (b1 * u + nx * ic), T(-0.5) * (b1 * v + ny * ic), T(0.5) * b1},
      {T(1) - b2, b1 * u, b1 * v, -b1},
      {T(0.5) * (b2 - un * ic), T(-0.5) * (b1 * u - nx * ic), T(-0.5) * (b1 * v - ny * ic), T(0.5) * b1},
      {-ut, -ny, nx, T(0)}};
  const T Rm[4][4] = {{T(1), T(1), T(1), T(0)},
                      {u - cc * nx, u, u + cc * nx, -ny},
                      {v - cc * ny, v, v + cc * ny, nx},
                      {hh - un * cc, T(0.5) * q2, hh + un * cc, ut}};
  const uint8_t fm = force ? force[e] : uint8_t(0);
  uint8_t bits = 0;
  const T eps = T(gp.eps), lo = T(gp.sw_lo), hi = T(gp.sw_hi);
  const T d1 = T(1.0 / 16.0), d2 = T(10.0 / 16.0), d3 = T(5.0 / 16.0);

  T wm0[4], wm1[4];
#pragma unroll 1
  for (int k = 0; k < 3 - LPE; ++k) {
    const int s = s0 + k;
    int id[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) id[t] = ldc(c.stg + (s == 0 ? t : 5 - t) * ne + e);
    // The 5-node Hermite row is the same for the four characteristic
    // components, so L (sum_t w5_t . data_t) is the projected Hermite value:
    // only the node values need projecting (for the smoothness indicators
    // and the 3-node values); the gradients enter through the physical sum.
    T w5[15];
#pragma unroll
    for (int j = 0; j < 15; ++j) w5[j] = ldc(c.w5 + int64_t(s * 15 + j) * ne + e);
    T cv[4][5], hs[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const V4<T> a = Gv[id[j]], bx = Gg[2 * int64_t(id[j])], by = Gg[2 * int64_t(id[j]) + 1];
      const T w[4] = {a.x, a.y, a.z, a.w};
      const T wx[4] = {bx.x, bx.y, bx.z, bx.w};
      const T wy[4] = {by.x, by.y, by.z, by.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cv[q][j] = L[q][0] * w[0] + L[q][1] * w[1] + L[q][2] * w[2] + L[q][3] * w[3];
        hs[q] += w5[3 * j] * w[q] + w5[3 * j + 1] * wx[q] + w5[3 * j + 2] * wy[q];
      }
    }
    T w3[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) w3[j] = ldc(c.w3 + int64_t(s * 9 + j) * ne + e);
    T C[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T c0 = cv[q][0], c1 = cv[q][1], c2 = cv[q][2], c3 = cv[q][3], c4 = cv[q][4];
      const T t1 = c0 - T(2) * c1 + c2, t2 = c0 - T(4) * c1 + T(3) * c2;
      const T t3 = c1 - T(2) * c2 + c3, t4 = c1 - c3;
      const T t5 = c2 - T(2) * c3 + c4, t6 = T(3) * c2 - T(4) * c3 + c4;
      const T be1 = T(13.0 / 12.0) * t1 * t1 + T(0.25) * t2 * t2;
      const T be2 = T(13.0 / 12.0) * t3 * t3 + T(0.25) * t4 * t4;
      const T be3 = T(13.0 / 12.0) * t5 * t5 + T(0.25) * t6 * t6;
      const T a1 = d1 / ((eps + be1) * (eps + be1));
      const T a2 = d2 / ((eps + be2) * (eps + be2));
      const T a3 = d3 / ((eps + be3) * (eps + be3));
      const T sa = a1 + a2 + a3;
      const T o1 = a1 / sa, o2 = a2 / sa, o3 = a3 / sa;
      bool weno;
      if (force) weno = (fm >> (4 * s + q)) & 1;
      else if (gp.sw == HFD_SWITCH_PAPER) weno = !(o1 > lo && o1 < hi);
      else weno = (gp.sw == HFD_SWITCH_WENO_ONLY);
      T val;
      if (weno) {
        val = o1 * (w3[0] * c0 + w3[1] * c1 + w3[2] * c2) +
              o2 * (w3[3] * c1 + w3[4] * c2 + w3[5] * c3) +
              o3 * (w3[6] * c2 + w3[7] * c3 + w3[8] * c4);
      } else {
        val = L[q][0] * hs[0] + L[q][1] * hs[1] + L[q][2] * hs[2] + L[q][3] * hs[3];
      }
      C[q] = val;
      bits |= uint8_t(weno ? 1 : 0) << (4 * s + q);
    }
    // back-projection w' = R C of this side
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const T x = Rm[r][0] * C[0] + Rm[r][1] * C[1] + Rm[r][2] * C[2] + Rm[r][3] * C[3];
      if (k == 0) wm0[r] = x;
      else wm1[r] = x;
    }
  }
  T wl[4], wr[4];
  if (LPE == 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      wl[q] = wm0[q];
      wr[q] = wm1[q];
    }
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T o = __shfl_xor(wm0[q], 1);
      wl[q] = s0 == 0 ? wm0[q] : o;
      wr[q] = s0 == 0 ? o : wm0[q];
    }
    bits |= uint8_t(__shfl_xor(int(bits), 1));
  }
  // Rusanov flux along n (perturbation form)
  T fl[4], gl[4], fr[4], gr[4], pl, rl, ul, vl, pr, rr, ur, vr;
  pert_flux<T>(wl, ref, gm1, fl, gl, &pl, &rl, &ul, &vl);
  pert_flux<T>(wr, ref, gm1, fr, gr, &pr, &rr, &ur, &vr);
  const T sl = fabs(ul * nx + vl * ny) + sqrt(gam * pl / rl);
  const T sr = fabs(ur * nx + vr * ny) + sqrt(gam * pr / rr);
  // NaN-propagating maximum: a non-physical state must not be hidden
  const T lam = (isnan(sl) || isnan(sr)) ? sl + sr : (sl > sr ? sl : sr);
  T h[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    h[q] = T(0.5) * ((fl[q] + fr[q]) * nx + (gl[q] + gr[q]) * ny) -
           T(0.5) * lam * (wr[q] - wl[q]);
  if (s0 == 0) {
    H[e] = V4<T>{h[0], h[1], h[2], h[3]};
    if (mask) mask[e] = bits;
    if (hsoa) {
#pragma unroll
      for (int q = 0; q < 4; ++q) hsoa[q * ne + e] = double(h[q]);
    }
  }
  if (wlr) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (LPE == 1 || s0 == 0) wlr[q * ne + e] = double(wl[q]) + gp.wref[q];
      if (LPE == 1 || s0 == 1) wlr[(4 + q) * ne + e] = double(wr[q]) + gp.wref[q];
    }
  }
}

// ---------------------------------------------------------------------------
// Vertex pass
// ---------------------------------------------------------------------------
constexpr int VL = HFD_VERTEX_LANES;   // lanes per vertex
constexpr int VPB = 256 / VL;          // vertices per block (256 threads)

template <class T>
__device__ inline void viscous_flux(const T w[4], const T wx[4], const T wy[4],
                                    const GasParams& gp, T fv[4], T gv[4]) {
  const T gm1 = T(gp.gamma - 1.0);
  const T rho = w[0], ir = T(1) / rho;
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

// Contribution of one vertex slot (node u of S(v)) to the 12 accumulators.
template <class T, bool VISC>
__device__ inline void vslot(const V4<T>& a, const V4<T>* gx, const T* d, const T* k,
                             const Ref<T>& ref, T gm1, const GasParams& gp, T acc[12]) {
  const T w[4] = {a.x, a.y, a.z, a.w};
  T f[4], g[4];
  pert_flux<T>(w, ref, gm1, f, g);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    acc[q] -= d[0] * f[q] + d[1] * g[q];
    acc[4 + q] -= d[2] * f[q] + d[3] * g[q];
    acc[8 + q] -= d[4] * f[q] + d[5] * g[q];
  }
  if (VISC) {
    const T wf[4] = {w[0] + ref.w[0], w[1] + ref.w[1], w[2] + ref.w[2], w[3] + ref.w[3]};
    const T wx[4] = {gx[0].x, gx[0].y, gx[0].z, gx[0].w};
    const T wy[4] = {gx[1].x, gx[1].y, gx[1].z, gx[1].w};
    T fv[4], gv[4];
    viscous_flux<T>(wf, wx, wy, gp, fv, gv);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc[q] += k[0] * fv[q] + k[1] * gv[q];
      acc[4 + q] += k[2] * fv[q] + k[3] * gv[q];
      acc[8 + q] += k[3] * fv[q] + k[4] * gv[q];
    }
  }
}

template <class T, bool VISC>
__global__ void __launch_bounds__(256)
k_vertex(int64_t nowned, int64_t nv, VertexCoef<T> c, GasParams gp,
         const V4<T>* __restrict__ Gv, const V4<T>* __restrict__ Gg,
         const V4<T>* __restrict__ H, int mode, double* __restrict__ dU, RkArgs rk,
         V4<T>* __restrict__ Gv_new, V4<T>* __restrict__ Gg_new,
         int32_t* __restrict__ flag) {
  __shared__ double sres[VPB][13];
  const int vl = threadIdx.x / VL, sub = threadIdx.x & (VL - 1);
  const int64_t v0 = xcd_block() * VPB;
  const int64_t v = v0 + vl;
  const Ref<T> ref = make_ref<T>(gp);
  const T gm1 = T(gp.gamma - 1.0);
  T acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = T(0);

  if (v < nowned) {
    // vertex slots, two per lane and iteration (all loads issued first)
    const int s0 = c.vptr[v], s1 = c.vptr[v + 1];
    for (int s = s0 + sub; s < s1; s += 2 * VL) {
      const int sb = (s + VL < s1) ? s + VL : s;
      const int ua = ldc(c.vg + s), ub = ldc(c.vg + sb);
      T da[6], db[6], ka[5], kb[5];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        da[q] = ldc(c.dv + int64_t(6) * s + q);
        db[q] = ldc(c.dv + int64_t(6) * sb + q);
      }
      if (VISC) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          ka[q] = ldc(c.dvis + int64_t(5) * s + q);
          kb[q] = ldc(c.dvis + int64_t(5) * sb + q);
        }
      }
      const V4<T> A = Gv[ua], B = Gv[ub];
      V4<T> gA[2], gB[2];
      if (VISC) {
        gA[0] = Gg[2 * int64_t(ua)];
        gA[1] = Gg[2 * int64_t(ua) + 1];
        gB[0] = Gg[2 * int64_t(ub)];
        gB[1] = Gg[2 * int64_t(ub) + 1];
      }
      vslot<T, VISC>(A, gA, da, ka, ref, gm1, gp, acc);
      if (sb != s) vslot<T, VISC>(B, gB, db, kb, ref, gm1, gp, acc);
    }
    // edge slots, four per lane and iteration
    const int e0 = c.eptr[v], e1 = c.eptr[v + 1];
    for (int s = e0 + sub; s < e1; s += 4 * VL) {
      int j[4];
      bool ok[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ok[k] = s + k * VL < e1;
        j[k] = ok[k] ? s + k * VL : s;
      }
      int m[4];
      T d[4][3];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        m[k] = ldc(c.ve + j[k]);
#pragma unroll
        for (int q = 0; q < 3; ++q) d[k][q] = ldc(c.de + int64_t(3) * j[k] + q);
      }
      V4<T> h[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) h[k] = H[m[k]];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (!ok[k]) continue;
        const T hq[4] = {h[k].x, h[k].y, h[k].z, h[k].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc[q] -= d[k][0] * hq[q];
          acc[4 + q] -= d[k][1] * hq[q];
          acc[8 + q] -= d[k][2] * hq[q];
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) {
#pragma unroll
    for (int o = VL / 2; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o);
  }
  T r = acc[0];
#pragma unroll
  for (int k = 1; k < 12; ++k)
    if (sub == k) r = acc[k];
  if (sub < 12) sres[vl][sub] = double(r);
  __syncthreads();

  // epilogue: thread (component cmp, vertex vl2), consecutive vertices in
  // consecutive lanes so every component row is written in 16-wide runs
  const int t = threadIdx.x;
  bool bad = false;
  if (t < 12 * VPB) {
    const int cmp = t / VPB, vl2 = t % VPB;
    const int64_t vv = v0 + vl2;
    if (vv < nowned) {
      const double rv = sres[vl2][cmp];
      const int64_t o = int64_t(cmp) * nv + vv;
      if (mode == 0) {
        dU[o] = rv;
        bad = !isfinite(rv);
      } else {
        const double dt = rk.dt_dev ? *rk.dt_dev : rk.dt;
        const double out = rk.a * rk.Un[o] + rk.b * (rk.Uk[o] + dt * rv);
        rk.Unew[o] = out;
        if (Gv_new) {
          const T g = T(out - (cmp < 4 ? gp.wref[cmp] : 0.0));
          if (cmp < 4) reinterpret_cast<T*>(Gv_new)[4 * vv + cmp] = g;
          else reinterpret_cast<T*>(Gg_new)[8 * vv + (cmp - 4)] = g;
        }
        bad = !isfinite(out);
        if (cmp < 4) sres[vl2][cmp] = out;
      }
    }
  }
  __syncthreads();
  if (mode == 1 && t < VPB && v0 + t < nowned) {
    // positivity of rho and p at the new state
    const double rho = sres[t][0], m = sres[t][1], n = sres[t][2], E = sres[t][3];
    const double p = (gp.gamma - 1.0) * (E - 0.5 * (m * m + n * n) / rho);
    bad = bad || !(rho > 0.0) || !(p > 0.0);
  }
  if (bad && flag) flag[0] = 1;
}

// State in the float64 [12][nv] layout -> gather layout (values [nv] of V4,
// gradients [2 nv] of V4), minus the reference state in the mixed form.
template <class T>
__global__ void k_to_gather(int64_t nv, const double* __restrict__ U, GasParams gp,
                            V4<T>* __restrict__ Gv, V4<T>* __restrict__ Gg) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  T w[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) w[q] = T(U[q * nv + i] - (q < 4 ? gp.wref[q] : 0.0));
  Gv[i] = V4<T>{w[0], w[1], w[2], w[3]};
  Gg[2 * i] = V4<T>{w[4], w[5], w[6], w[7]};
  Gg[2 * i + 1] = V4<T>{w[8], w[9], w[10], w[11]};
}

template <class T>
__global__ void k_copy_gather_rows(int64_t nrows, const int32_t* __restrict__ rows,
                                   const V4<T>* __restrict__ fv, const V4<T>* __restrict__ fg,
                                   V4<T>* __restrict__ tv, V4<T>* __restrict__ tg) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nrows) return;
  const int64_t r = rows[k];
  tv[r] = fv[r];
  tg[2 * r] = fg[2 * r];
  tg[2 * r + 1] = fg[2 * r + 1];
}

// ---------------------------------------------------------------------------
// Helpers
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_copy_rows(int64_t nrows, const int32_t* __restrict__ rows,
                            const int32_t* __restrict__ src, int64_t nv,
                            const T* from, T* to) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nrows * 12) return;
  const int64_t k = i / 12, q = i % 12;
  const int32_t dst = rows[k], s = src ? src[k] : rows[k];
  to[q * nv + dst] = from[q * nv + s];
}

__global__ void k_zero_rows(int64_t nowned, int64_t nv, double* __restrict__ dU) {
  const int64_t ng = nv - nowned;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= 12 * ng) return;
  const int64_t q = i / ng, k = i % ng;
  dU[q * nv + nowned + k] = 0.0;
}

constexpr int DT_BLOCK = 256;

__global__ void __launch_bounds__(DT_BLOCK)
k_dt_partial(int64_t nowned, int64_t nv, const double* __restrict__ U,
             const double* __restrict__ hmin, double gamma,
             double* __restrict__ partial) {
  __shared__ double red[DT_BLOCK / 64];
  double best = INFINITY;
  for (int64_t v = int64_t(blockIdx.x) * DT_BLOCK + threadIdx.x; v < nowned;
       v += int64_t(gridDim.x) * DT_BLOCK) {
    const double rho = U[v], u = U[nv + v] / rho, w = U[2 * nv + v] / rho;
    const double p = (gamma - 1.0) * (U[3 * nv + v] - 0.5 * rho * (u * u + w * w));
    const double lam = sqrt(u * u + w * w) + sqrt(gamma * p / rho);
    best = fmin(best, hmin[v] / lam);
  }
  for (int o = 32; o > 0; o >>= 1) best = fmin(best, __shfl_xor(best, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = red[0];
    for (int k = 1; k < DT_BLOCK / 64; ++k) b = fmin(b, red[k]);
    partial[blockIdx.x] = b;
  }
}

__global__ void __launch_bounds__(DT_BLOCK)
k_dt_final(int64_t np, const double* __restrict__ partial, double cfl,
           double* __restrict__ dt) {
  __shared__ double red[DT_BLOCK / 64];
  double best = INFINITY;
  for (int64_t i = threadIdx.x; i < np; i += DT_BLOCK) best = fmin(best, partial[i]);
  for (int o = 32; o > 0; o >>= 1) best = fmin(best, __shfl_xor(best, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = red[0];
    for (int k = 1; k < DT_BLOCK / 64; ++k) b = fmin(b, red[k]);
    dt[0] = cfl * b;
  }
}

__global__ void k_axpbypcz(int64_t n, double a, const double* __restrict__ x, double b,
                           const double* __restrict__ y, double c, const double* __restrict__ z,
                           double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double r = a * x[i] + b * y[i];
  if (z) r += c * z[i];
  out[i] = r;
}

// one thread per (source row, component)
__global__ void k_adj_copy_ghosts(int64_t nsrc, const int32_t* __restrict__ sptr,
                                  const int32_t* __restrict__ srows,
                                  const int32_t* __restrict__ gsts, int64_t nv,
                                  double* __restrict__ lam) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nsrc * 12) return;
  const int64_t k = i / 12, q = i % 12;
  const int64_t src = srows[k];
  double acc = lam[q * nv + src];
  for (int j = sptr[k]; j < sptr[k + 1]; ++j) {
    acc += lam[q * nv + gsts[j]];
    lam[q * nv + gsts[j]] = 0.0;
  }
  lam[q * nv + src] = acc;
}

__global__ void k_cast(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = float(a[i]);
}

__global__ void k_widen(int64_t n, const float* __restrict__ a, double* __restrict__ b) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = double(a[i]);
}

inline unsigned nblocks(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

}  // namespace

template <class T>
hipError_t launch_edge(int64_t ne, const EdgeCoef<T>& c, const GasParams& gp,
                       const V4<T>* Gv, const V4<T>* Gg, const uint8_t* force, V4<T>* H,
                       double* hsoa, double* wlr, uint8_t* mask, hipStream_t st) {
  if (ne == 0) return hipSuccess;
  // float: one lane per edge; double: two (one per side), register budget
  constexpr int lpe = sizeof(T) == 8 ? 2 : 1;
  hipLaunchKernelGGL((k_edge<T, lpe>), dim3(nblocks(lpe * ne, 256)), dim3(256), 0, st, ne, c,
                     gp, Gv, Gg, force, H, hsoa, wlr, mask);
  return hipGetLastError();
}
template hipError_t launch_edge<double>(int64_t, const EdgeCoef<double>&, const GasParams&,
                                        const V4<double>*, const V4<double>*, const uint8_t*,
                                        V4<double>*, double*, double*, uint8_t*, hipStream_t);
template hipError_t launch_edge<float>(int64_t, const EdgeCoef<float>&, const GasParams&,
                                       const V4<float>*, const V4<float>*, const uint8_t*,
                                       V4<float>*, double*, double*, uint8_t*, hipStream_t);

template <class T>
hipError_t launch_vertex(int64_t nowned, int64_t nv, const VertexCoef<T>& c,
                         const GasParams& gp, const V4<T>* Gv, const V4<T>* Gg,
                         const V4<T>* H, int mode, double* dU, const RkArgs& rk,
                         V4<T>* Gv_new, V4<T>* Gg_new, int32_t* flag, hipStream_t st) {
  if (nowned == 0) return hipSuccess;
  const unsigned nb = nblocks(nowned, VPB);
  if (c.dvis)
    hipLaunchKernelGGL((k_vertex<T, true>), dim3(nb), dim3(VL * VPB), 0, st, nowned, nv, c,
                       gp, Gv, Gg, H, mode, dU, rk, Gv_new, Gg_new, flag);
  else
    hipLaunchKernelGGL((k_vertex<T, false>), dim3(nb), dim3(VL * VPB), 0, st, nowned, nv, c,
                       gp, Gv, Gg, H, mode, dU, rk, Gv_new, Gg_new, flag);
  return hipGetLastError();
}
template hipError_t launch_vertex<double>(int64_t, int64_t, const VertexCoef<double>&,
                                          const GasParams&, const V4<double>*,
                                          const V4<double>*, const V4<double>*, int, double*,
                                          const RkArgs&, V4<double>*, V4<double>*, int32_t*,
                                          hipStream_t);
template hipError_t launch_vertex<float>(int64_t, int64_t, const VertexCoef<float>&,
                                         const GasParams&, const V4<float>*, const V4<float>*,
                                         const V4<float>*, int, double*, const RkArgs&,
                                         V4<float>*, V4<float>*, int32_t*, hipStream_t);

template <class T>
hipError_t launch_to_gather(int64_t nv, const double* U, const GasParams& gp, V4<T>* Gv,
                            V4<T>* Gg, hipStream_t st) {
  hipLaunchKernelGGL(k_to_gather<T>, dim3(nblocks(nv, 256)), dim3(256), 0, st, nv, U, gp,
                     Gv, Gg);
  return hipGetLastError();
}
template hipError_t launch_to_gather<double>(int64_t, const double*, const GasParams&,
                                             V4<double>*, V4<double>*, hipStream_t);
template hipError_t launch_to_gather<float>(int64_t, const double*, const GasParams&,
                                            V4<float>*, V4<float>*, hipStream_t);

template <class T>
hipError_t launch_copy_gather_rows(int64_t nrows, const int32_t* rows, const V4<T>* fv,
                                   const V4<T>* fg, V4<T>* tv, V4<T>* tg, hipStream_t st) {
  if (nrows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_gather_rows<T>, dim3(nblocks(nrows, 256)), dim3(256), 0, st,
                     nrows, rows, fv, fg, tv, tg);
  return hipGetLastError();
}
template hipError_t launch_copy_gather_rows<double>(int64_t, const int32_t*,
                                                    const V4<double>*, const V4<double>*,
                                                    V4<double>*, V4<double>*, hipStream_t);
template hipError_t launch_copy_gather_rows<float>(int64_t, const int32_t*, const V4<float>*,
                                                   const V4<float>*, V4<float>*, V4<float>*,
                                                   hipStream_t);

template <class T>
hipError_t launch_copy_rows(int64_t nrows, const int32_t* rows, const int32_t* src,
                            int64_t nv, const T* from, T* to, hipStream_t st) {
  if (nrows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_rows<T>, dim3(nblocks(nrows * 12, 256)), dim3(256), 0, st,
                     nrows, rows, src, nv, from, to);
  return hipGetLastError();
}
template hipError_t launch_copy_rows<double>(int64_t, const int32_t*, const int32_t*,
                                             int64_t, const double*, double*, hipStream_t);
template hipError_t launch_copy_rows<float>(int64_t, const int32_t*, const int32_t*,
                                            int64_t, const float*, float*, hipStream_t);

hipError_t launch_zero_ghost_rows(int64_t nowned, int64_t nv, double* dU,
                                  hipStream_t st) {
  if (nv == nowned) return hipSuccess;
  hipLaunchKernelGGL(k_zero_rows, dim3(nblocks(12 * (nv - nowned), 256)), dim3(256),
                     0, st, nowned, nv, dU);
  return hipGetLastError();
}

hipError_t launch_stable_dt(int64_t nowned, int64_t nv, const double* U,
                            const double* hmin, double gamma, double cfl,
                            double* partial, int64_t npartial, double* dt,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_dt_partial, dim3(unsigned(npartial)), dim3(DT_BLOCK), 0, st,
                     nowned, nv, U, hmin, gamma, partial);
  hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(DT_BLOCK), 0, st, npartial, partial,
                     cfl, dt);
  return hipGetLastError();
}

hipError_t launch_axpbypcz(int64_t n, double a, const double* x, double b, const double* y,
                           double c, const double* z, double* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpbypcz, dim3(nblocks(n, 256)), dim3(256), 0, st, n, a, x, b, y, c, z,
                     out);
  return hipGetLastError();
}

hipError_t launch_adj_copy_ghosts(int64_t nsrc, const int32_t* sptr, const int32_t* srows,
                                  const int32_t* gsts, int64_t nv, double* lam,
                                  hipStream_t st) {
  if (nsrc == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_copy_ghosts, dim3(nblocks(nsrc * 12, 256)), dim3(256), 0, st, nsrc,
                     sptr, srows, gsts, nv, lam);
  return hipGetLastError();
}

hipError_t launch_cast(int64_t n, const double* a, float* b, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast, dim3(nblocks(n, 256)), dim3(256), 0, st, n, a, b);
  return hipGetLastError();
}

hipError_t launch_widen(int64_t n, const float* a, double* b, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_widen, dim3(nblocks(n, 256)), dim3(256), 0, st, n, a, b);
  return hipGetLastError();
}

}  // namespace hfd
