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

namespace hfd {
namespace {

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

// ---------------------------------------------------------------------------
// Edge pass
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256)
k_edge(int64_t ne, int64_t nv, EdgeCoef<T> c, GasParams gp,
       const T* __restrict__ U, const uint8_t* __restrict__ force,
       T* __restrict__ H, double* __restrict__ wlr, uint8_t* __restrict__ mask) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const Ref<T> ref = make_ref<T>(gp);
  const T gam = T(gp.gamma), gm1 = T(gp.gamma - 1.0);
  int id[6];
#pragma unroll
  for (int t = 0; t < 6; ++t) id[t] = c.stg[t * ne + e];
  const T nx = c.n[e], ny = c.n[ne + e];

  // Roe average of the two end states (nodes i, i+1)
  T u, v, hh, cc;
  {
    T ra = ref.w[0] + U[id[2]], rb = ref.w[0] + U[id[3]];
    T ua = (ref.w[1] + U[nv + id[2]]) / ra, ub = (ref.w[1] + U[nv + id[3]]) / rb;
    T va = (ref.w[2] + U[2 * nv + id[2]]) / ra, vb = (ref.w[2] + U[2 * nv + id[3]]) / rb;
    T Ea = ref.w[3] + U[3 * nv + id[2]], Eb = ref.w[3] + U[3 * nv + id[3]];
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

  // characteristic values / gradients at the six nodes
  T cv[4][6], cx[4][6], cy[4][6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    T w[4], wx[4], wy[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      w[q] = U[q * nv + id[j]];
      wx[q] = U[(4 + q) * nv + id[j]];
      wy[q] = U[(8 + q) * nv + id[j]];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cv[q][j] = L[q][0] * w[0] + L[q][1] * w[1] + L[q][2] * w[2] + L[q][3] * w[3];
      cx[q][j] = L[q][0] * wx[0] + L[q][1] * wx[1] + L[q][2] * wx[2] + L[q][3] * wx[3];
      cy[q][j] = L[q][0] * wy[0] + L[q][1] * wy[1] + L[q][2] * wy[2] + L[q][3] * wy[3];
    }
  }

  const uint8_t fm = force ? force[e] : uint8_t(0);
  uint8_t bits = 0;
  T C[2][4];
  const T eps = T(gp.eps), lo = T(gp.sw_lo), hi = T(gp.sw_hi);
  const T d1 = T(1.0 / 16.0), d2 = T(10.0 / 16.0), d3 = T(5.0 / 16.0);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    // side nodes: left (0,1,2,3,4), right (5,4,3,2,1)
    int ix[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) ix[t] = s == 0 ? t : 5 - t;
    T w5[15], w3[9];
#pragma unroll
    for (int k = 0; k < 15; ++k) w5[k] = c.w5[int64_t(s * 15 + k) * ne + e];
#pragma unroll
    for (int k = 0; k < 9; ++k) w3[k] = c.w3[int64_t(s * 9 + k) * ne + e];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T c0 = cv[q][ix[0]], c1 = cv[q][ix[1]], c2 = cv[q][ix[2]],
              c3 = cv[q][ix[3]], c4 = cv[q][ix[4]];
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
        val = T(0);
#pragma unroll
        for (int t = 0; t < 5; ++t)
          val += w5[3 * t] * cv[q][ix[t]] + w5[3 * t + 1] * cx[q][ix[t]] +
                 w5[3 * t + 2] * cy[q][ix[t]];
      }
      C[s][q] = val;
      bits |= uint8_t(weno ? 1 : 0) << (4 * s + q);
    }
  }
  // back-projection w' = R C
  T wl[4], wr[4];
  {
    const T Rm[4][4] = {{T(1), T(1), T(1), T(0)},
                        {u - cc * nx, u, u + cc * nx, -ny},
                        {v - cc * ny, v, v + cc * ny, nx},
                        {hh - un * cc, T(0.5) * q2, hh + un * cc, ut}};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      wl[r] = Rm[r][0] * C[0][0] + Rm[r][1] * C[0][1] + Rm[r][2] * C[0][2] + Rm[r][3] * C[0][3];
      wr[r] = Rm[r][0] * C[1][0] + Rm[r][1] * C[1][1] + Rm[r][2] * C[1][2] + Rm[r][3] * C[1][3];
    }
  }
  // Rusanov flux along n (perturbation form)
  T fl[4], gl[4], fr[4], gr[4], pl, rl, ul, vl, pr, rr, ur, vr;
  pert_flux<T>(wl, ref, gm1, fl, gl, &pl, &rl, &ul, &vl);
  pert_flux<T>(wr, ref, gm1, fr, gr, &pr, &rr, &ur, &vr);
  const T sl = fabs(ul * nx + vl * ny) + sqrt(gam * pl / rl);
  const T sr = fabs(ur * nx + vr * ny) + sqrt(gam * pr / rr);
  // NaN-propagating maximum: a non-physical state must not be hidden
  const T lam = (isnan(sl) || isnan(sr)) ? sl + sr : (sl > sr ? sl : sr);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    T h = T(0.5) * ((fl[q] + fr[q]) * nx + (gl[q] + gr[q]) * ny) -
          T(0.5) * lam * (wr[q] - wl[q]);
    H[q * ne + e] = h;
  }
  if (wlr) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      wlr[q * ne + e] = double(wl[q]) + gp.wref[q];
      wlr[(4 + q) * ne + e] = double(wr[q]) + gp.wref[q];
    }
  }
  if (mask) mask[e] = bits;
}

// ---------------------------------------------------------------------------
// Vertex pass
// ---------------------------------------------------------------------------
constexpr int VL = 16;  // lanes per vertex

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

template <class T, bool VISC>
__global__ void __launch_bounds__(256)
k_vertex(int64_t nowned, int64_t nv, VertexCoef<T> c, GasParams gp,
         const T* __restrict__ U, const T* __restrict__ H, int64_t ne, int mode,
         double* __restrict__ dU, RkArgs rk, int32_t* __restrict__ flag) {
  const int sub = threadIdx.x & (VL - 1);
  const int64_t v = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / VL;
  if (v >= nowned) return;
  const Ref<T> ref = make_ref<T>(gp);
  const T gm1 = T(gp.gamma - 1.0);
  T acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = T(0);

  const int s0 = c.vptr[v], s1 = c.vptr[v + 1];
  for (int s = s0 + sub; s < s1; s += VL) {
    const int u = c.vg[s];
    T w[4], f[4], g[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = U[q * nv + u];
    pert_flux<T>(w, ref, gm1, f, g);
    const T* d = c.dv + int64_t(6) * s;
    const T d0f = d[0], d0g = d[1], dxf = d[2], dxg = d[3], dyf = d[4], dyg = d[5];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc[q] -= d0f * f[q] + d0g * g[q];
      acc[4 + q] -= dxf * f[q] + dxg * g[q];
      acc[8 + q] -= dyf * f[q] + dyg * g[q];
    }
    if (VISC) {
      T wf[4], wx[4], wy[4], fv[4], gv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        wf[q] = w[q] + ref.w[q];
        wx[q] = U[(4 + q) * nv + u];
        wy[q] = U[(8 + q) * nv + u];
      }
      viscous_flux<T>(wf, wx, wy, gp, fv, gv);
      const T* k = c.dvis + int64_t(5) * s;
      const T k0 = k[0], k1 = k[1], k2 = k[2], k3 = k[3], k4 = k[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc[q] += k0 * fv[q] + k1 * gv[q];
        acc[4 + q] += k2 * fv[q] + k3 * gv[q];
        acc[8 + q] += k3 * fv[q] + k4 * gv[q];
      }
    }
  }
  const int e0 = c.eptr[v], e1 = c.eptr[v + 1];
  for (int s = e0 + sub; s < e1; s += VL) {
    const int m = c.ve[s];
    const T* d = c.de + int64_t(3) * s;
    const T d0 = d[0], dx = d[1], dy = d[2];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T h = H[q * ne + m];
      acc[q] -= d0 * h;
      acc[4 + q] -= dx * h;
      acc[8 + q] -= dy * h;
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
  const int comp = sub < 12 ? sub : 0;
  bool bad = false;
  double out = 0.0;
  if (mode == 0) {
    out = double(r);
    if (sub < 12) dU[int64_t(comp) * nv + v] = out;
    bad = !isfinite(out);
  } else {
    const double dt = rk.dt_dev ? *rk.dt_dev : rk.dt;
    const int64_t o = int64_t(comp) * nv + v;
    out = rk.a * rk.Un[o] + rk.b * (rk.Uk[o] + dt * double(r));
    if (sub < 12) {
      rk.Unew[o] = out;
      if (rk.Us_new) rk.Us_new[o] = float(out - (comp < 4 ? gp.wref[comp] : 0.0));
    }
    bad = !isfinite(out);
    // positivity of rho and p at the new state
    const double rho = __shfl(out, 0, VL), m = __shfl(out, 1, VL),
                 n = __shfl(out, 2, VL), E = __shfl(out, 3, VL);
    if (sub == 0) {
      const double p = (gp.gamma - 1.0) * (E - 0.5 * (m * m + n * n) / rho);
      bad = bad || !(rho > 0.0) || !(p > 0.0);
    }
  }
  if (bad && sub < 12 && flag) flag[0] = 1;
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

__global__ void k_to_shadow(int64_t nv, const double* __restrict__ U,
                            GasParams gp, float* __restrict__ Us) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= 12 * nv) return;
  const int64_t q = i / nv;
  Us[i] = float(U[i] - (q < 4 ? gp.wref[q] : 0.0));
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

hipError_t launch_edge64(int64_t ne, int64_t nv, const EdgeCoef<double>& c,
                         const GasParams& gp, const double* U,
                         const uint8_t* force, double* H, double* wlr,
                         uint8_t* mask, hipStream_t st) {
  if (ne == 0) return hipSuccess;
  hipLaunchKernelGGL(k_edge<double>, dim3(nblocks(ne, 256)), dim3(256), 0, st, ne,
                     nv, c, gp, U, force, H, wlr, mask);
  return hipGetLastError();
}

hipError_t launch_edge32(int64_t ne, int64_t nv, const EdgeCoef<float>& c,
                         const GasParams& gp, const float* Us,
                         const uint8_t* force, float* H, double* wlr,
                         uint8_t* mask, hipStream_t st) {
  if (ne == 0) return hipSuccess;
  hipLaunchKernelGGL(k_edge<float>, dim3(nblocks(ne, 256)), dim3(256), 0, st, ne,
                     nv, c, gp, Us, force, H, wlr, mask);
  return hipGetLastError();
}

template <class T>
static hipError_t launch_vertex(int64_t nowned, int64_t nv, const VertexCoef<T>& c,
                                const GasParams& gp, const T* U, const T* H,
                                int64_t ne, int mode, double* dU, const RkArgs& rk,
                                int32_t* flag, hipStream_t st) {
  if (nowned == 0) return hipSuccess;
  const unsigned nb = nblocks(nowned * VL, 256);
  if (c.dvis)
    hipLaunchKernelGGL((k_vertex<T, true>), dim3(nb), dim3(256), 0, st, nowned, nv,
                       c, gp, U, H, ne, mode, dU, rk, flag);
  else
    hipLaunchKernelGGL((k_vertex<T, false>), dim3(nb), dim3(256), 0, st, nowned,
                       nv, c, gp, U, H, ne, mode, dU, rk, flag);
  return hipGetLastError();
}

hipError_t launch_vertex64(int64_t nowned, int64_t nv, const VertexCoef<double>& c,
                           const GasParams& gp, const double* U, const double* H,
                           int64_t ne, int mode, double* dU, const RkArgs& rk,
                           int32_t* flag, hipStream_t st) {
  return launch_vertex<double>(nowned, nv, c, gp, U, H, ne, mode, dU, rk, flag, st);
}

hipError_t launch_vertex32(int64_t nowned, int64_t nv, const VertexCoef<float>& c,
                           const GasParams& gp, const float* Us, const float* H,
                           int64_t ne, int mode, double* dU, const RkArgs& rk,
                           int32_t* flag, hipStream_t st) {
  return launch_vertex<float>(nowned, nv, c, gp, Us, H, ne, mode, dU, rk, flag, st);
}

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

hipError_t launch_to_shadow(int64_t nv, const double* U, const GasParams& gp,
                            float* Us, hipStream_t st) {
  hipLaunchKernelGGL(k_to_shadow, dim3(nblocks(12 * nv, 256)), dim3(256), 0, st, nv,
                     U, gp, Us);
  return hipGetLastError();
}

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
