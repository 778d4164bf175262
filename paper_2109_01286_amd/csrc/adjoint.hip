// Hand-written adjoint (vector-Jacobian product) of the residual, float64.
//
// The residual R(U) of eq. HWENO is a composition of
//   (1) the edge pass: h_e = Rusanov(w_L(e), w_R(e); n_e), w_L / w_R the
//       Hermite or WENO midpoint states of Algorithm 1 (Roe-characteristic
//       projection, uniform WENO5 weights, switch of eq. 2d_hweno_intp);
//   (2) the vertex pass: R_v = - sum_slots D (f(w_u), g(w_u)) - sum_edges D h_m
//       (eq. flux_polynomials and the rows d0, dx, dy).
// Its transpose applied to lambda is computed in three deterministic
// gathers (no atomics), using transposed maps built at first use:
//   k_adj_edge_flux:  lambda_h(m) = -sum_{(v,s): m in M(v)} de[s] . lambda(v)
//   k_adj_edge:       recompute the edge pass and run it backwards, giving
//                     the contribution of h_e to the 72 data (w, w_x, w_y at
//                     the six stencil nodes) of edge e
//   k_adj_vertex:     lambda_U(u) = sum over the edges whose stencils contain
//                     u of those contributions + A_f(w_u)^T lambda_f(u) +
//                     A_g(w_u)^T lambda_g(u), lambda_f/g(u) gathered from the
//                     rows of the vertices whose stencils contain u.
// The switch and the WENO weights are differentiated through the branch the
// forward pass takes; the maximum in the Rusanov flux through its larger
// argument.  Euler only (viscous fluxes are not differentiated).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace hfd {
namespace {

// derivative of F(w).n transposed, applied to g: out += A_n(w)^T g
__device__ inline void flux_jac_t(const double w[4], double nx, double ny, double gm1,
                                  const double g[4], double out[4]) {
  const double rho = w[0], ir = 1.0 / rho, u = w[1] * ir, v = w[2] * ir;
  const double un = u * nx + v * ny;
  const double p = gm1 * (w[3] - 0.5 * rho * (u * u + v * v));
  // d un / dw, d p / dw
  const double dun[4] = {-un * ir, nx * ir, ny * ir, 0.0};
  const double dp[4] = {gm1 * 0.5 * (u * u + v * v), -gm1 * u, -gm1 * v, gm1};
  const double m = w[1], n = w[2], E = w[3];
  for (int k = 0; k < 4; ++k) {
    double s = 0.0;
    // component 0: rho un = m nx + n ny
    s += g[0] * (k == 1 ? nx : (k == 2 ? ny : 0.0));
    // component 1: m un + p nx
    s += g[1] * ((k == 1 ? un : 0.0) + m * dun[k] + nx * dp[k]);
    // component 2: n un + p ny
    s += g[2] * ((k == 2 ? un : 0.0) + n * dun[k] + ny * dp[k]);
    // component 3: (E + p) un
    s += g[3] * (un * ((k == 3 ? 1.0 : 0.0) + dp[k]) + (E + p) * dun[k]);
    out[k] += s;
  }
}

// d(|u.n| + c)/dw
__device__ inline void speed_grad(const double w[4], double nx, double ny, double gam,
                                  double out[4]) {
  const double gm1 = gam - 1.0;
  const double rho = w[0], ir = 1.0 / rho, u = w[1] * ir, v = w[2] * ir;
  const double un = u * nx + v * ny;
  const double p = gm1 * (w[3] - 0.5 * rho * (u * u + v * v));
  const double c = sqrt(gam * p * ir);
  const double sg = un > 0.0 ? 1.0 : (un < 0.0 ? -1.0 : 0.0);
  const double dun[4] = {-un * ir, nx * ir, ny * ir, 0.0};
  const double dp[4] = {gm1 * 0.5 * (u * u + v * v), -gm1 * u, -gm1 * v, gm1};
  const double k = gam / (2.0 * c * rho);
  for (int j = 0; j < 4; ++j) out[j] = sg * dun[j] + k * (dp[j] - (j == 0 ? p * ir : 0.0));
}

__device__ inline void cart_flux_n(const double w[4], double nx, double ny, double gm1,
                                   double f[4], double* sp, double gam) {
  const double rho = w[0], ir = 1.0 / rho, u = w[1] * ir, v = w[2] * ir;
  const double un = u * nx + v * ny;
  const double p = gm1 * (w[3] - 0.5 * rho * (u * u + v * v));
  f[0] = rho * un;
  f[1] = w[1] * un + p * nx;
  f[2] = w[2] * un + p * ny;
  f[3] = (w[3] + p) * un;
  *sp = fabs(un) + sqrt(gam * p * ir);
}

}  // namespace

// ---------------------------------------------------------------------------
// lambda_h(m) = - sum over (v, s) of de[s] . lambda(v)
// ---------------------------------------------------------------------------
__global__ void k_adj_edge_flux(int64_t ne, const int32_t* __restrict__ tptr,
                                const int32_t* __restrict__ tv, const int32_t* __restrict__ ts,
                                const double* __restrict__ de, const V4<double>* __restrict__ Lv,
                                const V4<double>* __restrict__ Lg, V4<double>* __restrict__ lh) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= ne) return;
  double a[4] = {0, 0, 0, 0};
  for (int k = tptr[m]; k < tptr[m + 1]; ++k) {
    const int64_t v = tv[k];
    const int64_t s = ts[k];
    const double d0 = de[3 * s], dx = de[3 * s + 1], dy = de[3 * s + 2];
    const V4<double> l0 = Lv[v], lx = Lg[2 * v], ly = Lg[2 * v + 1];
    a[0] -= d0 * l0.x + dx * lx.x + dy * ly.x;
    a[1] -= d0 * l0.y + dx * lx.y + dy * ly.y;
    a[2] -= d0 * l0.z + dx * lx.z + dy * ly.z;
    a[3] -= d0 * l0.w + dx * lx.w + dy * ly.w;
  }
  lh[m] = V4<double>{a[0], a[1], a[2], a[3]};
}

// ---------------------------------------------------------------------------
// Edge pass forward + reverse: out[e][j][12] = d h_e / d(data of node j)^T lh
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256, 1)
k_adj_edge(int64_t ne, EdgeCoef<double> c, GasParams gp, const V4<double>* __restrict__ Gv,
           const V4<double>* __restrict__ Gg, const uint8_t* __restrict__ force,
           const V4<double>* __restrict__ lh, double* __restrict__ out) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const double gam = gp.gamma, gm1 = gam - 1.0;
  int id[6];
  for (int t = 0; t < 6; ++t) id[t] = c.stg[t * ne + e];
  const double nx = c.n[e], ny = c.n[ne + e];
  double W[6][4], X[6][4], Y[6][4];
  for (int j = 0; j < 6; ++j) {
    const V4<double> a = Gv[id[j]], bx = Gg[2 * int64_t(id[j])], by = Gg[2 * int64_t(id[j]) + 1];
    W[j][0] = a.x; W[j][1] = a.y; W[j][2] = a.z; W[j][3] = a.w;
    X[j][0] = bx.x; X[j][1] = bx.y; X[j][2] = bx.z; X[j][3] = bx.w;
    Y[j][0] = by.x; Y[j][1] = by.y; Y[j][2] = by.z; Y[j][3] = by.w;
  }
  // ---- forward: Roe average --------------------------------------------------
  const double* A = W[2];
  const double* B = W[3];
  const double ra = A[0], rb = B[0];
  const double sa = sqrt(ra), sb = sqrt(rb), D = sa + sb;
  const double pa = gm1 * (A[3] - 0.5 * (A[1] * A[1] + A[2] * A[2]) / ra);
  const double pb = gm1 * (B[3] - 0.5 * (B[1] * B[1] + B[2] * B[2]) / rb);
  const double Pa = A[1] / sa, Pb = B[1] / sb, Qa = A[2] / sa, Qb = B[2] / sb;
  const double Ka = (A[3] + pa) / sa, Kb = (B[3] + pb) / sb;
  const double u = (Pa + Pb) / D, v = (Qa + Qb) / D, H = (Ka + Kb) / D;
  const double q2 = u * u + v * v;
  const double cc = sqrt(gm1 * (H - 0.5 * q2));
  const double un = u * nx + v * ny, ut = -u * ny + v * nx;
  const double b1 = gm1 / (cc * cc), b2 = 0.5 * b1 * q2, ic = 1.0 / cc;
  const double L[4][4] = {
      {0.5 * (b2 + un * ic), -0.5 * (b1 * u + nx * ic), -0.5 * (b1 * v + ny * ic), 0.5 * b1},
      {1.0 - b2, b1 * u, b1 * v, -b1},
      {0.5 * (b2 - un * ic), -0.5 * (b1 * u - nx * ic), -0.5 * (b1 * v - ny * ic), 0.5 * b1},
      {-ut, -ny, nx, 0.0}};
  const double R[4][4] = {{1.0, 1.0, 1.0, 0.0},
                          {u - cc * nx, u, u + cc * nx, -ny},
                          {v - cc * ny, v, v + cc * ny, nx},
                          {H - un * cc, 0.5 * q2, H + un * cc, ut}};
  const double eps = gp.eps;
  const double dw[3] = {1.0 / 16.0, 10.0 / 16.0, 5.0 / 16.0};
  const uint8_t fm = force ? force[e] : uint8_t(0);
  double wm[2][4], C[2][4], hs[2][4];
  double cv[2][4][5];
  bool weno[2][4];
  double om[2][4][3], Sk[2][4][3];
  for (int s = 0; s < 2; ++s) {
    int ix[5];
    for (int t = 0; t < 5; ++t) ix[t] = s == 0 ? t : 5 - t;
    for (int q = 0; q < 4; ++q) hs[s][q] = 0.0;
    for (int t = 0; t < 5; ++t) {
      const double w0 = c.w5[int64_t(s * 15 + 3 * t) * ne + e];
      const double w1 = c.w5[int64_t(s * 15 + 3 * t + 1) * ne + e];
      const double w2 = c.w5[int64_t(s * 15 + 3 * t + 2) * ne + e];
      for (int q = 0; q < 4; ++q) {
        cv[s][q][t] = L[q][0] * W[ix[t]][0] + L[q][1] * W[ix[t]][1] + L[q][2] * W[ix[t]][2] +
                      L[q][3] * W[ix[t]][3];
        hs[s][q] += w0 * W[ix[t]][q] + w1 * X[ix[t]][q] + w2 * Y[ix[t]][q];
      }
    }
    for (int q = 0; q < 4; ++q) {
      const double* cq = cv[s][q];
      const double t1 = cq[0] - 2 * cq[1] + cq[2], t2 = cq[0] - 4 * cq[1] + 3 * cq[2];
      const double t3 = cq[1] - 2 * cq[2] + cq[3], t4 = cq[1] - cq[3];
      const double t5 = cq[2] - 2 * cq[3] + cq[4], t6 = 3 * cq[2] - 4 * cq[3] + cq[4];
      const double be[3] = {13.0 / 12.0 * t1 * t1 + 0.25 * t2 * t2,
                            13.0 / 12.0 * t3 * t3 + 0.25 * t4 * t4,
                            13.0 / 12.0 * t5 * t5 + 0.25 * t6 * t6};
      double al[3], sal = 0.0;
      for (int k = 0; k < 3; ++k) {
        al[k] = dw[k] / ((eps + be[k]) * (eps + be[k]));
        sal += al[k];
      }
      for (int k = 0; k < 3; ++k) om[s][q][k] = al[k] / sal;
      bool wq;
      if (force) wq = (fm >> (4 * s + q)) & 1;
      else if (gp.sw == HFD_SWITCH_PAPER) wq = !(om[s][q][0] > gp.sw_lo && om[s][q][0] < gp.sw_hi);
      else wq = (gp.sw == HFD_SWITCH_WENO_ONLY);
      weno[s][q] = wq;
      for (int k = 0; k < 3; ++k) {
        double sk = 0.0;
        for (int t = 0; t < 3; ++t) sk += c.w3[int64_t(s * 9 + 3 * k + t) * ne + e] * cq[k + t];
        Sk[s][q][k] = sk;
      }
      C[s][q] = wq ? om[s][q][0] * Sk[s][q][0] + om[s][q][1] * Sk[s][q][1] + om[s][q][2] * Sk[s][q][2]
                   : L[q][0] * hs[s][0] + L[q][1] * hs[s][1] + L[q][2] * hs[s][2] + L[q][3] * hs[s][3];
    }
    for (int r = 0; r < 4; ++r)
      wm[s][r] = R[r][0] * C[s][0] + R[r][1] * C[s][1] + R[r][2] * C[s][2] + R[r][3] * C[s][3];
  }
  double fl[4], fr[4], sl, sr;
  cart_flux_n(wm[0], nx, ny, gm1, fl, &sl, gam);
  cart_flux_n(wm[1], nx, ny, gm1, fr, &sr, gam);
  const double lam = sl >= sr ? sl : sr;

  // ---- reverse ---------------------------------------------------------------
  const V4<double> g4 = lh[e];
  const double gh[4] = {g4.x, g4.y, g4.z, g4.w};
  double gw[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
  double glam = 0.0;
  for (int q = 0; q < 4; ++q) {
    glam -= 0.5 * gh[q] * (wm[1][q] - wm[0][q]);
    gw[0][q] += 0.5 * lam * gh[q];
    gw[1][q] -= 0.5 * lam * gh[q];
  }
  const double half[4] = {0.5 * gh[0], 0.5 * gh[1], 0.5 * gh[2], 0.5 * gh[3]};
  flux_jac_t(wm[0], nx, ny, gm1, half, gw[0]);
  flux_jac_t(wm[1], nx, ny, gm1, half, gw[1]);
  {
    double ds[4];
    const int act = sl >= sr ? 0 : 1;
    speed_grad(wm[act], nx, ny, gam, ds);
    for (int k = 0; k < 4; ++k) gw[act][k] += glam * ds[k];
  }
  double gL[4][4] = {}, gR[4][4] = {};
  double gW[6][4] = {}, gX[6][4] = {}, gY[6][4] = {};
  for (int s = 0; s < 2; ++s) {
    int ix[5];
    for (int t = 0; t < 5; ++t) ix[t] = s == 0 ? t : 5 - t;
    double gC[4];
    for (int q = 0; q < 4; ++q) {
      gC[q] = R[0][q] * gw[s][0] + R[1][q] * gw[s][1] + R[2][q] * gw[s][2] + R[3][q] * gw[s][3];
      for (int r = 0; r < 4; ++r) gR[r][q] += gw[s][r] * C[s][q];
    }
    double ghs[4] = {0, 0, 0, 0};
    double gcv[4][5] = {};
    for (int q = 0; q < 4; ++q) {
      if (!weno[s][q]) {
        for (int k = 0; k < 4; ++k) {
          gL[q][k] += gC[q] * hs[s][k];
          ghs[k] += gC[q] * L[q][k];
        }
        continue;
      }
      const double* cq = cv[s][q];
      double gS[3], gom[3];
      for (int k = 0; k < 3; ++k) {
        gS[k] = gC[q] * om[s][q][k];
        gom[k] = gC[q] * Sk[s][q][k];
      }
      for (int k = 0; k < 3; ++k)
        for (int t = 0; t < 3; ++t)
          gcv[q][k + t] += gS[k] * c.w3[int64_t(s * 9 + 3 * k + t) * ne + e];
      // omega = alpha / sum(alpha), alpha = d / (eps + beta)^2
      const double t1 = cq[0] - 2 * cq[1] + cq[2], t2 = cq[0] - 4 * cq[1] + 3 * cq[2];
      const double t3 = cq[1] - 2 * cq[2] + cq[3], t4 = cq[1] - cq[3];
      const double t5 = cq[2] - 2 * cq[3] + cq[4], t6 = 3 * cq[2] - 4 * cq[3] + cq[4];
      const double be[3] = {13.0 / 12.0 * t1 * t1 + 0.25 * t2 * t2,
                            13.0 / 12.0 * t3 * t3 + 0.25 * t4 * t4,
                            13.0 / 12.0 * t5 * t5 + 0.25 * t6 * t6};
      double al[3], sal = 0.0;
      for (int k = 0; k < 3; ++k) {
        al[k] = dw[k] / ((eps + be[k]) * (eps + be[k]));
        sal += al[k];
      }
      double dot = 0.0;
      for (int k = 0; k < 3; ++k) dot += gom[k] * om[s][q][k];
      double gbe[3];
      for (int k = 0; k < 3; ++k) {
        const double gal = (gom[k] - dot) / sal;
        gbe[k] = -2.0 * gal * al[k] / (eps + be[k]);
      }
      const double gt1 = gbe[0] * (13.0 / 6.0) * t1, gt2 = gbe[0] * 0.5 * t2;
      const double gt3 = gbe[1] * (13.0 / 6.0) * t3, gt4 = gbe[1] * 0.5 * t4;
      const double gt5 = gbe[2] * (13.0 / 6.0) * t5, gt6 = gbe[2] * 0.5 * t6;
      gcv[q][0] += gt1 + gt2;
      gcv[q][1] += -2.0 * gt1 - 4.0 * gt2 + gt3 + gt4;
      gcv[q][2] += gt1 + 3.0 * gt2 - 2.0 * gt3 + gt5 + 3.0 * gt6;
      gcv[q][3] += gt3 - gt4 - 2.0 * gt5 - 4.0 * gt6;
      gcv[q][4] += gt5 + gt6;
    }
    // hs = sum_t w5 . data ; cv[q][t] = L[q] . W_t
    for (int t = 0; t < 5; ++t) {
      const double w0 = c.w5[int64_t(s * 15 + 3 * t) * ne + e];
      const double w1 = c.w5[int64_t(s * 15 + 3 * t + 1) * ne + e];
      const double w2 = c.w5[int64_t(s * 15 + 3 * t + 2) * ne + e];
      for (int k = 0; k < 4; ++k) {
        gW[ix[t]][k] += w0 * ghs[k];
        gX[ix[t]][k] += w1 * ghs[k];
        gY[ix[t]][k] += w2 * ghs[k];
      }
      for (int q = 0; q < 4; ++q) {
        if (gcv[q][t] == 0.0) continue;
        for (int k = 0; k < 4; ++k) {
          gL[q][k] += gcv[q][t] * W[ix[t]][k];
          gW[ix[t]][k] += gcv[q][t] * L[q][k];
        }
      }
    }
  }
  // ---- L, R -> (u, v, H, c) ----------------------------------------------------
  double gu = 0, gv = 0, gH = 0, gc = 0;
  // R
  gu += gR[1][0] + gR[1][1] + gR[1][2] + gR[3][0] * (-nx * cc) + gR[3][1] * u +
        gR[3][2] * (nx * cc) + gR[3][3] * (-ny);
  gv += gR[2][0] + gR[2][1] + gR[2][2] + gR[3][0] * (-ny * cc) + gR[3][1] * v +
        gR[3][2] * (ny * cc) + gR[3][3] * nx;
  gH += gR[3][0] + gR[3][2];
  gc += gR[1][0] * (-nx) + gR[1][2] * nx + gR[2][0] * (-ny) + gR[2][2] * ny +
        gR[3][0] * (-un) + gR[3][2] * un;
  // L (b1 = gm1/c^2, b2 = b1 q2/2, ic = 1/c)
  const double ic2 = ic * ic;
  gu += gL[0][0] * 0.5 * (b1 * u + nx * ic) + gL[0][1] * (-0.5 * b1) +
        gL[1][0] * (-b1 * u) + gL[1][1] * b1 + gL[2][0] * 0.5 * (b1 * u - nx * ic) +
        gL[2][1] * (-0.5 * b1) + gL[3][0] * ny;
  gv += gL[0][0] * 0.5 * (b1 * v + ny * ic) + gL[0][2] * (-0.5 * b1) +
        gL[1][0] * (-b1 * v) + gL[1][2] * b1 + gL[2][0] * 0.5 * (b1 * v - ny * ic) +
        gL[2][2] * (-0.5 * b1) + gL[3][0] * (-nx);
  gc += gL[0][0] * 0.5 * (-2.0 * b2 * ic - un * ic2) + gL[0][1] * 0.5 * (2.0 * b1 * u * ic + nx * ic2) +
        gL[0][2] * 0.5 * (2.0 * b1 * v * ic + ny * ic2) + gL[0][3] * (-b1 * ic) +
        gL[1][0] * (2.0 * b2 * ic) + gL[1][1] * (-2.0 * b1 * u * ic) +
        gL[1][2] * (-2.0 * b1 * v * ic) + gL[1][3] * (2.0 * b1 * ic) +
        gL[2][0] * 0.5 * (-2.0 * b2 * ic + un * ic2) + gL[2][1] * 0.5 * (2.0 * b1 * u * ic - nx * ic2) +
        gL[2][2] * 0.5 * (2.0 * b1 * v * ic - ny * ic2) + gL[2][3] * (-b1 * ic);
  // c = sqrt(gm1 (H - q2/2))
  gH += gc * gm1 / (2.0 * cc);
  gu += gc * (-gm1 * u / (2.0 * cc));
  gv += gc * (-gm1 * v / (2.0 * cc));
  // ---- Roe average -> end states -------------------------------------------------
  const double gP = gu / D, gQ = gv / D, gK = gH / D;
  const double gD = -(gu * u + gv * v + gH * H) / D;
  for (int side = 0; side < 2; ++side) {
    const double* S = side == 0 ? A : B;
    double* g = gW[side == 0 ? 2 : 3];
    const double r = S[0], s_ = side == 0 ? sa : sb, p = side == 0 ? pa : pb;
    double gs = gD;
    // P = m/s, Q = n/s, K = (E + p)/s
    g[1] += gP / s_;
    g[2] += gQ / s_;
    gs += -(gP * S[1] + gQ * S[2] + gK * (S[3] + p)) / (s_ * s_);
    const double gE = gK / s_, gp = gK / s_;
    g[3] += gE;
    // p = gm1 (E - (m^2 + n^2) / (2 r))
    g[3] += gm1 * gp;
    g[1] += -gm1 * gp * S[1] / r;
    g[2] += -gm1 * gp * S[2] / r;
    g[0] += gm1 * gp * 0.5 * (S[1] * S[1] + S[2] * S[2]) / (r * r);
    // s = sqrt(r)
    g[0] += gs / (2.0 * s_);
  }
  double* o = out + int64_t(e) * 72;
  for (int j = 0; j < 6; ++j)
    for (int k = 0; k < 4; ++k) {
      o[12 * j + k] = gW[j][k];
      o[12 * j + 4 + k] = gX[j][k];
      o[12 * j + 8 + k] = gY[j][k];
    }
}

// ---------------------------------------------------------------------------
// lambda_U(u) for owned u
// ---------------------------------------------------------------------------
__global__ void k_adj_vertex(int64_t nowned, int64_t nv, GasParams gp, const double* __restrict__ U,
                             const int32_t* __restrict__ vtp, const int32_t* __restrict__ vtv,
                             const int32_t* __restrict__ vts, const double* __restrict__ dv,
                             const int32_t* __restrict__ ntp, const int32_t* __restrict__ nte,
                             const int8_t* __restrict__ ntj, const double* __restrict__ bnode,
                             const V4<double>* __restrict__ Lv, const V4<double>* __restrict__ Lg,
                             double* __restrict__ out) {
  const int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (u >= nowned) return;
  const double gm1 = gp.gamma - 1.0;
  double acc[12] = {};
  // edge-pass contributions
  for (int k = ntp[u]; k < ntp[u + 1]; ++k) {
    const double* b = bnode + int64_t(nte[k]) * 72 + 12 * ntj[k];
    for (int q = 0; q < 12; ++q) acc[q] += b[q];
  }
  // vertex fluxes: lambda_f, lambda_g from the rows containing u
  double lf[4] = {0, 0, 0, 0}, lg[4] = {0, 0, 0, 0};
  for (int k = vtp[u]; k < vtp[u + 1]; ++k) {
    const int64_t v = vtv[k], s = vts[k];
    const double* d = dv + 6 * s;
    const V4<double> l0 = Lv[v], lx = Lg[2 * v], ly = Lg[2 * v + 1];
    const double a0[4] = {l0.x, l0.y, l0.z, l0.w};
    const double ax[4] = {lx.x, lx.y, lx.z, lx.w};
    const double ay[4] = {ly.x, ly.y, ly.z, ly.w};
    for (int q = 0; q < 4; ++q) {
      lf[q] -= d[0] * a0[q] + d[2] * ax[q] + d[4] * ay[q];
      lg[q] -= d[1] * a0[q] + d[3] * ax[q] + d[5] * ay[q];
    }
  }
  double w[4];
  for (int q = 0; q < 4; ++q) w[q] = U[q * nv + u];
  // A_f^T lf + A_g^T lg = A_n^T with n = (1,0) and (0,1)
  flux_jac_t(w, 1.0, 0.0, gm1, lf, acc);
  flux_jac_t(w, 0.0, 1.0, gm1, lg, acc);
  for (int q = 0; q < 12; ++q) out[q * nv + u] = acc[q];
}

hipError_t launch_adjoint_residual(const AdjointArgs& a, hipStream_t st) {
  if (a.ne > 0) {
    hipLaunchKernelGGL(k_adj_edge_flux, dim3(unsigned((a.ne + 255) / 256)), dim3(256), 0, st,
                       a.ne, a.etp, a.etv, a.ets, a.de, a.Lv, a.Lg, a.lh);
    hipLaunchKernelGGL(k_adj_edge, dim3(unsigned((a.ne + 255) / 256)), dim3(256), 0, st, a.ne,
                       a.ec, a.gp, a.Gv, a.Gg, a.force, a.lh, a.bnode);
  }
  if (a.nowned > 0)
    hipLaunchKernelGGL(k_adj_vertex, dim3(unsigned((a.nowned + 255) / 256)), dim3(256), 0, st,
                       a.nowned, a.nv, a.gp, a.U, a.vtp, a.vtv, a.vts, a.dv, a.ntp, a.nte,
                       a.ntj, a.bnode, a.Lv, a.Lg, a.out);
  return hipGetLastError();
}

}  // namespace hfd
