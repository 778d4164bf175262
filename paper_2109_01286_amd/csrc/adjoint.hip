// Hand-written adjoint (vector-Jacobian product) of the residual, float64 or
// float32 (the mixed form: float32 arithmetic on its own stage states, the
// per-vertex sums written to float64).
//
// The residual R(U) of eq. HWENO is a composition of
//   (1) the edge pass: h_e = Rusanov(w_L(e), w_R(e); n_e), w_L / w_R the
//       Hermite or WENO midpoint states of Algorithm 1 (Roe-characteristic
//       projection, uniform WENO5 weights, switch of eq. 2d_hweno_intp);
//   (2) the vertex pass: R_v = - sum_slots D (f(w_u), g(w_u)) - sum_edges D h_m
//       (eq. flux_polynomials and the rows d0, dx, dy).
// Its transpose applied to lambda is computed in two deterministic
// gathers (no atomics), using transposed maps built at first use (de and dv
// are read from copies in the transposed order):
//   k_adj_edge:       lambda_h(e) = -sum_{(v,s): e in M(v)} de[s] . lambda(v),
//                     then recompute the edge pass and run it backwards,
//                     giving the contribution of h_e to the 72 data (w, w_x,
//                     w_y at the six stencil nodes) of edge e
//   k_adj_vertex:     lambda_U(u) = sum over the edges whose stencils contain
//                     u of those contributions + A_f(w_u)^T lambda_f(u) +
//                     A_g(w_u)^T lambda_g(u), lambda_f/g(u) gathered from the
//                     rows of the vertices whose stencils contain u; with
//                     viscosity + the viscous flux derivative at
//                     (w_u, w_x(u), w_y(u)) applied to Lambda_fv/gv(u),
//                     gathered the same way from the viscous rows.
// The switch and the WENO weights are differentiated through the branch the
// forward pass takes; the maximum in the Rusanov flux through its larger
// argument.
#include <hip/hip_runtime.h>

#include "gas.h"
#include "kernels.h"

#ifndef ADJ_EDGE_WAVES
#define ADJ_EDGE_WAVES 2  // waves per SIMD of the edge reverse (register budget)
#endif

namespace hfd {
namespace {

// lambda_h entries per lane and batch in the edge reverse (measured: 4 is
// faster in float32, 2 in float64, whose registers are scarcer)
template <class T>
constexpr int kAdjGatherBatch = sizeof(T) == 4 ? 4 : 2;
// values per stencil node in the edge reverse's rows: (w, w_x, w_y), or w
// alone when the switch takes WENO everywhere (the gradients get nothing)
template <int SWM>
constexpr int kAdjNodeValues = SWM == HFD_SWITCH_WENO_ONLY ? 4 : 12;

// Forward-mode dual number: a value and its derivative along one direction.
// The adjoint of the Roe and HLLC fluxes runs their code (gas.h) on it, one
// direction per component of the lane's interface state, so that every
// branch the flux takes (entropy fix, wave-speed minimum and maximum, HLLC
// region) is differentiated as taken.
// (the overloads below would hide the plain ones inside namespace hfd)
using ::fabs;
using ::fmax;
using ::fmin;
using ::isnan;
using ::sqrt;

template <class B>
struct Dual {
  B v, d;
  Dual() = default;
  __device__ Dual(B x) : v(x), d(B(0)) {}
  __device__ Dual(B x, B y) : v(x), d(y) {}
};
template <class B>
__device__ inline Dual<B> operator+(Dual<B> a, Dual<B> b) { return {a.v + b.v, a.d + b.d}; }
template <class B>
__device__ inline Dual<B> operator-(Dual<B> a, Dual<B> b) { return {a.v - b.v, a.d - b.d}; }
template <class B>
__device__ inline Dual<B> operator-(Dual<B> a) { return {-a.v, -a.d}; }
template <class B>
__device__ inline Dual<B> operator*(Dual<B> a, Dual<B> b) {
  return {a.v * b.v, a.d * b.v + a.v * b.d};
}
template <class B>
__device__ inline Dual<B> operator/(Dual<B> a, Dual<B> b) {
  const B q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
template <class B>
__device__ inline Dual<B>& operator+=(Dual<B>& a, Dual<B> b) { return a = a + b; }
template <class B>
__device__ inline bool operator<(Dual<B> a, Dual<B> b) { return a.v < b.v; }
template <class B>
__device__ inline bool operator>(Dual<B> a, Dual<B> b) { return a.v > b.v; }
template <class B>
__device__ inline bool operator<=(Dual<B> a, Dual<B> b) { return a.v <= b.v; }
template <class B>
__device__ inline bool operator>=(Dual<B> a, Dual<B> b) { return a.v >= b.v; }
template <class B>
__device__ inline Dual<B> sqrt(Dual<B> a) {
  const B r = sqrt(a.v);
  return {r, a.d / (B(2) * r)};
}
template <class B>
__device__ inline Dual<B> fabs(Dual<B> a) { return a.v < B(0) ? -a : a; }
template <class B>
__device__ inline Dual<B> fmin(Dual<B> a, Dual<B> b) { return b.v < a.v ? b : a; }
template <class B>
__device__ inline Dual<B> fmax(Dual<B> a, Dual<B> b) { return b.v > a.v ? b : a; }
template <class B>
__device__ inline bool isnan(Dual<B> a) { return isnan(a.v); }

// derivative of F(w).n transposed, applied to g: out += A_n(w)^T g
template <class T>
__device__ inline void flux_jac_t(const T w[4], T nx, T ny, T gm1,
                                  const T g[4], T out[4]) {
  const T rho = w[0], ir = frcp(rho), u = w[1] * ir, v = w[2] * ir;
  const T un = u * nx + v * ny;
  const T p = gm1 * (w[3] - T(0.5) * rho * (u * u + v * v));
  // d un / dw, d p / dw
  const T dun[4] = {-un * ir, nx * ir, ny * ir, T(0.0)};
  const T dp[4] = {gm1 * T(0.5) * (u * u + v * v), -gm1 * u, -gm1 * v, gm1};
  const T m = w[1], n = w[2], E = w[3];
  for (int k = 0; k < 4; ++k) {
    T s = T(0.0);
    // component 0: rho un = m nx + n ny
    s += g[0] * (k == 1 ? nx : (k == 2 ? ny : T(0.0)));
    // component 1: m un + p nx
    s += g[1] * ((k == 1 ? un : T(0.0)) + m * dun[k] + nx * dp[k]);
    // component 2: n un + p ny
    s += g[2] * ((k == 2 ? un : T(0.0)) + n * dun[k] + ny * dp[k]);
    // component 3: (E + p) un
    s += g[3] * (un * ((k == 3 ? T(1.0) : T(0.0)) + dp[k]) + (E + p) * dun[k]);
    out[k] += s;
  }
}

// d(|u.n| + c)/dw
template <class T>
__device__ inline void speed_grad(const T w[4], T nx, T ny, T gam,
                                  T out[4]) {
  const T gm1 = gam - T(1.0);
  const T rho = w[0], ir = frcp(rho), u = w[1] * ir, v = w[2] * ir;
  const T un = u * nx + v * ny;
  const T p = gm1 * (w[3] - T(0.5) * rho * (u * u + v * v));
  const T c = fsqrt(gam * p * ir);
  const T sg = un > T(0.0) ? T(1.0) : (un < T(0.0) ? -T(1.0) : T(0.0));
  const T dun[4] = {-un * ir, nx * ir, ny * ir, T(0.0)};
  const T dp[4] = {gm1 * T(0.5) * (u * u + v * v), -gm1 * u, -gm1 * v, gm1};
  const T k = T(0.5) * gam * frcp(c) * ir;
  for (int j = 0; j < 4; ++j) out[j] = sg * dun[j] + k * (dp[j] - (j == 0 ? p * ir : T(0.0)));
}

template <class T>
__device__ inline void cart_flux_n(const T w[4], T nx, T ny, T gm1,
                                   T f[4], T* sp, T gam) {
  const T rho = w[0], ir = frcp(rho), u = w[1] * ir, v = w[2] * ir;
  const T un = u * nx + v * ny;
  const T p = gm1 * (w[3] - T(0.5) * rho * (u * u + v * v));
  f[0] = rho * un;
  f[1] = w[1] * un + p * nx;
  f[2] = w[2] * un + p * ny;
  f[3] = (w[3] + p) * un;
  *sp = fabs(un) + fsqrt(gam * p * ir);
}

// x, opaque to the optimiser (no code): values derived from it after this
// point are recomputed rather than reused from before.
template <class T>
__device__ inline T launder(T x) {
  asm volatile("" : "+v"(x));
  return x;
}

}  // namespace

// ---------------------------------------------------------------------------
// Edge pass forward + reverse: out[e][j][12] = d h_e / d(data of node j)^T lambda_h(e)
// ---------------------------------------------------------------------------
// Two lanes per edge: lane s recomputes side s (left: nodes 0..4, right:
// nodes 5..1, at positions t = 0..4) and runs it backwards; both lanes hold
// the Roe average and the flux.  The pair exchanges the interface states,
// the four scalar gradients of the Roe state (u, v, H, c) and the
// contributions to the nodes both sides share, then lane 0 writes nodes
// 0, 1, 2 and lane 1 nodes 5, 4, 3 (positions 0, 1, 2 of each lane).
// (the Roe and HLLC variants carry the dual-number flux: one wave per SIMD,
// the whole register file)
// SWM: the switch mode (hfd_switch), or kSwForced for the decisions of a
// forced mask, fixed at compile time.
template <class T, int FLUX, int SWM>
__global__ void __launch_bounds__(256, FLUX == HFD_FLUX_RUSANOV ? ADJ_EDGE_WAVES : 1)
k_adj_edge(int64_t ne, EdgeCoef<T> c, GasParams gp, const V4<T>* __restrict__ Gv,
           const V4<T>* __restrict__ Gg, const uint8_t* __restrict__ force,
           const int32_t* __restrict__ tptr, const int32_t* __restrict__ tv,
           const T* __restrict__ de_t, const V4<T>* __restrict__ Lv,
           const V4<T>* __restrict__ Lg, const int32_t* __restrict__ lrp,
           const int32_t* __restrict__ lrow, const uint16_t* __restrict__ lpos,
           T* __restrict__ out) {
  // With WENO everywhere no Hermite value is formed: the Hermite rows are not
  // read and the node gradients get no contribution, so each node's part of
  // the row is its 4 value entries instead of 12.
  constexpr bool HERM = SWM != HFD_SWITCH_WENO_ONLY;
  constexpr int NW = kAdjNodeValues<SWM>;
  // The block's output rows (6 NW values per edge) go through LDS; before
  // that, the same LDS holds the staged lambda rows.
  constexpr int RW = 6 * NW;
  __shared__ __attribute__((aligned(32))) T obuf[kAdjEdgesPerBlock * RW];
  static_assert(kAdjStageRows * 12 <= kAdjEdgesPerBlock * RW, "staged rows fit in obuf");
  const int s = threadIdx.x & 1;
  const int64_t eb = int64_t(blockIdx.x) * kAdjEdgesPerBlock;
  // lanes past the last edge recompute the last edge (both lanes of a pair
  // alike) and their results are not written
  const int64_t e = eb + threadIdx.x / 2 < ne ? eb + threadIdx.x / 2 : ne - 1;
  // Staging: the (lambda, lambda_x, lambda_y) rows of the distinct vertices
  // the block's entries name go to LDS once; the entries read them by
  // position.
  const bool stg = lrp != nullptr;
  V4<T>* lam_s = reinterpret_cast<V4<T>*>(obuf);
  if (stg) {
    const int r0 = lrp[blockIdx.x], nr = lrp[blockIdx.x + 1] - r0;
    for (int k = int(threadIdx.x); k < nr; k += int(blockDim.x)) {
      const int64_t u = lrow[r0 + k];
      lam_s[3 * k] = Lv[u];
      lam_s[3 * k + 1] = Lg[2 * u];
      lam_s[3 * k + 2] = Lg[2 * u + 1];
    }
    __syncthreads();
  }
  // lambda_h(e) = - sum over the (v, s') entries whose rows read h_e of
  // de[s'] . (lambda, lambda_x, lambda_y)(v): the lanes take alternate
  // entries (transposed order, contiguous per edge; every active edge has
  // one, so k1 - 1 is an entry: a lane past the end loads it again with zero
  // weight), kAdjGatherBatch per lane and batch, loads issued here so that
  // they overlap the forward recompute, and add their partial sums with one
  // lane swap
  T gh[4] = {T(0.0), T(0.0), T(0.0), T(0.0)};
  {
    const int k0 = tptr[e], k1 = tptr[e + 1];
    for (int b = k0 + s; b < k1; b += 2 * kAdjGatherBatch<T>) {
      constexpr int NB = kAdjGatherBatch<T>;
      int kk[NB];
      bool ok[NB];
      for (int i = 0; i < NB; ++i) {
        ok[i] = b + 2 * i < k1;
        kk[i] = ok[i] ? b + 2 * i : k1 - 1;
      }
      int v[NB];
      T d[NB][3];
      for (int i = 0; i < NB; ++i) {
        v[i] = stg ? int(lpos[kk[i]]) : tv[kk[i]];
        for (int q = 0; q < 3; ++q) d[i][q] = de_t[3 * int64_t(kk[i]) + q];
      }
      V4<T> l0[NB], lx[NB], ly[NB];
      for (int i = 0; i < NB; ++i) {
        if (stg) {
          l0[i] = lam_s[3 * v[i]];
          lx[i] = lam_s[3 * v[i] + 1];
          ly[i] = lam_s[3 * v[i] + 2];
        } else {
          l0[i] = Lv[v[i]];
          lx[i] = Lg[2 * int64_t(v[i])];
          ly[i] = Lg[2 * int64_t(v[i]) + 1];
        }
      }
      for (int i = 0; i < NB; ++i) {
        const T d0 = ok[i] ? d[i][0] : T(0.0), dx = ok[i] ? d[i][1] : T(0.0),
                dy = ok[i] ? d[i][2] : T(0.0);
        gh[0] -= d0 * l0[i].x + dx * lx[i].x + dy * ly[i].x;
        gh[1] -= d0 * l0[i].y + dx * lx[i].y + dy * ly[i].y;
        gh[2] -= d0 * l0[i].z + dx * lx[i].z + dy * ly[i].z;
        gh[3] -= d0 * l0[i].w + dx * lx[i].w + dy * ly[i].w;
      }
    }
    // the pair's sums agree bit for bit (a + b and b + a)
    for (int q = 0; q < 4; ++q) {
      gh[q] = launder(gh[q]);
      gh[q] += dpp_mov<0xB1>(gh[q]);
    }
  }
  // (the staged rows are read; the LDS takes the output rows later)
  if (stg) __syncthreads();
  const T gam = gpar<T>(gp.gamma, gp.f_gamma), gm1 = gpar<T>(gp.gamma - 1.0, gp.f_gm1);
  const T nx = c.n[2 * e], ny = c.n[2 * e + 1];
  const int ia = c.stg[2 * ne + e], ib = c.stg[3 * ne + e];
  int id[5];
  for (int t = 0; t < 5; ++t) id[t] = c.stg[(s == 0 ? t : 5 - t) * ne + e];
  const T eps = gpar<T>(gp.eps, gp.f_eps);
  const uint8_t fm = SWM == kSwForced ? force[e] : uint8_t(0);
  // The float32 form stores the perturbation w - w_ref of the values (the
  // gradients unchanged); the reverse works on the full state.
  auto full = [&](T x, int q) -> T {
    if constexpr (sizeof(T) == 4) return x + gp.f_wref[q];
    else return x;
  };
  // Roe average of nodes 2 and 3 and the eigenvector matrices L (rows), R
  auto roe = [&](T A[4], T B[4], T& sa, T& sb, T& D, T& pa,
                 T& pb, T& u, T& v, T& H, T& cc) {
    const V4<T> a = Gv[launder(ia)], b = Gv[launder(ib)];
    A[0] = a.x; A[1] = a.y; A[2] = a.z; A[3] = a.w;
    B[0] = b.x; B[1] = b.y; B[2] = b.z; B[3] = b.w;
    for (int q = 0; q < 4; ++q) {
      A[q] = full(A[q], q);
      B[q] = full(B[q], q);
    }
    const T ra = A[0], rb = B[0];
    const T ira = frcp(ra), irb = frcp(rb);
    sa = fsqrt(ra);
    sb = fsqrt(rb);
    D = sa + sb;
    pa = gm1 * (A[3] - T(0.5) * (A[1] * A[1] + A[2] * A[2]) * ira);
    pb = gm1 * (B[3] - T(0.5) * (B[1] * B[1] + B[2] * B[2]) * irb);
    // 1/sqrt(r) = sqrt(r)/r
    const T isa = sa * ira, isb = sb * irb, iD = frcp(D);
    const T Pa = A[1] * isa, Pb = B[1] * isb, Qa = A[2] * isa, Qb = B[2] * isb;
    const T Ka = (A[3] + pa) * isa, Kb = (B[3] + pb) * isb;
    u = (Pa + Pb) * iD;
    v = (Qa + Qb) * iD;
    H = (Ka + Kb) * iD;
    cc = fsqrt(gm1 * (H - T(0.5) * (u * u + v * v)));
  };
  auto eig = [&](T u, T v, T H, T cc, T L[4][4], T R[4][4]) {
    const T q2 = u * u + v * v;
    const T un = u * nx + v * ny, ut = -u * ny + v * nx;
    const T ic = frcp(cc), b1 = gm1 * ic * ic, b2 = T(0.5) * b1 * q2;
    const T Lv[4][4] = {
        {T(0.5) * (b2 + un * ic), -T(0.5) * (b1 * u + nx * ic), -T(0.5) * (b1 * v + ny * ic), T(0.5) * b1},
        {T(1.0) - b2, b1 * u, b1 * v, -b1},
        {T(0.5) * (b2 - un * ic), -T(0.5) * (b1 * u - nx * ic), -T(0.5) * (b1 * v - ny * ic), T(0.5) * b1},
        {-ut, -ny, nx, T(0.0)}};
    const T Rv[4][4] = {{T(1.0), T(1.0), T(1.0), T(0.0)},
                             {u - cc * nx, u, u + cc * nx, -ny},
                             {v - cc * ny, v, v + cc * ny, nx},
                             {H - un * cc, T(0.5) * q2, H + un * cc, ut}};
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        L[i][j] = Lv[i][j];
        R[i][j] = Rv[i][j];
      }
  };
  // this side's node values and coefficient rows.  The indices and the base
  // pointers pass through launder() at every use, so that the compiler
  // recomputes the addresses there instead of keeping them in registers.
  const T* w5p = c.w5 + (int64_t(s) * ne + e) * 15;
  const T* w3p = c.w3 + (int64_t(s) * ne + e) * 9;
  auto load_W = [&](T W[5][4]) {
    for (int t = 0; t < 5; ++t) {
      const V4<T> a = Gv[launder(id[t])];
      W[t][0] = full(a.x, 0); W[t][1] = full(a.y, 1); W[t][2] = full(a.z, 2);
      W[t][3] = full(a.w, 3);
    }
  };
  auto load_w5 = [&](T w5[5][3]) {
    const T* b = launder(w5p);
    for (int t = 0; t < 5; ++t)
      for (int k = 0; k < 3; ++k) w5[t][k] = b[3 * t + k];
  };
  auto load_w3 = [&](T w3[9]) {
    const T* b = launder(w3p);
    for (int j = 0; j < 9; ++j) w3[j] = b[j];
  };
  // projected node values of component q
  auto proj = [&](const T L[4][4], const T W[5][4], int q, T cq[5]) {
    for (int t = 0; t < 5; ++t)
      cq[t] = L[q][0] * W[t][0] + L[q][1] * W[t][1] + L[q][2] * W[t][2] + L[q][3] * W[t][3];
  };
  // smoothness indicators, WENO weights and 3-node values of component q
  // the forward passes' weights (shared code: the same decisions)
  auto weno_parts = [&](const T w3[9], const T cq[5], T be[3], T om[3], T Sk[3]) {
    weno_weights<T>(cq, eps, be, om);
    for (int k = 0; k < 3; ++k) {
      T sk = T(0.0);
      for (int t = 0; t < 3; ++t) sk += w3[3 * k + t] * cq[k + t];
      Sk[k] = sk;
    }
  };

  // ---- forward ---------------------------------------------------------------------
  bool weno[4];
  T hs[4] = {0, 0, 0, 0}, C[4], wm[4], wl[4], wr[4], sl, sr, lam;
  {
    T A[4], B[4], sa, sb, D, pa, pb, u, v, H, cc, L[4][4], R[4][4];
    roe(A, B, sa, sb, D, pa, pb, u, v, H, cc);
    eig(u, v, H, cc, L, R);
    T W[5][4], w3[9];
    load_W(W);
    load_w3(w3);
    if constexpr (HERM) {
      T w5[5][3];
      load_w5(w5);
      for (int t = 0; t < 5; ++t) {
        const V4<T> bx = Gg[2 * int64_t(id[t])], by = Gg[2 * int64_t(id[t]) + 1];
        const T X[4] = {bx.x, bx.y, bx.z, bx.w}, Y[4] = {by.x, by.y, by.z, by.w};
        for (int q = 0; q < 4; ++q)
          hs[q] += w5[t][0] * W[t][q] + w5[t][1] * X[q] + w5[t][2] * Y[q];
      }
    }
    for (int q = 0; q < 4; ++q) {
      T cq[5], be[3], om[3], Sk[3];
      proj(L, W, q, cq);
      weno_parts(w3, cq, be, om, Sk);
      bool wq;
      if constexpr (SWM == kSwForced) wq = (fm >> (4 * s + q)) & 1;
      else if constexpr (SWM == HFD_SWITCH_PAPER)
        wq = !weno_in<T>(be, eps, gpar<T>(gp.sw_lo, gp.f_sw_lo), gpar<T>(gp.sw_hi, gp.f_sw_hi));
      else wq = (SWM == HFD_SWITCH_WENO_ONLY);
      weno[q] = wq;
      C[q] = wq ? om[0] * Sk[0] + om[1] * Sk[1] + om[2] * Sk[2]
                : L[q][0] * hs[0] + L[q][1] * hs[1] + L[q][2] * hs[2] + L[q][3] * hs[3];
    }
    for (int r = 0; r < 4; ++r) wm[r] = R[r][0] * C[0] + R[r][1] * C[1] + R[r][2] * C[2] + R[r][3] * C[3];
    for (int r = 0; r < 4; ++r) {
      const T o = dpp_mov<0xB1>(wm[r]);  // the partner lane's state
      wl[r] = s == 0 ? wm[r] : o;
      wr[r] = s == 0 ? o : wm[r];
    }
    if constexpr (FLUX == HFD_FLUX_RUSANOV) {
      T fl[4], fr[4];
      cart_flux_n(wl, nx, ny, gm1, fl, &sl, gam);
      cart_flux_n(wr, nx, ny, gm1, fr, &sr, gam);
      lam = sl >= sr ? sl : sr;
    } else {
      sl = sr = lam = T(0);
    }
  }
  // The reverse reads the node values and coefficient rows again (cache hits)
  // and recomputes the Roe state where it needs them, instead of holding
  // them in registers through the forward pass: the compiler barriers keep
  // it from reusing the forward's copies.
  asm volatile("" ::: "memory");
  T u, v, H, cc, L[4][4], R[4][4];
  {
    T A[4], B[4], sa, sb, D, pa, pb;
    roe(A, B, sa, sb, D, pa, pb, u, v, H, cc);
  }
  eig(u, v, H, cc, L, R);
  const T q2 = u * u + v * v;
  const T un = u * nx + v * ny;
  const T ic = frcp(cc), b1 = gm1 * ic * ic, b2 = T(0.5) * b1 * q2;

  // ---- reverse: Riemann flux -> this side's state ------------------------------------
  T gw[4];
  if constexpr (FLUX == HFD_FLUX_RUSANOV) {
    T glam = T(0.0);
    for (int q = 0; q < 4; ++q) {
      glam -= T(0.5) * gh[q] * (wr[q] - wl[q]);
      gw[q] = (s == 0 ? T(0.5) : -T(0.5)) * lam * gh[q];
    }
    const T half[4] = {T(0.5) * gh[0], T(0.5) * gh[1], T(0.5) * gh[2], T(0.5) * gh[3]};
    flux_jac_t(wm, nx, ny, gm1, half, gw);
    if ((sl >= sr ? 0 : 1) == s) {
      T ds[4];
      speed_grad(wm, nx, ny, gam, ds);
      for (int k = 0; k < 4; ++k) gw[k] += glam * ds[k];
    }
  } else {
    // gw[k] = gh . dh/d(w_side)[k]: the flux on dual numbers seeded with
    // direction k of this lane's state (full states, zero reference)
    GasParams gz = gp;
    for (int q = 0; q < 4; ++q) gz.wref[q] = gz.f_wref[q] = 0.0;
    gz.uref = gz.vref = gz.etr_ref = 0.0;
    gz.f_uref = gz.f_vref = gz.f_etr_ref = 0.0f;
    const Ref<Dual<T>> rz = make_ref<Dual<T>>(gz);
    for (int k = 0; k < 4; ++k) {
      Dual<T> Ld[4], Rd[4], hd[4];
      for (int q = 0; q < 4; ++q) {
        Ld[q] = Dual<T>(wl[q], s == 0 && q == k ? T(1) : T(0));
        Rd[q] = Dual<T>(wr[q], s == 1 && q == k ? T(1) : T(0));
      }
      if constexpr (FLUX == HFD_FLUX_ROE)
        roe_flux<Dual<T>>(Ld, Rd, Dual<T>(nx), Dual<T>(ny), rz, Dual<T>(gm1), hd);
      else
        hllc_flux<Dual<T>>(Ld, Rd, Dual<T>(nx), Dual<T>(ny), rz, Dual<T>(gam), Dual<T>(gm1), hd);
      gw[k] = gh[0] * hd[0].d + gh[1] * hd[1].d + gh[2] * hd[2].d + gh[3] * hd[3].d;
    }
  }
  // ---- reverse: this side's reconstruction ----------------------------------------------
  // Gradients of R and L are folded into those of the Roe state (u, v, H, c)
  // as they arise (this side's part; the pair's parts are summed below).
  const T ic2 = ic * ic;
  T gu = 0, gv = 0, gH = 0, gc = 0;
  auto foldL = [&](int q, const T z[4]) {  // z = gradient of row q of L
    if (q == 0) {
      gu += z[0] * T(0.5) * (b1 * u + nx * ic) + z[1] * (-T(0.5) * b1);
      gv += z[0] * T(0.5) * (b1 * v + ny * ic) + z[2] * (-T(0.5) * b1);
      gc += z[0] * T(0.5) * (-T(2.0) * b2 * ic - un * ic2) + z[1] * T(0.5) * (T(2.0) * b1 * u * ic + nx * ic2) +
            z[2] * T(0.5) * (T(2.0) * b1 * v * ic + ny * ic2) + z[3] * (-b1 * ic);
    } else if (q == 1) {
      gu += z[0] * (-b1 * u) + z[1] * b1;
      gv += z[0] * (-b1 * v) + z[2] * b1;
      gc += z[0] * (T(2.0) * b2 * ic) + z[1] * (-T(2.0) * b1 * u * ic) + z[2] * (-T(2.0) * b1 * v * ic) +
            z[3] * (T(2.0) * b1 * ic);
    } else if (q == 2) {
      gu += z[0] * T(0.5) * (b1 * u - nx * ic) + z[1] * (-T(0.5) * b1);
      gv += z[0] * T(0.5) * (b1 * v - ny * ic) + z[2] * (-T(0.5) * b1);
      gc += z[0] * T(0.5) * (-T(2.0) * b2 * ic + un * ic2) + z[1] * T(0.5) * (T(2.0) * b1 * u * ic - nx * ic2) +
            z[2] * T(0.5) * (T(2.0) * b1 * v * ic - ny * ic2) + z[3] * (-b1 * ic);
    } else {
      gu += z[0] * ny;
      gv += z[0] * (-nx);
    }
  };
  {
    T gR[4][4];
    for (int r = 0; r < 4; ++r)
      for (int q = 0; q < 4; ++q) gR[r][q] = gw[r] * C[q];
    gu += gR[1][0] + gR[1][1] + gR[1][2] + gR[3][0] * (-nx * cc) + gR[3][1] * u +
          gR[3][2] * (nx * cc) + gR[3][3] * (-ny);
    gv += gR[2][0] + gR[2][1] + gR[2][2] + gR[3][0] * (-ny * cc) + gR[3][1] * v +
          gR[3][2] * (ny * cc) + gR[3][3] * nx;
    gH += gR[3][0] + gR[3][2];
    gc += gR[1][0] * (-nx) + gR[1][2] * nx + gR[2][0] * (-ny) + gR[2][2] * ny +
          gR[3][0] * (-un) + gR[3][2] * un;
  }
  T gC[4];
  for (int q = 0; q < 4; ++q)
    gC[q] = R[0][q] * gw[0] + R[1][q] * gw[1] + R[2][q] * gw[2] + R[3][q] * gw[3];
  T W[5][4], w3[9];
  load_W(W);
  load_w3(w3);
  T gW[5][4] = {}, ghs[4] = {0, 0, 0, 0};
  for (int q = 0; q < 4; ++q) {
    const T gCq = gC[q];
    T z[4];
    if (!weno[q]) {
      // C_q = L_q . hs
      for (int k = 0; k < 4; ++k) {
        z[k] = gCq * hs[k];
        ghs[k] += gCq * L[q][k];
      }
      foldL(q, z);
      continue;
    }
    T cq[5], be[3], om[3], Sk[3];
    proj(L, W, q, cq);
    weno_parts(w3, cq, be, om, Sk);
    T gcv[5] = {0, 0, 0, 0, 0}, gS[3], gom[3];
    for (int k = 0; k < 3; ++k) {
      gS[k] = gCq * om[k];
      gom[k] = gCq * Sk[k];
    }
    for (int k = 0; k < 3; ++k)
      for (int t = 0; t < 3; ++t) gcv[k + t] += gS[k] * w3[3 * k + t];
    // omega = alpha / sum(alpha), alpha = d / (eps + beta)^2: d omega_j /
    // d alpha_k = (delta_jk - omega_j) / sum(alpha) and d alpha_k / d beta_k
    // = -2 alpha_k / (eps + beta_k), so with alpha_k / sum(alpha) = omega_k
    // the adjoint of beta_k is -2 (g_k - sum_j g_j omega_j) omega_k / (eps + beta_k)
    T dot = T(0.0);
    for (int k = 0; k < 3; ++k) dot += gom[k] * om[k];
    T gbe[3];
    for (int k = 0; k < 3; ++k) gbe[k] = -T(2.0) * (gom[k] - dot) * om[k] * frcp(eps + be[k]);
    const T t1 = cq[0] - 2 * cq[1] + cq[2], t2 = cq[0] - 4 * cq[1] + 3 * cq[2];
    const T t3 = cq[1] - 2 * cq[2] + cq[3], t4 = cq[1] - cq[3];
    const T t5 = cq[2] - 2 * cq[3] + cq[4], t6 = 3 * cq[2] - 4 * cq[3] + cq[4];
    const T gt1 = gbe[0] * (T(13.0) / T(6.0)) * t1, gt2 = gbe[0] * T(0.5) * t2;
    const T gt3 = gbe[1] * (T(13.0) / T(6.0)) * t3, gt4 = gbe[1] * T(0.5) * t4;
    const T gt5 = gbe[2] * (T(13.0) / T(6.0)) * t5, gt6 = gbe[2] * T(0.5) * t6;
    gcv[0] += gt1 + gt2;
    gcv[1] += -T(2.0) * gt1 - T(4.0) * gt2 + gt3 + gt4;
    gcv[2] += gt1 + T(3.0) * gt2 - T(2.0) * gt3 + gt5 + T(3.0) * gt6;
    gcv[3] += gt3 - gt4 - T(2.0) * gt5 - T(4.0) * gt6;
    gcv[4] += gt5 + gt6;
    // cv[q][t] = L[q] . W_t
    for (int k = 0; k < 4; ++k) z[k] = T(0.0);
    for (int t = 0; t < 5; ++t)
      for (int k = 0; k < 4; ++k) {
        z[k] += gcv[t] * W[t][k];
        gW[t][k] += gcv[t] * L[q][k];
      }
    foldL(q, z);
  }
  // hs = sum_t w5 . data: the value part here, the gradient parts at output
  asm volatile("" ::: "memory");
  T w5[5][3];
  if constexpr (HERM) {
    load_w5(w5);
    for (int t = 0; t < 5; ++t)
      for (int k = 0; k < 4; ++k) gW[t][k] += w5[t][0] * ghs[k];
  }
  // sum over the pair in a fixed order (left part + right part)
  {
    const T ou = dpp_mov<0xB1>(gu), ov = dpp_mov<0xB1>(gv), oH = dpp_mov<0xB1>(gH),
                 oc = dpp_mov<0xB1>(gc);
    gu = s == 0 ? gu + ou : ou + gu;
    gv = s == 0 ? gv + ov : ov + gv;
    gH = s == 0 ? gH + oH : oH + gH;
    gc = s == 0 ? gc + oc : oc + gc;
  }
  // c = sqrt(gm1 (H - q2/2))
  {
    const T hc = gc * gm1 * T(0.5) * ic;
    gH += hc;
    gu -= hc * u;
    gv -= hc * v;
  }
  // ---- Roe average -> this lane's end state (node 2 or 3, position 2) ---------------
  {
    T A[4], B[4], sa, sb, D, pa, pb, u_, v_, H_, cc_;
    roe(A, B, sa, sb, D, pa, pb, u_, v_, H_, cc_);
    const T iD = frcp(D);
    const T gP = gu * iD, gQ = gv * iD, gK = gH * iD;
    const T gD = -(gu * u + gv * v + gH * H) * iD;
    const T* S = s == 0 ? A : B;
    T* g = gW[2];
    const T r = S[0], s_ = s == 0 ? sa : sb, p = s == 0 ? pa : pb;
    // 1/r, and 1/s = s/r (s = sqrt(r))
    const T ir = frcp(r), is = s_ * ir;
    T gs = gD;
    // P = m/s, Q = n/s, K = (E + p)/s
    g[1] += gP * is;
    g[2] += gQ * is;
    gs += -(gP * S[1] + gQ * S[2] + gK * (S[3] + p)) * is * is;
    const T gE = gK * is, gp_ = gK * is;
    g[3] += gE;
    // p = gm1 (E - (m^2 + n^2) / (2 r))
    g[3] += gm1 * gp_;
    g[1] += -gm1 * gp_ * S[1] * ir;
    g[2] += -gm1 * gp_ * S[2] * ir;
    g[0] += gm1 * gp_ * T(0.5) * (S[1] * S[1] + S[2] * S[2]) * ir * ir;
    // s = sqrt(r)
    g[0] += gs * T(0.5) * is;
  }
  // ---- shared nodes: position p (1, 2) of one lane is position 5 - p of the
  // other; each lane adds the partner's contribution to its positions 1, T(2.)
  // The gradient parts are w5[t][1] ghs and w5[t][2] ghs.
  T pghs[4], pw5[3][2];
  if constexpr (HERM) {
    for (int k = 0; k < 4; ++k) pghs[k] = dpp_mov<0xB1>(ghs[k]);
  }
  for (int p = 1; p <= 2; ++p) {
    if constexpr (HERM) {
      pw5[p][0] = dpp_mov<0xB1>(w5[5 - p][1]);
      pw5[p][1] = dpp_mov<0xB1>(w5[5 - p][2]);
    }
    for (int k = 0; k < 4; ++k) gW[p][k] += dpp_mov<0xB1>(gW[5 - p][k]);
  }
  // The block's rows (6 NW values per edge) go through LDS and out as one
  // contiguous run: stored directly, the lanes' rows lie 6 NW values apart
  // and every store instruction would touch 64 cache lines.
  T* o = obuf + (threadIdx.x / 2) * RW;
  for (int p = 0; p < 3; ++p) {
    const int j = s == 0 ? p : 5 - p;
    for (int k = 0; k < 4; ++k) {
      o[NW * j + k] = gW[p][k];
      if constexpr (HERM) {
        T gx = w5[p][1] * ghs[k], gy = w5[p][2] * ghs[k];
        if (p > 0) {
          gx += pw5[p][0] * pghs[k];
          gy += pw5[p][1] * pghs[k];
        }
        o[NW * j + 4 + k] = gx;
        o[NW * j + 8 + k] = gy;
      }
    }
  }
  __syncthreads();
  {
    const int64_t ce = ne - eb < kAdjEdgesPerBlock ? ne - eb : kAdjEdgesPerBlock;
    // (6 NW values per edge: whole 16-byte units)
    const int nvec = int(ce * RW * int64_t(sizeof(T)) / 16);
    const uint4* src = reinterpret_cast<const uint4*>(obuf);
    uint4* dst = reinterpret_cast<uint4*>(out + eb * RW);
    for (int i = threadIdx.x; i < nvec; i += blockDim.x) dst[i] = src[i];
  }
}

// ---------------------------------------------------------------------------
// lambda_U(u) for owned u
// ---------------------------------------------------------------------------
// 16 lanes per vertex, 16 vertices per block.  Lanes stride over (1) the
// (edge, position) entries of u, summing the 12 edge-pass contributions, and
// (2) the (v, s) entries with u in S(v), summing lambda_f and lambda_g from
// the transposed rows dv_t (contiguous per u), two entries per lane and
// batch.  With viscosity the same entries also sum Lambda_fv and Lambda_gv,
// the adjoints of the viscous fluxes at u, from the transposed viscous rows
// dvis_t.  A transposed DPP reduction leaves the 20 (28) sums in LDS; one
// lane per vertex applies the flux Jacobians, one thread per (vertex, input
// component) the viscous flux derivative (a dual-number evaluation of the
// viscous flux seeded at that component), and the 12 output rows are
// written in 16-wide runs.
template <class T, bool VISC, int NW>
__global__ void __launch_bounds__(256)
k_adj_vertex(int64_t nowned, int64_t nv, GasParams gp, const double* __restrict__ U,
             const int32_t* __restrict__ vtp, const int32_t* __restrict__ vtv,
             const T* __restrict__ dv_t, const T* __restrict__ dvis_t,
             const int32_t* __restrict__ ntp, const int32_t* __restrict__ nte,
             const int8_t* __restrict__ ntj, const T* __restrict__ bnode,
             const V4<T>* __restrict__ Lv, const V4<T>* __restrict__ Lg,
             double* __restrict__ out, AdjCombine<T> rc) {
  constexpr int VPB = 16, NS = VISC ? 28 : 20;
  __shared__ T sres[VPB][NS + 1];
  const int t = threadIdx.x, vl = t / 16, sub = t & 15;
  const int64_t u0 = int64_t(blockIdx.x) * VPB, u = u0 + vl;
  T acc[32];
  for (int k = 0; k < 32; ++k) acc[k] = T(0.0);
  if (u < nowned) {
    // (1) edge-pass contributions; every owned vertex is a stencil node of
    // some edge and lies in its own S(u), so k1 - 1 is an entry in both loops
    {
      const int k0 = ntp[u], k1 = ntp[u + 1];
      for (int b = k0 + sub; b < k1; b += 32) {
        int kk[2];
        bool ok[2];
        for (int i = 0; i < 2; ++i) {
          ok[i] = b + 16 * i < k1;
          kk[i] = ok[i] ? b + 16 * i : k1 - 1;
        }
        const T* src[2];
        for (int i = 0; i < 2; ++i)
          src[i] = bnode + int64_t(nte[kk[i]]) * (6 * NW) + NW * ntj[kk[i]];
        T x[2][NW];
        for (int i = 0; i < 2; ++i)
          for (int q = 0; q < NW; ++q) x[i][q] = src[i][q];
        for (int i = 0; i < 2; ++i)
          for (int q = 0; q < NW; ++q) acc[q] += ok[i] ? x[i][q] : T(0.0);
      }
    }
    // (2) lambda_f (12..15), lambda_g (16..19)
    {
      const int k0 = vtp[u], k1 = vtp[u + 1];
      for (int b = k0 + sub; b < k1; b += 32) {
        int kk[2];
        bool ok[2];
        for (int i = 0; i < 2; ++i) {
          ok[i] = b + 16 * i < k1;
          kk[i] = ok[i] ? b + 16 * i : k1 - 1;
        }
        int v[2];
        T d[2][6];
        for (int i = 0; i < 2; ++i) {
          v[i] = vtv[kk[i]];
          for (int q = 0; q < 6; ++q) d[i][q] = dv_t[6 * int64_t(kk[i]) + q];
        }
        T kv[2][5];
        if (VISC)
          for (int i = 0; i < 2; ++i)
            for (int q = 0; q < 5; ++q) kv[i][q] = dvis_t[5 * int64_t(kk[i]) + q];
        V4<T> l0[2], lx[2], ly[2];
        for (int i = 0; i < 2; ++i) {
          l0[i] = Lv[v[i]];
          lx[i] = Lg[2 * int64_t(v[i])];
          ly[i] = Lg[2 * int64_t(v[i]) + 1];
        }
        for (int i = 0; i < 2; ++i) {
          T dd[6];
          for (int q = 0; q < 6; ++q) dd[q] = ok[i] ? d[i][q] : T(0.0);
          const T a0[4] = {l0[i].x, l0[i].y, l0[i].z, l0[i].w};
          const T ax[4] = {lx[i].x, lx[i].y, lx[i].z, lx[i].w};
          const T ay[4] = {ly[i].x, ly[i].y, ly[i].z, ly[i].w};
          for (int q = 0; q < 4; ++q) {
            acc[12 + q] -= dd[0] * a0[q] + dd[2] * ax[q] + dd[4] * ay[q];
            acc[16 + q] -= dd[1] * a0[q] + dd[3] * ax[q] + dd[5] * ay[q];
          }
          if (VISC) {
            // the forward adds k0 fv + k1 gv, k2 fv + k3 gv, k3 fv + k4 gv
            T k[5];
            for (int q = 0; q < 5; ++q) k[q] = ok[i] ? kv[i][q] : T(0.0);
            for (int q = 0; q < 4; ++q) {
              acc[20 + q] += k[0] * a0[q] + k[2] * ax[q] + k[3] * ay[q];
              acc[24 + q] += k[1] * a0[q] + k[3] * ax[q] + k[4] * ay[q];
            }
          }
        }
      }
    }
  }
  reduce_stage<3, 32>(acc, sub);
  reduce_stage<2, 16>(acc, sub);
  reduce_stage<1, 8>(acc, sub);
  reduce_stage<0, 4>(acc, sub);
  // lane sub holds sums 2 sub and 2 sub + 1
  for (int i = 0; i < 2; ++i)
    if (2 * sub + i < NS) sres[vl][2 * sub + i] = acc[i];
  __syncthreads();
  if (t < VPB && u0 + t < nowned) {
    // A_f^T lambda_f + A_g^T lambda_g at w_u (n = (1, 0) and (0, 1))
    const int64_t uu = u0 + t;
    const T gm1 = gpar<T>(gp.gamma - 1.0, gp.f_gm1);
    T w[4], lf[4], lg[4], o[4] = {0, 0, 0, 0};
    for (int q = 0; q < 4; ++q) {
      w[q] = T(U[q * nv + uu]);
      lf[q] = sres[t][12 + q];
      lg[q] = sres[t][16 + q];
    }
    flux_jac_t(w, T(1.0), T(0.0), gm1, lf, o);
    flux_jac_t(w, T(0.0), T(1.0), gm1, lg, o);
    for (int q = 0; q < 4; ++q) sres[t][q] += o[q];
  }
  __syncthreads();
  if (t < 12 * VPB) {
    const int q = t / VPB, vl2 = t % VPB;
    const int64_t uu = u0 + vl2;
    if (uu < nowned) {
      const int64_t o = q * nv + uu;
      T xs = sres[vl2][q];
      if (VISC) {
        // sum_r Lambda_fv[r] dfv_r/dx_q + Lambda_gv[r] dgv_r/dx_q, x = (w, w_x, w_y)
        using D = Dual<T>;
        D x3[12];
        for (int r = 0; r < 12; ++r) x3[r] = D(T(U[r * nv + uu]), r == q ? T(1) : T(0));
        D fv[4], gv[4];
        viscous_flux<D>(x3, x3 + 4, x3 + 8, gp, fv, gv);
        for (int r = 0; r < 4; ++r) xs += sres[vl2][20 + r] * fv[r].d + sres[vl2][24 + r] * gv[r].d;
      }
      const double x = double(xs);
      if (out) out[o] = x;
      if (rc.lam_k) {
        const double lk = rc.lam_k[o];
        if (rc.nxt) {
          const double n = rc.ca * lk + rc.cb * x;
          rc.nxt[o] = n;
          if (q < 4) reinterpret_cast<T*>(rc.nGv)[4 * uu + q] = T(n);
          else reinterpret_cast<T*>(rc.nGg)[8 * uu + (q - 4)] = T(n);
        }
        double a = rc.cd * lk + rc.ce * x;
        if (rc.cc != 0.0) a += rc.cc * rc.acc[o];
        rc.acc[o] = a;
      }
    }
  }
}

// dst[i][0..w) = src[idx[i]][0..w), i < n
__global__ void k_take_rows(int64_t n, int w, const int32_t* __restrict__ idx,
                            const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n * w) return;
  const int64_t r = i / w, q = i % w;
  dst[i] = src[int64_t(idx[r]) * w + q];
}

// The three stage states of a Runge-Kutta step (U, U1, U2, float64 [12][nv])
// in gather layout, in one pass: the same conversion as the forward passes
// (minus the reference state in the mixed form).  The Dirichlet rows
// [d0, d1) of the two stages take U's values, as in the forward step.
template <class T>
__global__ void k_stage_gathers(int64_t nv, int64_t d0, int64_t d1, const double* __restrict__ U,
                                const double* __restrict__ U1, const double* __restrict__ U2,
                                GasParams gp, StageGathers<T> g) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  const bool dir = i >= d0 && i < d1;
  const double* src[3] = {U, dir ? U : U1, dir ? U : U2};
  for (int k = 0; k < 3; ++k) {
    T w[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) w[q] = T(src[k][q * nv + i] - (q < 4 ? gp.wref[q] : 0.0));
    g.v[k][i] = V4<T>{w[0], w[1], w[2], w[3]};
    g.g[k][2 * i] = V4<T>{w[4], w[5], w[6], w[7]};
    g.g[k][2 * i + 1] = V4<T>{w[8], w[9], w[10], w[11]};
  }
}

template <class T>
hipError_t launch_stage_gathers(int64_t nv, int64_t d0, int64_t d1, const double* U,
                                const double* U1, const double* U2, const GasParams& gp,
                                const StageGathers<T>& g, hipStream_t st) {
  if (nv == 0) return hipSuccess;
  hipLaunchKernelGGL(k_stage_gathers<T>, dim3(unsigned((nv + 255) / 256)), dim3(256), 0, st, nv,
                     d0, d1, U, U1, U2, gp, g);
  return hipGetLastError();
}
template hipError_t launch_stage_gathers<double>(int64_t, int64_t, int64_t, const double*,
                                                 const double*, const double*, const GasParams&,
                                                 const StageGathers<double>&, hipStream_t);
template hipError_t launch_stage_gathers<float>(int64_t, int64_t, int64_t, const double*,
                                                const double*, const double*, const GasParams&,
                                                const StageGathers<float>&, hipStream_t);

template <class T, int FLUX>
hipError_t launch_adj_edge(const AdjointArgs<T>& a, hipStream_t st) {
  const dim3 grid(unsigned((a.ne + kAdjEdgesPerBlock - 1) / kAdjEdgesPerBlock));
  const int swm = a.force ? kSwForced : a.gp.sw;
  if (swm == kSwForced)
    hipLaunchKernelGGL((k_adj_edge<T, FLUX, kSwForced>), grid, dim3(256), 0, st, a.ne, a.ec,
                       a.gp, a.Gv, a.Gg, a.force, a.etp, a.etv, a.de_t, a.Lv, a.Lg, a.lrp, a.lrow, a.lpos, a.bnode);
  else if (swm == HFD_SWITCH_PAPER)
    hipLaunchKernelGGL((k_adj_edge<T, FLUX, HFD_SWITCH_PAPER>), grid, dim3(256), 0, st, a.ne,
                       a.ec, a.gp, a.Gv, a.Gg, a.force, a.etp, a.etv, a.de_t, a.Lv, a.Lg, a.lrp, a.lrow, a.lpos, a.bnode);
  else if (swm == HFD_SWITCH_SMOOTH_ONLY)
    hipLaunchKernelGGL((k_adj_edge<T, FLUX, HFD_SWITCH_SMOOTH_ONLY>), grid, dim3(256), 0, st,
                       a.ne, a.ec, a.gp, a.Gv, a.Gg, a.force, a.etp, a.etv, a.de_t, a.Lv, a.Lg,
                       a.lrp, a.lrow, a.lpos, a.bnode);
  else if (swm == HFD_SWITCH_WENO_ONLY)
    hipLaunchKernelGGL((k_adj_edge<T, FLUX, HFD_SWITCH_WENO_ONLY>), grid, dim3(256), 0, st,
                       a.ne, a.ec, a.gp, a.Gv, a.Gg, a.force, a.etp, a.etv, a.de_t, a.Lv, a.Lg,
                       a.lrp, a.lrow, a.lpos, a.bnode);
  else
    return hipErrorInvalidValue;
  return hipSuccess;
}

template <class T>
hipError_t launch_adjoint_residual(const AdjointArgs<T>& a, hipStream_t st) {
  if (a.ne > 0) {
    hipError_t err;
    if (a.gp.flux == HFD_FLUX_ROE) err = launch_adj_edge<T, HFD_FLUX_ROE>(a, st);
    else if (a.gp.flux == HFD_FLUX_HLLC) err = launch_adj_edge<T, HFD_FLUX_HLLC>(a, st);
    else err = launch_adj_edge<T, HFD_FLUX_RUSANOV>(a, st);
    if (err != hipSuccess) return err;
  }
  if (a.nowned > 0) {
    const dim3 grid(unsigned((a.nowned + 15) / 16));
    // the edge reverse's row layout follows its switch mode
    const bool compact = !a.force && a.gp.sw == HFD_SWITCH_WENO_ONLY;
    constexpr int NC = kAdjNodeValues<HFD_SWITCH_WENO_ONLY>, NF = kAdjNodeValues<kSwForced>;
    if (a.dvis_t && compact)
      hipLaunchKernelGGL((k_adj_vertex<T, true, NC>), grid, dim3(256), 0, st, a.nowned, a.nv,
                         a.gp, a.U, a.vtp, a.vtv, a.dv_t, a.dvis_t, a.ntp, a.nte, a.ntj, a.bnode,
                         a.Lv, a.Lg, a.out, a.rc);
    else if (a.dvis_t)
      hipLaunchKernelGGL((k_adj_vertex<T, true, NF>), grid, dim3(256), 0, st, a.nowned, a.nv,
                         a.gp, a.U, a.vtp, a.vtv, a.dv_t, a.dvis_t, a.ntp, a.nte, a.ntj, a.bnode,
                         a.Lv, a.Lg, a.out, a.rc);
    else if (compact)
      hipLaunchKernelGGL((k_adj_vertex<T, false, NC>), grid, dim3(256), 0, st, a.nowned, a.nv,
                         a.gp, a.U, a.vtp, a.vtv, a.dv_t, a.dvis_t, a.ntp, a.nte, a.ntj, a.bnode,
                         a.Lv, a.Lg, a.out, a.rc);
    else
      hipLaunchKernelGGL((k_adj_vertex<T, false, NF>), grid, dim3(256), 0, st, a.nowned, a.nv,
                         a.gp, a.U, a.vtp, a.vtv, a.dv_t, a.dvis_t, a.ntp, a.nte, a.ntj, a.bnode,
                         a.Lv, a.Lg, a.out, a.rc);
  }
  return hipGetLastError();
}
template hipError_t launch_adjoint_residual<double>(const AdjointArgs<double>&, hipStream_t);
template hipError_t launch_adjoint_residual<float>(const AdjointArgs<float>&, hipStream_t);

hipError_t launch_take_rows(int64_t n, int w, const int32_t* idx, const double* src,
                            double* dst, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_take_rows, dim3(unsigned((n * w + 255) / 256)), dim3(256), 0, st, n, w,
                     idx, src, dst);
  return hipGetLastError();
}

}  // namespace hfd
