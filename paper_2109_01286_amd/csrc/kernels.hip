// Hot-path kernels of the Hermite finite-difference method (gfx950).
//
// Edge pass (Section 2.2 / 2.3, Algorithm 1, eq. 2d_hweno_intp): two lanes per
// active edge (one per side, sharing the six stencil nodes; a one-lane kernel
// for float32 is kept as an alternative).  Roe average of the edge's end states, characteristic
// projection of values and gradients at the six stencil nodes, per side and
// characteristic component the WENO5 smoothness indicators and the switch,
// the 5-node Hermite value (15-term dot product with the stored row) or the
// omega-weighted 3-node values, back-projection, Riemann flux along the edge.
// Each edge kernel is compiled once per switch mode (the paper's switch,
// Hermite everywhere, WENO everywhere, a forced mask): no run-time branches
// on the mode, and no work that the mode does not need.
//
// Vertex pass (eq. flux_polynomials and the rows d0, dx, dy; viscous
// vertex-only rows; three-stage TVD Runge-Kutta): a block of 16 owned
// vertices first copies its distinct state rows and edge fluxes into LDS;
// then 16 lanes per vertex stride over the vertex slots (analytic fluxes
// recomputed from the staged state, dotted with the coefficient record of
// the slot) and the edge slots (staged edge flux), all loads of a batch in
// flight together; a transposed DPP reduction gives the twelve right-hand
// sides, staged in LDS so that the float64 Runge-Kutta update is written
// row by row.  No atomics: every output has exactly one writer.
//
// Two precisions share the code: float64 throughout, or float32 arithmetic
// on a float32 perturbation state w' = w - w_ref (gradients unchanged) with
// fluxes in perturbation form F(w) - F(w_ref), written so that nothing large
// cancels, and float64 accumulation of the Runge-Kutta state.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "gas.h"

// Tuning parameters (compile-time).
#ifndef HFD_VERTEX_LANES32
#define HFD_VERTEX_LANES32 16 // lanes per vertex in the float32 vertex pass
#endif
#ifndef HFD_VERTEX_LANES64
#define HFD_VERTEX_LANES64 16 // lanes per vertex in the float64 vertex pass
#endif
#ifndef HFD_VERTEX_WAVES
#define HFD_VERTEX_WAVES 7    // waves per SIMD of the float32 vertex kernel (Euler)
#endif
#ifndef HFD_EDGE_WAVES
#define HFD_EDGE_WAVES 2      // waves per SIMD of the one-lane (float32) edge kernel
#endif
#ifndef HFD_EDGE2_WAVES64
#define HFD_EDGE2_WAVES64 2   // waves per SIMD of the two-lane edge kernel, float64
#endif
#ifndef HFD_EDGE2_WAVES32
#define HFD_EDGE2_WAVES32 5   // the same in float32 (80 VGPRs: 6 fit)
#endif
#ifndef HFD_EDGE32_TWO_LANES
#define HFD_EDGE32_TWO_LANES 1 // 0: the float32 edge pass uses the one-lane kernel
#endif
// vertex and edge slots per lane and batch of the vertex pass (16 lanes per
// vertex), per precision
#ifndef HFD_VERTEX_NVS32
#define HFD_VERTEX_NVS32 2
#endif
#ifndef HFD_VERTEX_NES32
#define HFD_VERTEX_NES32 4
#endif
#ifndef HFD_VERTEX_NVS32V
#define HFD_VERTEX_NVS32V 1   // (float32 with the viscous rows)
#endif
#ifndef HFD_VERTEX_NES32V
#define HFD_VERTEX_NES32V 4
#endif
#ifndef HFD_VERTEX_NVS64
#define HFD_VERTEX_NVS64 1
#endif
#ifndef HFD_VERTEX_NES64
#define HFD_VERTEX_NES64 3
#endif
#ifndef HFD_EDGE1_STAGE
#define HFD_EDGE1_STAGE 1     // 1: the one-lane edge kernel stages its stencil rows in LDS
#endif
#ifndef HFD_XCD_REMAP
#define HFD_XCD_REMAP 1       // 1: contiguous block ranges per XCD
#endif

namespace hfd {
namespace {

// base[uoff] plus a per-lane byte offset, with the wave-uniform element
// offset pinned in scalar registers: the load then takes a scalar base and
// one 32-bit vector register for its address.
template <class P>
__device__ inline const P* at(const P* base, int64_t uoff, uint32_t byte_off) {
  const uint64_t u = uint64_t(uoff) * sizeof(P);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(u));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(u >> 32));
  const char* b = reinterpret_cast<const char*>(base) + (uint64_t(lo) | (uint64_t(hi) << 32));
  return reinterpret_cast<const P*>(b + byte_off);
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
// Switch of one characteristic component q of side s from the smoothness
// indicators be of its five projected node values: true for the
// omega-weighted 3-node values, false for the 5-node Hermite value.  SWM is
// the switch mode (hfd_switch) or kSwForced (the bits fm of a forced mask),
// fixed at compile time so that the edge kernels carry no branches on it.
template <class T, int SWM>
__device__ inline bool comp_switch(const T be[3], const GasParams& gp, int s, int q,
                                   uint8_t fm) {
  if constexpr (SWM == kSwForced) return (fm >> (4 * s + q)) & 1;
  else if constexpr (SWM == HFD_SWITCH_PAPER)
    return !weno_in<T>(be, gpar<T>(gp.eps, gp.f_eps), gpar<T>(gp.sw_lo, gp.f_sw_lo),
                      gpar<T>(gp.sw_hi, gp.f_sw_hi));
  else return SWM == HFD_SWITCH_WENO_ONLY;
}

// Interface value of one characteristic component: the omega-weighted 3-node
// values (w3: the side's three 3-node rows) or the Hermite value hq (the
// component of L hs, hs the side's 5-node Hermite sum in physical variables;
// the row is the same for all components).
template <class T>
__device__ inline T comp_value(bool weno, const T c[5], const T o[3], const T w3[9], T hq) {
  if (weno)
    return o[0] * (w3[0] * c[0] + w3[1] * c[1] + w3[2] * c[2]) +
           o[1] * (w3[3] * c[1] + w3[4] * c[2] + w3[5] * c[3]) +
           o[2] * (w3[6] * c[2] + w3[7] * c[3] + w3[8] * c[4]);
  return hq;
}

// One side's decisions (bits 4 s + q) from its indicators.
template <class T, int SWM>
__device__ inline uint8_t side_decide(const T be[4][3], const GasParams& gp, int s, uint8_t fm) {
  uint8_t bits = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    bits |= uint8_t(comp_switch<T, SWM>(be[q], gp, s, q, fm) ? 1 : 0) << (4 * s + q);
  return bits;
}

// The side's interface state (back-projected).  Only when some component of
// the side takes the 3-node branch are the side's 3-node rows read and its
// WENO weights formed; otherwise every component is the Hermite value.
template <class T, class RowFn>
__device__ inline void side_state(uint8_t b, int s, const T be[4][3], const T cv[4][5],
                                  const T hs[4], const RoeState<T>& F, const GasParams& gp,
                                  RowFn w3row, T out[4]) {
  T C[4];
  F.proj(hs, C);
  if (b) {
    T w3[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) w3[j] = w3row(j);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T o[3];
      weno_omega<T>(be[q], gpar<T>(gp.eps, gp.f_eps), o);
      C[q] = comp_value<T>((b >> (4 * s + q)) & 1, cv[q], o, w3, C[q]);
    }
  }
  F.back(C, out);
}

template <class T>
__device__ inline void store_edge(int64_t ne, int64_t e, const T h[4], const T wl[4],
                                  const T wr[4], uint8_t bits, const GasParams& gp,
                                  V4<T>* H, double* hsoa, double* wlr, uint8_t* mask,
                                  bool left, bool right) {
  if (left) {
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
      if (left) wlr[q * ne + e] = double(wl[q]) + gp.wref[q];
      if (right) wlr[(4 + q) * ne + e] = double(wr[q]) + gp.wref[q];
    }
  }
}

// Dynamic LDS of the staging kernels (the edge pass's stencil rows, the
// vertex pass's state rows and edge fluxes).
extern __shared__ __attribute__((aligned(32))) unsigned char hfd_stage_lds[];

// Waves per SIMD each edge kernel is compiled for (register budget 512/waves).
template <class T> struct EdgeWaves { static constexpr int value = 2; };
template <> struct EdgeWaves<float> { static constexpr int value = HFD_EDGE_WAVES; };
template <class T> struct Edge2Waves { static constexpr int value = HFD_EDGE2_WAVES64; };
template <> struct Edge2Waves<float> { static constexpr int value = HFD_EDGE2_WAVES32; };

// One lane per edge.  The six stencil nodes are gathered and projected once
// and serve both sides: the left state interpolates from nodes 0..4
// (i-2 .. i+2), the right state from nodes 5..1 (i+3 .. i-1).  All loads of
// an edge are issued before its arithmetic.
// STG: blocks of kEdgeStageEdges edges first copy their distinct stencil
// rows to LDS, and the lanes read their nodes there by 2-byte position.
template <class T, int SWM, bool STG>
__global__ void __launch_bounds__(256, EdgeWaves<T>::value)
k_edge1(int64_t ne, EdgeCoef<T> c, GasParams gp, const V4<T>* __restrict__ Gv,
        const V4<T>* __restrict__ Gg, const uint8_t* __restrict__ force,
        V4<T>* __restrict__ H, double* __restrict__ hsoa, double* __restrict__ wlr,
        uint8_t* __restrict__ mask) {
  const int64_t e0 = xcd_block() * blockDim.x;
  int64_t e = e0 + threadIdx.x;
  if constexpr (!STG) {
    if (e >= ne) return;
  } else {
    if (e >= ne) e = ne - 1;  // (reaches the staging barrier, stores nothing)
  }
  const Ref<T> ref = make_ref<T>(gp);
  const T gam = gpar<T>(gp.gamma, gp.f_gamma), gm1 = gpar<T>(gp.gamma - 1.0, gp.f_gm1);
  // Row r of a [rows][ne] index array at this edge: the row base of the
  // block is uniform, the lane adds a 32-bit byte offset (one register for
  // all rows).
  const uint32_t li = uint32_t(e - e0) * 4u;
  int id[6];
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    if constexpr (STG) id[t] = *at(c.epos, t * ne + e0, 2u * uint32_t(e - e0));
    else id[t] = *at(c.stg, t * ne + e0, li);
  }
  const T nx = c.n[2 * e], ny = c.n[2 * e + 1];
  T w5[2][15];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int j = 0; j < 15; ++j) w5[s][j] = c.w5[(int64_t(s) * ne + e) * 15 + j];
  }
  const uint8_t fm = SWM == kSwForced ? force[e] : uint8_t(0);
  V4<T>* lv = reinterpret_cast<V4<T>*>(hfd_stage_lds);  // (staged: [rows][3] w, w_x, w_y)
  if constexpr (STG) {
    const int64_t b = e0 / kEdgeStageEdges;
    const int r0 = c.erp[b], nr = c.erp[b + 1] - r0;
    for (int k = int(threadIdx.x); k < nr; k += int(blockDim.x)) {
      const int64_t rw = c.erow[r0 + k];
      lv[3 * k] = Gv[rw];
      if constexpr (SWM != HFD_SWITCH_WENO_ONLY) {  // (WENO everywhere reads no gradient)
        lv[3 * k + 1] = Gg[2 * rw];
        lv[3 * k + 2] = Gg[2 * rw + 1];
      }
    }
    __syncthreads();
  }
  T w[6][4], wx[6][4], wy[6][4];
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    const int64_t i = id[t];
    V4<T> a, bx, by;
    if constexpr (STG) {
      a = lv[3 * i];
      bx = lv[3 * i + 1];
      by = lv[3 * i + 2];
    } else {
      a = Gv[i];
      bx = Gg[2 * i];
      by = Gg[2 * i + 1];
    }
    w[t][0] = a.x, w[t][1] = a.y, w[t][2] = a.z, w[t][3] = a.w;
    wx[t][0] = bx.x, wx[t][1] = bx.y, wx[t][2] = bx.z, wx[t][3] = bx.w;
    wy[t][0] = by.x, wy[t][1] = by.y, wy[t][2] = by.z, wy[t][3] = by.w;
  }
  const RoeState<T> F = roe_state<T>(V4<T>{w[2][0], w[2][1], w[2][2], w[2][3]},
                                     V4<T>{w[3][0], w[3][1], w[3][2], w[3][3]}, nx, ny, ref, gm1);
  // Hermite sums in physical variables: the 5-node row is the same for the
  // four characteristic components, so L (sum_t w5_t . data_t) is the
  // projected Hermite value
  T hs[2][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    hs[0][q] = T(0);
    hs[1][q] = T(0);
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      hs[0][q] += w5[0][3 * p] * w[p][q] + w5[0][3 * p + 1] * wx[p][q] + w5[0][3 * p + 2] * wy[p][q];
      const int n = 5 - p;
      hs[1][q] += w5[1][3 * p] * w[n][q] + w5[1][3 * p + 1] * wx[n][q] + w5[1][3 * p + 2] * wy[n][q];
    }
  }
  // characteristic projection of the six node values; side 0 takes nodes
  // 0..4, side 1 nodes 5..1
  T cv[4][6];
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    T pc[4];
    F.proj(w[t], pc);
#pragma unroll
    for (int q = 0; q < 4; ++q) cv[q][t] = pc[q];
  }
  // smoothness indicators of both sides (shared differences), then per side
  // the decisions and, only if some component takes that branch, the 3-node
  // rows and weights; then the interface state
  T be[2][4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q) weno_beta_pair<T>(cv[q], be[0][q], be[1][q]);
  uint8_t bits = 0;
  T wl[4], wr[4];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    T c5[4][5];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int p = 0; p < 5; ++p) c5[q][p] = cv[q][s == 0 ? p : 5 - p];
    }
    const uint8_t b = side_decide<T, SWM>(be[s], gp, s, fm);
    side_state<T>(b, s, be[s], c5, hs[s], F, gp, [&](int j) { return c.w3[(int64_t(s) * ne + e) * 9 + j]; },
                  s == 0 ? wl : wr);
    bits |= b;
  }
  T h[4];
  riemann<T>(gp.flux, wl, wr, nx, ny, ref, gam, gm1, h);
  const bool real = !STG || e0 + int64_t(threadIdx.x) < ne;
  store_edge<T>(ne, e, h, wl, wr, bits, gp, H, hsoa, wlr, mask, real, real);
}

// Roe state of an edge whose end states are held by a lane pair (lane 0
// node i, lane 1 node i+1; w in the kernel's form, perturbation in float32):
// each lane forms its node's square-root weights sqrt(rho) (1, u, v, H), the
// pair swaps them and both add the two.  The weights are rounded before the
// swap, so both lanes add the same two numbers and hold the same state.
template <class T>
__device__ inline RoeState<T> roe_state_pair(const T w[4], T nx, T ny, const Ref<T>& ref,
                                             T gm1) {
  const T r = ref.w[0] + w[0], ir = frcp(r);
  const T u = (ref.w[1] + w[1]) * ir, v = (ref.w[2] + w[2]) * ir;
  const T E = ref.w[3] + w[3];
  const T p = gm1 * (E - T(0.5) * r * (u * u + v * v));
  const T sq = fsqrt(r);
  T x[4] = {sq, sq * u, sq * v, sq * (E + p) * ir};
  T sum[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    asm volatile("" : "+v"(x[q]));  // (rounded: no product fused into the sum)
    sum[q] = x[q] + dpp_mov<0xB1>(x[q]);
  }
  const T iw = frcp(sum[0]);
  const T ur = sum[1] * iw, vr = sum[2] * iw, hh = sum[3] * iw;
  const T q2 = ur * ur + vr * vr;
  const T cc = fsqrt(gm1 * (hh - T(0.5) * q2));
  const T un = ur * nx + vr * ny, ut = -ur * ny + vr * nx;
  const T ic = frcp(cc), b1 = gm1 * ic * ic, b2 = T(0.5) * b1 * q2;
  return RoeState<T>{ur, vr, hh, cc, un, ut, b1, b2, ic, nx, ny};
}

// Two lanes per edge, lane s interpolating side s.  Each stencil node is
// gathered and projected once: lane 0 takes nodes 0, 1, 2 and lane 1 nodes
// 5, 4, 3 (its j-th node is node 5 - j), which are the first three nodes of
// each side in the side's own order.  The partner supplies the side's last
// two projected nodes and its partial Hermite sum over them (its own nodes
// j = 1, 2 lie on the other side, side-local nodes 4 and 3), and the edge's
// other end for the Roe average (node j = 2 of both lanes); the pair then
// swaps the interface states and both evaluate the flux (lane 0 stores it).
// All exchanges are DPP moves between lanes 2k and 2k+1.
// STG: the block's distinct stencil rows (values and gradients) are first
// copied to LDS, and the lanes read their nodes there by 2-byte position.
template <class T, int SWM, bool STG>
__global__ void __launch_bounds__(256, Edge2Waves<T>::value)
k_edge2(int64_t ne, EdgeCoef<T> c, GasParams gp, const V4<T>* __restrict__ Gv,
        const V4<T>* __restrict__ Gg, const uint8_t* __restrict__ force,
        V4<T>* __restrict__ H, double* __restrict__ hsoa, double* __restrict__ wlr,
        uint8_t* __restrict__ mask) {
  const int64_t e0 = xcd_block() * (blockDim.x / 2);
  const int s = int(threadIdx.x & 1);
  int64_t e = e0 + threadIdx.x / 2;
  if constexpr (!STG) {
    if (e >= ne) return;  // (both lanes of an edge leave together)
  } else {
    // every thread reaches the staging barrier: lanes past the last edge
    // recompute it and store nothing
    if (e >= ne) e = ne - 1;
  }
  const Ref<T> ref = make_ref<T>(gp);
  const T gam = gpar<T>(gp.gamma, gp.f_gamma), gm1 = gpar<T>(gp.gamma - 1.0, gp.f_gm1);
  // coefficient rows as in k_edge1, the pair of lanes sharing the edge.  A
  // side's Hermite weights (15 values) and 3-node rows (9) are one record
  // per edge, read with wide loads; the stencil positions are addressed from
  // a per-lane pointer formed once, plus the row's wave-uniform offset.
  const T* w5own = c.w5 + (int64_t(s) * ne + e) * 15;
  const T* w5oth = c.w5 + (int64_t(1 - s) * ne + e) * 15;
  const T* w3own = c.w3 + (int64_t(s) * ne + e) * 9;
  // this lane's stencil nodes j = 0, 1, 2: rows j (lane 0) or 5 - j (lane 1)
  const int64_t jstep = s == 0 ? ne : -ne;
  int id[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if constexpr (STG)
      id[j] = (c.epos + (s == 0 ? 0 : 5 * ne) + e)[j * jstep];
    else
      id[j] = (c.stg + (s == 0 ? 0 : 5 * ne) + e)[j * jstep];
  }
  const T nx = c.n[2 * e], ny = c.n[2 * e + 1];
  const uint8_t fm = SWM == kSwForced ? force[e] : uint8_t(0);
  // Hermite rows: own side at its nodes 0..2; other side at its nodes 3 + m,
  // which are own nodes j = 2 - m (m = 0, 1)
  T wo[9], wt[6];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
#pragma unroll
    for (int k = 0; k < 3; ++k) wo[3 * j + k] = w5own[3 * j + k];
  }
#pragma unroll
  for (int m = 0; m < 2; ++m) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
      wt[3 * m + k] = w5oth[3 * (3 + m) + k];
  }
  // (staged: the block's rows in LDS, [rows][3] records w, w_x, w_y)
  V4<T>* lv = reinterpret_cast<V4<T>*>(hfd_stage_lds);
  if constexpr (STG) {
    const int64_t b = e0 / kEdgeStageEdges;
    const int r0 = c.erp[b], nr = c.erp[b + 1] - r0;
    for (int k = int(threadIdx.x); k < nr; k += int(blockDim.x)) {
      const int64_t rw = c.erow[r0 + k];
      lv[3 * k] = Gv[rw];
      if constexpr (SWM != HFD_SWITCH_WENO_ONLY) {  // (WENO everywhere reads no gradient)
        lv[3 * k + 1] = Gg[2 * rw];
        lv[3 * k + 2] = Gg[2 * rw + 1];
      }
    }
    __syncthreads();
  }
  T w[3][4], gx[3][4], gy[3][4];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int64_t t = id[j];
    V4<T> a, bx, by;
    if constexpr (STG) {
      a = lv[3 * t];
      bx = lv[3 * t + 1];
      by = lv[3 * t + 2];
    } else {
      a = Gv[t];
      bx = Gg[2 * t];
      by = Gg[2 * t + 1];
    }
    w[j][0] = a.x, w[j][1] = a.y, w[j][2] = a.z, w[j][3] = a.w;
    gx[j][0] = bx.x, gx[j][1] = bx.y, gx[j][2] = bx.z, gx[j][3] = bx.w;
    gy[j][0] = by.x, gy[j][1] = by.y, gy[j][2] = by.z, gy[j][3] = by.w;
  }
  // Hermite partial sums in physical variables: own side over own nodes,
  // other side over own nodes j = 1, 2
  T hso[4], hst[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    hso[q] = T(0);
    hst[q] = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j)
      hso[q] += wo[3 * j] * w[j][q] + wo[3 * j + 1] * gx[j][q] + wo[3 * j + 2] * gy[j][q];
#pragma unroll
    for (int m = 0; m < 2; ++m)
      hst[q] += wt[3 * m] * w[2 - m][q] + wt[3 * m + 1] * gx[2 - m][q] +
                wt[3 * m + 2] * gy[2 - m][q];
  }
  // Roe frame of the edge's end states: lane 0 holds node 2, lane 1 node 3
  const RoeState<T> F = roe_state_pair<T>(w[2], nx, ny, ref, gm1);
  T hs[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) hs[q] = hso[q] + dpp_mov<0xB1>(hst[q]);
  // projected values of the side's five nodes: own j = 0..2, then the
  // partner's j = 2 and 1
  T cv[4][5];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    T pc[4];
    F.proj(w[j], pc);
#pragma unroll
    for (int q = 0; q < 4; ++q) cv[q][j] = pc[q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    cv[q][3] = dpp_mov<0xB1>(cv[q][2]);
    cv[q][4] = dpp_mov<0xB1>(cv[q][1]);
  }
  // decisions, then the 3-node rows and weights only where some component
  // of the side takes that branch
  T be[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q) weno_beta<T>(cv[q], be[q]);
  const uint8_t b = side_decide<T, SWM>(be, gp, s, fm);
  T wm[4];
  side_state<T>(b, s, be, cv, hs, F, gp, [&](int j) { return w3own[j]; }, wm);
  T wl[4], wr[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const T x = dpp_mov<0xB1>(wm[q]);
    wl[q] = s == 0 ? wm[q] : x;
    wr[q] = s == 0 ? x : wm[q];
  }
  const uint8_t bits = uint8_t(b | uint8_t(__builtin_amdgcn_update_dpp(0, int(b), 0xB1, 0xF, 0xF, false)));
  T h[4];
  if (gp.flux == HFD_FLUX_RUSANOV) {
    // each lane its own side's normal flux and speed, then swapped; only
    // lane 0 stores h, so both lanes join as lane 0 (left = own side)
    T fn[4], fo[4], sp;
    rusanov_side<T>(wm, nx, ny, ref, gam, gm1, fn, sp);
#pragma unroll
    for (int q = 0; q < 4; ++q) fo[q] = dpp_mov<0xB1>(fn[q]);
    rusanov_join<T>(wl, wr, fn, fo, sp, dpp_mov<0xB1>(sp), h);
  } else {
    riemann<T>(gp.flux, wl, wr, nx, ny, ref, gam, gm1, h);
  }
  const bool real = !STG || e0 + int64_t(threadIdx.x / 2) < ne;
  store_edge<T>(ne, e, h, wl, wr, bits, gp, H, hsoa, wlr, mask, real && s == 0, real && s == 1);
}

// Midpoint derivatives of the two interface states (hfd_edge_states only, not
// on the residual's path).  Two lanes per edge, lane s takes side s.  Per
// characteristic component, the branch recorded in the mask: the 5-node
// derivative rows applied to the side's physical data and projected (L_q G,
// the rows being the same for the four components), or the omega-weighted
// derivative rows of the three 3-node interpolants applied to the projected
// values; then back-projected with R.  The rows are float64 and annihilate
// constants, so the mixed form's perturbation data give the same sums.
template <class T>
__global__ void __launch_bounds__(256)
k_edge_grad(int64_t ne, EdgeCoef<T> c, const double* __restrict__ w5g,
            const double* __restrict__ w3g, GasParams gp, const V4<T>* __restrict__ Gv,
            const V4<T>* __restrict__ Gg, const uint8_t* __restrict__ mask,
            double* __restrict__ grad) {
  const int64_t e = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / 2;
  const int s = int(threadIdx.x & 1);
  if (e >= ne) return;
  const Ref<T> ref = make_ref<T>(gp);
  const T gm1 = gpar<T>(gp.gamma - 1.0, gp.f_gm1);
  const T nx = c.n[2 * e], ny = c.n[2 * e + 1];
  const RoeState<T> F = roe_state<T>(Gv[c.stg[2 * ne + e]], Gv[c.stg[3 * ne + e]], nx, ny, ref, gm1);
  const uint8_t fm = mask[e];
  T cv[4][5], G[2][4];
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int q = 0; q < 4; ++q) G[d][q] = T(0);
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const int64_t id = c.stg[int64_t(s == 0 ? j : 5 - j) * ne + e];
    const V4<T> a = Gv[id], bx = Gg[2 * id], by = Gg[2 * id + 1];
    const T w[4] = {a.x, a.y, a.z, a.w};
    const T wx[4] = {bx.x, bx.y, bx.z, bx.w};
    const T wy[4] = {by.x, by.y, by.z, by.w};
    T pc[4];
    F.proj(w, pc);
#pragma unroll
    for (int q = 0; q < 4; ++q) cv[q][j] = pc[q];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const double* r = w5g + int64_t((s * 2 + d) * 15 + 3 * j) * ne + e;
      const T gv = T(r[0]), gx = T(r[ne]), gy = T(r[2 * ne]);
#pragma unroll
      for (int q = 0; q < 4; ++q) G[d][q] += gv * w[q] + gx * wx[q] + gy * wy[q];
    }
  }
  T gc[2][4];
  F.proj(G[0], gc[0]);
  F.proj(G[1], gc[1]);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const bool weno = (fm >> (4 * s + q)) & 1;
    T o[3] = {T(0), T(0), T(0)};
    if (weno) {
      T be[3];
      weno_weights<T>(cv[q], gpar<T>(gp.eps, gp.f_eps), be, o);
    }
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      if (weno) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double* r = w3g + int64_t(((s * 3 + k) * 2 + d) * 3) * ne + e;
          acc += o[k] * (T(r[0]) * cv[q][k] + T(r[ne]) * cv[q][k + 1] +
                         T(r[2 * ne]) * cv[q][k + 2]);
        }
        gc[d][q] = acc;
      }
    }
  }
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    T out[4];
    F.back(gc[d], out);
#pragma unroll
    for (int q = 0; q < 4; ++q) grad[int64_t(8 * s + 4 * d + q) * ne + e] = double(out[q]);
  }
}

// ---------------------------------------------------------------------------
// Vertex pass
// ---------------------------------------------------------------------------
// Lanes per vertex (8 or 16) and vertices per 256-thread block, per precision.
template <class T> struct VertexLanes { static constexpr int value = HFD_VERTEX_LANES64; };
template <> struct VertexLanes<float> { static constexpr int value = HFD_VERTEX_LANES32; };

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

// A coefficient record of N values (loaded as one aggregate).
template <class T, int N>
struct Rec {
  T v[N];
};


// Waves per SIMD the vertex kernel is compiled for (register budget 512/waves).
template <class T> struct VertexWaves { static constexpr int value = 4; };
template <> struct VertexWaves<float> { static constexpr int value = HFD_VERTEX_WAVES; };

// Slot id of a coefficient stream at byte base b, slot r: a global row or
// edge (IB = 0, int32) or a position in the block's staged list (1 or 2 bytes).
template <int IB>
__device__ inline int slot_id(const char* b, uint32_t r) {
  if constexpr (IB == 0) return *reinterpret_cast<const int32_t*>(b + 4u * r);
  else if constexpr (IB == 1) return *reinterpret_cast<const uint8_t*>(b + r);
  else return *reinterpret_cast<const uint16_t*>(b + 2u * r);
}

template <class T, bool VISC, int IB>
__global__ void __launch_bounds__(256, VISC ? 2 : VertexWaves<T>::value)
k_vertex(int64_t nowned, int64_t nv, VertexCoef<T> c, GasParams gp,
         const V4<T>* __restrict__ Gv, const V4<T>* __restrict__ Gg,
         const V4<T>* __restrict__ H, int mode, double* __restrict__ dU, RkArgs rk,
         V4<T>* __restrict__ Gv_new, V4<T>* __restrict__ Gg_new,
         int32_t* __restrict__ flag) {
  constexpr int VL = VertexLanes<T>::value, VPB = 256 / VL;
  static_assert(VL == 8 || VL == 16, "8 or 16 lanes per vertex");
  static_assert(IB == 0 || VPB == kStageVertices, "staged lists are per 16 vertices");
  // slots per lane and iteration: every load of a batch is issued before any
  // of its data is used
  constexpr int NVS = VL != 16 ? 3
                      : sizeof(T) == 4 ? (VISC ? HFD_VERTEX_NVS32V : HFD_VERTEX_NVS32)
                                       : HFD_VERTEX_NVS64;
  constexpr int NES = VL != 16 ? 6
                      : sizeof(T) == 4 ? (VISC ? HFD_VERTEX_NES32V : HFD_VERTEX_NES32)
                                       : HFD_VERTEX_NES64;
  __shared__ double sres[VPB][13];
  const int t = threadIdx.x;
  const int vl = t / VL, sub = t & (VL - 1);
  const int64_t v0 = xcd_block() * VPB;
  const int64_t v = v0 + vl;

  // The epilogue gives element p = t + 256 i (i < NEP) of the block's
  // 12 x VPB results to thread t: component p / VPB of vertex v0 + p % VPB,
  // consecutive vertices in consecutive lanes so that every component row is
  // written in VPB-wide runs.  Its Runge-Kutta operands are loaded first, so
  // that their latency overlaps the slot loads.
  constexpr int NEP = (12 * VPB + 255) / 256;
  double un[NEP], uk[NEP];
  double dt = 0.0;
#pragma unroll
  for (int i = 0; i < NEP; ++i) {
    const int p = t + 256 * i;
    const int64_t vv = v0 + p % VPB;
    un[i] = uk[i] = 0.0;
    if (mode == 1 && p < 12 * VPB && vv < nowned) {
      const int64_t o = int64_t(p / VPB) * nv + vv;
      // (U^n has no weight in the first stage)
      if (rk.a != 0.0) un[i] = rk.Un[o];
      uk[i] = rk.Uk[o];
    }
  }
  if (mode == 1) dt = rk.dt_dev ? *rk.dt_dev : rk.dt;

  // Staging: the block's distinct state rows (and gradient rows) and edge
  // fluxes go to LDS once; the slots then read them by local id.
  const V4<T>* sV = Gv;
  const V4<T>* sG = Gg;
  const V4<T>* sH = H;
  if constexpr (IB > 0) {
    V4<T>* lv = reinterpret_cast<V4<T>*>(hfd_stage_lds);
    V4<T>* lg = lv + c.max_rows;
    V4<T>* lh = lv + (VISC ? 3 : 1) * c.max_rows;
    const int64_t b = v0 / VPB;
    const int r0 = c.hrp[b], nr = c.hrp[b + 1] - r0;
    const int q0 = c.hep[b], nq = c.hep[b + 1] - q0;
    // every block has at least one row and one edge (a vertex's own row and
    // an edge of it): lanes past a list's end load its last entry again and
    // do not store it
    const int nk = nr > nq ? nr : nq;
    for (int k = t; k < nk; k += 256) {
      const int64_t row = c.hrow[r0 + (k < nr ? k : nr - 1)];
      const int64_t ed = c.hedge[q0 + (k < nq ? k : nq - 1)];
      const V4<T> a = Gv[row];
      V4<T> g0, g1;
      if (VISC) {
        g0 = Gg[2 * row];
        g1 = Gg[2 * row + 1];
      }
      const V4<T> hh = H[ed];
      if (k < nr) {
        lv[k] = a;
        if (VISC) {
          lg[2 * k] = g0;
          lg[2 * k + 1] = g1;
        }
      }
      if (k < nq) lh[k] = hh;
    }
    __syncthreads();
    sV = lv;
    sG = lg;
    sH = lh;
  }

  const Ref<T> ref = make_ref<T>(gp);
  const T gm1 = gpar<T>(gp.gamma - 1.0, gp.f_gm1);
  T acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = T(0);

  if (v < nowned) {
    // S(v) holds v itself and M(v) at least one edge of v (the setup rejects
    // meshes where the rows cannot be built), so s1 - 1 and e1 - 1 are slots
    // of v: lanes past the end load them again and give them zero weight.
    const int s0 = c.vptr[v], s1 = c.vptr[v + 1];
    const int e0 = c.eptr[v], e1 = c.eptr[v + 1];
    // The coefficient streams are addressed from the block's first slots
    // (uniform) with 32-bit byte offsets: one register per address.
    const int sb = c.vptr[v0], eb = c.eptr[v0];
    const char* vgb = IB ? reinterpret_cast<const char*>(c.vloc) + IB * sb
                         : reinterpret_cast<const char*>(c.vg + sb);
    // staged: positions in the block's lists are v's base plus the slot's id
    const uint32_t lb = IB ? c.lbase[v] : 0u;
    const int rbase = int(lb & 0xffffu), ebase = int(lb >> 16);
    const char* dvb = reinterpret_cast<const char*>(c.dv + int64_t(6) * sb);
    const char* dkb = VISC ? reinterpret_cast<const char*>(c.dvis + int64_t(5) * sb) : nullptr;
    const char* veb = IB ? reinterpret_cast<const char*>(c.eloc) + IB * eb
                         : reinterpret_cast<const char*>(c.ve + eb);
    const char* deb = reinterpret_cast<const char*>(c.de + int64_t(3) * eb);
    // vertex slots, then edge slots (separate batches: fewer values in
    // flight per wave, more waves per SIMD)
    for (int bs = s0 + sub; bs < s1; bs += NVS * VL) {
      int js[NVS];
      bool oks[NVS];
#pragma unroll
      for (int k = 0; k < NVS; ++k) {
        oks[k] = bs + k * VL < s1;
        js[k] = oks[k] ? bs + k * VL : s1 - 1;
      }
      int u[NVS];
      T d[NVS][6], kv[NVS][5];
#pragma unroll
      for (int k = 0; k < NVS; ++k) {
        const uint32_t r = uint32_t(js[k] - sb);
        u[k] = rbase + slot_id<IB>(vgb, r);
        const Rec<T, 6> dr = *reinterpret_cast<const Rec<T, 6>*>(dvb + uint32_t(6 * sizeof(T)) * r);
#pragma unroll
        for (int q = 0; q < 6; ++q) d[k][q] = dr.v[q];
        if (VISC) {
          const Rec<T, 5> kr = *reinterpret_cast<const Rec<T, 5>*>(dkb + uint32_t(5 * sizeof(T)) * r);
#pragma unroll
          for (int q = 0; q < 5; ++q) kv[k][q] = kr.v[q];
        }
      }
      V4<T> A[NVS], G[NVS][2];
#pragma unroll
      for (int k = 0; k < NVS; ++k) {
        A[k] = sV[u[k]];
        if (VISC) {
          G[k][0] = sG[2 * int64_t(u[k])];
          G[k][1] = sG[2 * int64_t(u[k]) + 1];
        }
      }
#pragma unroll
      for (int k = 0; k < NVS; ++k) {
#pragma unroll
        for (int q = 0; q < 6; ++q) d[k][q] = oks[k] ? d[k][q] : T(0);
        if (VISC) {
#pragma unroll
          for (int q = 0; q < 5; ++q) kv[k][q] = oks[k] ? kv[k][q] : T(0);
        }
        vslot<T, VISC>(A[k], G[k], d[k], kv[k], ref, gm1, gp, acc);
      }
    }
    for (int be = e0 + sub; be < e1; be += NES * VL) {
      int je[NES];
      bool oke[NES];
#pragma unroll
      for (int k = 0; k < NES; ++k) {
        oke[k] = be + k * VL < e1;
        je[k] = oke[k] ? be + k * VL : e1 - 1;
      }
      int m[NES];
      T de[NES][3];
#pragma unroll
      for (int k = 0; k < NES; ++k) {
        const uint32_t r = uint32_t(je[k] - eb);
        m[k] = ebase + slot_id<IB>(veb, r);
        const Rec<T, 3> er = *reinterpret_cast<const Rec<T, 3>*>(deb + uint32_t(3 * sizeof(T)) * r);
#pragma unroll
        for (int q = 0; q < 3; ++q) de[k][q] = er.v[q];
      }
      V4<T> Hh[NES];
#pragma unroll
      for (int k = 0; k < NES; ++k) Hh[k] = sH[m[k]];
#pragma unroll
      for (int k = 0; k < NES; ++k) {
        const T w0 = oke[k] ? de[k][0] : T(0), w1 = oke[k] ? de[k][1] : T(0),
                w2 = oke[k] ? de[k][2] : T(0);
        const T hq[4] = {Hh[k].x, Hh[k].y, Hh[k].z, Hh[k].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc[q] -= w0 * hq[q];
          acc[4 + q] -= w1 * hq[q];
          acc[8 + q] -= w2 * hq[q];
        }
      }
    }
  }
  if constexpr (VL == 16) {
    reduce_stage<3, 16>(acc, sub);
    reduce_stage<2, 8>(acc, sub);
    reduce_stage<1, 4>(acc, sub);
    reduce_stage<0, 2>(acc, sub);
  } else {
    reduce_stage<2, 16>(acc, sub);
    reduce_stage<1, 8>(acc, sub);
    reduce_stage<0, 4>(acc, sub);
  }
  constexpr int CPL = 16 / VL;
#pragma unroll
  for (int i = 0; i < CPL; ++i)
    if (CPL * sub + i < 12) sres[vl][CPL * sub + i] = double(acc[i]);
  __syncthreads();

  bool bad = false;
#pragma unroll
  for (int i = 0; i < NEP; ++i) {
    const int p = t + 256 * i;
    const int cmp = p / VPB, vl2 = p % VPB;
    const int64_t vv = v0 + vl2;
    if (p >= 12 * VPB || vv >= nowned) continue;
    const int64_t o = int64_t(cmp) * nv + vv;
    const double rv = sres[vl2][cmp];
    if (mode == 0) {
      dU[o] = rv;
      bad = bad || !isfinite(rv);
    } else {
      const double out = rk.a * un[i] + rk.b * (uk[i] + dt * rv);
      rk.Unew[o] = out;
      if (Gv_new) {
        const T g = T(out - (cmp < 4 ? gp.wref[cmp] : 0.0));
        if (cmp < 4) reinterpret_cast<T*>(Gv_new)[4 * vv + cmp] = g;
        else reinterpret_cast<T*>(Gg_new)[8 * vv + (cmp - 4)] = g;
      }
      bad = bad || !isfinite(out);
      if (cmp < 4) sres[vl2][cmp] = out;
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

template <class T, int SWM>
void launch_edge_swm(int64_t ne, const EdgeCoef<T>& c, const GasParams& gp, const V4<T>* Gv,
                     const V4<T>* Gg, const uint8_t* force, V4<T>* H, double* hsoa,
                     double* wlr, uint8_t* mask, hipStream_t st) {
  // two lanes per edge (one per side); in float32 one lane per edge when
  // HFD_EDGE32_TWO_LANES is 0
  if constexpr (sizeof(T) == 8 || HFD_EDGE32_TWO_LANES) {
    if (c.erp)
      hipLaunchKernelGGL((k_edge2<T, SWM, true>), dim3(nblocks(2 * ne, 256)), dim3(256),
                         size_t(c.max_rows) * 3 * sizeof(V4<T>), st, ne, c, gp, Gv, Gg, force,
                         H, hsoa, wlr, mask);
    else
      hipLaunchKernelGGL((k_edge2<T, SWM, false>), dim3(nblocks(2 * ne, 256)), dim3(256), 0, st,
                         ne, c, gp, Gv, Gg, force, H, hsoa, wlr, mask);
  }
  else if (HFD_EDGE1_STAGE && c.erp)
    hipLaunchKernelGGL((k_edge1<T, SWM, true>), dim3(nblocks(ne, kEdgeStageEdges)),
                       dim3(kEdgeStageEdges), size_t(c.max_rows) * 3 * sizeof(V4<T>), st, ne, c,
                       gp, Gv, Gg, force, H, hsoa, wlr, mask);
  else
    hipLaunchKernelGGL((k_edge1<T, SWM, false>), dim3(nblocks(ne, 256)), dim3(256), 0, st, ne,
                       c, gp, Gv, Gg, force, H, hsoa, wlr, mask);
}

template <class T>
hipError_t launch_edge(int64_t ne, const EdgeCoef<T>& c, const GasParams& gp,
                       const V4<T>* Gv, const V4<T>* Gg, const uint8_t* force, V4<T>* H,
                       double* hsoa, double* wlr, uint8_t* mask, hipStream_t st) {
  if (ne == 0) return hipSuccess;
  if (force)
    launch_edge_swm<T, kSwForced>(ne, c, gp, Gv, Gg, force, H, hsoa, wlr, mask, st);
  else if (gp.sw == HFD_SWITCH_PAPER)
    launch_edge_swm<T, HFD_SWITCH_PAPER>(ne, c, gp, Gv, Gg, force, H, hsoa, wlr, mask, st);
  else if (gp.sw == HFD_SWITCH_SMOOTH_ONLY)
    launch_edge_swm<T, HFD_SWITCH_SMOOTH_ONLY>(ne, c, gp, Gv, Gg, force, H, hsoa, wlr, mask, st);
  else if (gp.sw == HFD_SWITCH_WENO_ONLY)
    launch_edge_swm<T, HFD_SWITCH_WENO_ONLY>(ne, c, gp, Gv, Gg, force, H, hsoa, wlr, mask, st);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
template hipError_t launch_edge<double>(int64_t, const EdgeCoef<double>&, const GasParams&,
                                        const V4<double>*, const V4<double>*, const uint8_t*,
                                        V4<double>*, double*, double*, uint8_t*, hipStream_t);
template hipError_t launch_edge<float>(int64_t, const EdgeCoef<float>&, const GasParams&,
                                       const V4<float>*, const V4<float>*, const uint8_t*,
                                       V4<float>*, double*, double*, uint8_t*, hipStream_t);

template <class T>
hipError_t launch_edge_grad(int64_t ne, const EdgeCoef<T>& c, const double* w5g,
                            const double* w3g, const GasParams& gp, const V4<T>* Gv,
                            const V4<T>* Gg, const uint8_t* mask, double* grad,
                            hipStream_t st) {
  if (ne == 0) return hipSuccess;
  hipLaunchKernelGGL(k_edge_grad<T>, dim3(nblocks(2 * ne, 256)), dim3(256), 0, st, ne, c, w5g,
                     w3g, gp, Gv, Gg, mask, grad);
  return hipGetLastError();
}
template hipError_t launch_edge_grad<double>(int64_t, const EdgeCoef<double>&, const double*,
                                             const double*, const GasParams&,
                                             const V4<double>*, const V4<double>*,
                                             const uint8_t*, double*, hipStream_t);
template hipError_t launch_edge_grad<float>(int64_t, const EdgeCoef<float>&, const double*,
                                            const double*, const GasParams&, const V4<float>*,
                                            const V4<float>*, const uint8_t*, double*,
                                            hipStream_t);

template <class T>
hipError_t launch_vertex(int64_t nowned, int64_t nv, const VertexCoef<T>& c,
                         const GasParams& gp, const V4<T>* Gv, const V4<T>* Gg,
                         const V4<T>* H, int mode, double* dU, const RkArgs& rk,
                         V4<T>* Gv_new, V4<T>* Gg_new, int32_t* flag, hipStream_t st) {
  if (nowned == 0) return hipSuccess;
  constexpr int VPB = 256 / VertexLanes<T>::value;
  const unsigned nb = nblocks(nowned, VPB);
  const size_t lds = c.idx_bytes ? size_t((c.dvis ? 3 : 1) * c.max_rows + c.max_edges) *
                                       sizeof(V4<T>)
                                 : 0;
#define HFD_LAUNCH_VERTEX(V, I)                                                              \
  hipLaunchKernelGGL((k_vertex<T, V, I>), dim3(nb), dim3(256), lds, st, nowned, nv, c, gp, Gv, \
                     Gg, H, mode, dU, rk, Gv_new, Gg_new, flag)
  if constexpr (VPB == kStageVertices) {
    if (c.dvis) {
      if (c.idx_bytes == 1) HFD_LAUNCH_VERTEX(true, 1);
      else if (c.idx_bytes == 2) HFD_LAUNCH_VERTEX(true, 2);
      else HFD_LAUNCH_VERTEX(true, 0);
    } else {
      if (c.idx_bytes == 1) HFD_LAUNCH_VERTEX(false, 1);
      else if (c.idx_bytes == 2) HFD_LAUNCH_VERTEX(false, 2);
      else HFD_LAUNCH_VERTEX(false, 0);
    }
  } else {
    // (8 lanes per vertex: 32-vertex blocks, no staging lists)
    if (c.idx_bytes != 0) return hipErrorInvalidValue;
    if (c.dvis) HFD_LAUNCH_VERTEX(true, 0);
    else HFD_LAUNCH_VERTEX(false, 0);
  }
#undef HFD_LAUNCH_VERTEX
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
