// Geometric precompute on the GPU in float64: the stored rows of every
// least-squares system of the method.
//
//  * Hermite 5-node rows (Section 2.2, eq. hintp_5): SVD of the 15 x 15
//    matrix P in the edge frame, rank = singular values above 1e-12 of the
//    largest (at most 14: P is singular for every stencil because the square
//    of the conic through the five nodes has zero value and gradient at all
//    of them), graded pseudo-inverse (the least-squares solution whose
//    degree-4 block is smallest), and the paper's dropping rule: while a
//    value weight of the row is >= 1 in magnitude, drop the smallest kept
//    singular value.  The anchor's value weight then absorbs
//    1 - sum(value weights).
//  * 3-node rows (eq. 3nodes_intp): the same on the 3 x 6 degree-2 system,
//    graded on the degree-2 block; optional dropping above a cap.
//  * On request, the midpoint derivatives: rows 2 and 3 (d/dx, d/dy) of the
//    same 5-node and 3-node operators at the final rank.
//  * Divergence rows (eq. flux_polynomials, rows d0, dx, dy): full-rank
//    least squares of degree 4 or 5 solved by Householder QR; a pseudo-inverse row
//    is Q [R^-T e; 0].  A rank-deficient system is reported as a mesh error.
//  * Viscous rows (vertex-only fit of degree 4): SVD + graded pseudo-inverse.
//
// SVDs are one-sided (Hestenes) Jacobi with the rows of the matrix spread
// over a group of lanes and the columns in LDS; every kernel runs blocks of
// exactly one wavefront, so synchronisation inside a group is wave-local.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace hfd {
namespace {

constexpr double kRtol = 1e-12;

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum and maximum over a group of G lanes (16 or 64), every lane receiving
// the same bits: within a 16-lane row by DPP (swap neighbours, swap pairs,
// mirror the half rows, mirror the row; each step combines two partial
// results that are equal up to the order of a commutative operation), across
// rows by lane exchange.  The lanes branch on these sums, so the bits must
// agree: the empty asm makes x an opaque register value, which keeps the
// compiler from fusing the caller's product into the first addition (a lane
// would then add its neighbour's rounded product to its own unrounded one).
template <int G>
__device__ inline double gsum(double x) {
  static_assert(G == 16 || G == 64, "group of 16 or 64 lanes");
  asm volatile("" : "+v"(x));
  x += dpp_mov<0xB1>(x);
  x += dpp_mov<0x4E>(x);
  x += dpp_mov<0x141>(x);
  x += dpp_mov<0x140>(x);
  if constexpr (G == 64) {
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
  }
  return x;
}

template <int G>
__device__ inline double gmax(double x) {
  static_assert(G == 16 || G == 64, "group of 16 or 64 lanes");
  x = fmax(x, dpp_mov<0xB1>(x));
  x = fmax(x, dpp_mov<0x4E>(x));
  x = fmax(x, dpp_mov<0x141>(x));
  x = fmax(x, dpp_mov<0x140>(x));
  if constexpr (G == 64) {
    x = fmax(x, __shfl_xor(x, 16));
    x = fmax(x, __shfl_xor(x, 32));
  }
  return x;
}

// Taylor-scaled monomials x^a y^b / (a! b!) ordered by total degree, then by
// decreasing power of x.  kind 0: value, 1: d/dx, 2: d/dy.
template <int DEG>
__device__ inline double mono(int c, int kind, double x, double y) {
  int d = 0, base = 0;
  while (base + d + 1 <= c) { base += d + 1; ++d; }
  int j = c - base;
  int a = d - j, b = j;
  if (kind == 1) { if (a == 0) return 0.0; a -= 1; }
  if (kind == 2) { if (b == 0) return 0.0; b -= 1; }
  double v = 1.0;
  for (int k = 1; k <= a; ++k) v *= x / double(k);
  for (int k = 1; k <= b; ++k) v *= y / double(k);
  return v;
}

// One-sided Jacobi on the m x n matrix A (LDS, column-major [n][G*RPL], the
// group's lane l holds rows l, l+G, ...).  On return A <- A V (orthogonal
// columns U*sigma) and V (LDS [n][G], lane j holds row j) is orthogonal.
// A pair is rotated unless its columns are orthogonal to 1e-15 (relative) or
// one of them has a squared norm below 1e-32 of the squared Frobenius norm
// of A.  The second test ends the iteration on rank-deficient matrices: the
// columns of zero singular values shrink geometrically as rounding noise
// whose angles to the other columns stay of order one, so the relative test
// alone never holds for them; rotating such a column changes the others
// below rounding.
template <int G, int RPL>
__device__ void jacobi(double* A, double* V, int m, int n, int lane) {
  constexpr int LD = G * RPL;
  for (int c = 0; c < n; ++c) V[c * G + lane] = (lane == c) ? 1.0 : 0.0;
  double fro = 0.0;
  for (int c = 0; c < n; ++c) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const double x = A[c * LD + lane + r * G];
      fro += x * x;
    }
  }
  const double tiny = 1e-32 * gsum<G>(fro);
  wave_sync();
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          int i = lane + r * G;
          double x = A[p * LD + i], y = A[q * LD + i];
          a += x * x;
          b += y * y;
          g += x * y;
        }
        a = gsum<G>(a);
        b = gsum<G>(b);
        g = gsum<G>(g);
        if (g == 0.0 || fmin(a, b) <= tiny || fabs(g) <= 1e-15 * sqrt(a * b)) continue;
        rotated = true;
        double zeta = (b - a) / (2.0 * g);
        double t = copysign(1.0, zeta) / (fabs(zeta) + hypot(1.0, zeta));
        double cs = 1.0 / sqrt(1.0 + t * t);
        double sn = cs * t;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          int i = lane + r * G;
          double x = A[p * LD + i], y = A[q * LD + i];
          A[p * LD + i] = cs * x - sn * y;
          A[q * LD + i] = sn * x + cs * y;
        }
        double x = V[p * G + lane], y = V[q * G + lane];
        V[p * G + lane] = cs * x - sn * y;
        V[q * G + lane] = sn * x + cs * y;
      }
    }
    if (!rotated) break;
  }
  wave_sync();
}

// Column norms of A (singular values) and their order, largest first.
template <int G, int RPL>
__device__ void sing_order(const double* A, int n, int lane, double* sig,
                           int* perm) {
  constexpr int LD = G * RPL;
  for (int c = 0; c < n; ++c) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      double x = A[c * LD + lane + r * G];
      s += x * x;
    }
    s = sqrt(gsum<G>(s));
    if (lane == 0) sig[c] = s;
  }
  wave_sync();
  if (lane == 0) {
    for (int c = 0; c < n; ++c) perm[c] = c;
    for (int i = 1; i < n; ++i) {  // insertion sort, descending, stable
      int k = perm[i];
      int j = i - 1;
      while (j >= 0 && sig[perm[j]] < sig[k]) { perm[j + 1] = perm[j]; --j; }
      perm[j + 1] = k;
    }
  }
  wave_sync();
}

// Workspace of the graded pseudo-inverse.
struct GradedWs {
  double* KT;   // [ntop][LD]
  double* Bt;   // [ntop][G]
  double* W;    // [ntop][G]
  double* sb;   // [ntop]
  int* pb;      // [ntop]
};

// Rows `rows` of the graded pseudo-inverse of rank r (see file comment):
//   K = K_r - N pinv(N_top) K_r[top],  K_r = V_r S_r^-1 U_r^T,
// with A holding U*sigma.  out: [nrows][LD] (lane rows).
template <int G, int RPL>
__device__ void graded_rows(const double* A, const double* V, const double* sig,
                            const int* perm, int m, int n, int r,
                            const int* top, int ntop, const int* rows,
                            int nrows, GradedWs ws, double* out, int lane) {
  constexpr int LD = G * RPL;
  // K_r rows for `top` and for `rows`
  for (int a = 0; a < ntop + nrows; ++a) {
    int j = a < ntop ? top[a] : rows[a - ntop];
    double* dst = a < ntop ? ws.KT + a * LD : out + (a - ntop) * LD;
#pragma unroll
    for (int rr = 0; rr < RPL; ++rr) {
      int i = lane + rr * G;
      double s = 0.0;
      for (int t = 0; t < r; ++t) {
        int c = perm[t];
        s += V[c * G + j] / (sig[c] * sig[c]) * A[c * LD + i];
      }
      dst[i] = (i < m) ? s : 0.0;
    }
  }
  wave_sync();
  const int k = n - r;
  if (k <= 0) return;
  // B^T (k x ntop): row t = lane, column a: V[top_a][perm[r + t]]
  for (int a = 0; a < ntop; ++a)
    ws.Bt[a * G + lane] = (lane < k) ? V[perm[r + lane] * G + top[a]] : 0.0;
  wave_sync();
  jacobi<G, 1>(ws.Bt, ws.W, k, ntop, lane);
  sing_order<G, 1>(ws.Bt, ntop, lane, ws.sb, ws.pb);
  double smax = ws.sb[ws.pb[0]];
  for (int jr = 0; jr < nrows; ++jr) {
    int j = rows[jr];
    double n0 = (lane < k) ? V[perm[r + lane] * G + j] : 0.0;
    double y[16];
#pragma unroll
    for (int a = 0; a < 16; ++a) y[a] = 0.0;
    for (int c = 0; c < ntop; ++c) {
      double gc = gsum<G>(n0 * ws.Bt[c * G + lane]);
      double s = ws.sb[c];
      double coef = (s > kRtol * smax) ? gc / (s * s) : 0.0;
#pragma unroll
      for (int a = 0; a < 16; ++a)
        if (a < ntop) y[a] += coef * ws.W[c * G + a];
    }
#pragma unroll
    for (int rr = 0; rr < RPL; ++rr) {
      int i = lane + rr * G;
      double s = out[jr * LD + i];
#pragma unroll
      for (int a = 0; a < 16; ++a)
        if (a < ntop) s -= y[a] * ws.KT[a * LD + i];
      out[jr * LD + i] = (i < m) ? s : 0.0;
    }
  }
  wave_sync();
}

// ---------------------------------------------------------------------------
// Edge weights: one 16-lane group per (edge, side); 4 groups per wavefront.
// ---------------------------------------------------------------------------
constexpr int EG = 16;

struct EdgeLds {
  double A[15 * EG];
  double V[15 * EG];
  double KT[5 * EG];
  double Bt[5 * EG];
  double W[5 * EG];
  double out[EG];
  double outg[2 * EG];
  double sig[16];
  double sb[8];
  int perm[16];
  int pb[8];
};

__global__ void __launch_bounds__(64)
k_edge_weights(int64_t ne, const double* __restrict__ pts,
               const double* __restrict__ eh, double w3_cap,
               double* __restrict__ w5, double* __restrict__ w3,
               int32_t* __restrict__ rank, int8_t* __restrict__ trunc3,
               double* __restrict__ w5g, double* __restrict__ w3g) {
  __shared__ EdgeLds lds_all[4];
  const int grp = threadIdx.x / EG, lane = threadIdx.x % EG;
  const int64_t item = int64_t(blockIdx.x) * 4 + grp;
  if (item >= 2 * ne) return;
  const int64_t e = item >> 1;
  const int side = int(item & 1);
  EdgeLds& L = lds_all[grp];
  // side nodes in the six-node stencil: left (0..4), right (5..1)
  int nodes[5];
  for (int t = 0; t < 5; ++t) nodes[t] = side == 0 ? t : 5 - t;
  const double* P = pts + 12 * e;

  // ---- 5-node Hermite ------------------------------------------------------
  {
    int i = lane;
    for (int c = 0; c < 15; ++c) {
      double v = 0.0;
      if (i < 15) {
        int nd = nodes[i / 3];
        v = mono<4>(c, i % 3, P[2 * nd], P[2 * nd + 1]);
      }
      L.A[c * EG + lane] = v;
    }
    wave_sync();
    jacobi<EG, 1>(L.A, L.V, 15, 15, lane);
    sing_order<EG, 1>(L.A, 15, lane, L.sig, L.perm);
    double smax = L.sig[L.perm[0]];
    int r = 0;
    for (int c = 0; c < 15; ++c) r += (L.sig[c] > kRtol * smax) ? 1 : 0;
    r = min(r, 14);
    const int top[5] = {10, 11, 12, 13, 14};
    const int rows[1] = {0};
    GradedWs ws{L.KT, L.Bt, L.W, L.sb, L.pb};
    for (;;) {
      graded_rows<EG, 1>(L.A, L.V, L.sig, L.perm, 15, 15, r, top, 5, rows, 1,
                         ws, L.out, lane);
      double wv = (lane < 15 && lane % 3 == 0) ? fabs(L.out[lane]) : 0.0;
      double mx = gmax<EG>(wv);
      if (mx >= 1.0 && r > 1) { --r; continue; }
      break;
    }
    double w = (lane < 15) ? L.out[lane] : 0.0;
    double sv = gsum<EG>((lane < 15 && lane % 3 == 0) ? w : 0.0);
    if (lane == 6) w += 1.0 - sv;  // anchor = node 2 of the side
    if (lane < 15) {
      if (lane % 3 != 0) w *= eh[e];
      w5[(int64_t(side) * ne + e) * 15 + lane] = w;
    }
    if (lane == 0) rank[int64_t(side) * ne + e] = r;
    // midpoint derivatives: rows 2 and 3 of the same operator at the final
    // rank; the anchor absorbs minus their value-weight sums (a constant has
    // zero gradient); value weights / h for physical units
    if (w5g) {
      const int grows[2] = {1, 2};
      graded_rows<EG, 1>(L.A, L.V, L.sig, L.perm, 15, 15, r, top, 5, grows, 2, ws,
                         L.outg, lane);
      for (int d = 0; d < 2; ++d) {
        double g = (lane < 15) ? L.outg[d * EG + lane] : 0.0;
        const double sg = gsum<EG>((lane < 15 && lane % 3 == 0) ? g : 0.0);
        if (lane == 6) g -= sg;
        if (lane < 15) {
          if (lane % 3 == 0) g /= eh[e];
          w5g[int64_t((side * 2 + d) * 15 + lane) * ne + e] = g;
        }
      }
      wave_sync();
    }
  }

  // ---- 3-node substencils (eq. 3nodes_intp) -----------------------------------
  for (int j = 0; j < 3; ++j) {
    // rows: the three nodes j, j+1, j+2 of the side; columns: degree-2 basis
    for (int c = 0; c < 6; ++c) {
      double v = 0.0;
      if (lane < 3) {
        int nd = nodes[j + lane];
        v = mono<2>(c, 0, P[2 * nd], P[2 * nd + 1]);
      }
      L.A[c * EG + lane] = v;
    }
    wave_sync();
    jacobi<EG, 1>(L.A, L.V, 3, 6, lane);
    sing_order<EG, 1>(L.A, 6, lane, L.sig, L.perm);
    double smax = L.sig[L.perm[0]];
    int r = 0;
    for (int c = 0; c < 6; ++c) r += (L.sig[c] > kRtol * smax) ? 1 : 0;
    const int top[3] = {3, 4, 5};
    const int rows[1] = {0};
    GradedWs ws{L.KT, L.Bt, L.W, L.sb, L.pb};
    int dropped = 0;
    for (;;) {
      graded_rows<EG, 1>(L.A, L.V, L.sig, L.perm, 3, 6, r, top, 3, rows, 1, ws,
                         L.out, lane);
      double mx = gmax<EG>(lane < 3 ? fabs(L.out[lane]) : 0.0);
      if (w3_cap > 0.0 && mx > w3_cap && r > 1) { --r; ++dropped; continue; }
      break;
    }
    double w = (lane < 3) ? L.out[lane] : 0.0;
    double sv = gsum<EG>(w);
    if (lane == 2 - j) w += 1.0 - sv;  // the side's anchor (node 2)
    if (lane < 3) w3[(int64_t(side) * ne + e) * 9 + j * 3 + lane] = w;
    if (lane == 0) trunc3[int64_t(side * 3 + j) * ne + e] = int8_t(dropped);
    if (w3g) {  // gradient of the interpolant at the midpoint, as for w5g
      const int grows[2] = {1, 2};
      graded_rows<EG, 1>(L.A, L.V, L.sig, L.perm, 3, 6, r, top, 3, grows, 2, ws, L.outg,
                         lane);
      for (int d = 0; d < 2; ++d) {
        double g = (lane < 3) ? L.outg[d * EG + lane] : 0.0;
        const double sg = gsum<EG>(g);
        if (lane == 2 - j) g -= sg;
        if (lane < 3) w3g[int64_t(((side * 3 + j) * 2 + d) * 3 + lane) * ne + e] = g / eh[e];
      }
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// Divergence rows: one wavefront per owned vertex, Householder QR.
// ---------------------------------------------------------------------------
// Terms of the divergence fit of degree DEG and its unknowns (a, b).
template <int DEG> constexpr int kDivTerms = (DEG + 1) * (DEG + 2) / 2;
template <int DEG> constexpr int kDivUnknowns = 2 * kDivTerms<DEG>;

// LD (a multiple of 8, at least the largest system's row count and NC5, at
// most 64 RPL) is the row stride of the matrix in dynamic LDS: sized to the mesh
// rather than to 64 RPL, it lets more blocks share a CU.  Rows i >= LD are
// never touched (they would be zero padding).
template <int RPL, int DEG>
__global__ void __launch_bounds__(64)
k_div_rows(int64_t nowned, int LD, const int64_t* __restrict__ vptr,
           const int64_t* __restrict__ eptr, const double* __restrict__ vpts,
           const double* __restrict__ mpts, const int32_t* __restrict__ sedge,
           const double* __restrict__ en, int64_t ne, const double* __restrict__ vh,
           double* __restrict__ dv, double* __restrict__ de,
           int32_t* __restrict__ status) {
  constexpr int NB5 = kDivTerms<DEG>, NC5 = kDivUnknowns<DEG>;
  extern __shared__ double div_lds[];
  double* A = div_lds;              // [NC5][LD]
  double* alpha = A + NC5 * LD;     // [NC5]
  double* vtvs = alpha + NC5;       // [NC5]
  double* yv = vtvs + NC5;          // [3][NC5]
  const int lane = threadIdx.x;
  const int64_t v = blockIdx.x;
  if (v >= nowned) return;
  const int64_t s0 = vptr[v], N = vptr[v + 1] - s0;
  const int64_t m0 = eptr[v], M = eptr[v + 1] - m0;
  const int m = int(2 * N + M);
  // ---- assemble (rows over lanes) ---------------------------------------------
  for (int rr = 0; rr < RPL; ++rr) {
    int i = lane + rr * 64;
    if (i >= LD) continue;
    double x = 0.0, y = 0.0, fa = 0.0, fb = 0.0;
    if (i < 2 * N) {
      int nd = i >> 1;
      x = vpts[2 * (s0 + nd)];
      y = vpts[2 * (s0 + nd) + 1];
      fa = (i & 1) ? 0.0 : 1.0;
      fb = (i & 1) ? 1.0 : 0.0;
    } else if (i < m) {
      int k = i - int(2 * N);
      x = mpts[2 * (m0 + k)];
      y = mpts[2 * (m0 + k) + 1];
      // the edge's unit direction (active-edge array, [2][ne])
      const int64_t je = sedge[m0 + k];
      fa = en[2 * je];
      fb = en[2 * je + 1];
    }
    for (int c = 0; c < NB5; ++c) {
      double p = (i < m) ? mono<DEG>(c, 0, x, y) : 0.0;
      A[c * LD + i] = p * fa;
      A[(NB5 + c) * LD + i] = p * fb;
    }
  }
  wave_sync();
  // ---- Householder QR: reflector v_j kept in column j, rows >= j -------------
  double dmax = 0.0;
  bool deficient = false;
  for (int j = 0; j < NC5; ++j) {
    double s2 = 0.0;
    for (int rr = 0; rr < RPL; ++rr) {
      int i = lane + rr * 64;
      double x = (i >= j && i < LD) ? A[j * LD + i] : 0.0;
      s2 += x * x;
    }
    s2 = gsum<64>(s2);
    double sig = sqrt(s2);
    double xj = A[j * LD + j];
    double al = (xj >= 0.0) ? -sig : sig;
    dmax = fmax(dmax, sig);
    if (sig == 0.0 || sig <= kRtol * dmax) deficient = true;
    double vtv = 2.0 * sig * (sig + fabs(xj));   // |x - al e_j|^2
    wave_sync();
    if (lane == (j % 64)) A[j * LD + j] = xj - al;
    if (lane == 0) { alpha[j] = al; vtvs[j] = vtv; }
    wave_sync();
    if (vtv > 0.0) {
      for (int c = j + 1; c < NC5; ++c) {
        double d = 0.0;
        for (int rr = 0; rr < RPL; ++rr) {
          int i = lane + rr * 64;
          if (i >= j && i < LD) d += A[j * LD + i] * A[c * LD + i];
        }
        d = gsum<64>(d);
        double f = 2.0 * d / vtv;
        for (int rr = 0; rr < RPL; ++rr) {
          int i = lane + rr * 64;
          if (i >= j && i < LD) A[c * LD + i] -= f * A[j * LD + i];
        }
      }
    }
    wave_sync();
  }
  if (deficient) {
    if (lane == 0) status[v] = 1;
    return;
  }
  // R[k][j] (k < j) is A[j][k], its diagonal alpha
  // three combinations of unknowns: (a_2 + b_3), (a_4 + b_5), (a_5 + b_6)
  // (1-based, a = f coefficients, b = g coefficients): y = R^-T e
  if (lane < 3) {
    const int ia = (lane == 0) ? 1 : (lane == 1 ? 3 : 4);
    const int ib = NB5 + ((lane == 0) ? 2 : (lane == 1 ? 4 : 5));
    double* y = yv + lane * NC5;
    for (int j = 0; j < NC5; ++j) {
      double s = (j == ia ? 1.0 : 0.0) + (j == ib ? 1.0 : 0.0);
      for (int k = 0; k < j; ++k) s -= A[j * LD + k] * y[k];
      y[j] = s / alpha[j];
    }
  }
  wave_sync();
  double z[3][RPL];
  for (int q = 0; q < 3; ++q)
    for (int rr = 0; rr < RPL; ++rr) {
      int i = lane + rr * 64;
      z[q][rr] = (i < NC5) ? yv[q * NC5 + i] : 0.0;
    }
  // z <- H_0 H_1 ... H_{n-1} [y; 0]
  for (int j = NC5 - 1; j >= 0; --j) {
    double vtv = vtvs[j];
    if (vtv == 0.0) continue;
    for (int q = 0; q < 3; ++q) {
      double d = 0.0;
      for (int rr = 0; rr < RPL; ++rr) {
        int i = lane + rr * 64;
        if (i >= j && i < m) d += A[j * LD + i] * z[q][rr];
      }
      d = gsum<64>(d);
      double f = 2.0 * d / vtv;
      for (int rr = 0; rr < RPL; ++rr) {
        int i = lane + rr * 64;
        if (i >= j && i < m) z[q][rr] -= f * A[j * LD + i];
      }
    }
  }
  const double h = vh[v];
  const double sc[3] = {1.0 / h, 1.0 / (h * h), 1.0 / (h * h)};
  // column i of the system -> (node, f|g) or edge slot
  for (int rr = 0; rr < RPL; ++rr) {
    int i = lane + rr * 64;
    if (i < 2 * N) {
      int nd = i >> 1, fg = i & 1;
      for (int q = 0; q < 3; ++q) dv[(s0 + nd) * 6 + 2 * q + fg] = z[q][rr] * sc[q];
    } else if (i < m) {
      int k = i - int(2 * N);
      for (int q = 0; q < 3; ++q) de[(m0 + k) * 3 + q] = z[q][rr] * sc[q];
    }
  }
  if (lane == 0) status[v] = 0;
}

// ---------------------------------------------------------------------------
// Viscous rows: one wavefront per owned vertex, SVD + graded pseudo-inverse.
// ---------------------------------------------------------------------------
struct VisLds {
  double A[15 * 64];
  double V[15 * 64];
  double KT[5 * 64];
  double Bt[5 * 64];
  double W[5 * 64];
  double out[5 * 64];
  double sig[16];
  double sb[8];
  int perm[16];
  int pb[8];
};

__global__ void __launch_bounds__(64)
k_visc_rows(int64_t nowned, const int64_t* __restrict__ vptr,
            const double* __restrict__ vpts, const double* __restrict__ vh,
            double* __restrict__ dvis, int32_t* __restrict__ status) {
  __shared__ VisLds L;
  const int lane = threadIdx.x;
  const int64_t v = blockIdx.x;
  if (v >= nowned) return;
  const int64_t s0 = vptr[v];
  const int N = int(vptr[v + 1] - s0);
  for (int c = 0; c < 15; ++c)
    L.A[c * 64 + lane] =
        (lane < N) ? mono<4>(c, 0, vpts[2 * (s0 + lane)], vpts[2 * (s0 + lane) + 1]) : 0.0;
  wave_sync();
  jacobi<64, 1>(L.A, L.V, N, 15, lane);
  sing_order<64, 1>(L.A, 15, lane, L.sig, L.perm);
  double smax = L.sig[L.perm[0]];
  int r = 0;
  for (int c = 0; c < 15; ++c) r += (L.sig[c] > kRtol * smax) ? 1 : 0;
  const int top[5] = {10, 11, 12, 13, 14};
  const int rows[5] = {1, 2, 3, 4, 5};
  GradedWs ws{L.KT, L.Bt, L.W, L.sb, L.pb};
  graded_rows<64, 1>(L.A, L.V, L.sig, L.perm, N, 15, r, top, 5, rows, 5, ws,
                     L.out, lane);
  const double h = vh[v];
  const double sc[5] = {1.0 / h, 1.0 / h, 1.0 / (h * h), 1.0 / (h * h), 1.0 / (h * h)};
  if (lane < N)
    for (int q = 0; q < 5; ++q) dvis[(s0 + lane) * 5 + q] = L.out[q * 64 + lane] * sc[q];
  if (lane == 0) status[v] = (r < 15) ? 2 : 0;
}

}  // namespace

hipError_t launch_edge_weights(int64_t ne, const double* pts, const double* eh,
                               double w3_cap, double* w5, double* w3,
                               int32_t* rank, int8_t* trunc3, double* w5g, double* w3g,
                               hipStream_t st) {
  if (ne == 0) return hipSuccess;
  int64_t blocks = (2 * ne + 3) / 4;
  hipLaunchKernelGGL(k_edge_weights, dim3(unsigned(blocks)), dim3(64), 0, st, ne,
                     pts, eh, w3_cap, w5, w3, rank, trunc3, w5g, w3g);
  return hipGetLastError();
}

hipError_t launch_div_rows(int64_t nowned, int msys, int deg, const int64_t* vptr,
                           const int64_t* eptr, const double* vpts,
                           const double* mpts, const int32_t* sedge,
                           const double* en, int64_t ne, const double* vh, double* dv,
                           double* de, int32_t* status, hipStream_t st) {
  if (nowned == 0) return hipSuccess;
  if (msys < 1 || msys > 192 || (deg != 4 && deg != 5)) return hipErrorInvalidValue;
  // at least NC rows, so that the diagonal A[j][j] (j < NC) lies in column j
  const int NC = deg == 5 ? kDivUnknowns<5> : kDivUnknowns<4>;
  const int LD = (std::max(msys, NC) + 7) / 8 * 8;
  const size_t lds = size_t(NC * LD + 5 * NC) * sizeof(double);
#define HFD_LAUNCH_DIV(R, D)                                                                \
  hipLaunchKernelGGL((k_div_rows<R, D>), dim3(unsigned(nowned)), dim3(64), lds, st, nowned, \
                     LD, vptr, eptr, vpts, mpts, sedge, en, ne, vh, dv, de, status)
  if (deg == 5) {
    if (LD <= 128) HFD_LAUNCH_DIV(2, 5);
    else HFD_LAUNCH_DIV(3, 5);
  } else {
    if (LD <= 128) HFD_LAUNCH_DIV(2, 4);
    else HFD_LAUNCH_DIV(3, 4);
  }
#undef HFD_LAUNCH_DIV
  return hipGetLastError();
}

hipError_t launch_visc_rows(int64_t nowned, const int64_t* vptr,
                            const double* vpts, const double* vh, double* dvis,
                            int32_t* status, hipStream_t st) {
  if (nowned == 0) return hipSuccess;
  hipLaunchKernelGGL(k_visc_rows, dim3(unsigned(nowned)), dim3(64), 0, st,
                     nowned, vptr, vpts, vh, dvis, status);
  return hipGetLastError();
}

}  // namespace hfd
