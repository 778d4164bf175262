// Launchers of the HIP kernels (internal to libhfd).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/hfd.h"

namespace hfd {

// Switch mode of the edge kernels when a forced mask gives the decisions
// (beside the hfd_switch values, which are the other modes).
constexpr int kSwForced = 3;

// ---- lane primitives (device) -----------------------------------------------
// Lane exchange through DPP (a VALU move, no LDS traffic).  0x140 mirrors a
// row of 16 lanes (the partner differs in bit 3 of the lane index), 0x141
// mirrors each half row (bit 2), the quad permutations 0x4E and 0xB1 swap
// lanes differing in bit 1 and in bit 0.
template <int CTRL>
__device__ inline float dpp_mov(float x) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_mov(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(uint32_t(b)), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(uint32_t(b >> 32)), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, uint64_t(uint32_t(lo)) | (uint64_t(uint32_t(hi)) << 32));
}

// One stage of the transposed lane reduction: of its N values the lane keeps
// the half selected by bit B of its index and adds the partner's copy of that
// half.  The four partner maps above pair disjoint lane sets at every stage,
// so after the stages for bits log2(VL)-1 .. 0 each value is a sum over all
// VL lanes, and lane `sub` holds accumulators (16/VL) sub + i.
template <int B, int N, class T>
__device__ inline void reduce_stage(T* a, int sub) {
  constexpr int CTRL = B == 3 ? 0x140 : B == 2 ? 0x141 : B == 1 ? 0x4E : 0xB1;
  const bool hi = (sub >> B) & 1;
#pragma unroll
  for (int j = 0; j < N / 2; ++j) {
    const T send = hi ? a[j] : a[N / 2 + j];
    const T keep = hi ? a[N / 2 + j] : a[j];
    a[j] = keep + dpp_mov<CTRL>(send);
  }
}

// ---- geometric precompute (float64) ----------------------------------------
// w5g, w3g: null, or the midpoint-derivative rows [2][2][15][ne], [2][3][2][3][ne]
hipError_t launch_edge_weights(int64_t ne, const double* pts, const double* eh,
                               double w3_cap, double* w5, double* w3,
                               int32_t* rank, int8_t* trunc3, double* w5g, double* w3g,
                               hipStream_t st);
// msys: the largest system's row count over the owned vertices (1..192);
// deg: degree of the fit (4 or 5)
hipError_t launch_div_rows(int64_t nowned, int msys, int deg, const int64_t* vptr,
                           const int64_t* eptr, const double* vpts,
                           const double* mpts, const int32_t* sedge,
                           const double* en, int64_t ne, const double* vh, double* dv,
                           double* de, int32_t* status, hipStream_t st);
hipError_t launch_visc_rows(int64_t nowned, const int64_t* vptr,
                            const double* vpts, const double* vh, double* dvis,
                            int32_t* status, hipStream_t st);

// ---- hot path ------------------------------------------------------------------
struct GasParams {
  double gamma, gas_R, mu, prandtl;
  double eps, sw_lo, sw_hi;
  double wref[4];   // FP32 form: reference state (zero in the FP64 form)
  double uref, vref, etr_ref;  // its velocity and E + p (set with wref)
  int sw;           // hfd_switch
  int flux;         // hfd_flux
  // the same values rounded to float once on the host: the float32 kernels
  // read these instead of converting on the vector ALUs
  float f_gamma, f_gm1, f_eps, f_sw_lo, f_sw_hi;
  float f_wref[4], f_uref, f_vref, f_etr_ref;
};

// Coefficients of the edge kernel, one precision.
template <class T>
struct EdgeCoef {
  const int32_t* stg;   // [6][ne] gather rows
  const T* n;           // [ne][2]: unit direction (one load per edge)
  const T* w5;          // [2][ne][15]: per side and edge its 15 Hermite weights
  const T* w3;          // [2][ne][9]: per side and edge its three 3-node rows
  // staging lists of the two-lane edge kernel (null: gathers from HBM): per
  // block of kEdgeStageEdges edges the sorted distinct stencil rows
  // (erow[erp[b] .. erp[b+1])), per stencil node its position in that list
  const int32_t* erp = nullptr;
  const int32_t* erow = nullptr;
  const uint16_t* epos = nullptr;  // [6][ne]
  int max_rows = 0;                // longest list
};
constexpr int kEdgeStageEdges = 128;

template <class T>
struct VertexCoef {
  const int32_t* vptr;     // [n_owned+1] (int32 slot offsets)
  const int32_t* eptr;     // [n_owned+1]
  const int32_t* vg;       // [n_vslots] gather rows
  const int32_t* ve;       // [n_eslots] edge index
  const T* dv;             // [n_vslots][6]
  const T* de;             // [n_eslots][3]
  const T* dvis;           // [n_vslots][5] or null
  // Staging of a block's neighbour data in LDS (idx_bytes 1 or 2; 0 = every
  // slot gathers from HBM through vg/ve).  Per block of 16
  // owned vertices: its distinct gather rows hrow[hrp[b] .. hrp[b+1]) and
  // distinct edges hedge[hep[b] .. hep[b+1]), sorted.  A slot's row (edge)
  // is at position base + vloc[slot] (eloc) of its block's list, where
  // lbase[v] = row base | edge base << 16 is the first position among v's
  // slots; vloc/eloc take idx_bytes bytes.
  const int32_t* hrp;      // [n_blocks+1]
  const int32_t* hrow;
  const int32_t* hep;      // [n_blocks+1]
  const int32_t* hedge;
  const uint32_t* lbase;   // [n_owned]
  const void* vloc;        // [n_vslots]
  const void* eloc;        // [n_eslots]
  int idx_bytes;
  int max_rows, max_edges; // longest lists (LDS size)
};

// Owned vertices per block of the vertex pass when its neighbour data is
// staged in LDS.
constexpr int kStageVertices = 16;

// Gather layout of a stage state: values Gv[nv] and gradients Gg[2 nv]
// (x then y) as 4-vectors, so that one vertex's data is one or two
// contiguous 16/32-byte loads.  In the mixed form it holds w - w_ref.
template <class T>
struct alignas(4 * sizeof(T)) V4 {
  T x, y, z, w;
};

// Edge pass: H[ne] (4 components per edge), optional float64 copies
// hsoa[4][ne], states wlr[8][ne] and WENO mask.
template <class T>
hipError_t launch_edge(int64_t ne, const EdgeCoef<T>& c, const GasParams& gp,
                       const V4<T>* Gv, const V4<T>* Gg, const uint8_t* force, V4<T>* H,
                       double* hsoa, double* wlr, uint8_t* mask, hipStream_t st);

// Midpoint derivatives of both sides of every edge, grad[16][ne] float64
// (row 8 side + 4 d + q: d/dx (d = 0) or d/dy of component q), with the
// branches recorded in mask (written by launch_edge before).
template <class T>
hipError_t launch_edge_grad(int64_t ne, const EdgeCoef<T>& c, const double* w5g,
                            const double* w3g, const GasParams& gp, const V4<T>* Gv,
                            const V4<T>* Gg, const uint8_t* mask, double* grad,
                            hipStream_t st);
// Vertex pass.  mode 0: dU = R (float64 rows [12][nv], owned vertices);
// mode 1: Unew = a*Un + b*(Uk + dt*R) in float64 (dt from dt_dev when
// non-null), plus the gather-layout copy of Unew when Gv_new is non-null.
struct RkArgs {
  const double* Un;
  const double* Uk;
  double* Unew;
  double a, b, dt;
  const double* dt_dev;
};
template <class T>
hipError_t launch_vertex(int64_t nowned, int64_t nv, const VertexCoef<T>& c,
                         const GasParams& gp, const V4<T>* Gv, const V4<T>* Gg,
                         const V4<T>* H, int mode, double* dU, const RkArgs& rk,
                         V4<T>* Gv_new, V4<T>* Gg_new, int32_t* flag, hipStream_t st);

template <class T>
hipError_t launch_to_gather(int64_t nv, const double* U, const GasParams& gp, V4<T>* Gv,
                            V4<T>* Gg, hipStream_t st);
template <class T>
hipError_t launch_copy_gather_rows(int64_t nrows, const int32_t* rows, const V4<T>* fv,
                                   const V4<T>* fg, V4<T>* tv, V4<T>* tg, hipStream_t st);

// Ghost rows and helpers.
template <class T>
hipError_t launch_copy_rows(int64_t nrows, const int32_t* rows, const int32_t* src,
                            int64_t nv, const T* from, T* to, hipStream_t st);
hipError_t launch_zero_ghost_rows(int64_t nowned, int64_t nv, double* dU,
                                  hipStream_t st);
hipError_t launch_stable_dt(int64_t nowned, int64_t nv, const double* U,
                            const double* hmin, double gamma, double cfl,
                            double* partial, int64_t npartial, double* dt,
                            hipStream_t st);
hipError_t launch_cast(int64_t n, const double* a, float* b, hipStream_t st);
hipError_t launch_widen(int64_t n, const float* a, double* b, hipStream_t st);

// ---- adjoint (float64, Euler) ---------------------------------------------------
// Runge-Kutta combination fused into the adjoint's vertex pass, owned rows
// o (x = (J^T lam)[o]): nxt = ca lam_k + cb x, also written in gather layout
// (nGv, nGg, the lambda of the next stage); acc = cc acc + cd lam_k + ce x
// (acc not read when cc == 0).  lam_k == null: nothing.
template <class T>
struct AdjCombine {
  const double* lam_k;
  double* nxt;
  V4<T>* nGv;
  V4<T>* nGg;
  double* acc;
  double ca, cb, cc, cd, ce;
};

// edges per block of the edge reverse (two lanes each: 256 threads)
constexpr int kAdjEdgesPerBlock = 128;
// longest staging list of the edge reverse: the lambda rows of that many
// vertices fit in the LDS of the block's output rows
constexpr int kAdjStageRows = 256;

template <class T>
struct AdjointArgs {
  int64_t ne, nowned, nv;
  const int32_t *etp, *etv;         // edge m <- (owner vertex, edge slot)
  const T* de_t;                    // de rows in the order of etv
  // staging lists of the edge reverse (null: lambda gathered from HBM): per
  // block of kAdjEdgesPerBlock edges the sorted distinct vertices of its
  // entries (lrow[lrp[b] .. lrp[b+1]), at most kAdjStageRows), per entry
  // (order of etv) its position in that list
  const int32_t* lrp;
  const int32_t* lrow;
  const uint16_t* lpos;
  const V4<T>* Lv;                  // lambda in gather layout
  const V4<T>* Lg;
  EdgeCoef<T> ec;
  GasParams gp;                     // float32: with the reference state of Gv
  const V4<T>* Gv;                  // state in gather layout
  const V4<T>* Gg;
  const uint8_t* force;
  T* bnode;                         // [ne][6][12] edge-pass contributions
  const double* U;                  // state [12][nv]
  const int32_t *vtp, *vtv;         // gather row <- (owner vertex, vertex slot)
  const T* dv_t;                    // dv rows in the order of vtv
  const T* dvis_t;                  // dvis rows in the order of vtv (null: mu == 0)
  const int32_t *ntp, *nte;         // gather row <- (edge, stencil position)
  const int8_t* ntj;
  double* out;                      // [12][nv], owned rows written, or null
  AdjCombine<T> rc;
};
template <class T>
hipError_t launch_adjoint_residual(const AdjointArgs<T>& a, hipStream_t st);
// Gather layouts of a step's input and two stages in one launch; the
// Dirichlet rows [d0, d1) of the stages come from U.
template <class T>
struct StageGathers {
  V4<T>* v[3];
  V4<T>* g[3];
};
template <class T>
hipError_t launch_stage_gathers(int64_t nv, int64_t d0, int64_t d1, const double* U,
                                const double* U1, const double* U2, const GasParams& gp,
                                const StageGathers<T>& g, hipStream_t st);
// dst[i][0..w) = src[idx[i]][0..w), i < n (transposed coefficient copies)
hipError_t launch_take_rows(int64_t n, int w, const int32_t* idx, const double* src,
                            double* dst, hipStream_t st);

// out[i] = a x[i] + b y[i] (+ c z[i] if z), i < n
hipError_t launch_axpbypcz(int64_t n, double a, const double* x, double b, const double* y,
                           double c, const double* z, double* out, hipStream_t st);
// lambda of a step's final ghost fill: src rows gather their copies, the
// copies' rows are cleared
hipError_t launch_adj_copy_ghosts(int64_t nsrc, const int32_t* sptr, const int32_t* srows,
                                  const int32_t* gsts, int64_t nv, double* lam,
                                  hipStream_t st);

}  // namespace hfd
