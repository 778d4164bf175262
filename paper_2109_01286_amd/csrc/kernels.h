// Launchers of the HIP kernels (internal to libhfd).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/hfd.h"

namespace hfd {

// ---- geometric precompute (float64) ----------------------------------------
hipError_t launch_edge_weights(int64_t ne, const double* pts, const double* eh,
                               double w3_cap, double* w5, double* w3,
                               int32_t* rank, int8_t* trunc3, hipStream_t st);
hipError_t launch_div_rows(int64_t nowned, int rpl, const int64_t* vptr,
                           const int64_t* eptr, const double* vpts,
                           const double* mpts, const double* mnrm,
                           const double* vh, double* dv, double* de,
                           int32_t* status, hipStream_t st);
hipError_t launch_visc_rows(int64_t nowned, const int64_t* vptr,
                            const double* vpts, const double* vh, double* dvis,
                            int32_t* status, hipStream_t st);

// ---- hot path ------------------------------------------------------------------
struct GasParams {
  double gamma, gas_R, mu, prandtl;
  double eps, sw_lo, sw_hi;
  double wref[4];   // FP32 form: reference state (zero in the FP64 form)
  int sw;           // hfd_switch
};

// Coefficients of the edge kernel, one precision.
template <class T>
struct EdgeCoef {
  const int32_t* stg;   // [6][ne] gather rows
  const T* n;           // [2][ne]
  const T* w5;          // [2][15][ne]
  const T* w3;          // [2][3][3][ne]
};

template <class T>
struct VertexCoef {
  const int32_t* vptr;     // [n_owned+1] (int32 slot offsets)
  const int32_t* eptr;     // [n_owned+1]
  const int32_t* vg;       // [n_vslots] gather rows
  const int32_t* ve;       // [n_eslots] edge index
  const T* dv;             // [n_vslots][6]
  const T* de;             // [n_eslots][3]
  const T* dvis;           // [n_vslots][5] or null
};

// Edge pass: H[4][ne] (and optional states / mask).  U is float64 in the FP64
// form (Us = null) or the float32 perturbation state in the mixed form.
hipError_t launch_edge64(int64_t ne, int64_t nv, const EdgeCoef<double>& c,
                         const GasParams& gp, const double* U,
                         const uint8_t* force, double* H, double* wlr,
                         uint8_t* mask, hipStream_t st);
hipError_t launch_edge32(int64_t ne, int64_t nv, const EdgeCoef<float>& c,
                         const GasParams& gp, const float* Us,
                         const uint8_t* force, float* H, double* wlr,
                         uint8_t* mask, hipStream_t st);

// Vertex pass.  mode 0: dU = R (float64 rows, owned vertices);
// mode 1: Unew = a*Un + b*(Uk + dt*R) in float64, plus the float32 shadow
// (mixed form).  dt is read from dt_dev when non-null.
struct RkArgs {
  const double* Un;
  const double* Uk;
  double* Unew;
  float* Us_new;       // mixed form: float32 perturbation shadow of Unew
  double a, b, dt;
  const double* dt_dev;
};
hipError_t launch_vertex64(int64_t nowned, int64_t nv, const VertexCoef<double>& c,
                           const GasParams& gp, const double* U, const double* H,
                           int64_t ne, int mode, double* dU, const RkArgs& rk,
                           int32_t* flag, hipStream_t st);
hipError_t launch_vertex32(int64_t nowned, int64_t nv, const VertexCoef<float>& c,
                           const GasParams& gp, const float* Us, const float* H,
                           int64_t ne, int mode, double* dU, const RkArgs& rk,
                           int32_t* flag, hipStream_t st);

// Ghost rows and helpers.
template <class T>
hipError_t launch_copy_rows(int64_t nrows, const int32_t* rows, const int32_t* src,
                            int64_t nv, const T* from, T* to, hipStream_t st);
hipError_t launch_to_shadow(int64_t nv, const double* U, const GasParams& gp,
                            float* Us, hipStream_t st);
hipError_t launch_zero_ghost_rows(int64_t nowned, int64_t nv, double* dU,
                                  hipStream_t st);
hipError_t launch_stable_dt(int64_t nowned, int64_t nv, const double* U,
                            const double* hmin, double gamma, double cfl,
                            double* partial, int64_t npartial, double* dt,
                            hipStream_t st);
hipError_t launch_cast(int64_t n, const double* a, float* b, hipStream_t st);
hipError_t launch_widen(int64_t n, const float* a, double* b, hipStream_t st);

}  // namespace hfd
