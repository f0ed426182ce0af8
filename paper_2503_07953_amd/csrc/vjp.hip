// vjp.hip -- dispatch of the RHS adjoint over the reconstruction variants
// (vjp_wv*.hip), and the adjoints of the field conversions and of the SSP-RK3
// stage combinations.
#include "vjp_impl.h"

namespace mfc {

MFC_EXTERN_VJP(0)
MFC_EXTERN_VJP(1)
MFC_EXTERN_VJP(2)
MFC_EXTERN_VJP(3)
MFC_EXTERN_VJP(4)

hipError_t launch_rhs_vjp(int nf, int ndim, const Params& pm, const double* q, const double* rbar, double* qbar,
                          const VjpScratch& sc, bool accumulate, hipStream_t s, PassTimer* tm, const StageEpi* epi) {
  StageEpi none{0, 0.0, nullptr, nullptr, nullptr};
  const StageEpi& ep = (epi && sc.all_axes) ? *epi : none;
  if (pm.nu[0] || pm.nu[1] || pm.nu[2])
    return launch_rhs_vjp_wv<kWvNonUniform>(nf, ndim, pm, q, rbar, qbar, sc, accumulate, s, tm, ep);
  switch (pm.weno_variant) {
    case 1: return launch_rhs_vjp_wv<1>(nf, ndim, pm, q, rbar, qbar, sc, accumulate, s, tm, ep);
    case 2: return launch_rhs_vjp_wv<2>(nf, ndim, pm, q, rbar, qbar, sc, accumulate, s, tm, ep);
    case 3: return launch_rhs_vjp_wv<3>(nf, ndim, pm, q, rbar, qbar, sc, accumulate, s, tm, ep);
    default: return launch_rhs_vjp_wv<0>(nf, ndim, pm, q, rbar, qbar, sc, accumulate, s, tm, ep);
  }
}

// ---------------------------------------------------------------------------
// per-cell conversions' adjoints
// ---------------------------------------------------------------------------
template <int NF, int D, bool TO_CONS>
__global__ __launch_bounds__(256) void convert_vjp_kernel(Params pm, const double* __restrict__ x,
                                                          const double* __restrict__ ybar, double* __restrict__ xbar,
                                                          int accumulate) {
  using R = Rows<NF, D>;
  constexpr int NEQ = R::NEQ;
  const long long nc = pm.ncell;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (long long)gridDim.x * blockDim.x) {
    double X[NEQ], Yb[NEQ], Xb[NEQ];
#pragma unroll
    for (int v = 0; v < NEQ; ++v) {
      X[v] = x[v * nc + c];
      Yb[v] = ybar[v * nc + c];
      Xb[v] = 0.0;
    }
    if constexpr (TO_CONS)
      prim_to_cons_vjp<NF, D>(pm, X, Yb, Xb);
    else
      cons_to_prim_vjp<NF, D>(pm, X, Yb, Xb);
#pragma unroll
    for (int v = 0; v < NEQ; ++v) {
      const long long e = v * nc + c;
      xbar[e] = accumulate ? xbar[e] + Xb[v] : Xb[v];
    }
  }
}

hipError_t launch_convert_vjp(int nf, int ndim, bool to_cons, const Params& pm, const double* x, const double* ybar,
                              double* xbar, bool accumulate, hipStream_t s) {
  long long nb = (pm.ncell + 255) / 256;
  if (nb > 65536) nb = 65536;
  dim3 grid((unsigned)nb), block(256);
  const int acc = accumulate ? 1 : 0;
#define MFC_CASE(NF, D)                                                                                       \
  if (nf == NF && ndim == D) {                                                                                \
    if (to_cons)                                                                                              \
      hipLaunchKernelGGL((convert_vjp_kernel<NF, D, true>), grid, block, 0, s, pm, x, ybar, xbar, acc);       \
    else                                                                                                      \
      hipLaunchKernelGGL((convert_vjp_kernel<NF, D, false>), grid, block, 0, s, pm, x, ybar, xbar, acc);      \
    return hipGetLastError();                                                                                 \
  }
  MFC_CASE(1, 1)
  MFC_CASE(1, 2)
  MFC_CASE(1, 3)
  MFC_CASE(2, 1)
  MFC_CASE(2, 2)
  MFC_CASE(2, 3)
#undef MFC_CASE
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// reverse SSP-RK3 combinations (Shu-Osher form)
//   qbar2 = 2/3 (qbar3 + dt v3),  qbarn  = 1/3 qbar3          (v3 = L^T(q2) qbar3)
//   qbar1 = 1/4 (qbar2 + dt v2),  qbarn += 3/4 qbar2          (v2 = L^T(q1) qbar2)
//   qbarn += qbar1 + dt v1                                    (v1 = L^T(qn) qbar1)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void adj_stage3_kernel(long long n, double dt, const double* __restrict__ a,
                                                         const double* __restrict__ v, double* __restrict__ b2,
                                                         double* __restrict__ qnb) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const double x = a[e];
    b2[e] = (2.0 / 3.0) * (x + dt * v[e]);
    qnb[e] = (1.0 / 3.0) * x;
  }
}
__global__ __launch_bounds__(256) void adj_stage2_kernel(long long n, double dt, const double* __restrict__ b2,
                                                         const double* __restrict__ v, double* __restrict__ b1,
                                                         double* __restrict__ qnb) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const double x = b2[e];
    b1[e] = 0.25 * (x + dt * v[e]);
    qnb[e] = qnb[e] + 0.75 * x;
  }
}
__global__ __launch_bounds__(256) void adj_stage1_kernel(long long n, double dt, const double* __restrict__ b1,
                                                         const double* __restrict__ v, double* __restrict__ qnb) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    qnb[e] = qnb[e] + (b1[e] + dt * v[e]);
}

hipError_t launch_adj_stage(int which, long long n, double dt, const double* x, const double* v, double* out,
                            double* qnb, hipStream_t s) {
  long long nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  dim3 grid((unsigned)nb), block(256);
  if (which == 3)
    hipLaunchKernelGGL(adj_stage3_kernel, grid, block, 0, s, n, dt, x, v, out, qnb);
  else if (which == 2)
    hipLaunchKernelGGL(adj_stage2_kernel, grid, block, 0, s, n, dt, x, v, out, qnb);
  else
    hipLaunchKernelGGL(adj_stage1_kernel, grid, block, 0, s, n, dt, x, v, qnb);
  return hipGetLastError();
}

}  // namespace mfc
