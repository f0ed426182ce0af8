// reduce.hip -- per-cell kernels outside the axis passes:
//   * signal-speed maximum for the CFL time step (two fixed-shape passes:
//     per-block maxima, then one block that also forms dt on the device);
//   * conservation sums (fixed reduction tree, so results are reproducible);
//   * primitive <-> conservative conversion of whole fields.
// All of these are HBM-bound streams over the state; each block walks one
// contiguous chunk of cells so that every load is a coalesced run.
#include "device.h"
#include "internal.h"

namespace mfc {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int NF, int D, typename Real>
__global__ __launch_bounds__(kReduceThreads) void max_signal_partial(Params pm, const Real* __restrict__ q,
                                                                     double* __restrict__ partial,
                                                                     int* __restrict__ flag) {
  using R = Rows<NF, D>;
  constexpr int NEQ = R::NEQ;
  const long long nc = pm.ncell;
  const long long chunk = (nc + gridDim.x - 1) / gridDim.x;
  const long long beg = (long long)blockIdx.x * chunk;
  const long long end = (beg + chunk < nc) ? beg + chunk : nc;
  double smax = 0.0;
  bool bad = false;
  for (long long c = beg + threadIdx.x; c < end; c += blockDim.x) {
    double U[NEQ], W[NEQ];
#pragma unroll
    for (int v = 0; v < NEQ; ++v) U[v] = double(q[v * nc + c]);
    cons_to_prim<NF, D>(pm, U, W);
    // 1/h per axis of this cell (tabulated on a non-uniform grid)
    const long long nx = pm.n[0], ny = pm.n[1];
    const int idx[3] = {(int)(c % nx), (int)((c / nx) % ny), (int)(c / (nx * ny))};
    double ih[D];
#pragma unroll
    for (int d = 0; d < D; ++d) ih[d] = inv_width(pm, d, idx[d]);
    bool b;
    const double s = cell_signal<NF, D>(pm, U, W, b, ih);
    bad |= b;
    smax = (s > smax) ? s : smax;  // NaN never wins; it is flagged instead
  }
  if (bad) atomicOr(flag, 1);
  __shared__ double red[kReduceThreads / 64];
  smax = wave_max(smax);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = smax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < kReduceThreads / 64; ++w) m = fmax(m, red[w]);
    partial[blockIdx.x] = m;
  }
}

__global__ __launch_bounds__(kReduceThreads) void finalize_dt(const double* __restrict__ partial, int nparts,
                                                              double cfl, double t_remaining,
                                                              double* __restrict__ smax_out,
                                                              double* __restrict__ dt_out,
                                                              double* __restrict__ dt_user) {
  // eight independent running maxima per thread keep eight loads in flight
  // (max is exact, so the order of the partials does not matter)
  double mk[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int bd = blockDim.x;
  int i = threadIdx.x;
  for (; i + 7 * bd < nparts; i += 8 * bd) {
#pragma unroll
    for (int k = 0; k < 8; ++k) mk[k] = fmax(mk[k], partial[i + k * bd]);
  }
  for (; i < nparts; i += bd) mk[0] = fmax(mk[0], partial[i]);
  double m = fmax(fmax(fmax(mk[0], mk[1]), fmax(mk[2], mk[3])), fmax(fmax(mk[4], mk[5]), fmax(mk[6], mk[7])));
  __shared__ double red[kReduceThreads / 64];
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kReduceThreads / 64; ++w) m = fmax(m, red[w]);
    m = fmax(m, red[0]);
    if (smax_out) *smax_out = m;
    if (cfl > 0.0) {
      double dt = cfl / m;
      if (t_remaining > 0.0 && dt > t_remaining) dt = t_remaining;
      if (dt_out) *dt_out = dt;
      if (dt_user) *dt_user = dt;
    }
  }
}

hipError_t launch_finalize_dt(const double* partial, int nparts, double cfl, double t_remaining, double* smax_out,
                              double* dt_out, double* dt_user, hipStream_t s) {
  hipLaunchKernelGGL(finalize_dt, dim3(1), dim3(kReduceThreads), 0, s, partial, nparts, cfl, t_remaining, smax_out,
                     dt_out, dt_user);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_max_signal(int nf, int ndim, const Params& pm, const Real* q, double* partial,
                             double* smax_out, double cfl, double t_remaining, double* dt_out,
                             double* dt_user, int* flag, hipStream_t s) {
  dim3 grid(kReduceBlocks), block(kReduceThreads);
#define MFC_CASE(NF, D)                                                                          \
  if (nf == NF && ndim == D) {                                                                   \
    hipLaunchKernelGGL((max_signal_partial<NF, D, Real>), grid, block, 0, s, pm, q, partial, flag); \
  } else
  MFC_CASE(1, 1) MFC_CASE(1, 2) MFC_CASE(1, 3) MFC_CASE(2, 1) MFC_CASE(2, 2) MFC_CASE(2, 3) {
    return hipErrorInvalidValue;
  }
#undef MFC_CASE
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(finalize_dt, dim3(1), block, 0, s, partial, kReduceBlocks, cfl, t_remaining, smax_out,
                     dt_out, dt_user);
  return hipGetLastError();
}

// Block sums of each row; on a non-uniform grid (NU) every cell is weighted by
// its own volume h_x h_y h_z (the finalize pass then scales by 1).
template <typename Real, bool NU>
__global__ __launch_bounds__(kReduceThreads) void sums_partial(Params pm, int neq, long long nc,
                                                               const Real* __restrict__ q,
                                                               double* __restrict__ partial) {
  const long long chunk = (nc + gridDim.x - 1) / gridDim.x;
  const long long beg = (long long)blockIdx.x * chunk;
  const long long end = (beg + chunk < nc) ? beg + chunk : nc;
  __shared__ double red[kReduceThreads / 64];
  for (int v = 0; v < neq; ++v) {
    double acc = 0.0;
    for (long long c = beg + threadIdx.x; c < end; c += blockDim.x) {
      if constexpr (NU) {
        const long long nx = pm.n[0], ny = pm.n[1];
        const double w = (1.0 / inv_width(pm, 0, (int)(c % nx))) * (1.0 / inv_width(pm, 1, (int)((c / nx) % ny))) *
                         (1.0 / inv_width(pm, 2, (int)(c / (nx * ny))));
        acc += double(q[v * nc + c]) * w;
      } else {
        acc += double(q[v * nc + c]);
      }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = red[0];
      for (int w = 1; w < kReduceThreads / 64; ++w) t += red[w];
      partial[(long long)v * gridDim.x + blockIdx.x] = t;
    }
    __syncthreads();
  }
}

__global__ void sums_finalize(int neq, int nparts, double vol, const double* __restrict__ partial,
                              double* __restrict__ out) {
  const int v = threadIdx.x;
  if (v >= neq) return;
  double t = 0.0;
  for (int i = 0; i < nparts; ++i) t += partial[(long long)v * nparts + i];
  out[v] = t * vol;
}

template <typename Real>
hipError_t launch_sums(int neq, const Params& pm, const Real* q, double vol, double* partial, double* sums_out,
                       hipStream_t s) {
  const bool nu = pm.nu[0] || pm.nu[1] || pm.nu[2];
  if (nu)
    hipLaunchKernelGGL((sums_partial<Real, true>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, pm, neq,
                       pm.ncell, q, partial);
  else
    hipLaunchKernelGGL((sums_partial<Real, false>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, pm, neq,
                       pm.ncell, q, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sums_finalize, dim3(1), dim3(64), 0, s, neq, kReduceBlocks, nu ? 1.0 : vol, partial, sums_out);
  return hipGetLastError();
}

// Field conversions (Sec. 2.1.1 mixture rules, Sec. 2.2 EOS), in double.
template <int NF, int D, typename Real, bool TO_CONS>
__global__ __launch_bounds__(256) void convert_kernel(Params pm, const Real* __restrict__ in,
                                                      Real* __restrict__ out) {
  using R = Rows<NF, D>;
  constexpr int NEQ = R::NEQ;
  const long long nc = pm.ncell;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < nc;
       c += (long long)gridDim.x * blockDim.x) {
    double X[NEQ], Y[NEQ];
#pragma unroll
    for (int v = 0; v < NEQ; ++v) X[v] = double(in[v * nc + c]);
    if constexpr (TO_CONS) {
      prim_to_cons<NF, D>(pm, X, Y);
    } else {
      cons_to_prim<NF, D>(pm, X, Y);
    }
#pragma unroll
    for (int v = 0; v < NEQ; ++v) out[v * nc + c] = Real(Y[v]);
  }
}

template <typename Real>
hipError_t launch_convert(int nf, int ndim, bool to_cons, const Params& pm, const Real* in, Real* out,
                          hipStream_t s) {
  long long nb = (pm.ncell + 255) / 256;
  if (nb > 65536) nb = 65536;
  dim3 grid((unsigned)nb), block(256);
#define MFC_CASE(NF, D)                                                                                  \
  if (nf == NF && ndim == D) {                                                                           \
    if (to_cons)                                                                                         \
      hipLaunchKernelGGL((convert_kernel<NF, D, Real, true>), grid, block, 0, s, pm, in, out);           \
    else                                                                                                 \
      hipLaunchKernelGGL((convert_kernel<NF, D, Real, false>), grid, block, 0, s, pm, in, out);          \
  } else
  MFC_CASE(1, 1) MFC_CASE(1, 2) MFC_CASE(1, 3) MFC_CASE(2, 1) MFC_CASE(2, 2) MFC_CASE(2, 3) {
    return hipErrorInvalidValue;
  }
#undef MFC_CASE
  return hipGetLastError();
}

__global__ void set_scalar_kernel(double* dst, double value) { *dst = value; }

hipError_t launch_set_scalar(double* dst, double value, hipStream_t s) {
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, s, dst, value);
  return hipGetLastError();
}

template hipError_t launch_max_signal<double>(int, int, const Params&, const double*, double*, double*, double,
                                              double, double*, double*, int*, hipStream_t);
template hipError_t launch_max_signal<float>(int, int, const Params&, const float*, double*, double*, double,
                                             double, double*, double*, int*, hipStream_t);
template hipError_t launch_sums<double>(int, const Params&, const double*, double, double*, double*, hipStream_t);
template hipError_t launch_sums<float>(int, const Params&, const float*, double, double*, double*, hipStream_t);
template hipError_t launch_convert<double>(int, int, bool, const Params&, const double*, double*, hipStream_t);
template hipError_t launch_convert<float>(int, int, bool, const Params&, const float*, float*, hipStream_t);

}  // namespace mfc
