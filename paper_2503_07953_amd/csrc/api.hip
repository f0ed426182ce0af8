// api.hip -- the C ABI declared in include/mfc355.h: problem validation,
// context and scratch ownership, argument checks, and the launch sequences of
// the right-hand side, the SSP-RK3 step and the diagnostics.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <mutex>
#include <utility>
#include <string>
#include <vector>

#include "../../include/mfc355.h"
#include "device.h"
#include "internal.h"

// Event pairs around every launch of an entry point (diagnostics).
struct EventTimer : mfc::PassTimer {
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  hipEvent_t pending = nullptr;
  hipError_t err = hipSuccess;

  hipEvent_t get() {
    if (used < pool.size()) return pool[used++];
    hipEvent_t e = nullptr;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      err = r;
      return nullptr;
    }
    pool.push_back(e);
    ++used;
    return e;
  }
  void begin(int, hipStream_t s) override {
    pending = get();
    if (pending) (void)hipEventRecord(pending, s);
  }
  void end(int kind, hipStream_t s) override {
    hipEvent_t e = get();
    if (!e || !pending) return;
    (void)hipEventRecord(e, s);
    recs.push_back({kind, pending, e});
    pending = nullptr;
  }
  hipError_t collect(double* ms, int64_t* cnt) {
    for (int k = 0; k < mfc::KIND_COUNT; ++k) {
      ms[k] = 0.0;
      cnt[k] = 0;
    }
    hipError_t r = err;
    for (const Rec& x : recs) {
      hipError_t e = hipEventSynchronize(x.b);
      float t = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, x.a, x.b);
      if (e != hipSuccess) {
        r = e;
        continue;
      }
      ms[x.kind] += t;
      cnt[x.kind] += 1;
    }
    recs.clear();
    used = 0;
    err = hipSuccess;
    return r;
  }
  ~EventTimer() override {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

struct mfc_ctx {
  mfc_problem prob;
  mfc::Params pm;
  int neq;
  long long ncell;
  size_t esize;       // bytes per element of q
  void* acc;          // RHS accumulator (neq*ncell elements)
  void* q1;           // stage state 1
  void* q2;           // stage state 2
  double* scal;       // [0] smax, [1] dt
  double* partial;    // reduction partials (see partial_len)
  int* flag;          // non-finite flag
  int device;
  std::string err;
  EventTimer* timer;  // non-null while timing is enabled
  // adjoint scratch (allocated on the first adjoint call)
  mfc::VjpScratch vjp;
  double* vbuf;       // L^T v
  double* b1;         // stage cotangents
  double* b2;
  // non-uniform grid (mfc_set_grid): face coordinates per axis (empty:
  // uniform spacing dx) and the device coefficient tables of every active axis
  std::vector<double> faces[3];
  double* nu_d[3];
  float* nu_f[3];
};

namespace {

int fail(mfc_ctx* c, int code, const char* msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(mfc_ctx* c, hipError_t e, const char* where) {
  if (c) {
    c->err = std::string(where) + ": " + hipGetErrorString(e);
  }
  return MFC_ERR_HIP;
}

// Per-axis face buffers (all axes in one face launch) are used while their sum
// stays within this many bytes; larger grids share one buffer across axes.
constexpr size_t kAllAxesFaceBudget = size_t(8) << 30;

void free_vjp_scratch(mfc_ctx* c) {
  for (int d = 0; d < 3; ++d) {
    if (c->vjp.Gd[d]) (void)hipFree(c->vjp.Gd[d]);
    if (c->vjp.UFd[d]) (void)hipFree(c->vjp.UFd[d]);
    c->vjp.Gd[d] = c->vjp.UFd[d] = nullptr;
  }
  void** bufs[] = {(void**)&c->vbuf, (void**)&c->b1, (void**)&c->b2};
  for (void** b : bufs) {
    if (*b) (void)hipFree(*b);
    *b = nullptr;
  }
  c->vjp.all_axes = false;
}

int ensure_vjp_scratch(mfc_ctx* c) {
  if (c->vjp.Gd[0]) return MFC_OK;
  long long faces[3] = {0, 0, 0}, maxfaces = 0, sumfaces = 0;
  for (int d = 0; d < c->prob.ndim; ++d) {
    const long long lines = c->ncell / c->prob.n[d];
    faces[d] = lines * (c->prob.n[d] + 1);
    if (faces[d] > maxfaces) maxfaces = faces[d];
    sumfaces += faces[d];
  }
  const size_t per_face = (size_t)(6 * c->neq + 1) * sizeof(double);
  size_t budget = kAllAxesFaceBudget;
  if (const char* env = getenv("MFC355_ADJOINT_FACE_BUDGET")) budget = (size_t)strtoull(env, nullptr, 10);
  const bool all_axes = (size_t)sumfaces * per_face <= budget;
  const size_t state = (size_t)c->neq * (size_t)c->ncell * sizeof(double);
  bool ok = true;
  for (int d = 0; d < (all_axes ? c->prob.ndim : 1) && ok; ++d) {
    const long long nf = all_axes ? faces[d] : maxfaces;
    ok = hipMalloc((void**)&c->vjp.Gd[d], (size_t)6 * c->neq * (size_t)nf * sizeof(double)) == hipSuccess &&
         hipMalloc((void**)&c->vjp.UFd[d], (size_t)nf * sizeof(double)) == hipSuccess;
  }
  ok = ok && hipMalloc((void**)&c->vbuf, state) == hipSuccess && hipMalloc((void**)&c->b1, state) == hipSuccess &&
       hipMalloc((void**)&c->b2, state) == hipSuccess;
  if (!ok) {
    // release whatever was obtained, so that a later call retries from scratch
    (void)hipGetLastError();
    free_vjp_scratch(c);
    c->err = "adjoint scratch allocation failed";
    return MFC_ERR_ALLOC;
  }
  c->vjp.all_axes = all_axes;
  return MFC_OK;
}

// ---------------------------------------------------------------------------
// Non-uniform grids (Sec. 4.2.2): reconstruction tables built on the host.
// For the centre cell at position c of an axis, with unit coordinate
// xi = (x - x_c)/h_c, candidate r (cells c - 2 + r .. c + r) is the quadratic
// m0 + m1 xi + m2 xi^2 with the data as its cell averages: m = A^-1 f, A the
// 3 x 3 matrix of cell averages of 1, xi, xi^2 over the stencil's cells.  The
// ideal weights at a face are the least-squares (here exact) solution of
// sum_r d_r v_r = v5, v_r the candidate's value functional at the face and v5
// that of the quartic with the five cells' averages.  Ghost cells take the
// width of the cell whose state they hold (ghost_index).
// ---------------------------------------------------------------------------
namespace {

// Solve the n x n system M X = B for X (k right-hand sides), Gaussian
// elimination with partial pivoting; M and B are overwritten.  False if singular.
bool solve_dense(int n, int k, double* M, double* B) {
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(M[r * n + col]) > fabs(M[piv * n + col])) piv = r;
    if (!(fabs(M[piv * n + col]) > 0.0)) return false;
    if (piv != col) {
      for (int j = 0; j < n; ++j) std::swap(M[col * n + j], M[piv * n + j]);
      for (int j = 0; j < k; ++j) std::swap(B[col * k + j], B[piv * k + j]);
    }
    for (int r = col + 1; r < n; ++r) {
      const double f = M[r * n + col] / M[col * n + col];
      for (int j = col; j < n; ++j) M[r * n + j] -= f * M[col * n + j];
      for (int j = 0; j < k; ++j) B[r * k + j] -= f * B[col * k + j];
    }
  }
  for (int col = n - 1; col >= 0; --col) {
    for (int j = 0; j < k; ++j) {
      double v = B[col * k + j];
      for (int c2 = col + 1; c2 < n; ++c2) v -= M[col * n + c2] * B[c2 * k + j];
      B[col * k + j] = v / M[col * n + col];
    }
  }
  return true;
}

// Inverse of the moment matrix of `deg + 1` cells with unit-coordinate faces
// e[0..deg+1]: row k of the result maps the cell averages to m_k.
bool moment_inverse(int deg, const double* e, double* inv) {
  const int n = deg + 1;
  double M[25], B[25];
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k) {
      const double a = e[j], b = e[j + 1];
      M[j * n + k] = (std::pow(b, k + 1) - std::pow(a, k + 1)) / ((k + 1) * (b - a));
      B[j * n + k] = (j == k) ? 1.0 : 0.0;
    }
  // M X = I gives X = M^-1 with X[k][j] the weight of average j in m_k
  if (!solve_dense(n, n, M, B)) return false;
  for (int i = 0; i < n * n; ++i) inv[i] = B[i];
  return true;
}

// Table of one axis: kNuCoefs rows of n + 6 entries (positions -3 .. n + 2).
bool build_axis_table(const mfc::Params& pm, int d, const std::vector<double>& faces, double dx,
                      std::vector<double>& tab) {
  const int n = pm.n[d];
  const long long st = n + 6;
  tab.assign((size_t)mfc::kNuCoefs * st, 0.0);
  auto width = [&](int pos) {
    if (faces.empty()) return dx;
    bool flip;
    const int i = mfc::ghost_index(pos, n, pm.bc_lo[d], pm.bc_hi[d], flip);
    return faces[i + 1] - faces[i];
  };
  for (int pos = -3; pos <= n + 2; ++pos) tab[mfc::NU_INVW * st + pos + 3] = 1.0 / width(pos);
  for (int pos = -1; pos <= n; ++pos) {
    const double hc = width(pos);
    double e[6];
    e[2] = -0.5;
    e[3] = 0.5;
    e[1] = e[2] - width(pos - 1) / hc;
    e[0] = e[1] - width(pos - 2) / hc;
    e[4] = e[3] + width(pos + 1) / hc;
    e[5] = e[4] + width(pos + 2) / hc;
    double inv3[3][9];
    for (int r = 0; r < 3; ++r) {
      if (!moment_inverse(2, &e[r], inv3[r])) return false;
      // m_k = sum_j inv[k][j] f_{r+j}; m0 - f_2 subtracts the centre (j = 2 - r)
      for (int k = 0; k < 3; ++k) {
        double w[3] = {inv3[r][k * 3 + 0], inv3[r][k * 3 + 1], inv3[r][k * 3 + 2]};
        if (k == 0) w[2 - r] -= 1.0;
        // zero-sum w: w . f = -w_0 (f_1 - f_0) + w_2 (f_2 - f_1) over the stencil
        const int row = (k == 0 ? mfc::NU_MU0 : k == 1 ? mfc::NU_M1 : mfc::NU_M2) + 2 * r;
        tab[row * st + pos + 3] = -w[0];
        tab[(row + 1) * st + pos + 3] = w[2];
      }
    }
    double inv5[25];
    if (!moment_inverse(4, e, inv5)) return false;
    for (int side = 0; side < 2; ++side) {
      const double xi = side == 0 ? 0.5 : -0.5;
      double v5[5] = {0, 0, 0, 0, 0}, V[3][5] = {};
      for (int j = 0; j < 5; ++j)
        for (int k = 0; k < 5; ++k) v5[j] += std::pow(xi, k) * inv5[k * 5 + j];
      for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k) V[r][r + j] += std::pow(xi, k) * inv3[r][k * 3 + j];
      double N[9], rhs[3];
      for (int a = 0; a < 3; ++a) {
        rhs[a] = 0.0;
        for (int j = 0; j < 5; ++j) rhs[a] += V[a][j] * v5[j];
        for (int b = 0; b < 3; ++b) {
          N[a * 3 + b] = 0.0;
          for (int j = 0; j < 5; ++j) N[a * 3 + b] += V[a][j] * V[b][j];
        }
      }
      if (!solve_dense(3, 1, N, rhs)) return false;
      const int row = side == 0 ? mfc::NU_DR : mfc::NU_DL;
      for (int r = 0; r < 3; ++r) tab[(row + r) * st + pos + 3] = rhs[r];
    }
  }
  return true;
}

}  // namespace

// Smallest accepted WENO eps: (4 eps)^8 stays far above the smallest normal
// double (2.2e-308) for every eps >= 1e-30.
constexpr double kMinWenoEps = 1e-30;

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int check_device(mfc_ctx* c) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device) {
    c->err = "the current HIP device is not the one the context was created on";
    return MFC_ERR_ARG;
  }
  return MFC_OK;
}

int check_array(mfc_ctx* c, const void* p, const char* name) {
  if (!p) {
    c->err = std::string("null pointer: ") + name;
    return MFC_ERR_ARG;
  }
  if (!aligned(p, c->esize)) {
    c->err = std::string("misaligned pointer: ") + name;
    return MFC_ERR_ARG;
  }
  return MFC_OK;
}

mfc::Params make_params(const mfc_problem& p) {
  mfc::Params pm;
  memset(&pm, 0, sizeof(pm));
  for (int d = 0; d < 3; ++d) {
    pm.n[d] = p.n[d];
    pm.bc_lo[d] = p.bc_lo[d];
    pm.bc_hi[d] = p.bc_hi[d];
    pm.inv_dx[d] = (d < p.ndim) ? 1.0 / p.dx[d] : 0.0;
  }
  for (int i = 0; i < 2; ++i) {
    const int k = (i < p.num_fluids) ? i : 0;
    pm.G[i] = 1.0 / (p.gamma[k] - 1.0);
    pm.P[i] = p.gamma[k] * p.pi_inf[k] / (p.gamma[k] - 1.0);
  }
  for (int i = 0; i < 2; ++i) {
    const int k = (i < p.num_fluids) ? i : 0;
    pm.gam[i] = p.gamma[k];
    pm.pinf[i] = p.pi_inf[k];
  }
  pm.eps = p.weno_eps;
  pm.weno_variant = p.weno_variant;
  pm.riemann = p.riemann_solver;
  pm.low_mach = p.low_mach;
  pm.model = p.model;
  pm.ncell = (long long)p.n[0] * p.n[1] * p.n[2];
  return pm;
}

}  // namespace

extern "C" {

int mfc_abi_version(void) { return MFC_ABI_VERSION; }

const char* mfc_status_string(int s) {
  switch (s) {
    case MFC_OK: return "ok";
    case MFC_ERR_ARG: return "invalid argument";
    case MFC_ERR_SHAPE: return "invalid shape";
    case MFC_ERR_UNSUPPORTED: return "unsupported configuration";
    case MFC_ERR_HIP: return "HIP error";
    case MFC_ERR_NONFINITE: return "non-finite state or non-positive squared sound speed";
    case MFC_ERR_ALLOC: return "device allocation failed";
    default: return "unknown status";
  }
}

int mfc_num_eqs(const mfc_problem* p) {
  if (!p) return MFC_ERR_ARG;
  if (p->ndim < 1 || p->ndim > 3) return MFC_ERR_UNSUPPORTED;
  if (p->num_fluids != 1 && p->num_fluids != 2) return MFC_ERR_UNSUPPORTED;
  return p->num_fluids + p->ndim + 1 + (p->num_fluids == 2 ? 2 : 0);
}

int mfc_validate(const mfc_problem* p) {
  if (!p) return MFC_ERR_ARG;
  if (p->abi_version != MFC_ABI_VERSION) return MFC_ERR_ARG;
  if (p->ndim < 1 || p->ndim > 3) return MFC_ERR_UNSUPPORTED;
  if (p->num_fluids != 1 && p->num_fluids != 2) return MFC_ERR_UNSUPPORTED;
  if (p->precision != MFC_FP64 && p->precision != MFC_FP32_MIXED) return MFC_ERR_UNSUPPORTED;
  long long ncell = 1;
  for (int d = 0; d < 3; ++d) {
    if (d < p->ndim) {
      if (p->n[d] < 3) return MFC_ERR_SHAPE;
      if (!(p->dx[d] > 0.0) || !(p->dx[d] < 1e300)) return MFC_ERR_ARG;
      if (p->bc_lo[d] < 0 || p->bc_lo[d] > 2 || p->bc_hi[d] < 0 || p->bc_hi[d] > 2) return MFC_ERR_ARG;
      if ((p->bc_lo[d] == MFC_BC_PERIODIC) != (p->bc_hi[d] == MFC_BC_PERIODIC)) return MFC_ERR_ARG;
    } else if (p->n[d] != 1) {
      return MFC_ERR_SHAPE;
    }
    ncell *= p->n[d];
  }
  // grid launch limits: the y and z extents index grid dimensions directly
  // (gridDim.y and gridDim.z are at most 65535)
  if (p->n[1] > 65535 || p->n[2] > 65535) return MFC_ERR_SHAPE;
  // 2^34 cells already exceed the device memory of any state; it also keeps
  // every one-dimensional grid (cells / 256 blocks) far inside its limit
  if (ncell > (1LL << 34)) return MFC_ERR_SHAPE;
  for (int i = 0; i < p->num_fluids; ++i)
    if (!(p->gamma[i] > 1.0) || !(p->pi_inf[i] >= 0.0) || !(p->pi_inf[i] < 1e300)) return MFC_ERR_ARG;
  // the double reconstructions normalize through products of up to eight
  // smoothness indicators, each at least 4 eps: eps below kMinWenoEps would
  // let that product underflow on flat data
  if (!(p->weno_eps >= kMinWenoEps) || !(p->weno_eps < 1e300)) return MFC_ERR_ARG;
  if (p->weno_variant < MFC_WENO_JS || p->weno_variant > MFC_WENO_M) return MFC_ERR_UNSUPPORTED;
  if (p->riemann_solver != MFC_HLLC && p->riemann_solver != MFC_HLL) return MFC_ERR_UNSUPPORTED;
  if (p->low_mach != MFC_LOW_MACH_NONE && p->low_mach != MFC_LOW_MACH_THORNBER && p->low_mach != MFC_LOW_MACH_CHEN_APC)
    return MFC_ERR_UNSUPPORTED;
  // the APC term corrects the HLLC star fluxes; HLL has no star region
  if (p->low_mach == MFC_LOW_MACH_CHEN_APC && p->riemann_solver != MFC_HLLC) return MFC_ERR_UNSUPPORTED;
  if (p->model != MFC_MODEL_ALLAIRE && p->model != MFC_MODEL_KAPILA) return MFC_ERR_UNSUPPORTED;
  // K couples the two phases' volume fractions
  if (p->model == MFC_MODEL_KAPILA && p->num_fluids != 2) return MFC_ERR_UNSUPPORTED;
  return MFC_OK;
}

// Partials buffer: the fixed-shape reductions (kReduceBlocks per row, up to
// 8 rows) and the signal maxima of the first axis pass of a CFL step.
static size_t partial_len(const mfc_problem& p) {
  const long long red = (long long)mfc::kReduceBlocks * 8;
  const long long sig = mfc::signal_partials(p.ndim, p.n);
  return (size_t)(red > sig ? red : sig);
}

int mfc_create(const mfc_problem* p, mfc_ctx** out) {
  if (!out) return MFC_ERR_ARG;
  *out = nullptr;
  int v = mfc_validate(p);
  if (v != MFC_OK) return v;
  mfc_ctx* c = new mfc_ctx();
  c->prob = *p;
  c->pm = make_params(*p);
  c->neq = mfc_num_eqs(p);
  c->ncell = c->pm.ncell;
  c->esize = (p->precision == MFC_FP64) ? sizeof(double) : sizeof(float);
  c->acc = c->q1 = c->q2 = nullptr;
  c->scal = c->partial = nullptr;
  c->flag = nullptr;
  c->timer = nullptr;
  c->vjp = mfc::VjpScratch{{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}, false};
  c->vbuf = c->b1 = c->b2 = nullptr;
  for (int d = 0; d < 3; ++d) {
    c->nu_d[d] = nullptr;
    c->nu_f[d] = nullptr;
  }
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return MFC_ERR_HIP;
  }
  const size_t bytes = (size_t)c->neq * (size_t)c->ncell * c->esize;
  bool ok = hipMalloc(&c->acc, bytes) == hipSuccess && hipMalloc(&c->q1, bytes) == hipSuccess &&
            hipMalloc(&c->q2, bytes) == hipSuccess &&
            hipMalloc((void**)&c->scal, 4 * sizeof(double)) == hipSuccess &&
            hipMalloc((void**)&c->partial, partial_len(c->prob) * sizeof(double)) == hipSuccess &&
            hipMalloc((void**)&c->flag, sizeof(int)) == hipSuccess;
  if (ok) ok = hipMemset(c->flag, 0, sizeof(int)) == hipSuccess;
  if (ok) ok = hipMemset(c->scal, 0, 4 * sizeof(double)) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    mfc_destroy(c);
    return MFC_ERR_ALLOC;
  }
  *out = c;
  return MFC_OK;
}

int mfc_destroy(mfc_ctx* c) {
  if (!c) return MFC_OK;
  int prev = -1;
  (void)hipGetDevice(&prev);
  const int dev = c->device;
  if (prev != dev) (void)hipSetDevice(dev);
  (void)hipDeviceSynchronize();
  if (c->acc) (void)hipFree(c->acc);
  if (c->q1) (void)hipFree(c->q1);
  if (c->q2) (void)hipFree(c->q2);
  if (c->scal) (void)hipFree(c->scal);
  if (c->partial) (void)hipFree(c->partial);
  if (c->flag) (void)hipFree(c->flag);
  for (int d = 0; d < 3; ++d) {
    if (c->nu_d[d]) (void)hipFree(c->nu_d[d]);
    if (c->nu_f[d]) (void)hipFree(c->nu_f[d]);
  }
  free_vjp_scratch(c);
  delete c->timer;
  delete c;
  if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
  return MFC_OK;
}

const char* mfc_last_error(const mfc_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

#define MFC_DISPATCH_REAL(c, CALL_D, CALL_F) \
  ((c)->prob.precision == MFC_FP64 ? (CALL_D) : (CALL_F))

int mfc_prim_to_cons(mfc_ctx* c, const void* w, void* q, void* stream) {
  if (!c) return MFC_ERR_ARG;
  if (int rd = check_device(c)) return rd;
  int r;
  if ((r = check_array(c, w, "w")) || (r = check_array(c, q, "q"))) return r;
  if (w == q) return fail(c, MFC_ERR_ARG, "w and q alias");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = MFC_DISPATCH_REAL(
      c, mfc::launch_convert<double>(c->prob.num_fluids, c->prob.ndim, true, c->pm, (const double*)w, (double*)q, s),
      mfc::launch_convert<float>(c->prob.num_fluids, c->prob.ndim, true, c->pm, (const float*)w, (float*)q, s));
  return e == hipSuccess ? MFC_OK : hip_fail(c, e, "prim_to_cons");
}

int mfc_cons_to_prim(mfc_ctx* c, const void* q, void* w, void* stream) {
  if (!c) return MFC_ERR_ARG;
  if (int rd = check_device(c)) return rd;
  int r;
  if ((r = check_array(c, w, "w")) || (r = check_array(c, q, "q"))) return r;
  if (w == q) return fail(c, MFC_ERR_ARG, "w and q alias");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = MFC_DISPATCH_REAL(
      c, mfc::launch_convert<double>(c->prob.num_fluids, c->prob.ndim, false, c->pm, (const double*)q, (double*)w, s),
      mfc::launch_convert<float>(c->prob.num_fluids, c->prob.ndim, false, c->pm, (const float*)q, (float*)w, s));
  return e == hipSuccess ? MFC_OK : hip_fail(c, e, "cons_to_prim");
}

int mfc_rhs(mfc_ctx* c, const void* q, void* rhs, void* stream) {
  if (!c) return MFC_ERR_ARG;
  if (int rd = check_device(c)) return rd;
  int r;
  if ((r = check_array(c, q, "q")) || (r = check_array(c, rhs, "rhs"))) return r;
  if (q == rhs) return fail(c, MFC_ERR_ARG, "q and rhs alias");
  hipStream_t s = (hipStream_t)stream;
  mfc::StageArgs st{0, 0.0, nullptr};
  hipError_t e = MFC_DISPATCH_REAL(
      c,
      mfc::launch_rhs<double>(c->prob.num_fluids, c->prob.ndim, c->pm, (const double*)q, (double*)rhs, nullptr,
                              nullptr, st, false, c->flag, s, c->timer),
      mfc::launch_rhs<float>(c->prob.num_fluids, c->prob.ndim, c->pm, (const float*)q, (float*)rhs, nullptr,
                             nullptr, st, false, c->flag, s, c->timer));
  return e == hipSuccess ? MFC_OK : hip_fail(c, e, "rhs");
}

int mfc_max_signal(mfc_ctx* c, const void* q, double* smax_dev, void* stream) {
  if (!c) return MFC_ERR_ARG;
  if (int rd = check_device(c)) return rd;
  int r;
  if ((r = check_array(c, q, "q"))) return r;
  if (!smax_dev || !aligned(smax_dev, sizeof(double))) return fail(c, MFC_ERR_ARG, "bad smax pointer");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = MFC_DISPATCH_REAL(
      c,
      mfc::launch_max_signal<double>(c->prob.num_fluids, c->prob.ndim, c->pm, (const double*)q, c->partial,
                                     smax_dev, 0.0, 0.0, nullptr, nullptr, c->flag, s),
      mfc::launch_max_signal<float>(c->prob.num_fluids, c->prob.ndim, c->pm, (const float*)q, c->partial,
                                    smax_dev, 0.0, 0.0, nullptr, nullptr, c->flag, s));
  return e == hipSuccess ? MFC_OK : hip_fail(c, e, "max_signal");
}

}  // extern "C"

namespace {
// Device buffers one SSP-RK3 step works in: the RHS accumulator, the two
// stage states, the reduction partials, [smax, dt] and the non-finite flag.
struct StepScratch {
  void* acc;
  void* q1;
  void* q2;
  double* partial;
  double* scal;
  int* flag;
};

template <typename Real>
hipError_t step_t(const mfc_problem& prob, const mfc::Params& pm, const StepScratch& sc, mfc::PassTimer* tm,
                  Real* q, double cfl, double dt_fixed, double t_remaining, double* dt_user, hipStream_t s) {
  const int nf = prob.num_fluids, nd = prob.ndim;
  hipError_t e;
  mfc::StageArgs st{1, dt_fixed, nullptr, nullptr};
  // 2D / 3D: the first axis pass of stage 1 forms the signal maxima while it
  // loads q^n, and dt is formed on the device before the x pass reads it
  mfc::SignalFuse sig{sc.partial, cfl, t_remaining, &sc.scal[0], &sc.scal[1], dt_user};
  const mfc::SignalFuse* sigp = nullptr;
  if (cfl > 0.0) {
    if (nd >= 2) {
      sigp = &sig;
    } else {
      if (tm) tm->begin(mfc::KIND_SIGNAL, s);
      e = mfc::launch_max_signal<Real>(nf, nd, pm, q, sc.partial, &sc.scal[0], cfl, t_remaining, &sc.scal[1],
                                       dt_user, sc.flag, s);
      if (tm) tm->end(mfc::KIND_SIGNAL, s);
      if (e != hipSuccess) return e;
    }
    st.dt_ptr = &sc.scal[1];
  } else if (dt_user) {
    e = mfc::launch_set_scalar(dt_user, dt_fixed, s);
    if (e != hipSuccess) return e;
  }
  Real* q1 = (Real*)sc.q1;
  Real* q2 = (Real*)sc.q2;
  Real* acc = (Real*)sc.acc;
  st.stage = 1;
  e = mfc::launch_rhs<Real>(nf, nd, pm, q, acc, q, q1, st, true, sc.flag, s, tm, sigp);
  if (e != hipSuccess) return e;
  st.stage = 2;
  e = mfc::launch_rhs<Real>(nf, nd, pm, q1, acc, q, q2, st, true, sc.flag, s, tm);
  if (e != hipSuccess) return e;
  st.stage = 3;
  e = mfc::launch_rhs<Real>(nf, nd, pm, q2, acc, q, q, st, true, sc.flag, s, tm);
  return e;
}

StepScratch ctx_scratch(mfc_ctx* c) { return StepScratch{c->acc, c->q1, c->q2, c->partial, c->scal, c->flag}; }

// Reverse sweep of one SSP-RK3 step given its stage states.
hipError_t step_reverse(mfc_ctx* c, const double* qn, const double* q1, const double* q2, double dt,
                        const double* qnp1_bar, double* qn_bar, hipStream_t s) {
  const int nf = c->prob.num_fluids, nd = c->prob.ndim;
  const long long n = (long long)c->neq * c->ncell;
  // with every axis gathered in one cell pass the stage combination is applied
  // there (no separate pass over v = vbuf); otherwise by launch_adj_stage
  const bool fused = c->vjp.all_axes;
  const mfc::StageEpi e3{3, dt, qnp1_bar, c->b2, qn_bar}, e2{2, dt, c->b2, c->b1, qn_bar}, e1{1, dt, c->b1, nullptr, qn_bar};
  hipError_t e = mfc::launch_rhs_vjp(nf, nd, c->pm, q2, qnp1_bar, c->vbuf, c->vjp, false, s, c->timer, &e3);
  if (e == hipSuccess && !fused) e = mfc::launch_adj_stage(3, n, dt, qnp1_bar, c->vbuf, c->b2, qn_bar, s);
  if (e == hipSuccess) e = mfc::launch_rhs_vjp(nf, nd, c->pm, q1, c->b2, c->vbuf, c->vjp, false, s, c->timer, &e2);
  if (e == hipSuccess && !fused) e = mfc::launch_adj_stage(2, n, dt, c->b2, c->vbuf, c->b1, qn_bar, s);
  if (e == hipSuccess) e = mfc::launch_rhs_vjp(nf, nd, c->pm, qn, c->b1, c->vbuf, c->vjp, false, s, c->timer, &e1);
  if (e == hipSuccess && !fused) e = mfc::launch_adj_stage(1, n, dt, c->b1, c->vbuf, nullptr, qn_bar, s);
  return e;
}
}  // namespace

extern "C" {

int mfc_step(mfc_ctx* c, void* q, double cfl, double dt_fixed, double t_remaining, double* dt_dev,
             void* stream) {
  if (!c) return MFC_ERR_ARG;
  if (int rd = check_device(c)) return rd;
  int r;
  if ((r = check_array(c, q, "q"))) return r;
  if ((cfl > 0.0) == (dt_fixed > 0.0)) return fail(c, MFC_ERR_ARG, "exactly one of cfl and dt_fixed must be > 0");
  if (!(cfl < 1e300) || !(dt_fixed < 1e300) || t_remaining != t_remaining)
    return fail(c, MFC_ERR_ARG, "non-finite step argument");
  if (dt_dev && !aligned(dt_dev, sizeof(double))) return fail(c, MFC_ERR_ARG, "misaligned dt pointer");
  hipStream_t s = (hipStream_t)stream;
  const StepScratch sc = ctx_scratch(c);
  hipError_t e = MFC_DISPATCH_REAL(
      c, step_t<double>(c->prob, c->pm, sc, c->timer, (double*)q, cfl, dt_fixed, t_remaining, dt_dev, s),
      step_t<float>(c->prob, c->pm, sc, c->timer, (float*)q, cfl, dt_fixed, t_remaining, dt_dev, s));
  return e == hipSuccess ? MFC_OK : hip_fail(c, e, "step");
}

int mfc_conserved_sums(mfc_ctx* c, const void* q, double* sums_dev, void* stream) {
  if (!c) return MFC_ERR_ARG;
  if (int rd = check_device(c)) return rd;
  int r;
  if ((r = check_array(c, q, "q"))) return r;
  if (!sums_dev || !aligned(sums_dev, sizeof(double))) return fail(c, MFC_ERR_ARG, "bad sums pointer");
  double vol = 1.0;
  for (int d = 0; d < c->prob.ndim; ++d) vol = vol * c->prob.dx[d];
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = MFC_DISPATCH_REAL(
      c, mfc::launch_sums<double>(c->neq, c->pm, (const double*)q, vol, c->partial, sums_dev, s),
      mfc::launch_sums<float>(c->neq, c->pm, (const float*)q, vol, c->partial, sums_dev, s));
  return e == hipSuccess ? MFC_OK : hip_fail(c, e, "conserved_sums");
}

int mfc_set_grid(mfc_ctx* c, int axis, const double* faces) {
  if (!c) return MFC_ERR_ARG;
  if (int rd = check_device(c)) return rd;
  if (axis < 0 || axis >= c->prob.ndim) return fail(c, MFC_ERR_ARG, "axis outside the problem's dimensions");
  const int n = c->prob.n[axis];
  if (faces) {
    if (c->prob.weno_variant != MFC_WENO_JS)
      return fail(c, MFC_ERR_UNSUPPORTED, "non-uniform grids take WENO5-JS weights");
    for (int i = 0; i < n; ++i)
      if (!(faces[i + 1] > faces[i]) || !std::isfinite(faces[i]) || !std::isfinite(faces[i + 1]) ||
          !std::isfinite(faces[i + 1] - faces[i]))
        return fail(c, MFC_ERR_ARG, "face coordinates must be finite and strictly increasing");
  }
  std::vector<double> keep = c->faces[axis];
  if (faces)
    c->faces[axis].assign(faces, faces + n + 1);
  else
    c->faces[axis].clear();
  const bool any = !c->faces[0].empty() || !c->faces[1].empty() || !c->faces[2].empty();
  if (!any) {
    // every axis uniform again: back to the uniform kernels
    for (int d = 0; d < 3; ++d) {
      c->pm.nu[d] = nullptr;
      c->pm.nuf[d] = nullptr;
    }
    return MFC_OK;
  }
  // every active axis gets a table (uniform axes: the uniform coefficients)
  for (int d = 0; d < c->prob.ndim; ++d) {
    std::vector<double> tab;
    if (!build_axis_table(c->pm, d, c->faces[d], c->prob.dx[d], tab)) {
      c->faces[axis] = keep;
      return fail(c, MFC_ERR_ARG, "degenerate grid: a reconstruction system is singular");
    }
    std::vector<float> tabf(tab.begin(), tab.end());
    const size_t nb = tab.size();
    if (!c->nu_d[d]) {
      if (hipMalloc((void**)&c->nu_d[d], nb * sizeof(double)) != hipSuccess ||
          hipMalloc((void**)&c->nu_f[d], nb * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        c->faces[axis] = keep;
        return fail(c, MFC_ERR_ALLOC, "grid table allocation failed");
      }
    }
    hipError_t e = hipMemcpy(c->nu_d[d], tab.data(), nb * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->nu_f[d], tabf.data(), nb * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "set_grid: copy");
    c->pm.nu[d] = c->nu_d[d];
    c->pm.nuf[d] = c->nu_f[d];
  }
  return MFC_OK;
}

int mfc_rhs_vjp(mfc_ctx* c, const void* q, const void* rhs_bar, void* q_bar, int accumulate, void* stream) {
  if (!c) return MFC_ERR_ARG;
  if (int rd = check_device(c)) return rd;
  if (c->prob.precision != MFC_FP64) return fail(c, MFC_ERR_UNSUPPORTED, "adjoint entry points are FP64 only");
  int r;
  if ((r = check_array(c, q, "q")) || (r = check_array(c, rhs_bar, "rhs_bar")) || (r = check_array(c, q_bar, "q_bar")))
    return r;
  if (q_bar == q || q_bar == rhs_bar) return fail(c, MFC_ERR_ARG, "q_bar aliases an input");
  if ((r = ensure_vjp_scratch(c))) return r;
  hipError_t e = mfc::launch_rhs_vjp(c->prob.num_fluids, c->prob.ndim, c->pm, (const double*)q,
                                     (const double*)rhs_bar, (double*)q_bar, c->vjp, accumulate != 0,
                                     (hipStream_t)stream, c->timer);
  return e == hipSuccess ? MFC_OK : hip_fail(c, e, "rhs_vjp");
}

int mfc_step_vjp(mfc_ctx* c, const void* q_n, double dt, const void* qnp1_bar, void* qn_bar, void* stream) {
  if (!c) return MFC_ERR_ARG;
  if (int rd = check_device(c)) return rd;
  if (c->prob.precision != MFC_FP64) return fail(c, MFC_ERR_UNSUPPORTED, "adjoint entry points are FP64 only");
  int r;
  if ((r = check_array(c, q_n, "q_n")) || (r = check_array(c, qnp1_bar, "qnp1_bar")) ||
      (r = check_array(c, qn_bar, "qn_bar")))
    return r;
  if (!(dt > 0.0) || !(dt < 1e300)) return fail(c, MFC_ERR_ARG, "dt must be positive and finite");
  if (qn_bar == q_n || qn_bar == qnp1_bar) return fail(c, MFC_ERR_ARG, "qn_bar aliases an input");
  if ((r = ensure_vjp_scratch(c))) return r;
  hipStream_t s = (hipStream_t)stream;
  const int nf = c->prob.num_fluids, nd = c->prob.ndim;
  const double* qn = (const double*)q_n;
  double* q1 = (double*)c->q1;
  double* q2 = (double*)c->q2;
  double* acc = (double*)c->acc;
  // recompute the stage states with the same dt
  mfc::StageArgs st{1, dt, nullptr};
  hipError_t e = mfc::launch_rhs<double>(nf, nd, c->pm, qn, acc, qn, q1, st, true, c->flag, s, c->timer);
  st.stage = 2;
  if (e == hipSuccess) e = mfc::launch_rhs<double>(nf, nd, c->pm, q1, acc, qn, q2, st, true, c->flag, s, c->timer);
  if (e == hipSuccess) e = step_reverse(c, qn, q1, q2, dt, (const double*)qnp1_bar, (double*)qn_bar, s);
  return e == hipSuccess ? MFC_OK : hip_fail(c, e, "step_vjp");
}

int mfc_step_save_stages(mfc_ctx* c, void* q, double dt, void* q1, void* q2, void* stream) {
  if (!c) return MFC_ERR_ARG;
  if (int rd = check_device(c)) return rd;
  if (c->prob.precision != MFC_FP64) return fail(c, MFC_ERR_UNSUPPORTED, "adjoint entry points are FP64 only");
  int r;
  if ((r = check_array(c, q, "q")) || (r = check_array(c, q1, "q1")) || (r = check_array(c, q2, "q2"))) return r;
  if (!(dt > 0.0) || !(dt < 1e300)) return fail(c, MFC_ERR_ARG, "dt must be positive and finite");
  if (q1 == q || q2 == q || q1 == q2) return fail(c, MFC_ERR_ARG, "q, q1 and q2 must be distinct");
  hipStream_t s = (hipStream_t)stream;
  const int nf = c->prob.num_fluids, nd = c->prob.ndim;
  double* qq = (double*)q;
  double* acc = (double*)c->acc;
  mfc::StageArgs st{1, dt, nullptr};
  hipError_t e = mfc::launch_rhs<double>(nf, nd, c->pm, qq, acc, qq, (double*)q1, st, true, c->flag, s, c->timer);
  st.stage = 2;
  if (e == hipSuccess)
    e = mfc::launch_rhs<double>(nf, nd, c->pm, (const double*)q1, acc, qq, (double*)q2, st, true, c->flag, s,
                                c->timer);
  st.stage = 3;
  if (e == hipSuccess)
    e = mfc::launch_rhs<double>(nf, nd, c->pm, (const double*)q2, acc, qq, qq, st, true, c->flag, s, c->timer);
  return e == hipSuccess ? MFC_OK : hip_fail(c, e, "step_save_stages");
}

int mfc_step_vjp_stages(mfc_ctx* c, const void* q_n, const void* q1, const void* q2, double dt,
                        const void* qnp1_bar, void* qn_bar, void* stream) {
  if (!c) return MFC_ERR_ARG;
  if (int rd = check_device(c)) return rd;
  if (c->prob.precision != MFC_FP64) return fail(c, MFC_ERR_UNSUPPORTED, "adjoint entry points are FP64 only");
  int r;
  if ((r = check_array(c, q_n, "q_n")) || (r = check_array(c, q1, "q1")) || (r = check_array(c, q2, "q2")) ||
      (r = check_array(c, qnp1_bar, "qnp1_bar")) || (r = check_array(c, qn_bar, "qn_bar")))
    return r;
  if (!(dt > 0.0) || !(dt < 1e300)) return fail(c, MFC_ERR_ARG, "dt must be positive and finite");
  if (qn_bar == q_n || qn_bar == qnp1_bar || qn_bar == q1 || qn_bar == q2)
    return fail(c, MFC_ERR_ARG, "qn_bar aliases an input");
  if ((r = ensure_vjp_scratch(c))) return r;
  hipError_t e = step_reverse(c, (const double*)q_n, (const double*)q1, (const double*)q2, dt,
                              (const double*)qnp1_bar, (double*)qn_bar, (hipStream_t)stream);
  return e == hipSuccess ? MFC_OK : hip_fail(c, e, "step_vjp_stages");
}

int mfc_cons_to_prim_vjp(mfc_ctx* c, const void* q, const void* w_bar, void* q_bar, int accumulate, void* stream) {
  if (!c) return MFC_ERR_ARG;
  if (int rd = check_device(c)) return rd;
  if (c->prob.precision != MFC_FP64) return fail(c, MFC_ERR_UNSUPPORTED, "adjoint entry points are FP64 only");
  int r;
  if ((r = check_array(c, q, "q")) || (r = check_array(c, w_bar, "w_bar")) || (r = check_array(c, q_bar, "q_bar")))
    return r;
  if (q_bar == q || q_bar == w_bar) return fail(c, MFC_ERR_ARG, "q_bar aliases an input");
  hipError_t e = mfc::launch_convert_vjp(c->prob.num_fluids, c->prob.ndim, false, c->pm, (const double*)q,
                                         (const double*)w_bar, (double*)q_bar, accumulate != 0, (hipStream_t)stream);
  return e == hipSuccess ? MFC_OK : hip_fail(c, e, "cons_to_prim_vjp");
}

int mfc_prim_to_cons_vjp(mfc_ctx* c, const void* w, const void* q_bar, void* w_bar, int accumulate, void* stream) {
  if (!c) return MFC_ERR_ARG;
  if (int rd = check_device(c)) return rd;
  if (c->prob.precision != MFC_FP64) return fail(c, MFC_ERR_UNSUPPORTED, "adjoint entry points are FP64 only");
  int r;
  if ((r = check_array(c, w, "w")) || (r = check_array(c, q_bar, "q_bar")) || (r = check_array(c, w_bar, "w_bar")))
    return r;
  if (w_bar == w || w_bar == q_bar) return fail(c, MFC_ERR_ARG, "w_bar aliases an input");
  hipError_t e = mfc::launch_convert_vjp(c->prob.num_fluids, c->prob.ndim, true, c->pm, (const double*)w,
                                         (const double*)q_bar, (double*)w_bar, accumulate != 0, (hipStream_t)stream);
  return e == hipSuccess ? MFC_OK : hip_fail(c, e, "prim_to_cons_vjp");
}

int mfc_set_timing(mfc_ctx* c, int enable) {
  if (!c) return MFC_ERR_ARG;
  if (int rd = check_device(c)) return rd;
  if (enable && !c->timer) c->timer = new EventTimer();
  if (!enable && c->timer) {
    delete c->timer;
    c->timer = nullptr;
  }
  return MFC_OK;
}

int mfc_get_timing(mfc_ctx* c, double* ms_sum, int64_t* counts) {
  if (!c || !ms_sum || !counts) return MFC_ERR_ARG;
  if (!c->timer) return fail(c, MFC_ERR_ARG, "timing is not enabled");
  hipError_t e = c->timer->collect(ms_sum, counts);
  return e == hipSuccess ? MFC_OK : hip_fail(c, e, "get_timing");
}

int mfc_check(mfc_ctx* c, void* stream) {
  if (!c) return MFC_ERR_ARG;
  if (int rd = check_device(c)) return rd;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "check: stream");
  int h = 0;
  e = hipMemcpy(&h, c->flag, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "check: flag");
  if (h) {
    e = hipMemset(c->flag, 0, sizeof(int));
    if (e != hipSuccess) return hip_fail(c, e, "check: reset");
    return fail(c, MFC_ERR_NONFINITE, "non-finite flux or c^2 <= 0 met");
  }
  return MFC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free step: the same kernels as mfc_step, working in a static
// device array instead of context scratch.  Every GPU the library runs on
// holds its own copy of `scratch` until the process ends; host code uses the
// per-device address returned by hipGetSymbolAddress, never the array's name.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[MFC_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's copy of `scratch` (resolved once per device, with
// that device current).
hipError_t static_scratch(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = (unsigned char*)g_scratch_ptr[dev];
  return hipSuccess;
}

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" {

int mfc_step_static(const mfc_problem* p, void* q, double cfl, double dt_fixed, double t_remaining,
                    double* dt_dev, int* flag_dev, void* stream) {
  int v = mfc_validate(p);
  if (v != MFC_OK) return v;
  const size_t esize = (p->precision == MFC_FP64) ? sizeof(double) : sizeof(float);
  if (!q || !aligned(q, esize)) return MFC_ERR_ARG;
  if (!flag_dev || !aligned(flag_dev, sizeof(int))) return MFC_ERR_ARG;
  if (dt_dev && !aligned(dt_dev, sizeof(double))) return MFC_ERR_ARG;
  if ((cfl > 0.0) == (dt_fixed > 0.0)) return MFC_ERR_ARG;
  if (!(cfl < 1e300) || !(dt_fixed < 1e300) || t_remaining != t_remaining) return MFC_ERR_ARG;
  // scratch layout: accumulator, stage 1, stage 2 (one state each), the
  // reduction partials, then [smax, dt]; each part starts on 256 bytes
  const mfc::Params pm = make_params(*p);
  const size_t state = round256((size_t)mfc_num_eqs(p) * (size_t)pm.ncell * esize);
  const size_t parts = round256(partial_len(*p) * sizeof(double));
  const size_t need = 3 * state + parts + 256;
  if (need > (size_t)MFC_STATIC_SCRATCH_BYTES) return MFC_ERR_SHAPE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return MFC_ERR_HIP;
  if (dev >= kMaxDevices) return MFC_ERR_UNSUPPORTED;
  unsigned char* base = nullptr;
  if (static_scratch(dev, &base) != hipSuccess) return MFC_ERR_HIP;
  const StepScratch sc{base, base + state, base + 2 * state, (double*)(base + 3 * state),
                       (double*)(base + 3 * state + parts), flag_dev};
  hipStream_t s = (hipStream_t)stream;
  hipError_t e =
      (p->precision == MFC_FP64)
          ? step_t<double>(*p, pm, sc, nullptr, (double*)q, cfl, dt_fixed, t_remaining, dt_dev, s)
          : step_t<float>(*p, pm, sc, nullptr, (float*)q, cfl, dt_fixed, t_remaining, dt_dev, s);
  return e == hipSuccess ? MFC_OK : MFC_ERR_HIP;
}

}  // extern "C"
