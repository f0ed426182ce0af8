// vjp_impl.h -- face and cell passes of the RHS adjoint, templated on the
// reconstruction variant WV; each vjp_wv*.hip instantiates one variant and
// vjp.hip dispatches among them.
#pragma once
//
// For rhs = L(q) and a cotangent rbar, mfc_rhs_vjp forms qbar = (dL/dq)^T rbar
// in deterministic passes (no atomics):
//   face pass   one thread per face f of an axis (low side of cell f, f = 0..n):
//               the six-cell stencil is staged in LDS (ghost remap, one
//               conversion per cell), WENO and HLLC are recomputed, the face
//               cotangents Fbar = (rbar_f - rbar_{f-1})/dx and
//               ufbar = sum_j (alpha_j rbar_alpha_j)_{f-1} - (...)_f (times 1/dx)
//               go through HLLC^T and WENO^T, and the primitive cotangents of
//               the six stencil positions are stored per face;
//   cell pass   one thread per interior cell p: sums the contributions of the six
//               faces whose stencils hold p, plus those of every ghost position
//               that the boundary condition fills from p (mirror-flipped normal
//               velocity cotangent for slip walls), applies cons->prim^T at the
//               state of p, adds the direct alpha term rbar_alpha div(u_f) and
//               writes qbar.
// When the per-axis face buffers fit the scratch budget, the face passes of
// all axes run as one launch and one cell pass sums every axis (a single
// cons->prim^T per cell); otherwise the axes run one after the other through
// one shared face buffer.
// A ghost holds the state of its source cell (normal momentum negated at a
// slip wall), so the ghost's primitive cotangent reaches the source through
// the source's own cons->prim^T once its normal-velocity entry is negated.

#include "adjoint.h"
#include "internal.h"

namespace mfc {

struct AxisGeom {
  int fx, fy, fz;   // extent of the enumerated grid
  long long count;  // fx*fy*fz
};

template <int DIR>
__device__ __forceinline__ int line_of(int i, int j, int k, int nx, int ny) {
  if constexpr (DIR == 0) return k * ny + j;
  else if constexpr (DIR == 1) return k * nx + i;
  else return j * nx + i;
}

// Face tile: FA consecutive faces along the axis times FB lines across it (x
// lanes for the y and z axes, so that every load is coalesced); 256 threads
// for every axis.  The primitives of the FA + 5 cells the stencils touch are
// converted once and staged in LDS; each face thread reads its six-cell
// stencil from there.
template <int DIR>
struct FaceTile {
  static constexpr int FA = (DIR == 0) ? 256 : 8;
  static constexpr int FB = (DIR == 0) ? 1 : 32;
  static constexpr int NT = FA * FB;
  static constexpr int CA = FA + 5;  // cells f0-3 .. f0+FA+1
};
constexpr int kFaceThreads = 256;
static_assert(FaceTile<0>::NT == kFaceThreads && FaceTile<1>::NT == kFaceThreads, "one block shape for all axes");

template <int DIR>
__device__ __forceinline__ int face_lds(int v, int c, int b) {
  using FT = FaceTile<DIR>;
  if constexpr (DIR == 0)
    return v * FT::CA + c;
  else
    return (v * FT::CA + c) * FT::FB + b;
}

template <int NEQ>
struct FaceLds {
  static constexpr int X = NEQ * FaceTile<0>::CA * FaceTile<0>::FB;
  static constexpr int YZ = NEQ * FaceTile<1>::CA * FaceTile<1>::FB;
  static constexpr int size = X > YZ ? X : YZ;
};

template <int DIR>
__device__ __forceinline__ long long cell_at(int pos, int i, int j, int k, int nx, int ny) {
  if constexpr (DIR == 0)
    return ((long long)k * ny + j) * nx + pos;
  else if constexpr (DIR == 1)
    return ((long long)k * ny + pos) * nx + i;
  else
    return ((long long)pos * ny + j) * nx + i;
}

// Tile counts of the face grid of axis DIR: (along the axis or x, ., .).
template <int DIR>
__host__ __device__ __forceinline__ void face_grid(const int* n, int& g0, int& g1, int& g2) {
  using FT = FaceTile<DIR>;
  if constexpr (DIR == 0) {
    g0 = (n[0] + 1 + FT::FA - 1) / FT::FA;
    g1 = n[1];
    g2 = n[2];
  } else {
    g0 = (n[0] + FT::FB - 1) / FT::FB;
    g1 = (n[DIR] + 1 + FT::FA - 1) / FT::FA;
    g2 = (DIR == 1) ? n[2] : n[1];
  }
}

// One face tile of axis DIR (tile coordinates t0, t1, t2 as in face_grid):
// face cotangents, HLLC^T and WENO^T, writing the six stencil positions'
// primitive cotangents of every face to G and the forward face velocity to UF.
template <int NF, int D, int DIR, int WV, int RS>
__device__ __forceinline__ void face_tile(const Params pm, const double* __restrict__ q,
                                          const double* __restrict__ rbar, double* __restrict__ G,
                                          double* __restrict__ UF, const AxisGeom& fg, int t0, int t1, int t2,
                                          int tid, double* __restrict__ sw) {
  using R = Rows<NF, D>;
  using FT = FaceTile<DIR>;
  constexpr int NEQ = R::NEQ;
  const int nx = pm.n[0], ny = pm.n[1];
  const int nd = pm.n[DIR];
  const long long nc = pm.ncell;
  // this thread's face (a along the axis, b across it) and its line
  int a, b, f0, i, j, k, ibase;
  if constexpr (DIR == 0) {
    a = tid;
    b = 0;
    f0 = t0 * FT::FA;
    ibase = 0;
    i = f0 + a;
    j = t1;
    k = t2;
  } else {
    b = tid % FT::FB;
    a = tid / FT::FB;
    f0 = t1 * FT::FA;
    ibase = t0 * FT::FB;
    i = ibase + b;
    if constexpr (DIR == 1) {
      j = f0 + a;
      k = t2;
    } else {
      j = t2;
      k = f0 + a;
    }
  }
  // stage the primitives of positions f0-3 .. f0+FA+1 (ghosts remapped); kept
  // rolled, since two unrolled trips would hold two cells' states at once
#pragma unroll 1
  for (int e = tid; e < FT::CA * FT::FB; e += FT::NT) {
    const int c = (DIR == 0) ? e : e / FT::FB;
    const int bb = (DIR == 0) ? 0 : e % FT::FB;
    const int pos = f0 - 3 + c;
    const int ii = ibase + bb;
    double Wv[NEQ];
    if (pos >= -3 && pos <= nd + 2 && (DIR == 0 || ii < nx)) {
      bool flip;
      const int g = ghost_index(pos, nd, pm.bc_lo[DIR], pm.bc_hi[DIR], flip);
      const long long cell = cell_at<DIR>(g, ii, j, k, nx, ny);
      double U[NEQ];
#pragma unroll
      for (int v = 0; v < NEQ; ++v) U[v] = q[v * nc + cell];
      if (flip) U[R::MOM + DIR] = -U[R::MOM + DIR];
      cons_to_prim<NF, D>(pm, U, Wv);
    } else {
#pragma unroll
      for (int v = 0; v < NEQ; ++v) Wv[v] = 0.0;
    }
#pragma unroll
    for (int v = 0; v < NEQ; ++v) sw[face_lds<DIR>(v, c, bb)] = Wv[v];
  }
  __syncthreads();
  const int f = f0 + a;
  if (f > nd || (DIR != 0 && i >= nx)) return;
  const long long id = ((long long)k * fg.fy + j) * fg.fx + i;
  // stencil slot s = 0..5 holds position f-3+s
  auto Ws = [&](int s, int v) -> double { return sw[face_lds<DIR>(v, a + s, b)]; };

  // face cotangents: Fbar = (rbar_f - rbar_{f-1})/dx over interior cells, and
  // ufbar from the alpha source of the two cells sharing the face
  // 1/h of the two cells sharing the face (tabulated on a non-uniform grid)
  const double ih0 = (WV == kWvNonUniform) ? inv_width(pm, DIR, f - 1) : pm.inv_dx[DIR];
  const double ih1 = (WV == kWvNonUniform) ? inv_width(pm, DIR, f) : pm.inv_dx[DIR];
  const bool in0 = f - 1 >= 0, in1 = f < nd;
  const long long c0 = cell_at<DIR>(in0 ? f - 1 : 0, i, j, k, nx, ny);
  const long long c1 = cell_at<DIR>(in1 ? f : 0, i, j, k, nx, ny);
  double Fb[NEQ];
  double ufb = 0.0;
  // the alpha rows' source factors of the two cells: alpha_i, or alpha_i +- K
  // with Kapila's K of that cell (RS_KAPILA)
  double K0 = 0.0, K1 = 0.0;
  if constexpr (NF == 2 && (RS & RS_KAPILA) != 0) {
    K0 = kapila_K(pm, Ws(2, R::E), Ws(2, R::ALPHA), Ws(2, R::ALPHA + 1));
    K1 = kapila_K(pm, Ws(3, R::E), Ws(3, R::ALPHA), Ws(3, R::ALPHA + 1));
  }
#pragma unroll
  for (int v = 0; v < NEQ; ++v) {
    const double r0 = in0 ? rbar[v * nc + c0] : 0.0;
    const double r1 = in1 ? rbar[v * nc + c1] : 0.0;
    Fb[v] = ih1 * r1 - ih0 * r0;
    if constexpr (NF == 2) {
      if (v == R::ALPHA) ufb += ih0 * ((Ws(2, v) + K0) * r0) - ih1 * ((Ws(3, v) + K1) * r1);
      if (v == R::ALPHA + 1) ufb += ih0 * ((Ws(2, v) - K0) * r0) - ih1 * ((Ws(3, v) - K1) * r1);
    }
  }

  // non-uniform grid: table entries of the centres f - 1 and f along the axis
  const long long nst = (long long)nd + 6;
  const double* cfa = nullptr;
  const double* cfb = nullptr;
  if constexpr (WV == kWvNonUniform) {
    cfa = pm.nu[DIR] + (f - 1 + 3);
    cfb = pm.nu[DIR] + (f + 3);
  }
  double WL[NEQ], WR[NEQ];
#pragma unroll
  for (int v = 0; v < NEQ; ++v) {
    double l, r, t;
    if constexpr (WV == kWvNonUniform) {
      weno5_nu(Ws(0, v), Ws(1, v), Ws(2, v), Ws(3, v), Ws(4, v), pm.eps, cfa, nst, l, t);
      weno5_nu(Ws(1, v), Ws(2, v), Ws(3, v), Ws(4, v), Ws(5, v), pm.eps, cfb, nst, t, r);
    } else {
      weno5<WV>(Ws(0, v), Ws(1, v), Ws(2, v), Ws(3, v), Ws(4, v), pm.eps, l, t);
      weno5<WV>(Ws(1, v), Ws(2, v), Ws(3, v), Ws(4, v), Ws(5, v), pm.eps, t, r);
    }
    WL[v] = l;
    WR[v] = r;
  }
  double WLb[NEQ], WRb[NEQ];
#pragma unroll
  for (int v = 0; v < NEQ; ++v) WLb[v] = WRb[v] = 0.0;
  double uf;
  // RS bit 1: the low-Mach correction precedes the face solver; its adjoint
  // follows the solver's
  double uL0 = 0.0, uR0 = 0.0;
  if constexpr ((RS & RS_THORNBER) != 0) {
    uL0 = WL[Rows<NF, D>::MOM + DIR];
    uR0 = WR[Rows<NF, D>::MOM + DIR];
    thornber<NF, D, DIR, double>(pm, WL, WR);
  }
  riemann_vjp<RS, NF, D, DIR>(pm, WL, WR, Fb, ufb, WLb, WRb, &uf);
  if constexpr ((RS & RS_THORNBER) != 0) thornber_vjp<NF, D, DIR>(pm, WL, WR, uL0, uR0, WLb, WRb);

  const long long nfc = fg.count;
  // compiler-only memory barrier: the stencil values are read from LDS again
  // below instead of being kept live in registers across the HLLC adjoint
  asm volatile("" ::: "memory");
#pragma unroll
  for (int v = 0; v < NEQ; ++v) {
    double g[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double gr[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (WV == kWvNonUniform) {
      // centre f - 1 gives the left state (its right-face value), centre f
      // the right state (its left-face value); gr holds centre f's stencil
      // in natural order, folded below as the reversed uniform stencils are
      weno_nu_vjp(Ws(0, v), Ws(1, v), Ws(2, v), Ws(3, v), Ws(4, v), pm.eps, cfa, nst, WLb[v], 0.0, g);
      double gb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      weno_nu_vjp(Ws(1, v), Ws(2, v), Ws(3, v), Ws(4, v), Ws(5, v), pm.eps, cfb, nst, 0.0, WRb[v], gb);
#pragma unroll
      for (int k = 0; k < 5; ++k) gr[4 - k] = gb[k];
    } else if constexpr (WV == 1) {
      weno_z_left_vjp(Ws(0, v), Ws(1, v), Ws(2, v), Ws(3, v), Ws(4, v), pm.eps, WLb[v], g);
      weno_z_left_vjp(Ws(5, v), Ws(4, v), Ws(3, v), Ws(2, v), Ws(1, v), pm.eps, WRb[v], gr);
    } else if constexpr (WV == 2) {
      teno_left_vjp(Ws(0, v), Ws(1, v), Ws(2, v), Ws(3, v), Ws(4, v), pm.eps, WLb[v], g);
      teno_left_vjp(Ws(5, v), Ws(4, v), Ws(3, v), Ws(2, v), Ws(1, v), pm.eps, WRb[v], gr);
    } else if constexpr (WV == 3) {
      weno_m_left_vjp(Ws(0, v), Ws(1, v), Ws(2, v), Ws(3, v), Ws(4, v), pm.eps, WLb[v], g);
      weno_m_left_vjp(Ws(5, v), Ws(4, v), Ws(3, v), Ws(2, v), Ws(1, v), pm.eps, WRb[v], gr);
    } else {
      weno_left_vjp(Ws(0, v), Ws(1, v), Ws(2, v), Ws(3, v), Ws(4, v), pm.eps, WLb[v], g);
      weno_left_vjp(Ws(5, v), Ws(4, v), Ws(3, v), Ws(2, v), Ws(1, v), pm.eps, WRb[v], gr);
    }
    g[1] += gr[4];
    g[2] += gr[3];
    g[3] += gr[2];
    g[4] += gr[1];
    g[5] += gr[0];
#pragma unroll
    for (int s = 0; s < 6; ++s) G[(long long)(s * NEQ + v) * nfc + id] = g[s];
  }
  UF[id] = uf;
}

template <int DIR>
__device__ __forceinline__ AxisGeom face_geom(const Params& pm) {
  AxisGeom fg{pm.n[0] + (DIR == 0), pm.n[1] + (DIR == 1), pm.n[2] + (DIR == 2), 0};
  fg.count = (long long)fg.fx * fg.fy * fg.fz;
  return fg;
}

template <int DIR>
__device__ __forceinline__ void unflatten_tile(int w, const Params& pm, int& t0, int& t1, int& t2) {
  int g0, g1, g2;
  face_grid<DIR>(pm.n, g0, g1, g2);
  (void)g2;
  t0 = w % g0;
  t1 = (w / g0) % g1;
  t2 = w / (g0 * g1);
}

// Face pass of one axis (sequential path).
template <int NF, int D, int DIR, int WV, int RS>
__global__ __launch_bounds__(kFaceThreads) void vjp_face_kernel(Params pm, const double* __restrict__ q,
                                                               const double* __restrict__ rbar,
                                                               double* __restrict__ G, double* __restrict__ UF) {
  __shared__ double sw[FaceLds<Rows<NF, D>::NEQ>::size];
  int t0, t1, t2;
  unflatten_tile<DIR>(blockIdx.x, pm, t0, t1, t2);
  face_tile<NF, D, DIR, WV, RS>(pm, q, rbar, G, UF, face_geom<DIR>(pm), t0, t1, t2, threadIdx.x, sw);
}

// Face passes of every axis in one launch: blocks [0, nb[0]) take x tiles,
// the next nb[1] y tiles, then z.  Each axis writes its own G and UF.
template <int NF, int D, int WV, int RS>
__global__ __launch_bounds__(kFaceThreads) void vjp_faces_all_kernel(Params pm, const double* __restrict__ q,
                                                                    const double* __restrict__ rbar, VjpScratch sc,
                                                                    int nb0, int nb1) {
  __shared__ double sw[FaceLds<Rows<NF, D>::NEQ>::size];
  int w = blockIdx.x, t0, t1, t2;
  if (w < nb0) {
    unflatten_tile<0>(w, pm, t0, t1, t2);
    face_tile<NF, D, 0, WV, RS>(pm, q, rbar, sc.Gd[0], sc.UFd[0], face_geom<0>(pm), t0, t1, t2, threadIdx.x, sw);
    return;
  }
  w -= nb0;
  if constexpr (D > 1) {
    if (w < nb1) {
      unflatten_tile<1>(w, pm, t0, t1, t2);
      face_tile<NF, D, 1, WV, RS>(pm, q, rbar, sc.Gd[1], sc.UFd[1], face_geom<1>(pm), t0, t1, t2, threadIdx.x, sw);
      return;
    }
    w -= nb1;
  }
  if constexpr (D > 2) {
    unflatten_tile<2>(w, pm, t0, t1, t2);
    face_tile<NF, D, 2, WV, RS>(pm, q, rbar, sc.Gd[2], sc.UFd[2], face_geom<2>(pm), t0, t1, t2, threadIdx.x, sw);
  }
}

template <int NF, int D, int DIR>
__device__ __forceinline__ void add_face_terms(const double* __restrict__ G, long long nfc, const AxisGeom& fg,
                                               int i, int j, int k, int pos, int nd, double* wb) {
  using R = Rows<NF, D>;
  constexpr int NEQ = R::NEQ;
  // faces holding position pos in their stencils: f = pos + 3 - s, s = 0..5
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int f = pos + 3 - s;
    if (f < 0 || f > nd) continue;
    int fi[3] = {i, j, k};
    fi[DIR] = f;
    const long long fid = ((long long)fi[2] * fg.fy + fi[1]) * fg.fx + fi[0];
#pragma unroll
    for (int v = 0; v < NEQ; ++v) wb[v] += G[(long long)(s * NEQ + v) * nfc + fid];
  }
}

// Primitive cotangent of cell (i, j, k) from the faces of axis DIR, including
// every ghost position the boundary condition fills from it (normal-velocity
// entry negated for slip walls), and that axis's part of the alpha-source
// divergence.
template <int NF, int D, int DIR>
__device__ __forceinline__ void gather_axis(const Params& pm, const double* __restrict__ G,
                                            const double* __restrict__ UF, int i, int j, int k, double* wb,
                                            double& div) {
  using R = Rows<NF, D>;
  constexpr int NEQ = R::NEQ;
  const AxisGeom fg = face_geom<DIR>(pm);
  const int nd = pm.n[DIR];
  const int idx[3] = {i, j, k};
  const int p = idx[DIR];
  add_face_terms<NF, D, DIR>(G, fg.count, fg, i, j, k, p, nd, wb);
  // ghost positions filled from this cell (only cells within three of an end,
  // or of the far end for periodic axes, have any)
  if (p < 3 || p >= nd - 3) {
#pragma unroll
    for (int gsl = 0; gsl < 6; ++gsl) {
      const int gp = gsl < 3 ? -1 - gsl : nd + gsl - 3;
      bool flip;
      if (ghost_index(gp, nd, pm.bc_lo[DIR], pm.bc_hi[DIR], flip) != p) continue;
      double wg[NEQ];
#pragma unroll
      for (int v = 0; v < NEQ; ++v) wg[v] = 0.0;
      add_face_terms<NF, D, DIR>(G, fg.count, fg, i, j, k, gp, nd, wg);
      if (flip) wg[R::MOM + DIR] = -wg[R::MOM + DIR];
#pragma unroll
      for (int v = 0; v < NEQ; ++v) wb[v] += wg[v];
    }
  }
  if constexpr (NF == 2) {
    int f0[3] = {i, j, k};
    f0[DIR] = p;
    const long long fid0 = ((long long)f0[2] * fg.fy + f0[1]) * fg.fx + f0[0];
    int f1[3] = {i, j, k};
    f1[DIR] = p + 1;
    const long long fid1 = ((long long)f1[2] * fg.fy + f1[1]) * fg.fx + f1[0];
    div += inv_width(pm, DIR, p) * (UF[fid1] - UF[fid0]);
  }
}

// Cell pass: cons->prim^T of the summed primitive cotangent plus the direct
// alpha term rbar_alpha * div u, for the axes in [D0, D1); qbar is written
// (or accumulated) once.
template <int NF, int D, int D0, int D1>
__global__ __launch_bounds__(256) void vjp_gather_kernel(Params pm, const double* __restrict__ q,
                                                         const double* __restrict__ rbar, VjpScratch sc,
                                                         double* __restrict__ qbar, int accumulate, StageEpi epi) {
  using R = Rows<NF, D>;
  constexpr int NEQ = R::NEQ;
  const long long nc = pm.ncell;
  const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= nc) return;
  const int nx = pm.n[0], ny = pm.n[1];
  const int i = (int)(cell % nx), j = (int)((cell / nx) % ny), k = (int)(cell / ((long long)nx * ny));
  double wb[NEQ];
#pragma unroll
  for (int v = 0; v < NEQ; ++v) wb[v] = 0.0;
  double div = 0.0;
  if constexpr (D0 <= 0 && 0 < D1) gather_axis<NF, D, 0>(pm, sc.Gd[0], sc.UFd[0], i, j, k, wb, div);
  if constexpr (D0 <= 1 && 1 < D1 && D > 1) gather_axis<NF, D, 1>(pm, sc.Gd[1], sc.UFd[1], i, j, k, wb, div);
  if constexpr (D0 <= 2 && 2 < D1 && D > 2) gather_axis<NF, D, 2>(pm, sc.Gd[2], sc.UFd[2], i, j, k, wb, div);
  double U[NEQ], Ub[NEQ];
#pragma unroll
  for (int v = 0; v < NEQ; ++v) {
    U[v] = q[v * nc + cell];
    Ub[v] = 0.0;
  }
  if constexpr (NF == 2) {
    // Kapila's K of the cell scales the summed divergence on both alpha rows,
    // (alpha_1 + K) and (alpha_2 - K): Kbar = div (rbar_alpha1 - rbar_alpha2),
    // pushed to the cell's primitive p and volume fractions
    if (pm.model == 1) {
      double W[NEQ];
      cons_to_prim<NF, D>(pm, U, W);
      double dp, da1, da2;
      kapila_K_grad(pm, W[R::E], W[R::ALPHA], W[R::ALPHA + 1], dp, da1, da2);
      const double Kb = div * (rbar[R::ALPHA * nc + cell] - rbar[(R::ALPHA + 1) * nc + cell]);
      wb[R::E] += Kb * dp;
      wb[R::ALPHA] += Kb * da1;
      wb[R::ALPHA + 1] += Kb * da2;
    }
  }
  cons_to_prim_vjp<NF, D>(pm, U, wb, Ub);
  if constexpr (NF == 2) {
#pragma unroll
    for (int a = 0; a < 2; ++a) Ub[R::ALPHA + a] += rbar[(R::ALPHA + a) * nc + cell] * div;
  }
  // qbar, or (epi.stage > 0) the reverse stage combination of v = Ub, the
  // same operations as launch_adj_stage's
#pragma unroll
  for (int v = 0; v < NEQ; ++v) {
    const long long e = v * nc + cell;
    if (epi.stage == 3) {
      const double x = epi.x[e];
      epi.out[e] = (2.0 / 3.0) * (x + epi.dt * Ub[v]);
      epi.qnb[e] = (1.0 / 3.0) * x;
    } else if (epi.stage == 2) {
      const double x = epi.x[e];
      epi.out[e] = 0.25 * (x + epi.dt * Ub[v]);
      epi.qnb[e] = epi.qnb[e] + 0.75 * x;
    } else if (epi.stage == 1) {
      epi.qnb[e] = epi.qnb[e] + (epi.x[e] + epi.dt * Ub[v]);
    } else {
      qbar[e] = accumulate ? qbar[e] + Ub[v] : Ub[v];
    }
  }
}

template <int DIR>
static int face_blocks(const Params& pm) {
  int g0, g1, g2;
  face_grid<DIR>(pm.n, g0, g1, g2);
  return g0 * g1 * g2;
}

// Sequential path: per axis, its face pass into the shared buffer Gd[0] /
// UFd[0], then its cell pass.
template <int NF, int D, int DIR, int WV, int RS>
static hipError_t launch_axis_vjp(const Params& pm, const double* q, const double* rbar, double* qbar,
                                  VjpScratch sc, bool accumulate, hipStream_t s) {
  hipLaunchKernelGGL((vjp_face_kernel<NF, D, DIR, WV, RS>), dim3((unsigned)face_blocks<DIR>(pm)), dim3(kFaceThreads), 0, s,
                     pm, q, rbar, sc.Gd[0], sc.UFd[0]);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the cell pass reads the axis's buffers through slot DIR
  VjpScratch one = sc;
  one.Gd[DIR] = sc.Gd[0];
  one.UFd[DIR] = sc.UFd[0];
  hipLaunchKernelGGL((vjp_gather_kernel<NF, D, DIR, DIR + 1>), dim3((unsigned)((pm.ncell + 255) / 256)), dim3(256), 0,
                     s, pm, q, rbar, one, qbar, accumulate ? 1 : 0, StageEpi{0, 0.0, nullptr, nullptr, nullptr});
  return hipGetLastError();
}

template <int NF, int D, int WV, int RS>
static hipError_t launch_rhs_vjp_t(const Params& pm, const double* q, const double* rbar, double* qbar,
                                   const VjpScratch& sc, bool accumulate, hipStream_t s, PassTimer* tm,
                                   const StageEpi& epi) {
  hipError_t e = hipSuccess;
  if (tm) tm->begin(KIND_VJP, s);
  if (sc.all_axes) {
    // every axis's faces in one launch, then one cell pass
    const int nb0 = face_blocks<0>(pm);
    const int nb1 = D > 1 ? face_blocks<(D > 1 ? 1 : 0)>(pm) : 0;
    const int nb2 = D > 2 ? face_blocks<(D > 2 ? 2 : 0)>(pm) : 0;
    hipLaunchKernelGGL((vjp_faces_all_kernel<NF, D, WV, RS>), dim3((unsigned)(nb0 + nb1 + nb2)), dim3(kFaceThreads), 0, s, pm,
                       q, rbar, sc, nb0, nb1);
    e = hipGetLastError();
    if (e == hipSuccess) {
      hipLaunchKernelGGL((vjp_gather_kernel<NF, D, 0, D>), dim3((unsigned)((pm.ncell + 255) / 256)), dim3(256), 0, s,
                         pm, q, rbar, sc, qbar, accumulate ? 1 : 0, epi);
      e = hipGetLastError();
    }
  } else {
    e = launch_axis_vjp<NF, D, 0, WV, RS>(pm, q, rbar, qbar, sc, accumulate, s);
    if (e == hipSuccess && D > 1) e = launch_axis_vjp<NF, D, (D > 1 ? 1 : 0), WV, RS>(pm, q, rbar, qbar, sc, true, s);
    if (e == hipSuccess && D > 2) e = launch_axis_vjp<NF, D, (D > 2 ? 2 : 0), WV, RS>(pm, q, rbar, qbar, sc, true, s);
  }
  if (tm) tm->end(KIND_VJP, s);
  return e;
}

// The face options are compile-time choices, as in the forward passes.
template <int NF, int D, int WV>
static hipError_t vjp_by_riemann(const Params& pm, const double* q, const double* rbar, double* qbar,
                                 const VjpScratch& sc, bool accumulate, hipStream_t s, PassTimer* tm,
                                 const StageEpi& epi) {
#define MFC_RS(B) \
  case B: return launch_rhs_vjp_t<NF, D, WV, B>(pm, q, rbar, qbar, sc, accumulate, s, tm, epi);
  switch (option_bits(pm)) {
    MFC_RS(0)
    MFC_RS(RS_HLL)
    MFC_RS(RS_THORNBER)
    MFC_RS(RS_HLL | RS_THORNBER)
    MFC_RS(RS_APC)
    default: break;
  }
  if constexpr (NF == 2) {
    switch (option_bits(pm)) {
      MFC_RS(RS_KAPILA)
      MFC_RS(RS_KAPILA | RS_HLL)
      MFC_RS(RS_KAPILA | RS_THORNBER)
      MFC_RS(RS_KAPILA | RS_HLL | RS_THORNBER)
      MFC_RS(RS_KAPILA | RS_APC)
      default: break;
    }
  }
#undef MFC_RS
  return hipErrorInvalidValue;
}

// Every grid of one reconstruction variant.
template <int WV>
hipError_t launch_rhs_vjp_wv(int nf, int ndim, const Params& pm, const double* q, const double* rbar, double* qbar,
                             const VjpScratch& sc, bool accumulate, hipStream_t s, PassTimer* tm,
                             const StageEpi& epi) {
#define MFC_CASE(NF, D) \
  if (nf == NF && ndim == D) return vjp_by_riemann<NF, D, WV>(pm, q, rbar, qbar, sc, accumulate, s, tm, epi);
  MFC_CASE(1, 1)
  MFC_CASE(1, 2)
  MFC_CASE(1, 3)
  MFC_CASE(2, 1)
  MFC_CASE(2, 2)
  MFC_CASE(2, 3)
#undef MFC_CASE
  return hipErrorInvalidValue;
}

#define MFC_VJP_DECL(KW, WV)                                                                                 \
  KW template hipError_t launch_rhs_vjp_wv<WV>(int, int, const Params&, const double*, const double*, double*, \
                                               const VjpScratch&, bool, hipStream_t, PassTimer*, const StageEpi&);
#define MFC_INSTANTIATE_VJP(WV) MFC_VJP_DECL(, WV)
#define MFC_EXTERN_VJP(WV) MFC_VJP_DECL(extern, WV)

}  // namespace mfc
