// sweep_impl.h -- the fused axis-pass kernel of the five-equation RHS and its
// launch sequence, templated on the reconstruction variant WV.  Each
// sweep_wv*.hip translation unit instantiates one variant (so that the
// variants compile in parallel); sweep.hip dispatches among them.
// One fused pass per grid axis of the five-equation RHS.
//
// A pass over axis DIR does, for a tile of cells, in one kernel:
//   (a) load the conservative state of the tile plus three ghost/halo cells on
//       each side along DIR (ghost layers by index remap, Sec. 3.3), convert it
//       to primitive variables (double pressure inversion) and stage it in LDS;
//   (b) WENO5-JS at every reconstruction centre of the tile (Sec. 3.2.1):
//       the left-biased value at c+1/2 and the right-biased value at c-1/2;
//   (c) HLLC at every face between two centres (Sec. 3.2.2): flux and face
//       velocity;
//   (d) the axis contribution of eq. eqn:rhs for every output cell:
//       (F_{-1/2} - F_{+1/2})/dx plus alpha (u_{+1/2} - u_{-1/2})/dx on the
//       volume-fraction rows, which is written to the RHS accumulator, added
//       to it, or (on the last axis of an SSP-RK3 stage) combined with the
//       stage states into the next stage state.
// Reconstructed states, fluxes and face velocities live only in registers
// and LDS; HBM sees one read of the stage state (plus halos), the RHS
// accumulator round trip and the stage combination.  In the x pass the
// values of neighbouring centres move between adjacent lanes (DPP) instead
// of through LDS, and the stage update takes the centre's state from the
// primitives still in LDS rather than reading q_k a second time.
//
// Tile shapes (wave64): along x the centres of a tile are the 64 lanes of a
// wave, one wave per x-row, 4 rows per block; along y and z, 32 x-lanes by 16
// centres along the sweep axis (512 threads; in FP64, 16 lanes by 16 centres
// for y in 3D and 16 lanes by 32 centres for z).  Every access to q is to x-
// contiguous runs, so all three passes read HBM coalesced without any
// transposition of the state.
#pragma once

#include "device.h"
#include "internal.h"

namespace mfc {

// Accumulator access with or without the non-temporal cache hint.
template <bool NT, typename Real>
__device__ __forceinline__ Real ld_acc(const Real* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
template <bool NT, typename Real>
__device__ __forceinline__ void st_acc(Real v, Real* p) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Exchange between adjacent lanes of a wave (DPP wave_shr:1 / wave_shl:1):
// lane i receives lane i-1's value (kFromPrev) or lane i+1's (kFromNext); the
// lane at the end with no source receives 0.  Called with every lane active.
constexpr int kFromPrev = 0x138;
constexpr int kFromNext = 0x130;
template <int CTRL>
__device__ __forceinline__ double lane_shift(double x) {
  const long long bits = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(bits & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float lane_shift(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}

template <int DIR, int D, typename Real>
struct Tile {
  // TA: reconstruction centres per tile along the sweep axis (outputs TA - 2)
  // TB: independent lines across the sweep axis (x lanes for y and z).  In
  // FP64 the y pass of a 3D stage runs 16 lanes (256-thread blocks, twice the
  // blocks per CU) and the z pass 32 centres x 16 lanes (halo loads 36 per 30
  // outputs instead of 20 per 14); both measured faster in FP64, slower in FP32.
  static constexpr bool kF64 = sizeof(Real) == 8;
  static constexpr int TA = (DIR == 0) ? 64 : ((DIR == 2 && kF64) ? 32 : 16);
  static constexpr int TB = (DIR == 0) ? ((D == 1) ? 1 : 4) : ((kF64 && (DIR == 2 || D == 3)) ? 16 : 32);
  static constexpr int NT = TA * TB;
  static constexpr int OUT = TA - 2;
  static constexpr int SA = TA + 4;  // LDS slots along the sweep axis
};

// LDS index of (row v, slot s along the sweep axis, line b).
template <int DIR, int D, typename Real>
__device__ __forceinline__ int lds_index(int v, int s, int b) {
  using TL = Tile<DIR, D, Real>;
  if constexpr (DIR == 0)
    return (v * TL::TB + b) * TL::SA + s;
  else
    return (v * TL::SA + s) * TL::TB + b;
}

template <int NF, int D, int DIR, typename Real, int MODE, int WV, int RS>
__global__ __launch_bounds__((Tile<DIR, D, Real>::NT)) void sweep_kernel(Params pm, const Real* __restrict__ qk,
                                                                 Real* __restrict__ acc,
                                                                 const Real* __restrict__ qn,
                                                                 Real* __restrict__ qout, StageArgs st,
                                                                 int* __restrict__ flag, long long block_base) {
  using R = Rows<NF, D>;
  using TL = Tile<DIR, D, Real>;
  constexpr int NEQ = R::NEQ;
  __shared__ Real sh[(NEQ + 1) * TL::SA * TL::TB];
  // x pass: a tile row is one wave of 64 centres, so the neighbours a - 1 and
  // a + 1 of centre a are the adjacent lanes.  The biased values and the
  // fluxes move between lanes by DPP and the LDS keeps the primitives to the
  // end (no barrier after the load); the double stage update takes the
  // centre's conservative values from them instead of a second read of q_k.
  constexpr bool kLaneX = DIR == 0;
  static_assert(!kLaneX || TL::TA == 64, "an x tile row is one wave");
  constexpr bool kCentreFromLds = kLaneX && sizeof(Real) == 8 && (MODE & MODE_STEP) != 0;

  const int nx = pm.n[0], ny = pm.n[1];
  const int nd = pm.n[DIR];
  const long long nc = pm.ncell;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;

  // tile origin (first output cell along DIR) and the fixed coordinates
  int a, b, org, cx = 0, cy = 0, cz = 0;
  if constexpr (DIR == 0 && D > 1) {
    // One-dimensional grid.  Blocks are dispatched to the eight XCDs in turn
    // (block L to XCD L mod 8); XCD k takes the x tiles of row group
    // 8 g + k in order (g = (L / 8) / tiles per row), so neighbouring x tiles,
    // which share the 128-byte lines at their edges and their halo, run on
    // one XCD one after the other, while the eight XCDs work on adjacent
    // row groups at any time.
    a = threadIdx.x;
    b = threadIdx.y;
    const long long ntx = (nx + TL::OUT - 1) / TL::OUT;
    const long long nrg_y = (ny + TL::TB - 1) / TL::TB;
    const long long L = block_base + blockIdx.x;  // launches come in chunks that start at multiples of 8
    const long long j = L >> 3;
    const long long g = j / ntx;
    const long long rg = g * 8 + (L & 7);
    if (rg >= nrg_y * pm.n[2]) return;  // padding blocks of the last group of eight
    org = (int)(j - g * ntx) * TL::OUT;
    cz = (int)(rg / nrg_y);
    cy = (int)(rg - cz * nrg_y) * TL::TB;  // + line
  } else if constexpr (DIR == 0) {
    a = threadIdx.x;
    b = threadIdx.y;
    org = blockIdx.x * TL::OUT;
    cy = blockIdx.y * TL::TB;  // + line
    cz = blockIdx.z;
  } else if constexpr (DIR == 1) {
    b = threadIdx.x;
    a = threadIdx.y;
    cx = blockIdx.x * TL::TB;
    org = blockIdx.y * TL::OUT;
    cz = blockIdx.z;
  } else {
    b = threadIdx.x;
    a = threadIdx.y;
    cx = blockIdx.x * TL::TB;
    cy = blockIdx.y;
    org = blockIdx.z * TL::OUT;
  }

  // ---- (a) load + convert the tile and its halo into LDS -------------------
  // MODE_SIGNAL: the signal speed of the tile's own cells (slots 3 .. 2 + OUT,
  // inside the grid) as well; the tiles partition the grid, so the block
  // maxima cover every cell once.
  constexpr bool kSignal = (MODE & MODE_SIGNAL) != 0;
  __shared__ double sred[kSignal ? TL::NT / 64 : 1];
  double smax = 0.0;
  bool sbad = false;
  // A thread holds at most kIt cells of the tile (kIt = 2 for every tile
  // shape).  In the x and z passes the loads of all of them are issued before
  // the first conversion, so that a thread with two cells waits for memory
  // once (x pass -1.2 %, z -0.8 %); the y pass, which prefetches its
  // accumulator behind this phase, measured 2.5 % slower that way and
  // converts each cell as it arrives.
  constexpr int kCells = TL::SA * TL::TB;
  constexpr int kIt = (kCells + TL::NT - 1) / TL::NT;
  constexpr bool kBatchLoads = DIR != 1;
  double U[kIt][NEQ];
  int slot[kIt], line[kIt], cpos[kIt], cix[kIt][3];
  bool live[kIt], flip[kIt];
  auto load_cell = [&](int it) {
    const int L = tid + it * TL::NT;
    int s, bb;
    if constexpr (DIR == 0) {
      bb = L / TL::SA;
      s = L - bb * TL::SA;
    } else {
      s = L / TL::TB;
      bb = L - s * TL::TB;
    }
    const int pos = org - 3 + s;
    int ix = cx, iy = cy, iz = cz;
    bool inb;
    if constexpr (DIR == 0) {
      iy += bb;
      inb = iy < ny;
    } else {
      ix += bb;
      inb = ix < nx;
    }
    live[it] = L < kCells && inb && pos <= nd + 2;
    slot[it] = s;
    line[it] = bb;
    cpos[it] = pos;
    flip[it] = false;
    if (!live[it]) return;
    const int g = ghost_index(pos, nd, pm.bc_lo[DIR], pm.bc_hi[DIR], flip[it]);
    if constexpr (DIR == 0) ix = g;
    else if constexpr (DIR == 1) iy = g;
    else iz = g;
    cix[it][0] = ix;
    cix[it][1] = iy;
    cix[it][2] = iz;
    const long long cell = ((long long)iz * ny + iy) * nx + ix;
#pragma unroll
    for (int v = 0; v < NEQ; ++v) U[it][v] = double(qk[v * nc + cell]);
  };
  auto convert_cell = [&](int it) {
    if (!live[it]) return;
    const int s = slot[it], bb = line[it];
    double W[NEQ];
    if (flip[it]) U[it][R::MOM + DIR] = -U[it][R::MOM + DIR];
    cons_to_prim<NF, D>(pm, U[it], W);
#pragma unroll
    for (int v = 0; v < NEQ; ++v) sh[lds_index<DIR, D, Real>(v, s, bb)] = Real(W[v]);
    if constexpr (kSignal) {
      if (s >= 3 && s < 3 + TL::OUT && cpos[it] < nd) {
        double ih[D];
#pragma unroll
        for (int d = 0; d < D; ++d) ih[d] = (WV == kWvNonUniform) ? inv_width(pm, d, cix[it][d]) : pm.inv_dx[d];
        bool b;
        const double sg = cell_signal<NF, D>(pm, U[it], W, b, ih);
        sbad |= b;
        smax = (sg > smax) ? sg : smax;  // NaN never wins; it is flagged instead
      }
    }
  };
  if constexpr (kBatchLoads) {
#pragma unroll
    for (int it = 0; it < kIt; ++it) load_cell(it);
#pragma unroll
    for (int it = 0; it < kIt; ++it) convert_cell(it);
  } else {
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      load_cell(it);
      convert_cell(it);
    }
  }
  if constexpr (kSignal) {
    if (sbad) atomicOr(flag, 1);
    smax = wave_max(smax);
    if ((tid & 63) == 0) sred[tid >> 6] = smax;
  }
  __syncthreads();
  if constexpr (kSignal) {
    if (tid == 0) {
      double m = sred[0];
      for (int w = 1; w < TL::NT / 64; ++w) m = fmax(m, sred[w]);
      st.sig_partial[blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z)] = m;
    }
  }

  // this thread's reconstruction centre and line
  const int c = org - 1 + a;
  int ox = cx, oy = cy, oz = cz;
  bool line_ok;
  if constexpr (DIR == 0) {
    oy += b;
    line_ok = oy < ny;
  } else {
    ox += b;
    line_ok = ox < nx;
  }
  const bool centre_ok = line_ok && c <= nd;

  // The accumulator of this thread's output cell is loaded here, so that its
  // latency hides behind the reconstruction: in the y pass, and in the float
  // x pass, which also loads q^n here (in the double x pass the 16 extra
  // VGPRs cost a wave per SIMD and the pass got 12 % slower; it issues those
  // loads together at the start of the update instead)
  constexpr bool kPrefetch =
      (DIR == 1 && MODE == MODE_ACC) || (DIR == 0 && D > 1 && (MODE & MODE_ACC) && sizeof(Real) == 4);
  // the y and z passes stream the accumulator with the non-temporal hint (the
  // y pass gained 4 % in FP64; in the x pass it cost 1.5-3 %)
  constexpr bool kNT = DIR != 0;
  Real pre[kPrefetch ? NEQ : 1];
  constexpr bool kPrefetchQn = kPrefetch && DIR == 0 && (MODE & MODE_STEP) != 0;
  Real preq[kPrefetchQn ? NEQ : 1];
  if constexpr (kPrefetch) {
    if (line_ok && a >= 1 && a <= TL::TA - 2 && c >= 0 && c < nd) {
      const long long cell = (DIR == 1) ? ((long long)oz * ny + c) * nx + ox : ((long long)oz * ny + oy) * nx + c;
#pragma unroll
      for (int v = 0; v < NEQ; ++v) pre[v] = ld_acc<kNT>(&acc[v * nc + cell]);
      if constexpr (kPrefetchQn) {
        if (st.stage != 1) {
#pragma unroll
          for (int v = 0; v < NEQ; ++v) preq[v] = qn[v * nc + cell];
        }
      }
    }
  }

  // ---- (b) WENO5-JS at centre c -----------------------------------------------
  // (lanes past the grid leave them unset: no face reads them)
  Real WLc[NEQ], WRc[NEQ];  // value at c+1/2 (left-biased) and at c-1/2 (right-biased)
  // volume fractions of the centre cell for the alpha source; with RS_KAPILA
  // they carry Kapila's K of the cell, (alpha_1 + K, alpha_2 - K)
  Real alpha_cell[2] = {Real(0), Real(0)};
  if (centre_ok) {
    const Real eps = Real(pm.eps);
    // non-uniform grid: the table entry of centre c along this axis
    const long long nst = (long long)nd + 6;
    const Real* cf = nullptr;
    if constexpr (WV == kWvNonUniform) {
      if constexpr (sizeof(Real) == 8)
        cf = (const Real*)pm.nu[DIR] + (c + 3);
      else
        cf = (const Real*)pm.nuf[DIR] + (c + 3);
    }
#pragma unroll
    for (int v = 0; v < NEQ; ++v) {
      const Real f0 = sh[lds_index<DIR, D, Real>(v, a + 0, b)];
      const Real f1 = sh[lds_index<DIR, D, Real>(v, a + 1, b)];
      const Real f2 = sh[lds_index<DIR, D, Real>(v, a + 2, b)];
      const Real f3 = sh[lds_index<DIR, D, Real>(v, a + 3, b)];
      const Real f4 = sh[lds_index<DIR, D, Real>(v, a + 4, b)];
      if constexpr (WV == kWvNonUniform)
        weno5_nu(f0, f1, f2, f3, f4, eps, cf, nst, WLc[v], WRc[v]);
      else
        weno5<WV>(f0, f1, f2, f3, f4, eps, WLc[v], WRc[v]);
    }
    if constexpr (NF == 2) {
      alpha_cell[0] = sh[lds_index<DIR, D, Real>(R::ALPHA, a + 2, b)];
      alpha_cell[1] = sh[lds_index<DIR, D, Real>(R::ALPHA + 1, a + 2, b)];
      if constexpr ((RS & RS_KAPILA) != 0) {
        const double K = kapila_K(pm, double(sh[lds_index<DIR, D, Real>(R::E, a + 2, b)]), double(alpha_cell[0]),
                                  double(alpha_cell[1]));
        alpha_cell[0] = Real(double(alpha_cell[0]) + K);
        alpha_cell[1] = Real(double(alpha_cell[1]) - K);
      }
    }
  }
  if constexpr (!kLaneX) {
    __syncthreads();
    if (centre_ok) {
#pragma unroll
      for (int v = 0; v < NEQ; ++v) sh[lds_index<DIR, D, Real>(v, a, b)] = WLc[v];
    }
    __syncthreads();
  }

  // ---- (c) HLLC at the face c-1/2 between centres c-1 (left) and c (right) ----
  Real F[NEQ];
  Real uf = Real(0);
  const bool face_ok = centre_ok && a >= 1;
  Real WL[NEQ];
  if constexpr (kLaneX) {
#pragma unroll
    for (int v = 0; v < NEQ; ++v) WL[v] = lane_shift<kFromPrev>(WLc[v]);
  }
  if (face_ok) {
    if constexpr (!kLaneX) {
#pragma unroll
      for (int v = 0; v < NEQ; ++v) WL[v] = sh[lds_index<DIR, D, Real>(v, a - 1, b)];
    }
    // RS: face solver and low-Mach treatment (RS_HLL, RS_THORNBER, RS_APC),
    // compile-time so that none costs registers where it is off
    if constexpr ((RS & RS_THORNBER) != 0) thornber<NF, D, DIR, Real>(pm, WL, WRc);
    const bool bad = riemann<RS, NF, D, DIR, Real>(pm, WL, WRc, F, uf);
    if (bad) atomicOr(flag, 1);
  }
  // the face c+1/2, high side of the output cell c (x pass: each flux row
  // moves from lane a + 1 where it is used, below, with every lane active)
  Real uhi = Real(0);
  if constexpr (kLaneX) {
    uhi = lane_shift<kFromNext>(uf);
  } else {
    __syncthreads();
    if (face_ok) {
#pragma unroll
      for (int v = 0; v < NEQ; ++v) sh[lds_index<DIR, D, Real>(v, a, b)] = F[v];
      sh[lds_index<DIR, D, Real>(NEQ, a, b)] = uf;
    }
    __syncthreads();
  }

  // ---- (d) axis contribution for output cell c --------------------------------
  const bool out_ok = line_ok && a >= 1 && a <= TL::TA - 2 && c >= 0 && c < nd;
  if constexpr (!kLaneX) {
    if (!out_ok) return;
  }
  if constexpr (DIR == 0) ox = c;
  else if constexpr (DIR == 1) oy = c;
  else oz = c;
  const long long cell = ((long long)oz * ny + oy) * nx + ox;
  // (x pass: every lane gets here, but only an output lane, 0 <= c < nd, may
  // read the width table)
  const Real inv_dx = Real((WV == kWvNonUniform) ? (out_ok ? inv_width(pm, DIR, c) : 0.0) : pm.inv_dx[DIR]);
  if constexpr (!kLaneX) uhi = sh[lds_index<DIR, D, Real>(NEQ, a + 1, b)];
  const Real div = inv_dx * (uhi - uf);
  // the centre's conservative values from its primitives (slot a + 2), each
  // where it is used: the partial densities and volume fractions are the
  // stored rows, momentum is rho u and the energy Gamma p + Pi + rho |u|^2/2
  auto centre_cons = [&](int v) -> double {
    auto w = [&](int r) { return double(sh[lds_index<DIR, D, Real>(r, a + 2, b)]); };
    if (v == R::E) {
      double Wc[NEQ], Uc[NEQ];
#pragma unroll
      for (int r = 0; r < NEQ; ++r) Wc[r] = w(r);
      prim_to_cons<NF, D>(pm, Wc, Uc);
      return Uc[R::E];
    }
    if (v >= R::MOM && v < R::MOM + D) return ((NF == 2) ? w(0) + w(1) : w(0)) * w(v);
    return w(v);
  };
  // the double x pass issues the accumulator and q^n loads of its output cell
  // together, before any of them is used
  constexpr bool kLoadsFirst = kLaneX && sizeof(Real) == 8 && (MODE & MODE_ACC) != 0;
  constexpr bool kQnFirst = kLoadsFirst && (MODE & MODE_STEP) != 0;
  // the float x pass takes q_k of its output cell from memory: those loads
  // are issued together too
  constexpr bool kQkFirst = kLaneX && sizeof(Real) == 4 && (MODE & MODE_STEP) != 0;
  Real accv[kLoadsFirst ? NEQ : 1];
  Real qnl[kQnFirst ? NEQ : 1];
  Real qkl[kQkFirst ? NEQ : 1];
  if constexpr (kQkFirst) {
    if (out_ok) {
#pragma unroll
      for (int v = 0; v < NEQ; ++v) qkl[v] = qk[v * nc + cell];
    }
  }
  if constexpr (kLoadsFirst) {
    if (out_ok) {
#pragma unroll
      for (int v = 0; v < NEQ; ++v) accv[v] = acc[v * nc + cell];
      if constexpr (kQnFirst) {
        if (st.stage != 1) {
#pragma unroll
          for (int v = 0; v < NEQ; ++v) qnl[v] = qn[v * nc + cell];
        }
      }
    }
  }
#pragma unroll
  for (int v = 0; v < NEQ; ++v) {
    Real fhi;
    if constexpr (kLaneX) {
      fhi = lane_shift<kFromNext>(F[v]);
      if (!out_ok) continue;
    } else {
      fhi = sh[lds_index<DIR, D, Real>(v, a + 1, b)];
    }
    Real Dv = inv_dx * (F[v] - fhi);
    if constexpr (NF == 2) {
      if (v == R::ALPHA) Dv = Dv + alpha_cell[0] * div;
      if (v == R::ALPHA + 1) Dv = Dv + alpha_cell[1] * div;
    }
    const long long e = v * nc + cell;
    Real r = Dv;
    if constexpr (kPrefetch)
      r = pre[v] + Dv;
    else if constexpr (kLoadsFirst)
      r = accv[v] + Dv;
    else if constexpr (MODE & MODE_ACC)
      r = ld_acc<kNT>(&acc[e]) + Dv;
    if constexpr (MODE & MODE_STEP) {
      // SSP-RK3, Shu-Osher form (Sec. 3.4), combined in double
      const double dt = st.dt_ptr ? *st.dt_ptr : st.dt;
      double uk;
      if constexpr (kCentreFromLds) {
        uk = centre_cons(v);
      } else if constexpr (kQkFirst) {
        uk = double(qkl[v]);
      } else {
        uk = double(qk[e]);
      }
      const double qs = uk + dt * double(r);
      double out;
      double qnv = 0.0;
      if (st.stage != 1) {
        if constexpr (kPrefetchQn)
          qnv = double(preq[v]);
        else if constexpr (kQnFirst)
          qnv = double(qnl[v]);
        else
          qnv = double(qn[e]);
      }
      if (st.stage == 1)
        out = qs;
      else if (st.stage == 2)
        out = 0.75 * qnv + 0.25 * qs;
      else
        out = (1.0 / 3.0) * qnv + (2.0 / 3.0) * qs;
      qout[e] = Real(out);
    } else {
      st_acc<kNT>(r, &acc[e]);
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <int NF, int D, int DIR, typename Real, int MODE, int WV, int RS>
static hipError_t launch_one(const Params& pm, const Real* qk, Real* acc, const Real* qn, Real* qout,
                             StageArgs st, int* flag, hipStream_t s, PassTimer* tm) {
  using TL = Tile<DIR, D, Real>;
  dim3 block, grid;
  const int nx = pm.n[0], ny = pm.n[1], nz = pm.n[2];
  if constexpr (DIR == 0 && D > 1) {
    // x tiles over groups of eight row groups, launched in chunks of at most
    // 2^24 blocks (64 x 2^24 work-items along x stays below 2^32); every chunk
    // starts at a multiple of 8 so that block L keeps XCD L mod 8
    block = dim3(TL::TA, TL::TB, 1);
    const long long groups = (long long)((ny + TL::TB - 1) / TL::TB) * nz;
    const long long total = (long long)((nx + TL::OUT - 1) / TL::OUT) * ((groups + 7) / 8) * 8;
    constexpr long long kChunk = 1ll << 24;
    hipError_t e = hipSuccess;
    if (tm) tm->begin(KIND_PASS_X, s);
    for (long long base = 0; base < total && e == hipSuccess; base += kChunk) {
      const long long nb = (total - base < kChunk) ? total - base : kChunk;
      hipLaunchKernelGGL((sweep_kernel<NF, D, DIR, Real, MODE, WV, RS>), dim3((unsigned)nb, 1, 1), block, 0, s, pm, qk,
                         acc, qn, qout, st, flag, base);
      e = hipGetLastError();
    }
    if (tm) tm->end(KIND_PASS_X, s);
    return e;
  } else if constexpr (DIR == 0) {
    block = dim3(TL::TA, TL::TB, 1);
    grid = dim3((nx + TL::OUT - 1) / TL::OUT, (ny + TL::TB - 1) / TL::TB, nz);
  } else if constexpr (DIR == 1) {
    block = dim3(TL::TB, TL::TA, 1);
    grid = dim3((nx + TL::TB - 1) / TL::TB, (ny + TL::OUT - 1) / TL::OUT, nz);
  } else {
    block = dim3(TL::TB, TL::TA, 1);
    grid = dim3((nx + TL::TB - 1) / TL::TB, ny, (nz + TL::OUT - 1) / TL::OUT);
  }
  if (tm) tm->begin(KIND_PASS_X + DIR, s);
  hipLaunchKernelGGL((sweep_kernel<NF, D, DIR, Real, MODE, WV, RS>), grid, block, 0, s, pm, qk, acc, qn, qout, st,
                     flag, 0ll);
  if (tm) tm->end(KIND_PASS_X + DIR, s);
  return hipGetLastError();
}

// Blocks of the first axis pass of a 2D / 3D evaluation (y in 2D, z in 3D).
template <int D, typename Real>
static long long first_pass_blocks(const int* n) {
  using TL = Tile<D - 1, D, Real>;
  const long long bx = (n[0] + TL::TB - 1) / TL::TB;
  if constexpr (D == 2)
    return bx * ((n[1] + TL::OUT - 1) / TL::OUT) * n[2];
  else
    return bx * n[1] * ((n[2] + TL::OUT - 1) / TL::OUT);
}

// All axes of one RHS evaluation, z (or y) first and x last.  final_step: the
// x pass combines into qout.  sig (2D / 3D): the first pass also forms the
// signal-speed block maxima and dt is formed before the x pass reads it.
template <int NF, int D, typename Real, int WV, int RS>
static hipError_t launch_rhs_t(const Params& pm, const Real* qk, Real* acc, const Real* qn, Real* qout,
                               StageArgs st, bool final_step, int* flag, hipStream_t s, PassTimer* tm,
                               const SignalFuse* sig) {
  hipError_t e = hipSuccess;
  if constexpr (D == 1) {
    if (sig) return hipErrorInvalidValue;
    if (final_step)
      e = launch_one<NF, D, 0, Real, MODE_STEP, WV, RS>(pm, qk, acc, qn, qout, st, flag, s, tm);
    else
      e = launch_one<NF, D, 0, Real, MODE_WRITE, WV, RS>(pm, qk, acc, qn, qout, st, flag, s, tm);
  } else {
    constexpr int FIRST = D - 1;
    if (sig) {
      StageArgs s1 = st;
      s1.sig_partial = sig->partial;
      e = launch_one<NF, D, FIRST, Real, MODE_WRITE | MODE_SIGNAL, WV, RS>(pm, qk, acc, qn, qout, s1, flag, s, tm);
      if (e != hipSuccess) return e;
      if (tm) tm->begin(KIND_SIGNAL, s);
      e = launch_finalize_dt(sig->partial, (int)first_pass_blocks<D, Real>(pm.n), sig->cfl, sig->t_remaining,
                             sig->smax_out, sig->dt_out, sig->dt_user, s);
      if (tm) tm->end(KIND_SIGNAL, s);
    } else {
      e = launch_one<NF, D, FIRST, Real, MODE_WRITE, WV, RS>(pm, qk, acc, qn, qout, st, flag, s, tm);
    }
    if (e != hipSuccess) return e;
    if constexpr (D == 3) {
      e = launch_one<NF, D, 1, Real, MODE_ACC, WV, RS>(pm, qk, acc, qn, qout, st, flag, s, tm);
      if (e != hipSuccess) return e;
    }
    if (final_step)
      e = launch_one<NF, D, 0, Real, MODE_ACC | MODE_STEP, WV, RS>(pm, qk, acc, qn, qout, st, flag, s, tm);
    else
      e = launch_one<NF, D, 0, Real, MODE_ACC, WV, RS>(pm, qk, acc, qn, qout, st, flag, s, tm);
  }
  return e;
}

// The face solver, the low-Mach treatment and the model are compile-time
// choices too (a run-time branch cost the double x pass 6 VGPRs and a wave per
// SIMD).  The APC term exists for HLLC only and Kapila's K for two fluids only
// (the problem validation rejects the other settings).
template <int NF, int D, typename Real, int WV>
static hipError_t by_riemann(const Params& pm, const Real* qk, Real* acc, const Real* qn, Real* qout, StageArgs st,
                             bool final_step, int* flag, hipStream_t s, PassTimer* tm, const SignalFuse* sig) {
#define MFC_RS(B) \
  case B: return launch_rhs_t<NF, D, Real, WV, B>(pm, qk, acc, qn, qout, st, final_step, flag, s, tm, sig);
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
template <int WV, typename Real>
hipError_t launch_rhs_wv(int nf, int ndim, const Params& pm, const Real* qk, Real* acc, const Real* qn, Real* qout,
                         StageArgs st, bool final_step, int* flag, hipStream_t s, PassTimer* tm,
                         const SignalFuse* sig) {
#define MFC_CASE(NF, D) \
  if (nf == NF && ndim == D) return by_riemann<NF, D, Real, WV>(pm, qk, acc, qn, qout, st, final_step, flag, s, tm, sig);
  MFC_CASE(1, 1)
  MFC_CASE(1, 2)
  MFC_CASE(1, 3)
  MFC_CASE(2, 1)
  MFC_CASE(2, 2)
  MFC_CASE(2, 3)
#undef MFC_CASE
  return hipErrorInvalidValue;
}

// Explicit instantiation (sweep_wv*.hip) and its extern declaration (sweep.hip).
#define MFC_SWEEP_DECL(KW, WV)                                                                                      \
  KW template hipError_t launch_rhs_wv<WV, double>(int, int, const Params&, const double*, double*, const double*, \
                                                   double*, StageArgs, bool, int*, hipStream_t, PassTimer*,       \
                                                   const SignalFuse*);                                            \
  KW template hipError_t launch_rhs_wv<WV, float>(int, int, const Params&, const float*, float*, const float*,     \
                                                  float*, StageArgs, bool, int*, hipStream_t, PassTimer*,         \
                                                  const SignalFuse*);
#define MFC_INSTANTIATE_SWEEP(WV) MFC_SWEEP_DECL(, WV)
#define MFC_EXTERN_SWEEP(WV) MFC_SWEEP_DECL(extern, WV)

}  // namespace mfc
