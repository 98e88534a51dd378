// Multigrid kernels for the pressure equation A phi = b (Sec. 2.4,
// eqs. pc_discretized, jacobi_pc, restriction, prolongation; Algorithm 1) and
// the flexible conjugate-gradient iteration that uses one V-cycle as its
// preconditioner.
//
// A x at an active cell = sum over faces c_f (x_P - x_N) / h_d^2.  Ghost and
// inactive cells of every level array hold 0 and are never written, so the
// same formula covers zero-value outlet faces (c_f = 2 there) and closed faces
// (c_f = 0).  Regular cells (all c_f = 1, neighbours inside the box) skip the
// coefficient loads.
#include <hip/hip_runtime.h>

#include "nfvm_device.hpp"

namespace nfvm {

constexpr int MBX = 64, MBY = 4, MBS = MBX * MBY;

__host__ inline dim3 lvl_grid(const Geom& g) {
  return dim3((g.nx + MBX - 1) / MBX, (g.ny + MBY - 1) / MBY, g.nz);
}

struct LevelView {
  Geom g;
  const uint8_t* cls;
  const float* cf0;
  const float* cf1;
  const float* cf2;
  const uint8_t* full;
};

__host__ inline LevelView view(const Level& l) {
  return LevelView{l.g, l.cls, l.cf[0], l.cf[1], l.g.dim == 3 ? l.cf[2] : l.cf[0], l.full};
}

// Coarse cells whose 26 neighbours are all active and inside the box: the
// prolongation from them needs no boundary or mask checks.
__global__ void k_mark_full(Geom g, const uint8_t* __restrict__ cls, uint8_t* __restrict__ full) {
  const int i = blockIdx.x * MBX + threadIdx.x, j = blockIdx.y * MBY + threadIdx.y, k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  bool f = true;
  const int kz = g.dim == 3 ? 1 : 0;
  for (int c = -kz; c <= kz && f; ++c)
    for (int b = -1; b <= 1 && f; ++b)
      for (int a = -1; a <= 1 && f; ++a) {
        const int ii = i + a, jj = j + b, kk = k + c;
        if (ii < 0 || jj < 0 || kk < 0 || ii >= g.nx || jj >= g.ny || kk >= g.nz ||
            cls[g.idx(ii, jj, kk)] == MG_INACTIVE)
          f = false;
      }
  full[g.idx(i, j, k)] = f ? 1 : 0;
}

void launch_mark_full(const Level& l, hipStream_t s) {
  hipLaunchKernelGGL(k_mark_full, lvl_grid(l.g), dim3(MBX, MBY), 0, s, l.g, l.cls, l.full);
}

// A x and the diagonal at cell P.
template <class S, class C>
__device__ __forceinline__ void apply_at(const LevelView& L, uint8_t cl, const S* __restrict__ x,
                                         int P, C xP, C& Ax, C& D) {
  const Geom& g = L.g;
  const C ih2x = (C)(1.0 / (g.hx * g.hx)), ih2y = (C)(1.0 / (g.hy * g.hy)),
          ih2z = (C)(1.0 / (g.hz * g.hz));
  if (cl == MG_REGULAR) {
    C s = ((C)2 * xP - St<S, C>::ld(x + P - 1) - St<S, C>::ld(x + P + 1)) * ih2x +
          ((C)2 * xP - St<S, C>::ld(x + P - g.sx) - St<S, C>::ld(x + P + g.sx)) * ih2y;
    C d = (C)2 * (ih2x + ih2y);
    if (g.dim == 3) {
      s += ((C)2 * xP - St<S, C>::ld(x + P - g.sxy) - St<S, C>::ld(x + P + g.sxy)) * ih2z;
      d += (C)2 * ih2z;
    }
    Ax = s;
    D = d;
    return;
  }
  const C cxl = (C)L.cf0[P], cxh = (C)L.cf0[P + 1];
  const C cyl = (C)L.cf1[P], cyh = (C)L.cf1[P + g.sx];
  C s = (cxl * (xP - St<S, C>::ld(x + P - 1)) + cxh * (xP - St<S, C>::ld(x + P + 1))) * ih2x +
        (cyl * (xP - St<S, C>::ld(x + P - g.sx)) + cyh * (xP - St<S, C>::ld(x + P + g.sx))) * ih2y;
  C d = (cxl + cxh) * ih2x + (cyl + cyh) * ih2y;
  if (g.dim == 3) {
    const C czl = (C)L.cf2[P], czh = (C)L.cf2[P + g.sxy];
    s += (czl * (xP - St<S, C>::ld(x + P - g.sxy)) + czh * (xP - St<S, C>::ld(x + P + g.sxy))) * ih2z;
    d += (czl + czh) * ih2z;
  }
  Ax = s;
  D = d;
}

// Tiles of a level for the column-walking kernels below.
__host__ inline Tiles lvl_tiles(const Level& l, int kid) {
  return make_tiles(l.g.nx, l.g.ny, l.g.nz, l.tt[kid]);
}

// A x and the diagonal at cell P, z neighbours given (the walking kernels
// keep them in registers).
template <class S, class C>
__device__ __forceinline__ void apply_z(const LevelView& L, uint8_t cl, const S* __restrict__ x,
                                        int P, C xP, C xm, C xp, C& Ax, C& D) {
  const Geom& g = L.g;
  const C ih2x = (C)(1.0 / (g.hx * g.hx)), ih2y = (C)(1.0 / (g.hy * g.hy)),
          ih2z = (C)(1.0 / (g.hz * g.hz));
  const bool d3 = g.dim == 3;
  if (cl == MG_REGULAR) {
    C s = ((C)2 * xP - St<S, C>::ld(x + P - 1) - St<S, C>::ld(x + P + 1)) * ih2x +
          ((C)2 * xP - St<S, C>::ld(x + P - g.sx) - St<S, C>::ld(x + P + g.sx)) * ih2y;
    C d = (C)2 * (ih2x + ih2y);
    if (d3) {
      s += ((C)2 * xP - xm - xp) * ih2z;
      d += (C)2 * ih2z;
    }
    Ax = s;
    D = d;
    return;
  }
  const C cxl = (C)L.cf0[P], cxh = (C)L.cf0[P + 1];
  const C cyl = (C)L.cf1[P], cyh = (C)L.cf1[P + g.sx];
  C s = (cxl * (xP - St<S, C>::ld(x + P - 1)) + cxh * (xP - St<S, C>::ld(x + P + 1))) * ih2x +
        (cyl * (xP - St<S, C>::ld(x + P - g.sx)) + cyh * (xP - St<S, C>::ld(x + P + g.sx))) * ih2y;
  C d = (cxl + cxh) * ih2x + (cyl + cyh) * ih2y;
  if (d3) {
    const C czl = (C)L.cf2[P], czh = (C)L.cf2[P + g.sxy];
    s += (czl * (xP - xm) + czh * (xP - xp)) * ih2z;
    d += (czl + czh) * ih2z;
  }
  Ax = s;
  D = d;
}

// ---- damped Jacobi sweep: x_out = x_in + w (b - A x_in) / D -------------------
// Each thread walks cz planes of one column with x(k-1), x(k), x(k+1) in
// registers; in-plane neighbours come through the cache.
template <class S, class C, bool ZERO>
__global__ __launch_bounds__(MBS) void k_smooth(LevelView L, Tiles T, const S* __restrict__ xin,
                                                S* __restrict__ xout, const S* __restrict__ b,
                                                C wj, const double* __restrict__ ctl) {
  if (ctl[S_DONE] != 0.0) return;
  int tx, ty, tz;
  if (!tile_of(T, tx, ty, tz)) return;
  const Geom& g = L.g;
  const int i = tx * MBX + threadIdx.x, j = ty * MBY + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const int k0 = tz * T.cz, k1 = min(g.nz, k0 + T.cz);
  const bool d3 = g.dim == 3;
  int P = g.idx(i, j, k0);
  C xm = 0, xc = 0;
  if (!ZERO) {
    xc = St<S, C>::ld(xin + P);
    if (d3) xm = St<S, C>::ld(xin + P - g.sxy);
  }
  for (int k = k0; k < k1; ++k, P += g.sxy) {
    C xp = 0;
    if (!ZERO && d3) xp = St<S, C>::ld(xin + P + g.sxy);
    const uint8_t cl = L.cls[P];
    if (cl != MG_INACTIVE) {
      const C bP = St<S, C>::ld(b + P);
      C Ax, D;
      if (ZERO) {
        apply_z<S, C>(L, cl, b, P, (C)0, (C)0, (C)0, Ax, D);
        St<S, C>::st(xout + P, wj * bP / D);
      } else {
        apply_z<S, C>(L, cl, xin, P, xc, xm, xp, Ax, D);
        St<S, C>::st(xout + P, xc + wj * (bP - Ax) / D);
      }
    }
    xm = xc;
    xc = xp;
  }
}

template <class S, class C>
void launch_smooth(const Level& l, const void* xin, void* xout, double wj, bool from_zero,
                   const double* ctl, hipStream_t s) {
  const Tiles T = lvl_tiles(l, from_zero ? TK_SMOOTH_ZERO : TK_SMOOTH);
  if (from_zero)
    hipLaunchKernelGGL((k_smooth<S, C, true>), dim3(T.grid), dim3(MBX, MBY), 0, s, view(l), T,
                       (const S*)xin, (S*)xout, (const S*)l.b, (C)wj, ctl);
  else
    hipLaunchKernelGGL((k_smooth<S, C, false>), dim3(T.grid), dim3(MBX, MBY), 0, s, view(l), T,
                       (const S*)xin, (S*)xout, (const S*)l.b, (C)wj, ctl);
}

// ---- residual and restriction: b_c = mean over the 2^dim children of (b - A x)
// One thread per fine column (64 x 4 fine columns = 32 x 2 coarse columns per
// workgroup), walking fine planes in pairs; the 2 x 2 in-plane sum uses a
// lane exchange (x) and LDS (y).  Tiles count coarse planes along z.
template <class S, class C, class SC>
__global__ __launch_bounds__(MBS) void k_resid_restrict(LevelView F, Tiles T,
                                                        const S* __restrict__ x,
                                                        const S* __restrict__ b, LevelView Cl,
                                                        SC* __restrict__ bc,
                                                        const double* __restrict__ ctl) {
  if (ctl[S_DONE] != 0.0) return;
  __shared__ C sh[MBY][MBX];
  int tx, ty, tz;
  if (!tile_of(T, tx, ty, tz)) return;  // uniform over the workgroup
  const Geom& g = F.g;
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int i = tx * MBX + lx, j = ty * MBY + ly;
  const bool in = i < g.nx && j < g.ny;
  const bool d3 = g.dim == 3;
  const int K0 = tz * T.cz, K1 = min(Cl.g.nz, K0 + T.cz);
  const int kz = d3 ? 2 : 1;
  int P = in ? g.idx(i, j, kz * K0) : 0;
  C xm = 0, xc = 0;
  if (in) {
    xc = St<S, C>::ld(x + P);
    if (d3) xm = St<S, C>::ld(x + P - g.sxy);
  }
  for (int K = K0; K < K1; ++K) {
    C r = 0;
    for (int c = 0; c < kz; ++c, P += g.sxy) {
      C xp = 0;
      if (in) {
        if (d3) xp = St<S, C>::ld(x + P + g.sxy);
        const uint8_t cl = F.cls[P];
        if (cl != MG_INACTIVE) {
          C Ax, D;
          apply_z<S, C>(F, cl, x, P, xc, xm, xp, Ax, D);
          r += St<S, C>::ld(b + P) - Ax;
        }
      }
      xm = xc;
      xc = xp;
    }
    r += __shfl_xor(r, 1);
    sh[ly][lx] = r;
    __syncthreads();
    if (in && !(lx & 1) && !(ly & 1)) {
      const int PC = Cl.g.idx(i >> 1, j >> 1, K);
      if (Cl.cls[PC] != MG_INACTIVE)
        St<SC, C>::st(bc + PC, (sh[ly][lx] + sh[ly + 1][lx]) * (C)(d3 ? 0.125 : 0.25));
    }
    __syncthreads();
  }
}

template <class S, class C, class SC>
void launch_resid_restrict(const Level& f, const Level& c, const double* ctl, hipStream_t s) {
  const Tiles T = make_tiles(f.g.nx, f.g.ny, c.g.nz, f.tt[TK_RESTRICT]);
  hipLaunchKernelGGL((k_resid_restrict<S, C, SC>), dim3(T.grid), dim3(MBX, MBY), 0, s, view(f),
                     T, (const S*)f.x[f.cur], (const S*)f.b, view(c), (SC*)c.b, ctl);
}

// ---- prolongation and correction: x_f += PROL(e_c) ------------------------------
// Cell-centred linear interpolation axis by axis (x, y, then z), weights 3/4
// and 1/4.  A neighbour outside the box contributes the boundary ghost
// (1 - c_f) e (c_f = 0: zero gradient, 2: zero value); an inactive neighbour
// is replaced by the cell it is interpolated from.
template <class SC, class C>
__device__ __forceinline__ bool act_at(const LevelView& L, int i, int j, int k) {
  if (i < 0 || j < 0 || k < 0 || i >= L.g.nx || j >= L.g.ny || k >= L.g.nz) return false;
  return L.cls[L.g.idx(i, j, k)] != MG_INACTIVE;
}

template <class S, class C, class SC>
__global__ __launch_bounds__(MBS) void k_prolong(LevelView F, Tiles T, S* __restrict__ x,
                                                 LevelView Cl, const SC* __restrict__ e,
                                                 const double* __restrict__ ctl) {
  if (ctl[S_DONE] != 0.0) return;
  int tx, ty, tz;
  if (!tile_of(T, tx, ty, tz)) return;
  const int i = tx * MBX + threadIdx.x, j = ty * MBY + threadIdx.y;
  if (i >= F.g.nx || j >= F.g.ny) return;
  const int k0 = tz * T.cz, k1 = min(F.g.nz, k0 + T.cz);
  for (int k = k0; k < k1; ++k) {
  const int P = F.g.idx(i, j, k);
  if (F.cls[P] == MG_INACTIVE) continue;
  const Geom& cg = Cl.g;
  const bool d3 = cg.dim == 3;
  const int I = i >> 1, J = j >> 1, K = d3 ? (k >> 1) : 0;
  const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
  const C w3 = (C)0.75, w1 = (C)0.25;
  const int PC = cg.idx(I, J, K);
  if (Cl.full[PC]) {
    // all corners active and inside: same axis-by-axis sums, no checks
    const int oy = sy * cg.sx, oz = sz * cg.sxy;
    C Y0, Z;
    {
      const C x00 = w3 * St<SC, C>::ld(e + PC) + w1 * St<SC, C>::ld(e + PC + sx);
      const C x01 = w3 * St<SC, C>::ld(e + PC + oy) + w1 * St<SC, C>::ld(e + PC + oy + sx);
      Y0 = w3 * x00 + w1 * x01;
    }
    if (d3) {
      const C x10 = w3 * St<SC, C>::ld(e + PC + oz) + w1 * St<SC, C>::ld(e + PC + oz + sx);
      const C x11 =
          w3 * St<SC, C>::ld(e + PC + oz + oy) + w1 * St<SC, C>::ld(e + PC + oz + oy + sx);
      const C Y1 = w3 * x10 + w1 * x11;
      Z = w3 * Y0 + w1 * Y1;
    } else {
      Z = Y0;
    }
    St<S, C>::st(x + P, St<S, C>::ld(x + P) + Z);
    continue;
  }
  C X[2][2] = {{0, 0}, {0, 0}};
  const int nzc = d3 ? 2 : 1;
  for (int cc = 0; cc < nzc; ++cc)
    for (int b = 0; b < 2; ++b) {
      const int qj = J + b * sy, qk = K + cc * sz;
      if (!act_at<SC, C>(Cl, I, qj, qk)) continue;
      const int Q = cg.idx(I, qj, qk);
      const C eq = St<SC, C>::ld(e + Q);
      C en;
      const int ri = I + sx;
      if (ri < 0 || ri >= cg.nx) {
        const C cfb = (C)Cl.cf0[sx > 0 ? Q + 1 : Q];
        en = ((C)1 - cfb) * eq;
      } else {
        en = Cl.cls[Q + sx] != MG_INACTIVE ? St<SC, C>::ld(e + Q + sx) : eq;
      }
      X[cc][b] = w3 * eq + w1 * en;
    }
  C Y[2] = {0, 0};
  for (int cc = 0; cc < nzc; ++cc) {
    const int qk = K + cc * sz;
    if (!act_at<SC, C>(Cl, I, J, qk)) continue;
    C yn;
    const int qj = J + sy;
    if (qj < 0 || qj >= cg.ny) {
      const int Q0 = cg.idx(I, J, qk);
      const C cfb = (C)Cl.cf1[sy > 0 ? Q0 + cg.sx : Q0];
      yn = ((C)1 - cfb) * X[cc][0];
    } else {
      yn = act_at<SC, C>(Cl, I, qj, qk) ? X[cc][1] : X[cc][0];
    }
    Y[cc] = w3 * X[cc][0] + w1 * yn;
  }
  C Z = Y[0];
  if (d3) {
    C zn;
    const int qk = K + sz;
    if (qk < 0 || qk >= cg.nz) {
      const int Q0 = cg.idx(I, J, K);
      const C cfb = (C)Cl.cf2[sz > 0 ? Q0 + cg.sxy : Q0];
      zn = ((C)1 - cfb) * Y[0];
    } else {
      zn = act_at<SC, C>(Cl, I, J, qk) ? Y[1] : Y[0];
    }
    Z = w3 * Y[0] + w1 * zn;
  }
  St<S, C>::st(x + P, St<S, C>::ld(x + P) + Z);
  }
}

template <class S, class C, class SC>
void launch_prolong(const Level& f, const Level& c, const double* ctl, hipStream_t s) {
  const Tiles T = lvl_tiles(f, TK_PROLONG);
  hipLaunchKernelGGL((k_prolong<S, C, SC>), dim3(T.grid), dim3(MBX, MBY), 0, s, view(f), T,
                     (S*)f.x[f.cur], view(c), (const SC*)c.x[c.cur], ctl);
}

// ---- coarsest level: x = A^-1 b with the dense inverse, one workgroup -------------
template <class SC, class C>
__global__ __launch_bounds__(256) void k_coarse_solve(const SC* __restrict__ b, SC* __restrict__ x,
                                                      const int* __restrict__ cmap,
                                                      const int* __restrict__ ncount,
                                                      const double* __restrict__ ainv, int max_n,
                                                      const double* __restrict__ ctl) {
  if (ctl[S_DONE] != 0.0) return;
  __shared__ C bs[512];
  const int n = *ncount;
  if (n > max_n) return;
  for (int a = threadIdx.x; a < n; a += blockDim.x) bs[a] = St<SC, C>::ld(b + cmap[a]);
  __syncthreads();
  for (int a = threadIdx.x; a < n; a += blockDim.x) {
    C s = 0;
    const double* row = ainv + (size_t)a * n;
    for (int q = 0; q < n; ++q) s += (C)row[q] * bs[q];
    St<SC, C>::st(x + cmap[a], s);
  }
}

template <class SC, class C>
void launch_coarse_solve(const Level& c, const int* cmap, const int* ncount, const double* ainv,
                         int max_n, const double* ctl, hipStream_t s) {
  hipLaunchKernelGGL((k_coarse_solve<SC, C>), dim3(1), dim3(256), 0, s, (const SC*)c.b,
                     (SC*)c.x[c.cur], cmap, ncount, ainv, max_n, ctl);
}

template <class S>
__global__ void k_fill_zero(Geom g, S* x, const double* __restrict__ ctl) {
  if (ctl[S_DONE] != 0.0) return;
  const int i = blockIdx.x * MBX + threadIdx.x, j = blockIdx.y * MBY + threadIdx.y, k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  S z;
  memset(&z, 0, sizeof z);
  x[g.idx(i, j, k)] = z;
}
template <class S>
void launch_fill_zero(const Level& l, void* x, const double* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero<S>, lvl_grid(l.g), dim3(MBX, MBY), 0, s, l.g, (S*)x, ctl);
}

// ---- flexible conjugate gradient on level 0 ---------------------------------------
// Vectors x (phi), r, p (two buffers, alternating by iteration parity), q in
// the outer precision O; z is the V-cycle result in the level-0 storage S; the
// level-0 right-hand side of the next V-cycle is r rounded to S.  Scalars and
// the stopping state live in red.out (ctl).  Every kernel walks column tiles
// and writes one partial per workgroup (tiles outside the grid write zeros).

// r = b - A x0 (x0 = 0 unless given), x = x0 on active cells, 0 elsewhere.
template <class O, class S>
__global__ __launch_bounds__(MBS) void k_fcg_start(LevelView L, Tiles T, const O* __restrict__ b,
                                                   const O* __restrict__ x0, O* __restrict__ r,
                                                   O* __restrict__ x, S* __restrict__ b0,
                                                   int have_x0, RedBuf red) {
  int tx, ty, tz;
  double bb = 0.0, rr = 0.0;
  if (tile_of(T, tx, ty, tz)) {
    const Geom& g = L.g;
    const int i = tx * MBX + threadIdx.x, j = ty * MBY + threadIdx.y;
    if (i < g.nx && j < g.ny) {
      const int k0 = tz * T.cz, k1 = min(g.nz, k0 + T.cz);
      for (int k = k0; k < k1; ++k) {
        const int P = g.idx(i, j, k);
        const uint8_t cl = L.cls[P];
        if (cl == MG_INACTIVE) continue;
        const O bP = b[P];
        O rP = bP, xP = 0;
        if (have_x0) {
          xP = x0[P];
          const O xm = g.dim == 3 ? x0[P - g.sxy] : (O)0, xp = g.dim == 3 ? x0[P + g.sxy] : (O)0;
          O Ax, D;
          apply_z<O, O>(L, cl, x0, P, xP, xm, xp, Ax, D);
          rP = bP - Ax;
        }
        r[P] = rP;
        x[P] = xP;
        St<S, O>::st(b0 + P, rP);
        bb += (double)bP * (double)bP;
        rr += (double)rP * (double)rP;
      }
    }
  }
  double vv[2] = {bb, rr};
  block_partial<2, R_SUM, MBS>(vv, red);
}

// Stopping rule, evaluated by one thread after ||r||^2 is known.
__device__ __forceinline__ void fcg_judge(double* ctl) {
  const double bb = ctl[S_BB], rr = ctl[S_RR], it = ctl[S_ITER];
  bool done;
  if (!isfinite(rr) || !isfinite(bb))
    done = true;
  else if (ctl[S_FORCED] >= 0.0)
    done = it >= ctl[S_FORCED];
  else
    done = bb == 0.0 || rr <= ctl[S_TOL2] * bb || it >= ctl[S_MAXIT];
  ctl[S_DONE] = done ? 1.0 : 0.0;
}

constexpr int FIN = 1024;  // threads of the finalising workgroup

template <int NV>
__device__ __forceinline__ void fin_sum(const RedBuf& red, int nb, double (&acc)[NV]) {
  __shared__ double sh[NV][FIN];
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  for (int i = threadIdx.x; i < nb; i += FIN)
    for (int q = 0; q < NV; ++q) acc[q] += red.partial[(size_t)i * NV + q];
  block_tree<NV, R_SUM, FIN>(acc, sh);
}

__global__ __launch_bounds__(FIN) void k_fin_start(RedBuf red, int nb, double tol2, double maxit,
                                                   double forced) {
  double acc[2];
  fin_sum<2>(red, nb, acc);
  if (threadIdx.x == 0) {
    red.out[S_BB] = acc[0];
    red.out[S_RR] = acc[1];
    red.out[S_ITER] = 0.0;
    red.out[S_TOL2] = tol2;
    red.out[S_MAXIT] = maxit;
    red.out[S_FORCED] = forced;
    fcg_judge(red.out);
  }
}

template <class O, class S>
void launch_fcg_start(const Level& l0, const O* b, const O* x0, O* r, O* x, const RedBuf& red,
                      bool have_x0, double tol, int max_cycles, int forced, hipStream_t s,
                      bool fin) {
  const Tiles T = lvl_tiles(l0, TK_START);
  hipLaunchKernelGGL((k_fcg_start<O, S>), dim3(T.grid), dim3(MBX, MBY), 0, s, view(l0), T, b, x0,
                     r, x, (S*)l0.b, have_x0 ? 1 : 0, red);
  if (fin)
    hipLaunchKernelGGL(k_fin_start, dim3(1), dim3(FIN), 0, s, red, T.grid, tol * tol,
                       (double)max_cycles, (double)forced);
}

// (z, r) and (z, q_prev)
template <class O, class S>
__global__ __launch_bounds__(MBS) void k_fcg_dots(LevelView L, Tiles T, const S* __restrict__ z,
                                                  const O* __restrict__ r, const O* __restrict__ q,
                                                  RedBuf red) {
  if (red.out[S_DONE] != 0.0) return;
  int tx, ty, tz;
  double zr = 0.0, zq = 0.0;
  if (tile_of(T, tx, ty, tz)) {
    const Geom& g = L.g;
    const int i = tx * MBX + threadIdx.x, j = ty * MBY + threadIdx.y;
    if (i < g.nx && j < g.ny) {
      const int k0 = tz * T.cz, k1 = min(g.nz, k0 + T.cz);
      for (int k = k0; k < k1; ++k) {
        const int P = g.idx(i, j, k);
        if (L.cls[P] == MG_INACTIVE) continue;
        const double zP = (double)St<S, O>::ld(z + P);
        zr += zP * (double)r[P];
        zq += zP * (double)q[P];
      }
    }
  }
  double vv[2] = {zr, zq};
  block_partial<2, R_SUM, MBS>(vv, red);
}

// sums of the last kernel's partials into slots (s0, s1); slot_par adds the
// iteration parity to both slots
template <int NV>
__global__ __launch_bounds__(FIN) void k_fin_sum(RedBuf red, int nb, int s0, int s1,
                                                 int slot_par) {
  if (red.out[S_DONE] != 0.0) return;
  double acc[NV];
  fin_sum<NV>(red, nb, acc);
  if (threadIdx.x == 0) {
    const int par = slot_par ? ((int)red.out[S_ITER] & 1) : 0;
    red.out[s0 + par] = acc[0];
    if (NV > 1) red.out[s1 + par] = acc[NV - 1];
  }
}

template <class O, class S>
void launch_fcg_dots(const Level& l0, const O* r, const O* q, const RedBuf& red, hipStream_t s,
                     bool fin) {
  const Tiles T = lvl_tiles(l0, TK_DOTS);
  hipLaunchKernelGGL((k_fcg_dots<O, S>), dim3(T.grid), dim3(MBX, MBY), 0, s, view(l0), T,
                     (const S*)l0.x[l0.cur], r, q, red);
  if (fin) hipLaunchKernelGGL(k_fin_sum<2>, dim3(1), dim3(FIN), 0, s, red, T.grid, S_ZR, S_ZQ, 0);
}

// p_new = z + beta p_old with beta = -alpha_prev (z, q_prev) / (z_prev, r_prev)
// = -(z, q_prev) / (p_prev, q_prev) (0 on the first iteration); q = A p_new,
// computed from z and p_old at the neighbours; (p_new, q) into S_PQ0 + parity.
// p_new is buffer (iteration parity), p_old the other one.
template <class O, class S>
__global__ __launch_bounds__(MBS) void k_fcg_dir(LevelView L, Tiles T, const S* __restrict__ z,
                                                 O* p0, O* p1, O* __restrict__ q, RedBuf red) {
  if (red.out[S_DONE] != 0.0) return;
  const int it = (int)red.out[S_ITER];
  const int par = it & 1;
  const bool first = it == 0;
  const O* __restrict__ pold = par ? p0 : p1;
  O* __restrict__ pnew = par ? p1 : p0;
  const O beta = first ? (O)0 : (O)(-red.out[S_ZQ] / red.out[par ? S_PQ0 : S_PQ1]);
  int tx, ty, tz;
  double pq = 0.0;
  if (tile_of(T, tx, ty, tz)) {
    const Geom& g = L.g;
    const int i = tx * MBX + threadIdx.x, j = ty * MBY + threadIdx.y;
    if (i < g.nx && j < g.ny) {
      const bool d3 = g.dim == 3;
      auto pn = [&](int N) -> O {
        return St<S, O>::ld(z + N) + (first ? (O)0 : beta * pold[N]);
      };
      const O ih2x = (O)(1.0 / (g.hx * g.hx)), ih2y = (O)(1.0 / (g.hy * g.hy)),
              ih2z = (O)(1.0 / (g.hz * g.hz));
      const int k0 = tz * T.cz, k1 = min(g.nz, k0 + T.cz);
      int P = g.idx(i, j, k0);
      O pm = d3 ? pn(P - g.sxy) : (O)0, pc = pn(P);
      for (int k = k0; k < k1; ++k, P += g.sxy) {
        const O pp = d3 ? pn(P + g.sxy) : (O)0;
        const uint8_t cl = L.cls[P];
        if (cl != MG_INACTIVE) {
          O cxl = 1, cxh = 1, cyl = 1, cyh = 1, czl = 1, czh = 1;
          if (cl != MG_REGULAR) {
            cxl = (O)L.cf0[P];
            cxh = (O)L.cf0[P + 1];
            cyl = (O)L.cf1[P];
            cyh = (O)L.cf1[P + g.sx];
            if (d3) {
              czl = (O)L.cf2[P];
              czh = (O)L.cf2[P + g.sxy];
            }
          }
          O Ap = (cxl * (pc - pn(P - 1)) + cxh * (pc - pn(P + 1))) * ih2x +
                 (cyl * (pc - pn(P - g.sx)) + cyh * (pc - pn(P + g.sx))) * ih2y;
          if (d3) Ap += (czl * (pc - pm) + czh * (pc - pp)) * ih2z;
          pnew[P] = pc;
          q[P] = Ap;
          pq += (double)pc * (double)Ap;
        }
        pm = pc;
        pc = pp;
      }
    }
  }
  double vv[1] = {pq};
  block_partial<1, R_SUM, MBS>(vv, red);
}

template <class O, class S>
void launch_fcg_dir(const Level& l0, O* p0, O* p1, O* q, const RedBuf& red, hipStream_t s,
                    bool fin) {
  const Tiles T = lvl_tiles(l0, TK_DIR);
  hipLaunchKernelGGL((k_fcg_dir<O, S>), dim3(T.grid), dim3(MBX, MBY), 0, s, view(l0), T,
                     (const S*)l0.x[l0.cur], p0, p1, q, red);
  if (fin)
    hipLaunchKernelGGL(k_fin_sum<1>, dim3(1), dim3(FIN), 0, s, red, T.grid, S_PQ0, S_PQ0, 1);
}

// alpha = (z, r)/(p, q); x += alpha p; r -= alpha q; ||r||^2; next V-cycle rhs.
template <class O, class S>
__global__ __launch_bounds__(MBS) void k_fcg_update(LevelView L, Tiles T, O* __restrict__ x,
                                                    O* __restrict__ r, const O* p0, const O* p1,
                                                    const O* __restrict__ q, S* __restrict__ b0,
                                                    RedBuf red) {
  if (red.out[S_DONE] != 0.0) return;
  const int par = (int)red.out[S_ITER] & 1;
  const O* __restrict__ pv = par ? p1 : p0;
  const O a = (O)(red.out[S_ZR] / red.out[par ? S_PQ1 : S_PQ0]);
  int tx, ty, tz;
  double rr = 0.0;
  if (tile_of(T, tx, ty, tz)) {
    const Geom& g = L.g;
    const int i = tx * MBX + threadIdx.x, j = ty * MBY + threadIdx.y;
    if (i < g.nx && j < g.ny) {
      const int k0 = tz * T.cz, k1 = min(g.nz, k0 + T.cz);
      for (int k = k0; k < k1; ++k) {
        const int P = g.idx(i, j, k);
        if (L.cls[P] == MG_INACTIVE) continue;
        x[P] += a * pv[P];
        const O rP = r[P] - a * q[P];
        r[P] = rP;
        St<S, O>::st(b0 + P, rP);
        rr += (double)rP * (double)rP;
      }
    }
  }
  double vv[1] = {rr};
  block_partial<1, R_SUM, MBS>(vv, red);
}

// ||r||^2, one more iteration done, stopping rule
__global__ __launch_bounds__(FIN) void k_fin_update(RedBuf red, int nb) {
  if (red.out[S_DONE] != 0.0) return;
  double acc[1];
  fin_sum<1>(red, nb, acc);
  if (threadIdx.x == 0) {
    red.out[S_RR] = acc[0];
    red.out[S_ITER] += 1.0;
    fcg_judge(red.out);
  }
}

template <class O, class S>
void launch_fcg_update(const Level& l0, O* x, O* r, O* p0, O* p1, const O* q, const RedBuf& red,
                       hipStream_t s, bool fin) {
  const Tiles T = lvl_tiles(l0, TK_UPDATE);
  hipLaunchKernelGGL((k_fcg_update<O, S>), dim3(T.grid), dim3(MBX, MBY), 0, s, view(l0), T, x, r,
                     p0, p1, q, (S*)l0.b, red);
  if (fin) hipLaunchKernelGGL(k_fin_update, dim3(1), dim3(FIN), 0, s, red, T.grid);
}

// ---- deterministic finalisation of block partials ---------------------------------
template <int NV, int OP>
__global__ __launch_bounds__(256) void k_finalize(RedBuf red, int nb, int s0, int s1) {
  __shared__ double sh[NV][256];
  double acc[NV];
  for (int q = 0; q < NV; ++q) acc[q] = rid<OP>();
  for (int i = threadIdx.x; i < nb; i += 256)
    for (int q = 0; q < NV; ++q) acc[q] = rop<OP>(acc[q], red.partial[(size_t)i * NV + q]);
  block_tree<NV, OP, 256>(acc, sh);
  if (threadIdx.x == 0) {
    red.out[s0] = acc[0];
    if (NV > 1) red.out[s1] = acc[NV - 1];
  }
}

void launch_finalize(int nv, int op, const RedBuf& red, int nblocks, int slot0, int slot1,
                     hipStream_t s) {
  if (nv == 1 && op == R_SUM)
    hipLaunchKernelGGL((k_finalize<1, R_SUM>), dim3(1), dim3(256), 0, s, red, nblocks, slot0, slot1);
  else if (nv == 1 && op == R_MAX)
    hipLaunchKernelGGL((k_finalize<1, R_MAX>), dim3(1), dim3(256), 0, s, red, nblocks, slot0, slot1);
  else if (nv == 2 && op == R_SUM)
    hipLaunchKernelGGL((k_finalize<2, R_SUM>), dim3(1), dim3(256), 0, s, red, nblocks, slot0, slot1);
  else
    hipLaunchKernelGGL((k_finalize<2, R_MIN>), dim3(1), dim3(256), 0, s, red, nblocks, slot0, slot1);
}

// ---- LDS bottom solver ----------------------------------------------------------------
// The same operators as the per-level kernels, on compact LDS arrays
// (index (k ny + j) nx + i; neighbours outside the box read as 0, inactive
// cells hold 0); coefficients and classes come from the level arrays.
template <class C>
__device__ __forceinline__ C lds_nb(const C* x, const BottomLevel& L, int i, int j, int k, int d,
                                    int s) {
  int q[3] = {i, j, k};
  q[d] += s;
  const int n3[3] = {L.g.nx, L.g.ny, L.g.nz};
  if (q[d] < 0 || q[d] >= n3[d]) return (C)0;
  return x[(q[2] * L.g.ny + q[1]) * L.g.nx + q[0]];
}

template <class C>
__device__ __forceinline__ void lds_apply(const BottomLevel& L, const C* x, int i, int j, int k,
                                          uint8_t cl, C xP, C& Ax, C& D) {
  const Geom& g = L.g;
  const C ih2[3] = {(C)(1.0 / (g.hx * g.hx)), (C)(1.0 / (g.hy * g.hy)), (C)(1.0 / (g.hz * g.hz))};
  const int P = g.idx(i, j, k);
  const int st[3] = {1, g.sx, g.sxy};
  const float* cf[3] = {L.cf0, L.cf1, L.cf2};
  C s = 0, d = 0;
  for (int a = 0; a < g.dim; ++a) {
    const C cl_ = cl == MG_REGULAR ? (C)1 : (C)cf[a][P];
    const C ch_ = cl == MG_REGULAR ? (C)1 : (C)cf[a][P + st[a]];
    s += (cl_ * (xP - lds_nb(x, L, i, j, k, a, -1)) + ch_ * (xP - lds_nb(x, L, i, j, k, a, 1))) *
         ih2[a];
    d += (cl_ + ch_) * ih2[a];
  }
  Ax = s;
  D = d;
}

template <class C>
__device__ __forceinline__ void lds_cell(const BottomLevel& L, int c, int& i, int& j, int& k) {
  i = c % L.g.nx;
  j = (c / L.g.nx) % L.g.ny;
  k = c / (L.g.nx * L.g.ny);
}

template <class SC, class C>
__global__ __launch_bounds__(1024) void k_bottom(Bottom B, const SC* __restrict__ btop,
                                                 SC* __restrict__ xtop,
                                                 const double* __restrict__ ctl) {
  if (ctl[S_DONE] != 0.0) return;
  extern __shared__ unsigned char lds_raw[];
  C* lds = (C*)lds_raw;
  const int t = threadIdx.x, NT = blockDim.x;
  const C wj = (C)B.wj;
  const int nl = B.nlev;
  for (int e = t; e < (int)(B.lds_bytes / sizeof(C)); e += NT) lds[e] = (C)0;
  __syncthreads();
  {
    const BottomLevel& L = B.lv[0];
    for (int c = t; c < L.n; c += NT) {
      int i, j, k;
      lds_cell<C>(L, c, i, j, k);
      lds[L.ob + c] = St<SC, C>::ld(btop + L.g.idx(i, j, k));
    }
  }
  __syncthreads();
  int cur[BOTTOM_MAX_LEVELS];
  // one damped-Jacobi sweep on level l from buffer cur (or from zero)
  auto sweep = [&](int l, bool zero) {
    const BottomLevel& L = B.lv[l];
    const C* xin = lds + (cur[l] ? L.ox1 : L.ox0);
    C* xout = lds + (zero ? L.ox0 : (cur[l] ? L.ox0 : L.ox1));
    const C* b = lds + L.ob;
    for (int c = t; c < L.n; c += NT) {
      int i, j, k;
      lds_cell<C>(L, c, i, j, k);
      const uint8_t cl = L.cls[L.g.idx(i, j, k)];
      if (cl == MG_INACTIVE) continue;
      C Ax, D;
      const C xP = zero ? (C)0 : xin[c];
      lds_apply<C>(L, zero ? b : xin, i, j, k, cl, xP, Ax, D);
      xout[c] = zero ? wj * b[c] / D : xP + wj * (b[c] - Ax) / D;
    }
    cur[l] = zero ? 0 : (cur[l] ^ 1);
    __syncthreads();
  };
  for (int l = 0; l < nl - 1; ++l) {
    cur[l] = 0;
    if (B.nu1 > 0) {
      sweep(l, true);
      for (int s = 1; s < B.nu1; ++s) sweep(l, false);
    } else {
      const BottomLevel& L = B.lv[l];
      for (int c = t; c < L.n; c += NT) lds[L.ox0 + c] = (C)0;
      __syncthreads();
    }
    // residual and restriction into level l + 1
    const BottomLevel& F = B.lv[l];
    const BottomLevel& Cc = B.lv[l + 1];
    const C* x = lds + (cur[l] ? F.ox1 : F.ox0);
    const int kz = Cc.g.dim == 3 ? 2 : 1;
    for (int c = t; c < Cc.n; c += NT) {
      int I, J, K;
      lds_cell<C>(Cc, c, I, J, K);
      if (Cc.cls[Cc.g.idx(I, J, K)] == MG_INACTIVE) continue;
      C sum = 0;
      for (int cc = 0; cc < kz; ++cc)
        for (int bb = 0; bb < 2; ++bb)
          for (int a = 0; a < 2; ++a) {
            const int i = 2 * I + a, j = 2 * J + bb, k = kz * K + cc;
            const uint8_t cl = F.cls[F.g.idx(i, j, k)];
            if (cl == MG_INACTIVE) continue;
            const int fc = (k * F.g.ny + j) * F.g.nx + i;
            C Ax, D;
            lds_apply<C>(F, x, i, j, k, cl, x[fc], Ax, D);
            sum += lds[F.ob + fc] - Ax;
          }
      lds[Cc.ob + c] = sum * (C)(kz == 2 ? 0.125 : 0.25);
    }
    __syncthreads();
  }
  // coarsest level: dense inverse
  {
    const int l = nl - 1;
    const BottomLevel& L = B.lv[l];
    const int n = *B.ncount;
    cur[l] = 0;
    if (n <= B.max_n) {
      for (int a = t; a < n; a += NT) {
        C s = 0;
        const double* row = B.ainv + (size_t)a * n;
        for (int q = 0; q < n; ++q) {
          const int P = B.cmap[q] - L.g.off;
          const int kk = P / L.g.sxy, jj = (P % L.g.sxy) / L.g.sx, ii = P % L.g.sx;
          s += (C)row[q] * lds[L.ob + (kk * L.g.ny + jj) * L.g.nx + ii];
        }
        const int P = B.cmap[a] - L.g.off;
        const int kk = P / L.g.sxy, jj = (P % L.g.sxy) / L.g.sx, ii = P % L.g.sx;
        lds[L.ox0 + (kk * L.g.ny + jj) * L.g.nx + ii] = s;
      }
    }
    __syncthreads();
  }
  // up the hierarchy: prolongation and post-smoothing
  for (int l = nl - 2; l >= 0; --l) {
    const BottomLevel& F = B.lv[l];
    const BottomLevel& Cc = B.lv[l + 1];
    C* x = lds + (cur[l] ? F.ox1 : F.ox0);
    const C* e = lds + (cur[l + 1] ? Cc.ox1 : Cc.ox0);
    const Geom& cg = Cc.g;
    const bool d3 = cg.dim == 3;
    auto act = [&](int I, int J, int K) -> bool {
      if (I < 0 || J < 0 || K < 0 || I >= cg.nx || J >= cg.ny || K >= cg.nz) return false;
      return Cc.cls[cg.idx(I, J, K)] != MG_INACTIVE;
    };
    auto ev = [&](int I, int J, int K) -> C { return e[(K * cg.ny + J) * cg.nx + I]; };
    for (int c = t; c < F.n; c += NT) {
      int i, j, k;
      lds_cell<C>(F, c, i, j, k);
      if (F.cls[F.g.idx(i, j, k)] == MG_INACTIVE) continue;
      const int I = i >> 1, J = j >> 1, K = d3 ? (k >> 1) : 0;
      const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
      const C w3 = (C)0.75, w1 = (C)0.25;
      C X[2][2] = {{0, 0}, {0, 0}};
      const int nzc = d3 ? 2 : 1;
      for (int cc = 0; cc < nzc; ++cc)
        for (int b = 0; b < 2; ++b) {
          const int qj = J + b * sy, qk = K + cc * sz;
          if (!act(I, qj, qk)) continue;
          const C eq = ev(I, qj, qk);
          C en;
          const int ri = I + sx;
          if (ri < 0 || ri >= cg.nx) {
            const int Q = cg.idx(I, qj, qk);
            en = ((C)1 - (C)Cc.cf0[sx > 0 ? Q + 1 : Q]) * eq;
          } else {
            en = act(ri, qj, qk) ? ev(ri, qj, qk) : eq;
          }
          X[cc][b] = w3 * eq + w1 * en;
        }
      C Y[2] = {0, 0};
      for (int cc = 0; cc < nzc; ++cc) {
        const int qk = K + cc * sz;
        if (!act(I, J, qk)) continue;
        C yn;
        const int qj = J + sy;
        if (qj < 0 || qj >= cg.ny) {
          const int Q0 = cg.idx(I, J, qk);
          yn = ((C)1 - (C)Cc.cf1[sy > 0 ? Q0 + cg.sx : Q0]) * X[cc][0];
        } else {
          yn = act(I, qj, qk) ? X[cc][1] : X[cc][0];
        }
        Y[cc] = w3 * X[cc][0] + w1 * yn;
      }
      C Z = Y[0];
      if (d3) {
        C zn;
        const int qk = K + sz;
        if (qk < 0 || qk >= cg.nz) {
          const int Q0 = cg.idx(I, J, K);
          zn = ((C)1 - (C)Cc.cf2[sz > 0 ? Q0 + cg.sxy : Q0]) * Y[0];
        } else {
          zn = act(I, J, qk) ? Y[1] : Y[0];
        }
        Z = w3 * Y[0] + w1 * zn;
      }
      x[c] += Z;
    }
    __syncthreads();
    for (int s = 0; s < B.nu2; ++s) sweep(l, false);
  }
  {
    const BottomLevel& L = B.lv[0];
    const C* x = lds + (cur[0] ? L.ox1 : L.ox0);
    for (int c = t; c < L.n; c += NT) {
      int i, j, k;
      lds_cell<C>(L, c, i, j, k);
      const int P = L.g.idx(i, j, k);
      if (L.cls[P] != MG_INACTIVE) St<SC, C>::st(xtop + P, x[c]);
    }
  }
}

template <class SC, class C>
void launch_bottom(const Bottom& B, const void* btop, void* xtop, const double* ctl,
                   hipStream_t s) {
  hipLaunchKernelGGL((k_bottom<SC, C>), dim3(1), dim3(1024), B.lds_bytes, s, B, (const SC*)btop,
                     (SC*)xtop, ctl);
}
template void launch_bottom<double, double>(const Bottom&, const void*, void*, const double*,
                                            hipStream_t);
template void launch_bottom<float, float>(const Bottom&, const void*, void*, const double*,
                                          hipStream_t);
template void launch_bottom<bf16, float>(const Bottom&, const void*, void*, const double*,
                                         hipStream_t);

// ---- instantiations ------------------------------------------------------------
#define INST_LEVEL(S, C)                                                                     \
  template void launch_smooth<S, C>(const Level&, const void*, void*, double, bool,         \
                                    const double*, hipStream_t);                             \
  template void launch_fill_zero<S>(const Level&, void*, const double*, hipStream_t);
INST_LEVEL(double, double)
INST_LEVEL(float, float)
template void launch_smooth<bf16, float>(const Level&, const void*, void*, double, bool,
                                         const double*, hipStream_t);
template void launch_fill_zero<bf16>(const Level&, void*, const double*, hipStream_t);

#define INST_PAIR(S, C, SC)                                                                 \
  template void launch_resid_restrict<S, C, SC>(const Level&, const Level&, const double*,   \
                                                hipStream_t);                                 \
  template void launch_prolong<S, C, SC>(const Level&, const Level&, const double*,          \
                                         hipStream_t);
INST_PAIR(double, double, double)
INST_PAIR(float, float, float)
INST_PAIR(float, float, bf16)
INST_PAIR(bf16, float, bf16)

template void launch_coarse_solve<double, double>(const Level&, const int*, const int*,
                                                  const double*, int, const double*, hipStream_t);
template void launch_coarse_solve<float, float>(const Level&, const int*, const int*,
                                                const double*, int, const double*, hipStream_t);
template void launch_coarse_solve<bf16, float>(const Level&, const int*, const int*,
                                               const double*, int, const double*, hipStream_t);

#define INST_FCG(O, S)                                                                          \
  template void launch_fcg_start<O, S>(const Level&, const O*, const O*, O*, O*, const RedBuf&, \
                                       bool, double, int, int, hipStream_t, bool);              \
  template void launch_fcg_dots<O, S>(const Level&, const O*, const O*, const RedBuf&,          \
                                      hipStream_t, bool);                                       \
  template void launch_fcg_dir<O, S>(const Level&, O*, O*, O*, const RedBuf&, hipStream_t,      \
                                     bool);                                                     \
  template void launch_fcg_update<O, S>(const Level&, O*, O*, O*, O*, const O*, const RedBuf&,  \
                                        hipStream_t, bool);
INST_FCG(double, double)
INST_FCG(float, float)
INST_FCG(double, float)

}  // namespace nfvm
