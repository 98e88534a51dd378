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
};

__host__ inline LevelView view(const Level& l) {
  return LevelView{l.g, l.cls, l.cf[0], l.cf[1], l.g.dim == 3 ? l.cf[2] : l.cf[0]};
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

// ---- damped Jacobi sweep: x_out = x_in + w (b - A x_in) / D -------------------
template <class S, class C, bool ZERO>
__global__ __launch_bounds__(MBS) void k_smooth(LevelView L, const S* __restrict__ xin,
                                                S* __restrict__ xout, const S* __restrict__ b,
                                                C wj) {
  const int i = blockIdx.x * MBX + threadIdx.x, j = blockIdx.y * MBY + threadIdx.y, k = blockIdx.z;
  if (i >= L.g.nx || j >= L.g.ny) return;
  const int P = L.g.idx(i, j, k);
  const uint8_t cl = L.cls[P];
  if (cl == MG_INACTIVE) return;
  const C bP = St<S, C>::ld(b + P);
  C Ax, D;
  if (ZERO) {
    // A applied to zero: only the diagonal matters
    C tmp;
    apply_at<S, C>(L, cl, b, P, (C)0, tmp, D);
    St<S, C>::st(xout + P, wj * bP / D);
  } else {
    const C xP = St<S, C>::ld(xin + P);
    apply_at<S, C>(L, cl, xin, P, xP, Ax, D);
    St<S, C>::st(xout + P, xP + wj * (bP - Ax) / D);
  }
}

template <class S, class C>
void launch_smooth(const Level& l, const void* xin, void* xout, double wj, bool from_zero,
                   hipStream_t s) {
  if (from_zero)
    hipLaunchKernelGGL((k_smooth<S, C, true>), lvl_grid(l.g), dim3(MBX, MBY), 0, s, view(l),
                       (const S*)xin, (S*)xout, (const S*)l.b, (C)wj);
  else
    hipLaunchKernelGGL((k_smooth<S, C, false>), lvl_grid(l.g), dim3(MBX, MBY), 0, s, view(l),
                       (const S*)xin, (S*)xout, (const S*)l.b, (C)wj);
}

// ---- residual and restriction: b_c = mean over the 2^dim children of (b - A x)
template <class S, class C, class SC>
__global__ __launch_bounds__(MBS) void k_resid_restrict(LevelView F, const S* __restrict__ x,
                                                        const S* __restrict__ b, LevelView Cl,
                                                        SC* __restrict__ bc) {
  const int I = blockIdx.x * MBX + threadIdx.x, J = blockIdx.y * MBY + threadIdx.y, K = blockIdx.z;
  if (I >= Cl.g.nx || J >= Cl.g.ny) return;
  const int PC = Cl.g.idx(I, J, K);
  if (Cl.cls[PC] == MG_INACTIVE) return;
  const int kz = Cl.g.dim == 3 ? 2 : 1;
  C sum = 0;
  for (int cc = 0; cc < kz; ++cc)
    for (int bb = 0; bb < 2; ++bb)
      for (int a = 0; a < 2; ++a) {
        const int P = F.g.idx(2 * I + a, 2 * J + bb, kz * K + cc);
        const uint8_t cl = F.cls[P];
        if (cl == MG_INACTIVE) continue;
        const C xP = St<S, C>::ld(x + P);
        C Ax, D;
        apply_at<S, C>(F, cl, x, P, xP, Ax, D);
        sum += St<S, C>::ld(b + P) - Ax;
      }
  St<SC, C>::st(bc + PC, sum * (C)(kz == 2 ? 0.125 : 0.25));
}

template <class S, class C, class SC>
void launch_resid_restrict(const Level& f, const Level& c, hipStream_t s) {
  hipLaunchKernelGGL((k_resid_restrict<S, C, SC>), lvl_grid(c.g), dim3(MBX, MBY), 0, s, view(f),
                     (const S*)f.x[f.cur], (const S*)f.b, view(c), (SC*)c.b);
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
__global__ __launch_bounds__(MBS) void k_prolong(LevelView F, S* __restrict__ x, LevelView Cl,
                                                 const SC* __restrict__ e) {
  const int i = blockIdx.x * MBX + threadIdx.x, j = blockIdx.y * MBY + threadIdx.y, k = blockIdx.z;
  if (i >= F.g.nx || j >= F.g.ny) return;
  const int P = F.g.idx(i, j, k);
  if (F.cls[P] == MG_INACTIVE) return;
  const Geom& cg = Cl.g;
  const bool d3 = cg.dim == 3;
  const int I = i >> 1, J = j >> 1, K = d3 ? (k >> 1) : 0;
  const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
  const C w3 = (C)0.75, w1 = (C)0.25;
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

template <class S, class C, class SC>
void launch_prolong(const Level& f, const Level& c, hipStream_t s) {
  hipLaunchKernelGGL((k_prolong<S, C, SC>), lvl_grid(f.g), dim3(MBX, MBY), 0, s, view(f),
                     (S*)f.x[f.cur], view(c), (const SC*)c.x[c.cur]);
}

// ---- coarsest level: x = A^-1 b with the dense inverse, one workgroup -------------
template <class SC, class C>
__global__ __launch_bounds__(256) void k_coarse_solve(const SC* __restrict__ b, SC* __restrict__ x,
                                                      const int* __restrict__ cmap,
                                                      const int* __restrict__ ncount,
                                                      const double* __restrict__ ainv, int max_n) {
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
                         int max_n, hipStream_t s) {
  hipLaunchKernelGGL((k_coarse_solve<SC, C>), dim3(1), dim3(256), 0, s, (const SC*)c.b,
                     (SC*)c.x[c.cur], cmap, ncount, ainv, max_n);
}

template <class S>
__global__ void k_fill_zero(Geom g, S* x) {
  const int i = blockIdx.x * MBX + threadIdx.x, j = blockIdx.y * MBY + threadIdx.y, k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  S z;
  memset(&z, 0, sizeof z);
  x[g.idx(i, j, k)] = z;
}
template <class S>
void launch_fill_zero(const Level& l, void* x, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero<S>, lvl_grid(l.g), dim3(MBX, MBY), 0, s, l.g, (S*)x);
}

// ---- flexible conjugate gradient on level 0 ---------------------------------------
// Vectors x (phi), r, p, q in the outer precision O; z is the V-cycle result
// in the level-0 storage S; the level-0 right-hand side of the next V-cycle is
// r rounded to S.  Scalars live in red.out.

// r = b - A x0 (x0 = 0 unless given), x = x0 on active cells, 0 elsewhere.
template <class O, class S>
__global__ __launch_bounds__(MBS) void k_fcg_start(LevelView L, const O* __restrict__ b,
                                                   const O* __restrict__ x0, O* __restrict__ r,
                                                   O* __restrict__ x, S* __restrict__ b0,
                                                   int have_x0, RedBuf red) {
  const int i = blockIdx.x * MBX + threadIdx.x, j = blockIdx.y * MBY + threadIdx.y, k = blockIdx.z;
  double bb = 0.0, rr = 0.0;
  if (i < L.g.nx && j < L.g.ny) {
    const int P = L.g.idx(i, j, k);
    const uint8_t cl = L.cls[P];
    if (cl != MG_INACTIVE) {
      const O bP = b[P];
      O rP = bP, xP = 0;
      if (have_x0) {
        xP = x0[P];
        O Ax, D;
        apply_at<O, O>(L, cl, x0, P, xP, Ax, D);
        rP = bP - Ax;
      }
      r[P] = rP;
      x[P] = xP;
      St<S, O>::st(b0 + P, rP);
      bb = (double)bP * (double)bP;
      rr = (double)rP * (double)rP;
    }
  }
  double vv[2] = {bb, rr};
  block_partial<2, R_SUM, MBS>(vv, red);
}

// x0 may alias x only when have_x0 == 0; the engine passes a separate buffer otherwise.
template <class O, class S>
void launch_fcg_start(const Level& l0, const O* b, const O* x0, O* r, O* x, const RedBuf& red,
                      bool have_x0, hipStream_t s) {
  const dim3 gr = lvl_grid(l0.g);
  hipLaunchKernelGGL((k_fcg_start<O, S>), gr, dim3(MBX, MBY), 0, s, view(l0), b, x0, r, x,
                     (S*)l0.b, have_x0 ? 1 : 0, red);
  launch_finalize(2, R_SUM, red, gr.x * gr.y * gr.z, S_BB, S_RR, s);
}

// (z, r) and (z, q_prev)
template <class O, class S>
__global__ __launch_bounds__(MBS) void k_fcg_dots(LevelView L, const S* __restrict__ z,
                                                  const O* __restrict__ r, const O* __restrict__ q,
                                                  RedBuf red) {
  const int i = blockIdx.x * MBX + threadIdx.x, j = blockIdx.y * MBY + threadIdx.y, k = blockIdx.z;
  double zr = 0.0, zq = 0.0;
  if (i < L.g.nx && j < L.g.ny) {
    const int P = L.g.idx(i, j, k);
    if (L.cls[P] != MG_INACTIVE) {
      const double zP = (double)St<S, O>::ld(z + P);
      zr = zP * (double)r[P];
      zq = zP * (double)q[P];
    }
  }
  double vv[2] = {zr, zq};
  block_partial<2, R_SUM, MBS>(vv, red);
}

template <class O, class S>
void launch_fcg_dots(const Level& l0, const O* r, const O* q, const RedBuf& red, hipStream_t s) {
  const dim3 gr = lvl_grid(l0.g);
  hipLaunchKernelGGL((k_fcg_dots<O, S>), gr, dim3(MBX, MBY), 0, s, view(l0),
                     (const S*)l0.x[l0.cur], r, q, red);
  launch_finalize(2, R_SUM, red, gr.x * gr.y * gr.z, S_ZR, S_ZQ, s);
}

// p_new = z + beta p_old with beta = -alpha_prev (z, q_prev) / (z_prev, r_prev)
// = -(z, q_prev) / (p_prev, q_prev) (0 on the first iteration); q = A p_new,
// computed from z and p_old at the neighbours; (p_new, q) into slot pq_out.
template <class O, class S>
__global__ __launch_bounds__(MBS) void k_fcg_dir(LevelView L, const S* __restrict__ z,
                                                 const O* __restrict__ pold, O* __restrict__ pnew,
                                                 O* __restrict__ q, int first, int pq_in,
                                                 int pq_out, RedBuf red) {
  const int i = blockIdx.x * MBX + threadIdx.x, j = blockIdx.y * MBY + threadIdx.y, k = blockIdx.z;
  const O beta = first ? (O)0 : (O)(-red.out[S_ZQ] / red.out[pq_in]);
  double pq = 0.0;
  if (i < L.g.nx && j < L.g.ny) {
    const int P = L.g.idx(i, j, k);
    const uint8_t cl = L.cls[P];
    if (cl != MG_INACTIVE) {
      const Geom& g = L.g;
      auto pn = [&](int N) -> O {
        return St<S, O>::ld(z + N) + (first ? (O)0 : beta * pold[N]);
      };
      const O pP = pn(P);
      const O ih2[3] = {(O)(1.0 / (g.hx * g.hx)), (O)(1.0 / (g.hy * g.hy)),
                        (O)(1.0 / (g.hz * g.hz))};
      const int st[3] = {1, g.sx, g.sxy};
      const float* cf[3] = {L.cf0, L.cf1, L.cf2};
      O Ap = 0;
      for (int d = 0; d < g.dim; ++d) {
        const O cl_ = cl == MG_REGULAR ? (O)1 : (O)cf[d][P];
        const O ch_ = cl == MG_REGULAR ? (O)1 : (O)cf[d][P + st[d]];
        Ap += (cl_ * (pP - pn(P - st[d])) + ch_ * (pP - pn(P + st[d]))) * ih2[d];
      }
      pnew[P] = pP;
      q[P] = Ap;
      pq = (double)pP * (double)Ap;
    }
  }
  double vv[1] = {pq};
  block_partial<1, R_SUM, MBS>(vv, red);
}

template <class O, class S>
void launch_fcg_dir(const Level& l0, const O* pold, O* pnew, O* q, const RedBuf& red, bool first,
                    int parity, hipStream_t s) {
  const int pq_out = parity ? S_PQ1 : S_PQ0, pq_in = parity ? S_PQ0 : S_PQ1;
  const dim3 gr = lvl_grid(l0.g);
  hipLaunchKernelGGL((k_fcg_dir<O, S>), gr, dim3(MBX, MBY), 0, s, view(l0),
                     (const S*)l0.x[l0.cur], pold, pnew, q, first ? 1 : 0, pq_in, pq_out, red);
  launch_finalize(1, R_SUM, red, gr.x * gr.y * gr.z, pq_out, pq_out, s);
}

// alpha = (z, r)/(p, q); x += alpha p; r -= alpha q; ||r||^2; next V-cycle rhs.
template <class O, class S>
__global__ __launch_bounds__(MBS) void k_fcg_update(LevelView L, O* __restrict__ x,
                                                    O* __restrict__ r, const O* __restrict__ pv,
                                                    const O* __restrict__ q, S* __restrict__ b0,
                                                    int pq_slot, RedBuf red) {
  const int i = blockIdx.x * MBX + threadIdx.x, j = blockIdx.y * MBY + threadIdx.y, k = blockIdx.z;
  const double alpha = red.out[S_ZR] / red.out[pq_slot];
  double rr = 0.0;
  if (i < L.g.nx && j < L.g.ny) {
    const int P = L.g.idx(i, j, k);
    if (L.cls[P] != MG_INACTIVE) {
      const O a = (O)alpha;
      x[P] += a * pv[P];
      const O rP = r[P] - a * q[P];
      r[P] = rP;
      St<S, O>::st(b0 + P, rP);
      rr = (double)rP * (double)rP;
    }
  }
  double vv[1] = {rr};
  block_partial<1, R_SUM, MBS>(vv, red);
}

template <class O, class S>
void launch_fcg_update(const Level& l0, O* x, O* r, const O* pv, const O* q, const RedBuf& red,
                       int parity, hipStream_t s) {
  const dim3 gr = lvl_grid(l0.g);
  hipLaunchKernelGGL((k_fcg_update<O, S>), gr, dim3(MBX, MBY), 0, s, view(l0), x, r, pv, q,
                     (S*)l0.b, parity ? S_PQ1 : S_PQ0, red);
  launch_finalize(1, R_SUM, red, gr.x * gr.y * gr.z, S_RR, S_RR, s);
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

// ---- instantiations ------------------------------------------------------------
#define INST_LEVEL(S, C)                                                                     \
  template void launch_smooth<S, C>(const Level&, const void*, void*, double, bool,         \
                                    hipStream_t);                                            \
  template void launch_fill_zero<S>(const Level&, void*, hipStream_t);
INST_LEVEL(double, double)
INST_LEVEL(float, float)
template void launch_smooth<bf16, float>(const Level&, const void*, void*, double, bool,
                                         hipStream_t);
template void launch_fill_zero<bf16>(const Level&, void*, hipStream_t);

#define INST_PAIR(S, C, SC)                                                             \
  template void launch_resid_restrict<S, C, SC>(const Level&, const Level&, hipStream_t); \
  template void launch_prolong<S, C, SC>(const Level&, const Level&, hipStream_t);
INST_PAIR(double, double, double)
INST_PAIR(float, float, float)
INST_PAIR(float, float, bf16)
INST_PAIR(bf16, float, bf16)

template void launch_coarse_solve<double, double>(const Level&, const int*, const int*,
                                                  const double*, int, hipStream_t);
template void launch_coarse_solve<float, float>(const Level&, const int*, const int*,
                                                const double*, int, hipStream_t);
template void launch_coarse_solve<bf16, float>(const Level&, const int*, const int*,
                                               const double*, int, hipStream_t);

#define INST_FCG(O, S)                                                                          \
  template void launch_fcg_start<O, S>(const Level&, const O*, const O*, O*, O*, const RedBuf&, \
                                       bool, hipStream_t);                                      \
  template void launch_fcg_dots<O, S>(const Level&, const O*, const O*, const RedBuf&,          \
                                      hipStream_t);                                             \
  template void launch_fcg_dir<O, S>(const Level&, const O*, O*, O*, const RedBuf&, bool, int,  \
                                     hipStream_t);                                              \
  template void launch_fcg_update<O, S>(const Level&, O*, O*, const O*, const O*,              \
                                        const RedBuf&, int, hipStream_t);
INST_FCG(double, double)
INST_FCG(float, float)
INST_FCG(double, float)

}  // namespace nfvm
