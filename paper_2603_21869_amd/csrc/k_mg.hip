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
// Multiply-adds are fused only where one source expression holds both
// (a * b + c), never across statements: the rounding of every result then
// follows from the source alone, so a single launch and a batched launch of
// the same body give bitwise the same values however the compiler unrolls or
// schedules each.
#pragma clang fp contract(on)

#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <type_traits>
#include <vector>

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
  const uint16_t* code;  // level 0: face codes (FACE_CODE_INACTIVE for inactive cells)
};

__host__ inline LevelView view(const Level& l) {
  return LevelView{l.g,  l.cls,  l.cf[0], l.cf[1], l.g.dim == 3 ? l.cf[2] : l.cf[0],
                   l.full, l.code};
}

// Coefficient of face f (0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+) from a face code.
template <class C>
__device__ __forceinline__ C face_c(uint32_t cd, int f) {
  return (C)(int)((cd >> (2 * f)) & 3u);
}

// A x and the diagonal at a cell from its face code and the six neighbour
// values (-x, +x, -y, +y, -z, +z): sum over faces of c_f (x_P - x_N) / h^2.
template <class C>
__device__ __forceinline__ void apply_code_v(const Geom& g, uint32_t cd, C xP, C xl, C xh, C xs,
                                             C xn, C xm, C xp, C& Ax, C& D) {
  const C ih2x = (C)(1.0 / (g.hx * g.hx)), ih2y = (C)(1.0 / (g.hy * g.hy)),
          ih2z = (C)(1.0 / (g.hz * g.hz));
  const C cxl = face_c<C>(cd, 0), cxh = face_c<C>(cd, 1);
  const C cyl = face_c<C>(cd, 2), cyh = face_c<C>(cd, 3);
  C s = (cxl * (xP - xl) + cxh * (xP - xh)) * ih2x + (cyl * (xP - xs) + cyh * (xP - xn)) * ih2y;
  C d = (cxl + cxh) * ih2x + (cyl + cyh) * ih2y;
  if (g.dim == 3) {
    const C czl = face_c<C>(cd, 4), czh = face_c<C>(cd, 5);
    s += (czl * (xP - xm) + czh * (xP - xp)) * ih2z;
    d += (czl + czh) * ih2z;
  }
  Ax = s;
  D = g.sd > 0.0 ? (C)g.sd : d;
}

// One damped Jacobi update at a cell from its face code and neighbours,
// x + wj (b - A x) / D.  Cells whose faces all have coefficient 1 (the
// regular interior: code 0x555 in 3D, 0x55 in 2D) take the plain stencil
// and the constant wj / D of the level, formed once per thread, in place of
// the coefficient form and a division per cell; every level-0 sweep kernel
// takes this function, so a cell gets the same value from each of them.
template <class C>
struct JacobiConst {
  C ih2x, ih2y, ih2z, wj, wjd;
  uint32_t reg;
};
template <class C>
__device__ __forceinline__ JacobiConst<C> jacobi_const(const Geom& g, C wj) {
  JacobiConst<C> k;
  k.ih2x = (C)(1.0 / (g.hx * g.hx));
  k.ih2y = (C)(1.0 / (g.hy * g.hy));
  k.ih2z = (C)(1.0 / (g.hz * g.hz));
  C d = (C)2 * k.ih2x + (C)2 * k.ih2y;
  if (g.dim == 3) d += (C)2 * k.ih2z;
  if (g.sd > 0.0) d = (C)g.sd;
  k.wj = wj;
  k.wjd = wj / d;
  k.reg = g.dim == 3 ? 0x555u : 0x55u;
  return k;
}
template <class C>
__device__ __forceinline__ C jacobi_code(const Geom& g, const JacobiConst<C>& k, uint32_t cd,
                                         C xP, C xl, C xh, C xs, C xn, C xm, C xp, C bP) {
  if (cd == k.reg) {
    C s = ((xP - xl) + (xP - xh)) * k.ih2x + ((xP - xs) + (xP - xn)) * k.ih2y;
    if (g.dim == 3) s += ((xP - xm) + (xP - xp)) * k.ih2z;
    return xP + (bP - s) * k.wjd;
  }
  C A, D;
  apply_code_v<C>(g, cd, xP, xl, xh, xs, xn, xm, xp, A, D);
  return xP + k.wj * (bP - A) / D;
}

// ... at cell P, the x and y neighbours loaded here, the z neighbours given
// (the walking kernels keep them in registers).
template <class S, class C>
__device__ __forceinline__ void apply_code(const Geom& g, uint32_t cd, const S* __restrict__ x,
                                           int P, C xP, C xm, C xp, C& Ax, C& D) {
  apply_code_v<C>(g, cd, xP, St<S, C>::ld(x + P - 1), St<S, C>::ld(x + P + 1),
                  St<S, C>::ld(x + P - g.sx), St<S, C>::ld(x + P + g.sx), xm, xp, Ax, D);
}

// Diagonal of A from a face code.
template <class C>
__device__ __forceinline__ C diag_code(const Geom& g, uint32_t cd) {
  const C ih2x = (C)(1.0 / (g.hx * g.hx)), ih2y = (C)(1.0 / (g.hy * g.hy)),
          ih2z = (C)(1.0 / (g.hz * g.hz));
  C d = (face_c<C>(cd, 0) + face_c<C>(cd, 1)) * ih2x + (face_c<C>(cd, 2) + face_c<C>(cd, 3)) * ih2y;
  if (g.dim == 3) d += (face_c<C>(cd, 4) + face_c<C>(cd, 5)) * ih2z;
  return g.sd > 0.0 ? (C)g.sd : d;
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
    D = g.sd > 0.0 ? (C)g.sd : d;
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
  D = g.sd > 0.0 ? (C)g.sd : d;
}

// Tiles of a level for the column-walking kernels below.
__host__ inline Tiles lvl_tiles(const Level& l, int kid) {
  return make_tiles(l.g.nx, l.g.ny, l.g.nz, l.tt[kid]);
}

// ---- single and batched launches ----------------------------------------------------
// Every level kernel is a body taking its arguments as one struct and the tile
// it works on.  A single launch covers one grid (block b takes tile
// tile_of(b)); a batched launch covers the tiles of up to MAXB grids, one
// after the other.  `pb` is the block index the tile has in a single launch of its grid, where
// a reduction kernel stores its partial: batched and single launches then sum
// the same partials in the same order.
struct TileCtx {
  int tx, ty, tz, pb;
};

__device__ __forceinline__ bool tile_single(const Tiles& T, TileCtx& c) {
  c.pb = blockIdx.x;
  return tile_of(T, c.tx, c.ty, c.tz);
}

__device__ __forceinline__ bool tile_of_index(const Tiles& T, int t, TileCtx& c) {
  const int per = T.grid >> 3;
  c.pb = (t % per) * 8 + t / per;
  c.tx = t % T.ntx;
  c.ty = (t / T.ntx) % T.nty;
  c.tz = t / (T.ntx * T.nty);
  return t < T.total;
}

// Arguments of a batched launch over up to MAXB grids, passed by value (in
// the kernel-argument segment, read with scalar loads like a single
// launch's): grid i owns the blocks [start[i], start[i + 1]).
constexpr int MAXB = 8;
template <class A>
struct Pack {
  A a[MAXB];
  int start[MAXB + 1];
  int n;
};

// Grid and tile index of this block in a batched launch (false past the
// end); block b takes entry (b mod 8) * (blocks / 8) + b / 8, so that each
// XCD gets a contiguous range of entries.
template <class A>
__device__ __forceinline__ bool pack_entry(const Pack<A>& p, int& g, int& t) {
  const int per = gridDim.x >> 3;
  const int b = blockIdx.x;
  const int q = (b & 7) * per + (b >> 3);
  if (q >= p.start[p.n]) return false;
  int i = 0;
  while (q >= p.start[i + 1]) ++i;
  g = i;
  t = q - p.start[i];
  return true;
}

// Defines the single kernel NAME(ARGS a) and the batched kernel
// NAME_batch(Pack<ARGS> p) around BODY(const ARGS&, const TileCtx&, bool
// valid); TPL / TPLA are the parenthesised template parameters / arguments of
// the kernels and ARGA the argument struct's template arguments; with PAD,
// blocks of tiles past the end still run the body (reductions store a zero
// partial there).
#define NFVM_PASS(...) __VA_ARGS__
#define NFVM_TILE_KERNELS(NAME, BODY, ARGS, ARGA, TPL, TPLA, THREADS, PAD)                    \
  template <NFVM_PASS TPL>                                                                    \
  __global__ __launch_bounds__(THREADS) void NAME(ARGS<NFVM_PASS ARGA> a) {                   \
    TileCtx c;                                                                                \
    const bool v = tile_single(a.T, c);                                                       \
    if (v || PAD) BODY<NFVM_PASS TPLA>(a, c, v);                                              \
  }                                                                                           \
  template <NFVM_PASS TPL>                                                                    \
  __global__ __launch_bounds__(THREADS) void NAME##_batch(Pack<ARGS<NFVM_PASS ARGA>> p) {     \
    int gi, t;                                                                                \
    if (!pack_entry(p, gi, t)) return;                                                        \
    const ARGS<NFVM_PASS ARGA>& a = p.a[gi];                                                  \
    TileCtx c;                                                                                \
    const bool v = tile_of_index(a.T, t, c);                                                  \
    if (v || PAD) BODY<NFVM_PASS TPLA>(a, c, v);                                              \
  }

// Coarse-level operator from class bytes and face coefficients.  The
// neighbourhood of cell P is loaded in one go, before its class byte is
// tested (coarse launches are small and latency-bound; every index lies in
// the padded arrays); the z neighbours come from the walking kernels'
// registers.
template <class C>
struct Nbhd {
  C xl, xh, xs, xn;              // x neighbours: -x, +x, -y, +y
  C cxl, cxh, cyl, cyh, czl, czh;  // face coefficients
};

// Levels up to this many cells load the face coefficients of every cell up
// front (latency-bound launches); larger ones only for irregular cells,
// after the class byte (12 extra bytes per cell would cost bandwidth).
constexpr long long NBHD_EAGER_CELLS = 1 << 20;

template <class C>
__device__ __forceinline__ void load_coef(const LevelView& L, int P, Nbhd<C>& n) {
  const Geom& g = L.g;
  n.cxl = (C)L.cf0[P];
  n.cxh = (C)L.cf0[P + 1];
  n.cyl = (C)L.cf1[P];
  n.cyh = (C)L.cf1[P + g.sx];
  n.czl = g.dim == 3 ? (C)L.cf2[P] : (C)0;
  n.czh = g.dim == 3 ? (C)L.cf2[P + g.sxy] : (C)0;
}

// Neighbour values (x null: none, for the diagonal alone) and, with eager,
// the face coefficients.  Without eager the caller loads the coefficients
// of irregular cells (load_coef) once the class byte is known.
template <class S, class C>
__device__ __forceinline__ void load_nbhd(const LevelView& L, const S* __restrict__ x, int P,
                                          bool eager, Nbhd<C>& n) {
  const Geom& g = L.g;
  n.xl = n.xh = n.xs = n.xn = (C)0;
  n.cxl = n.cxh = n.cyl = n.cyh = n.czl = n.czh = (C)0;
  if (x) {
    n.xl = St<S, C>::ld(x + P - 1);
    n.xh = St<S, C>::ld(x + P + 1);
    n.xs = St<S, C>::ld(x + P - g.sx);
    n.xn = St<S, C>::ld(x + P + g.sx);
  }
  if (eager) load_coef<C>(L, P, n);
}

// A x at an active cell: regular cells (every face coefficient 1) take the
// plain form, others the coefficient form.
template <class C>
__device__ __forceinline__ C apply_cls(const Geom& g, bool regular, const Nbhd<C>& n, C xP, C xm,
                                       C xp) {
  const C ih2x = (C)(1.0 / (g.hx * g.hx)), ih2y = (C)(1.0 / (g.hy * g.hy)),
          ih2z = (C)(1.0 / (g.hz * g.hz));
  C s;
  if (regular) {
    s = ((C)2 * xP - n.xl - n.xh) * ih2x + ((C)2 * xP - n.xs - n.xn) * ih2y;
    if (g.dim == 3) s += ((C)2 * xP - xm - xp) * ih2z;
  } else {
    s = (n.cxl * (xP - n.xl) + n.cxh * (xP - n.xh)) * ih2x +
        (n.cyl * (xP - n.xs) + n.cyh * (xP - n.xn)) * ih2y;
    if (g.dim == 3) s += (n.czl * (xP - xm) + n.czh * (xP - xp)) * ih2z;
  }
  return s;
}

// Diagonal of A at an active cell, formed as apply_cls forms it.
template <class C>
__device__ __forceinline__ C diag_cls(const Geom& g, bool regular, const Nbhd<C>& n) {
  const C ih2x = (C)(1.0 / (g.hx * g.hx)), ih2y = (C)(1.0 / (g.hy * g.hy)),
          ih2z = (C)(1.0 / (g.hz * g.hz));
  C d;
  if (regular) {
    d = (C)2 * (ih2x + ih2y);
    if (g.dim == 3) d += (C)2 * ih2z;
  } else {
    d = (n.cxl + n.cxh) * ih2x + (n.cyl + n.cyh) * ih2y;
    if (g.dim == 3) d += (n.czl + n.czh) * ih2z;
  }
  return g.sd > 0.0 ? (C)g.sd : d;
}

// Diagonal of A at cell P (active), formed as diag_cls forms it, with the
// coefficients loaded here.
template <class C>
__device__ __forceinline__ C diag_at(const LevelView& L, uint8_t cl, int P) {
  const Geom& g = L.g;
  const C ih2x = (C)(1.0 / (g.hx * g.hx)), ih2y = (C)(1.0 / (g.hy * g.hy)),
          ih2z = (C)(1.0 / (g.hz * g.hz));
  if (g.sd > 0.0) return (C)g.sd;
  if (cl == MG_REGULAR) {
    C d = (C)2 * (ih2x + ih2y);
    if (g.dim == 3) d += (C)2 * ih2z;
    return d;
  }
  C d = ((C)L.cf0[P] + (C)L.cf0[P + 1]) * ih2x + ((C)L.cf1[P] + (C)L.cf1[P + g.sx]) * ih2y;
  if (g.dim == 3) d += ((C)L.cf2[P] + (C)L.cf2[P + g.sxy]) * ih2z;
  return d;
}

// The same diagonal with the coefficients loaded whatever the class, so the
// loads need not wait for the class byte (small, latency-bound levels).
template <class C>
__device__ __forceinline__ C diag_eager(const LevelView& L, uint8_t cl, int P) {
  const Geom& g = L.g;
  const C ih2x = (C)(1.0 / (g.hx * g.hx)), ih2y = (C)(1.0 / (g.hy * g.hy)),
          ih2z = (C)(1.0 / (g.hz * g.hz));
  const C fx0 = (C)L.cf0[P], fx1 = (C)L.cf0[P + 1], fy0 = (C)L.cf1[P], fy1 = (C)L.cf1[P + g.sx];
  const C fz0 = g.dim == 3 ? (C)L.cf2[P] : (C)0, fz1 = g.dim == 3 ? (C)L.cf2[P + g.sxy] : (C)0;
  C dr = (C)2 * (ih2x + ih2y);
  if (g.dim == 3) dr += (C)2 * ih2z;
  C di = (fx0 + fx1) * ih2x + (fy0 + fy1) * ih2y;
  if (g.dim == 3) di += (fz0 + fz1) * ih2z;
  return g.sd > 0.0 ? (C)g.sd : (cl == MG_REGULAR ? dr : di);
}

// The first sweep from zero of a coarse cell whose right-hand side has just
// been formed: w bc / D with bc rounded to storage as the store rounds it.
template <class SC, class C>
__device__ __forceinline__ C zero_sweep_of(C bc, C wj, C D) {
  SC s;
  St<SC, C>::st(&s, bc);
  return wj * St<SC, C>::ld(&s) / D;
}

// ---- damped Jacobi sweep: x_out = x_in + w (b - A x_in) / D -------------------
template <class S, class C>
struct SmoothArgs {
  LevelView L;
  Tiles T;
  const S* xin;
  S* xout;
  const S* b;
  C wj;
  const double* ctl;
};

// Each thread walks cz planes of one column with x(k-1), x(k), x(k+1) in
// registers; in-plane neighbours come through the cache.
template <class S, class C, bool ZERO>
__device__ __forceinline__ void smooth_body(const SmoothArgs<S, C>& a, const TileCtx& c, bool) {
  // Coarse levels are small and their launches latency-bound: every load of
  // a plane (stopping flag, class byte, right-hand side, neighbourhood) goes
  // out at once, and the flag and the class are tested only before the
  // store.
  const LevelView& L = a.L;
  const S* __restrict__ xin = a.xin;
  S* __restrict__ xout = a.xout;
  const S* __restrict__ b = a.b;
  const C wj = a.wj;
  const Geom& g = L.g;
  const bool done = a.ctl[S_DONE] != 0.0;
  const int i = c.tx * MBX + threadIdx.x, j = c.ty * MBY + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const int k0 = c.tz * a.T.cz, k1 = min(g.nz, k0 + a.T.cz);
  const bool d3 = g.dim == 3;
  const bool eager = g.cells() <= NBHD_EAGER_CELLS;
  int P = g.idx(i, j, k0);
  C xm = 0, xc = 0;
  if (!ZERO) {
    xc = St<S, C>::ld(xin + P);
    if (d3) xm = St<S, C>::ld(xin + P - g.sxy);
  }
  for (int k = k0; k < k1; ++k, P += g.sxy) {
    const uint8_t cl = L.cls[P];
    const C bP = St<S, C>::ld(b + P);
    Nbhd<C> n;
    load_nbhd<S, C>(L, ZERO ? nullptr : xin, P, eager, n);
    C xp = 0;
    if (!ZERO && d3) xp = St<S, C>::ld(xin + P + g.sxy);
    if (!eager && cl == MG_IRREGULAR) load_coef<C>(L, P, n);
    if (!done && cl != MG_INACTIVE) {
      const bool reg = cl == MG_REGULAR;
      const C D = diag_cls<C>(g, reg, n);
      if (ZERO)
        St<S, C>::st(xout + P, wj * bP / D);
      else
        St<S, C>::st(xout + P, xc + wj * (bP - apply_cls<C>(g, reg, n, xc, xm, xp)) / D);
    }
    xm = xc;
    xc = xp;
  }
}
NFVM_TILE_KERNELS(k_smooth, smooth_body, SmoothArgs, (S, C), (class S, class C, bool ZERO),
                  (S, C, ZERO), MBS, false)

// Level-0 sweep from face codes: no branch on the cell kind, and the loads of
// two planes are issued before their arithmetic.
template <class S, class C, bool ZERO>
__device__ __forceinline__ void smooth_code_body(const SmoothArgs<S, C>& a, const TileCtx& c,
                                                 bool) {
  // the stopping flag is read with the first plane's loads and tested
  // before the first store (no barrier in this kernel)
  const bool done = a.ctl[S_DONE] != 0.0;
  const LevelView& L = a.L;
  const S* __restrict__ xin = a.xin;
  S* __restrict__ xout = a.xout;
  const S* __restrict__ b = a.b;
  const C wj = a.wj;
  const Geom& g = L.g;
  const int i = c.tx * MBX + threadIdx.x, j = c.ty * MBY + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const int k0 = c.tz * a.T.cz, k1 = min(g.nz, k0 + a.T.cz);
  const bool d3 = g.dim == 3;
  int P = g.idx(i, j, k0);
  if (ZERO) {
    for (int k = k0; k < k1; ++k, P += g.sxy) {
      const uint32_t cd = L.code[P];
      const C bP = St<S, C>::ld(b + P);
      if (done) return;
      if (cd != FACE_CODE_INACTIVE) St<S, C>::st(xout + P, wj * bP / diag_code<C>(g, cd));
    }
    return;
  }
  const JacobiConst<C> jk = jacobi_const<C>(g, wj);
  auto ld = [&](int Q) { return St<S, C>::ld(xin + Q); };
  C xc = St<S, C>::ld(xin + P);
  C xm = d3 ? St<S, C>::ld(xin + P - g.sxy) : (C)0;
  int k = k0;
  for (; k + 1 < k1; k += 2, P += 2 * g.sxy) {  // 3D only (a 2D level has one plane)
    const int Q = P + g.sxy;
    const uint32_t c0 = L.code[P], c1 = L.code[Q];
    const C b0 = St<S, C>::ld(b + P), b1 = St<S, C>::ld(b + Q);
    const C xp = St<S, C>::ld(xin + Q), xpp = St<S, C>::ld(xin + Q + g.sxy);
    const C y0 = jacobi_code<C>(g, jk, c0, xc, ld(P - 1), ld(P + 1), ld(P - g.sx), ld(P + g.sx),
                                xm, xp, b0);
    const C y1 = jacobi_code<C>(g, jk, c1, xp, ld(Q - 1), ld(Q + 1), ld(Q - g.sx), ld(Q + g.sx),
                                xc, xpp, b1);
    if (done) return;
    if (c0 != FACE_CODE_INACTIVE) St<S, C>::st(xout + P, y0);
    if (c1 != FACE_CODE_INACTIVE) St<S, C>::st(xout + Q, y1);
    xm = xp;
    xc = xpp;
  }
  if (k < k1) {
    const uint32_t cd = L.code[P];
    const C bP = St<S, C>::ld(b + P);
    const C xp = d3 ? St<S, C>::ld(xin + P + g.sxy) : (C)0;
    const C y = jacobi_code<C>(g, jk, cd, xc, ld(P - 1), ld(P + 1), ld(P - g.sx), ld(P + g.sx),
                               xm, xp, bP);
    if (done) return;
    if (cd != FACE_CODE_INACTIVE) St<S, C>::st(xout + P, y);
  }
}
NFVM_TILE_KERNELS(k_smooth_code, smooth_code_body, SmoothArgs, (S, C),
                  (class S, class C, bool ZERO), (S, C, ZERO), MBS, false)

// Level-0 sweep over four consecutive x cells per thread (nx a multiple of
// 4): one aligned 4-wide load per row (the centre row, the rows at y +- 1 and
// the plane above), the two x neighbours past the ends, the four face codes
// in one 8-byte load; a wave covers 256 cells of a row.  Inactive cells are
// written as 0 (the value they always hold).  Per cell the arithmetic is
// apply_code's.
template <class S>
struct Quad {
  typedef S V __attribute__((ext_vector_type(4)));
};
// level-0 storage types (coarse-only BF16 has no four-wide form)
template <class S>
constexpr bool has_quad = !std::is_same<S, bf16>::value;

// One sweep of four consecutive cells (k_smooth_code4's arithmetic; inactive
// cells are 0).
template <class S, class C>
__device__ __forceinline__ typename Quad<S>::V sweep_quad_at(const Geom& g,
                                                             const JacobiConst<C>& jk, uint2 cw,
                                                             typename Quad<S>::V xc, C xl, C xr,
                                                             typename Quad<S>::V xs,
                                                             typename Quad<S>::V xn,
                                                             typename Quad<S>::V xm,
                                                             typename Quad<S>::V xp,
                                                             typename Quad<S>::V bb) {
  typedef typename Quad<S>::V V4;
  const uint32_t cd[4] = {cw.x & 0xFFFFu, cw.x >> 16, cw.y & 0xFFFFu, cw.y >> 16};
  const C xv[6] = {xl, (C)xc[0], (C)xc[1], (C)xc[2], (C)xc[3], xr};
  V4 out;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const C y = jacobi_code<C>(g, jk, cd[q], xv[q + 1], xv[q], xv[q + 2], (C)xs[q], (C)xn[q],
                               (C)xm[q], (C)xp[q], (C)bb[q]);
    out[q] = cd[q] != FACE_CODE_INACTIVE ? (S)y : (S)0;
  }
  return out;
}

template <class S, class C>
__device__ __forceinline__ void smooth_code4_body(const SmoothArgs<S, C>& a, const TileCtx& c,
                                                  bool) {
  typedef typename Quad<S>::V V4;
  const bool done = a.ctl[S_DONE] != 0.0;
  const LevelView& L = a.L;
  const S* __restrict__ xin = a.xin;
  S* __restrict__ xout = a.xout;
  const S* __restrict__ b = a.b;
  const C wj = a.wj;
  const Geom& g = L.g;
  const int i0 = 4 * (c.tx * MBX + threadIdx.x), j = c.ty * MBY + threadIdx.y;
  if (i0 >= g.nx || j >= g.ny) return;
  const int k0 = c.tz * a.T.cz, k1 = min(g.nz, k0 + a.T.cz);
  const bool d3 = g.dim == 3;
  int P = g.idx(i0, j, k0);
  const JacobiConst<C> jk = jacobi_const<C>(g, wj);
  V4 xc = *(const V4*)(xin + P);
  V4 xm = d3 ? *(const V4*)(xin + P - g.sxy) : V4(0);
  for (int k = k0; k < k1; ++k, P += g.sxy) {
    const V4 xp = d3 ? *(const V4*)(xin + P + g.sxy) : V4(0);
    const V4 xs = *(const V4*)(xin + P - g.sx), xn = *(const V4*)(xin + P + g.sx);
    const V4 bb = *(const V4*)(b + P);
    const C xl = St<S, C>::ld(xin + P - 1), xr = St<S, C>::ld(xin + P + 4);
    const uint2 cw = *(const uint2*)(L.code + P);
    if (done) return;
    *(V4*)(xout + P) = sweep_quad_at<S, C>(g, jk, cw, xc, xl, xr, xs, xn, xm, xp, bb);
    xm = xc;
    xc = xp;
  }
}
NFVM_TILE_KERNELS(k_smooth_code4, smooth_code4_body, SmoothArgs, (S, C), (class S, class C),
                  (S, C), MBS, false)

// Whether a level-0 sweep takes the four-cells-per-thread kernel.
__host__ inline bool sweep_quad(const Level& l, bool from_zero) {
  return l.code && !from_zero && l.g.nx % 4 == 0;
}

// Coarse-level sweep over four consecutive x cells per thread, for the large
// coarse levels (bandwidth-bound, unlike the small ones smooth_body serves):
// one 4-wide load per row (centre, y +- 1, the plane above) and of the
// right-hand side, the four class bytes in one 4-byte load, the two x
// neighbours past the ends; irregular cells load their face coefficients
// after the class test, as smooth_body does for levels of this size.  Per
// cell the arithmetic is smooth_body's; inactive cells are written as 0, the
// value they hold.
template <class S, class C>
__device__ __forceinline__ void smooth4_body(const SmoothArgs<S, C>& a, const TileCtx& c, bool) {
  typedef typename Quad<S>::V V4;
  const bool done = a.ctl[S_DONE] != 0.0;
  const LevelView& L = a.L;
  const S* __restrict__ xin = a.xin;
  S* __restrict__ xout = a.xout;
  const S* __restrict__ b = a.b;
  const C wj = a.wj;
  const Geom& g = L.g;
  const int i0 = 4 * (c.tx * MBX + threadIdx.x), j = c.ty * MBY + threadIdx.y;
  if (i0 >= g.nx || j >= g.ny) return;
  const int k0 = c.tz * a.T.cz, k1 = min(g.nz, k0 + a.T.cz);
  const bool d3 = g.dim == 3;
  int P = g.idx(i0, j, k0);
  V4 xc = *(const V4*)(xin + P);
  V4 xm = d3 ? *(const V4*)(xin + P - g.sxy) : V4(0);
  for (int k = k0; k < k1; ++k, P += g.sxy) {
    const V4 xp = d3 ? *(const V4*)(xin + P + g.sxy) : V4(0);
    const V4 xs = *(const V4*)(xin + P - g.sx), xn = *(const V4*)(xin + P + g.sx);
    const V4 bb = *(const V4*)(b + P);
    const C xl = St<S, C>::ld(xin + P - 1), xr = St<S, C>::ld(xin + P + 4);
    const uint32_t cw = *(const uint32_t*)(L.cls + P);
    if (done) return;
    const C xv[6] = {xl, (C)xc[0], (C)xc[1], (C)xc[2], (C)xc[3], xr};
    V4 out;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint8_t cl = (uint8_t)(cw >> (8 * q));
      Nbhd<C> n;
      n.xl = xv[q];
      n.xh = xv[q + 2];
      n.xs = (C)xs[q];
      n.xn = (C)xn[q];
      n.cxl = n.cxh = n.cyl = n.cyh = n.czl = n.czh = (C)0;
      if (cl == MG_IRREGULAR) load_coef<C>(L, P + q, n);
      const bool reg = cl == MG_REGULAR;
      const C D = diag_cls<C>(g, reg, n);
      const C Ax = apply_cls<C>(g, reg, n, xv[q + 1], (C)xm[q], (C)xp[q]);
      out[q] = cl != MG_INACTIVE ? (S)(xv[q + 1] + wj * ((C)bb[q] - Ax) / D) : (S)0;
    }
    *(V4*)(xout + P) = out;
    xm = xc;
    xc = xp;
  }
}
NFVM_TILE_KERNELS(k_smooth4, smooth4_body, SmoothArgs, (S, C), (class S, class C), (S, C), MBS,
                  false)

// Whether a coarse-level sweep takes k_smooth4.
template <class S>
__host__ inline bool coarse_quad(const Level& l, bool from_zero) {
  return has_quad<S> && !l.code && !from_zero && l.g.nx % 4 == 0 &&
         l.g.cells() > NBHD_EAGER_CELLS;
}

template <class S, class C>
SmoothArgs<S, C> smooth_args(const Level& l, const void* xin, void* xout, double wj, bool from_zero,
                             const double* ctl) {
  const int tk = from_zero ? TK_SMOOTH_ZERO : TK_SMOOTH;
  const Tiles T = sweep_quad(l, from_zero) || coarse_quad<S>(l, from_zero)
                      ? make_tiles(l.g.nx / 4, l.g.ny, l.g.nz, l.tt[tk])
                      : lvl_tiles(l, tk);
  return SmoothArgs<S, C>{view(l), T, (const S*)xin, (S*)xout, (const S*)l.b, (C)wj, ctl};
}

template <class S, class C>
void launch_smooth(const Level& l, const void* xin, void* xout, double wj, bool from_zero,
                   const double* ctl, hipStream_t s) {
  const SmoothArgs<S, C> a = smooth_args<S, C>(l, xin, xout, wj, from_zero, ctl);
  const dim3 G(a.T.grid), B(MBX, MBY);
  if (l.code) {
    if (from_zero)
      NFVM_LAUNCH((k_smooth_code<S, C, true>), G, B, 0, s, a);
    else if (sweep_quad(l, false)) {
      if constexpr (has_quad<S>) NFVM_LAUNCH((k_smooth_code4<S, C>), G, B, 0, s, a);
    } else {
      NFVM_LAUNCH((k_smooth_code<S, C, false>), G, B, 0, s, a);
    }
  } else if (from_zero) {
    NFVM_LAUNCH((k_smooth<S, C, true>), G, B, 0, s, a);
  } else if (coarse_quad<S>(l, false)) {
    if constexpr (has_quad<S>) NFVM_LAUNCH((k_smooth4<S, C>), G, B, 0, s, a);
  } else {
    NFVM_LAUNCH((k_smooth<S, C, false>), G, B, 0, s, a);
  }
}

// ---- two level-0 sweeps in one pass ------------------------------------------------
// x2 = S(S(x0)), S(x) = x + wj (b - A x) / D, four cells per thread as in
// k_smooth_code4: half the HBM bytes of two single sweeps (x0, b and the
// face code read once, x2 written once).  Each thread owns two rows of four
// columns and walks the planes of its column tile: per plane it forms the
// first sweep one plane ahead for its rows (registers) and puts it in LDS;
// the first and last waves of the workgroup also form it for the row past
// their side of the tile.  A wave's first and last lanes are halo lanes:
// they form the first sweep of the four columns past each side of the tile
// and write no result, so a tile is 62 four-cell columns wide and every lane
// runs the same instructions.  After one barrier per plane the second sweep
// reads its in-plane neighbours from LDS and its z neighbours from
// registers.  Both sweeps take
// k_smooth_code4's arithmetic on the same values and the first is rounded to
// the storage type before the second reads it, so the result is bitwise that
// of two single sweeps.  The first sweep is 0 outside the box and on
// inactive cells, as a single sweep leaves them.  LDS holds three planes, so
// one barrier per plane suffices: a wave that writes plane k + 1 has passed
// the barrier of plane k - 1, which every wave reaches only after reading
// plane k - 2, the buffer plane k + 1 reuses.
constexpr int S2_ROW = 4 * MBX;          // the cells of a wave's 64 four-cell columns
constexpr int S2_ROWS = 2 * MBY;         // rows of a workgroup (two per thread)
constexpr int S2_QX = MBX - 2;           // four-cell columns a tile writes

// The first sweep of a row's quad at one plane, with the plane's right-hand
// side and face codes (kept for the second sweep there).
template <class S>
struct FirstQuad {
  typename Quad<S>::V x1, bb;
  uint2 cw;
};

template <class S, class C>
__device__ __forceinline__ void smooth2_body(const SmoothArgs<S, C>& a, const TileCtx& c, bool) {
  typedef typename Quad<S>::V V4;
  __shared__ S lx[3][S2_ROWS + 2][S2_ROW];
  if (a.ctl[S_DONE] != 0.0) return;  // (uniform: every thread reads the same flag)
  const LevelView& L = a.L;
  const S* __restrict__ x = a.xin;
  S* __restrict__ xout = a.xout;
  const S* __restrict__ b = a.b;
  const Geom& g = L.g;
  const JacobiConst<C> jk = jacobi_const<C>(g, a.wj);
  const bool d3 = g.dim == 3;
  const int lane = threadIdx.x, wy = threadIdx.y;
  const int i0 = 4 * (c.tx * S2_QX + lane - 1);  // (lane 0: the halo left of the tile)
  const int jt = S2_ROWS * c.ty;  // first row of the workgroup
  const int j0 = jt + 2 * wy;     // this thread's rows j0, j0 + 1
  const bool col = i0 >= 0 && i0 < g.nx;
  const bool halo = lane == 0 || lane == MBX - 1;  // no result of its own
  const bool live[2] = {col && j0 < g.ny, col && j0 + 1 < g.ny};
  const int k0 = c.tz * a.T.cz, k1 = min(g.nz, k0 + a.T.cz);
  // the row past the workgroup's side of the tile (first wave: above the
  // first row, last wave: below the last), 0 outside the box
  const int jx = wy == 0 ? jt - 1 : jt + S2_ROWS;
  const bool xrow = (wy == 0 || wy == MBY - 1) && col && jx >= 0 && jx < g.ny;
  auto first4 = [&](int r, int m) -> FirstQuad<S> {
    const int P = g.idx(i0, r, m);
    const V4 xc = *(const V4*)(x + P);
    const V4 xm = d3 ? *(const V4*)(x + P - g.sxy) : V4(0);
    const V4 xp = d3 ? *(const V4*)(x + P + g.sxy) : V4(0);
    const V4 xs = *(const V4*)(x + P - g.sx), xn = *(const V4*)(x + P + g.sx);
    const C xl = St<S, C>::ld(x + P - 1), xr = St<S, C>::ld(x + P + 4);
    FirstQuad<S> f;
    f.bb = *(const V4*)(b + P);
    f.cw = *(const uint2*)(L.code + P);
    f.x1 = sweep_quad_at<S, C>(g, jk, f.cw, xc, xl, xr, xs, xn, xm, xp, f.bb);
    return f;
  };
  // x0 of this thread's rows as the walk carries it: planes m - 1 and m of
  // the next plane m whose first sweep is formed (each plane loaded once;
  // the rows' in-plane neighbours j0 + 1 and j0 are each other's centres)
  auto ldp = [&](int r, int m) -> V4 {
    return (m >= -1 && m <= g.nz && (d3 || m == 0)) ? *(const V4*)(x + g.idx(i0, r, m)) : V4(0);
  };
  V4 xa[2], xb[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    xa[h] = live[h] ? ldp(j0 + h, k0 - 2) : V4(0);
    xb[h] = live[h] ? ldp(j0 + h, k0 - 1) : V4(0);
  }
  // the first sweep of this thread's rows at plane m (0 outside the box);
  // advances the carried planes by one
  auto own2 = [&](int m, FirstQuad<S> (&f)[2]) {
    V4 xn[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) xn[h] = live[h] ? ldp(j0 + h, m + 1) : V4(0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (live[h] && m >= 0 && m < g.nz) {
        const int P = g.idx(i0, j0 + h, m);
        const V4 ys = h == 0 ? *(const V4*)(x + P - g.sx) : xb[0];
        const V4 yn = h == 1 ? *(const V4*)(x + P + g.sx) : xb[1];
        const C xl = St<S, C>::ld(x + P - 1), xr = St<S, C>::ld(x + P + 4);
        f[h].bb = *(const V4*)(b + P);
        f[h].cw = *(const uint2*)(L.code + P);
        f[h].x1 = sweep_quad_at<S, C>(g, jk, f[h].cw, xb[h], xl, xr, ys, yn, xa[h], xn[h],
                                      f[h].bb);
      } else {
        f[h].x1 = f[h].bb = V4(0);
        f[h].cw = make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      xa[h] = xb[h];
      xb[h] = xn[h];
    }
  };
  // plane m of the first sweep into LDS buffer m % 3 (the own quads given)
  auto to_lds = [&](int m, const V4& q0, const V4& q1) {
    S(*row)[S2_ROW] = lx[m % 3];
    *(V4*)&row[2 * wy + 1][4 * lane] = q0;
    *(V4*)&row[2 * wy + 2][4 * lane] = q1;
    if (wy == 0 || wy == MBY - 1) {
      const V4 e = xrow ? first4(jx, m).x1 : V4(0);
      *(V4*)&row[wy == 0 ? 0 : S2_ROWS + 1][4 * lane] = e;
    }
  };
  // prologue: planes k0 - 1 (registers) and k0 (registers and LDS)
  V4 ym[2], yc[2];
  V4 bc[2];
  uint2 cc[2];
  {
    FirstQuad<S> f[2];
    own2(k0 - 1, f);
#pragma unroll
    for (int h = 0; h < 2; ++h) ym[h] = f[h].x1;
    own2(k0, f);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      yc[h] = f[h].x1;
      bc[h] = f[h].bb;
      cc[h] = f[h].cw;
    }
  }
  to_lds(k0, yc[0], yc[1]);
  for (int k = k0; k < k1; ++k) {
    // the first sweep one plane ahead (LDS only if a later plane of this
    // tile reads it in-plane)
    FirstQuad<S> fp[2];
    own2(k + 1, fp);
    if (k + 1 < k1) to_lds(k + 1, fp[0].x1, fp[1].x1);
    __syncthreads();
    S(*row)[S2_ROW] = lx[k % 3];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (live[h] && !halo) {
        const int lr = 2 * wy + 1 + h;  // this row's LDS row
        const V4 ys = *(const V4*)&row[lr - 1][4 * lane];
        const V4 yn = *(const V4*)&row[lr + 1][4 * lane];
        const C yl = (C)row[lr][4 * lane - 1];
        const C yr = (C)row[lr][4 * lane + 4];
        *(V4*)(xout + g.idx(i0, j0 + h, k)) =
            sweep_quad_at<S, C>(g, jk, cc[h], yc[h], yl, yr, ys, yn, ym[h], fp[h].x1, bc[h]);
      }
      ym[h] = yc[h];
      yc[h] = fp[h].x1;
      bc[h] = fp[h].bb;
      cc[h] = fp[h].cw;
    }
  }
}
NFVM_TILE_KERNELS(k_smooth2_code4, smooth2_body, SmoothArgs, (S, C), (class S, class C),
                  (S, C), MBS, false)

// Whether level l takes two-sweep passes (level 0 with four-cell rows).
bool sweep_pair(const Level& l) { return l.code && l.g.nx % 4 == 0; }

template <class S, class C>
void launch_smooth2(const Level& l, const void* xin, void* xout, double wj, const double* ctl,
                    hipStream_t s) {
  if constexpr (has_quad<S>) {
    // tiles of 62 four-cell columns (make_tiles counts 64 per tile) by 8
    // rows (two per thread)
    const int nq = l.g.nx / 4, ntx = (nq + S2_QX - 1) / S2_QX;
    const Tiles T = make_tiles(ntx * MBX, (l.g.ny + 1) / 2, l.g.nz, l.tt[TK_SMOOTH2]);
    const SmoothArgs<S, C> a{view(l), T, (const S*)xin, (S*)xout, (const S*)l.b, (C)wj, ctl};
    NFVM_LAUNCH((k_smooth2_code4<S, C>), dim3(T.grid), dim3(MBX, MBY), 0, s, a);
  }
}

// ---- residual and restriction: b_c = mean over the 2^dim children of (b - A x)
// One thread per fine column i and coarse row J: it walks the two fine rows
// 2J, 2J + 1 plane by plane (the z neighbours of both rows stay in
// registers) and sums each row over the two fine planes of a coarse plane;
// the x pair is summed by a lane exchange, so no workgroup barrier is
// needed.  A workgroup covers 64 fine columns by 4 coarse rows; tiles count
// coarse rows along y and coarse planes along z.  Sum order per coarse cell:
// ((row 2J over planes) + (x partner's)) + ((row 2J + 1 over planes) + (x
// partner's)).
template <class S, class C, class SC>
struct RestrictArgs {
  LevelView F;
  Tiles T;  // fine columns, coarse rows, coarse planes
  const S* x;
  const S* b;
  LevelView Cl;
  SC* bc;
  SC* zc;  // coarse level's first sweep from zero (null: not fused)
  C wj;
  const double* ctl;
};

// b - A x at fine cell P (0 for inactive cells), z neighbours given.
template <class S, class C>
__device__ __forceinline__ C resid_at(const LevelView& F, const S* __restrict__ x,
                                      const S* __restrict__ b, int P, C xc, C xm, C xp) {
  C Ax, D;
  if (F.code) {
    const uint32_t cd = F.code[P];
    const C bP = St<S, C>::ld(b + P);
    apply_code<S, C>(F.g, cd, x, P, xc, xm, xp, Ax, D);
    return cd != FACE_CODE_INACTIVE ? bP - Ax : (C)0;
  }
  // coarse levels: every load goes out before the class byte is tested
  const uint8_t cl = F.cls[P];
  const C bP = St<S, C>::ld(b + P);
  const bool eager = F.g.cells() <= NBHD_EAGER_CELLS;
  Nbhd<C> n;
  load_nbhd<S, C>(F, x, P, eager, n);
  if (!eager && cl == MG_IRREGULAR) load_coef<C>(F, P, n);
  if (cl == MG_INACTIVE) return (C)0;
  (void)D;
  return bP - apply_cls<C>(F.g, cl == MG_REGULAR, n, xc, xm, xp);
}

template <class S, class C, class SC>
__device__ __forceinline__ void restrict_body(const RestrictArgs<S, C, SC>& a, const TileCtx& c,
                                              bool) {
  // the stopping flag (uniform over the workgroup) is read with the first
  // loads and tested before the first store; no barrier in this kernel
  const bool done = a.ctl[S_DONE] != 0.0;
  const LevelView& F = a.F;
  const LevelView& Cl = a.Cl;
  const S* __restrict__ x = a.x;
  const S* __restrict__ b = a.b;
  const Geom& g = F.g;
  const int lx = threadIdx.x;
  const int i = c.tx * MBX + lx, J = c.ty * MBY + threadIdx.y;
  // lanes past the box still take part in the lane exchange
  const bool in = i < g.nx && J < Cl.g.ny;
  const bool d3 = g.dim == 3;
  const int K0 = c.tz * a.T.cz, K1 = min(Cl.g.nz, K0 + a.T.cz);
  const int kz = d3 ? 2 : 1;
  int P0 = in ? g.idx(i, 2 * J, kz * K0) : 0, P1 = P0 + g.sx;
  C xm0 = 0, xc0 = 0, xm1 = 0, xc1 = 0;
  if (in) {
    xc0 = St<S, C>::ld(x + P0);
    xc1 = St<S, C>::ld(x + P1);
    if (d3) {
      xm0 = St<S, C>::ld(x + P0 - g.sxy);
      xm1 = St<S, C>::ld(x + P1 - g.sxy);
    }
  }
  const bool lead = in && !(lx & 1);  // the lane that stores the coarse cell
  const bool ceager = Cl.g.cells() <= NBHD_EAGER_CELLS;
  const int dz = d3 ? g.sxy : 0;  // (2D: the one plane read twice, counted once)
  for (int K = K0; K < K1; ++K) {
    // the coarse cell's class byte and diagonal go out with the fine loads
    const int PC = lead ? Cl.g.idx(i >> 1, J, K) : 0;
    const uint8_t ccl = lead ? Cl.cls[PC] : (uint8_t)MG_INACTIVE;
    const C dge = (lead && ceager) ? diag_eager<C>(Cl, ccl, PC) : (C)1;
    C r0 = 0, r1 = 0;
    if (in) {
      // both fine planes of the coarse plane: every load of the four cells
      // before their arithmetic
      const C xp0 = St<S, C>::ld(x + P0 + dz), xp1 = St<S, C>::ld(x + P1 + dz);
      const C xq0 = St<S, C>::ld(x + P0 + 2 * dz), xq1 = St<S, C>::ld(x + P1 + 2 * dz);
      const C a0 = resid_at<S, C>(F, x, b, P0, xc0, xm0, xp0);
      const C a1 = resid_at<S, C>(F, x, b, P1, xc1, xm1, xp1);
      const C c0 = resid_at<S, C>(F, x, b, P0 + dz, xp0, xc0, xq0);
      const C c1 = resid_at<S, C>(F, x, b, P1 + dz, xp1, xc1, xq1);
      r0 += a0;
      r1 += a1;
      if (d3) {
        r0 += c0;
        r1 += c1;
      }
      xm0 = xp0;
      xc0 = xq0;
      xm1 = xp1;
      xc1 = xq1;
      P0 += kz * g.sxy;
      P1 += kz * g.sxy;
    }
    r0 += __shfl_xor(r0, 1);
    r1 += __shfl_xor(r1, 1);
    if (done) return;
    if (lead && ccl != MG_INACTIVE) {
      const C bc = (r0 + r1) * (C)(d3 ? 0.125 : 0.25);
      St<SC, C>::st(a.bc + PC, bc);
      // first pre-smoothing sweep (from zero) of the coarse level
      if (a.zc)
        St<SC, C>::st(a.zc + PC, zero_sweep_of<SC, C>(bc, a.wj,
                                                      ceager ? dge : diag_at<C>(Cl, ccl, PC)));
    }
  }
}
NFVM_TILE_KERNELS(k_resid_restrict, restrict_body, RestrictArgs, (S, C, SC),
                  (class S, class C, class SC), (S, C, SC), MBS, false)

// Level 0 with nx a multiple of 4: one thread per four fine columns (two
// coarse cells) and coarse row J, with four-wide loads of the rows 2J - 1 ..
// 2J + 2, the right-hand sides and the face codes.  The sums are formed in
// the order of restrict_body, so the results are the same.
template <class S, class C, class SC>
__device__ __forceinline__ void restrict4_body(const RestrictArgs<S, C, SC>& a, const TileCtx& c,
                                               bool) {
  typedef typename Quad<S>::V V4;
  const bool done = a.ctl[S_DONE] != 0.0;
  const LevelView& F = a.F;
  const LevelView& Cl = a.Cl;
  const S* __restrict__ x = a.x;
  const S* __restrict__ b = a.b;
  const Geom& g = F.g;
  const int i0 = 4 * (c.tx * MBX + threadIdx.x), J = c.ty * MBY + threadIdx.y;
  if (i0 >= g.nx || J >= Cl.g.ny) return;
  const bool d3 = g.dim == 3;
  const int K0 = c.tz * a.T.cz, K1 = min(Cl.g.nz, K0 + a.T.cz);
  const int kz = d3 ? 2 : 1;
  int P0 = g.idx(i0, 2 * J, kz * K0);  // row 2J; row 2J + 1 is P0 + sx
  // centre and lower plane of both rows
  V4 xc0 = *(const V4*)(x + P0), xc1 = *(const V4*)(x + P0 + g.sx);
  V4 xm0 = d3 ? *(const V4*)(x + P0 - g.sxy) : V4(0);
  V4 xm1 = d3 ? *(const V4*)(x + P0 + g.sx - g.sxy) : V4(0);
  const bool ceager = Cl.g.cells() <= NBHD_EAGER_CELLS;
  for (int K = K0; K < K1; ++K) {
    // the coarse cells' class bytes (and, on small levels, diagonals) go out
    // with the fine loads
    const int PC0 = Cl.g.idx(i0 >> 1, J, K);
    const uint8_t ccl[2] = {Cl.cls[PC0], Cl.cls[PC0 + 1]};
    C dge[2] = {(C)1, (C)1};
    if (ceager) {
      dge[0] = diag_eager<C>(Cl, ccl[0], PC0);
      dge[1] = diag_eager<C>(Cl, ccl[1], PC0 + 1);
    }
    C r[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    for (int cc = 0; cc < kz; ++cc, P0 += g.sxy) {
      const int P1 = P0 + g.sx;
      const V4 xp0 = d3 ? *(const V4*)(x + P0 + g.sxy) : V4(0);
      const V4 xp1 = d3 ? *(const V4*)(x + P1 + g.sxy) : V4(0);
      const V4 ys = *(const V4*)(x + P0 - g.sx), yn = *(const V4*)(x + P1 + g.sx);
      const V4 b0 = *(const V4*)(b + P0), b1 = *(const V4*)(b + P1);
      const uint2 w0 = *(const uint2*)(F.code + P0), w1 = *(const uint2*)(F.code + P1);
      const C l0 = St<S, C>::ld(x + P0 - 1), h0 = St<S, C>::ld(x + P0 + 4);
      const C l1 = St<S, C>::ld(x + P1 - 1), h1 = St<S, C>::ld(x + P1 + 4);
      const uint32_t cd0[4] = {w0.x & 0xFFFFu, w0.x >> 16, w0.y & 0xFFFFu, w0.y >> 16};
      const uint32_t cd1[4] = {w1.x & 0xFFFFu, w1.x >> 16, w1.y & 0xFFFFu, w1.y >> 16};
      const C v0[6] = {l0, (C)xc0[0], (C)xc0[1], (C)xc0[2], (C)xc0[3], h0};
      const C v1[6] = {l1, (C)xc1[0], (C)xc1[1], (C)xc1[2], (C)xc1[3], h1};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        C A, D;
        // row 2J: y neighbours are row 2J - 1 and row 2J + 1
        apply_code_v<C>(g, cd0[e], v0[e + 1], v0[e], v0[e + 2], (C)ys[e], (C)xc1[e], (C)xm0[e],
                        (C)xp0[e], A, D);
        r[0][e] += cd0[e] != FACE_CODE_INACTIVE ? (C)b0[e] - A : (C)0;
        // row 2J + 1: y neighbours are row 2J and row 2J + 2
        apply_code_v<C>(g, cd1[e], v1[e + 1], v1[e], v1[e + 2], (C)xc0[e], (C)yn[e], (C)xm1[e],
                        (C)xp1[e], A, D);
        r[1][e] += cd1[e] != FACE_CODE_INACTIVE ? (C)b1[e] - A : (C)0;
      }
      xm0 = xc0;
      xc0 = xp0;
      xm1 = xc1;
      xc1 = xp1;
    }
    if (done) return;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (ccl[h] == MG_INACTIVE) continue;
      const int PC = PC0 + h;
      const C s0 = r[0][2 * h] + r[0][2 * h + 1], s1 = r[1][2 * h] + r[1][2 * h + 1];
      const C bc = (s0 + s1) * (C)(d3 ? 0.125 : 0.25);
      St<SC, C>::st(a.bc + PC, bc);
      // first pre-smoothing sweep (from zero) of the coarse level
      if (a.zc)
        St<SC, C>::st(a.zc + PC, zero_sweep_of<SC, C>(
                                     bc, a.wj, ceager ? dge[h] : diag_at<C>(Cl, ccl[h], PC)));
    }
  }
}
NFVM_TILE_KERNELS(k_resid_restrict4, restrict4_body, RestrictArgs, (S, C, SC),
                  (class S, class C, class SC), (S, C, SC), MBS, false)

// Whether the restriction from fine level f takes the four-column kernel.
__host__ inline bool restrict_quad(const Level& f) { return f.code && f.g.nx % 4 == 0; }

template <class S, class C, class SC>
RestrictArgs<S, C, SC> restrict_args(const Level& f, const Level& c, const double* ctl, void* zc,
                                     double wj) {
  return RestrictArgs<S, C, SC>{view(f),
                                make_tiles(restrict_quad(f) ? f.g.nx / 4 : f.g.nx, c.g.ny,
                                           c.g.nz, f.tt[TK_RESTRICT]),
                                (const S*)f.x[f.cur],
                                (const S*)f.b,
                                view(c),
                                (SC*)c.b,
                                (SC*)zc,
                                (C)wj,
                                ctl};
}

template <class S, class C, class SC>
void launch_resid_restrict(const Level& f, const Level& c, const double* ctl, hipStream_t s,
                           void* zc, double wj) {
  const RestrictArgs<S, C, SC> a = restrict_args<S, C, SC>(f, c, ctl, zc, wj);
  if (restrict_quad(f)) {
    if constexpr (has_quad<S>)
      NFVM_LAUNCH((k_resid_restrict4<S, C, SC>), dim3(a.T.grid), dim3(MBX, MBY), 0, s, a);
  } else {
    NFVM_LAUNCH((k_resid_restrict<S, C, SC>), dim3(a.T.grid), dim3(MBX, MBY), 0, s, a);
  }
}

// ---- prolongation and correction: x_f += PROL(e_c) ------------------------------
// Cell-centred linear interpolation axis by axis (x, y, then z), weights 3/4
// and 1/4.  A neighbour outside the box contributes the boundary ghost
// (1 - c_f) e (c_f = 0: zero gradient, 2: zero value); an inactive neighbour
// is replaced by the cell it is interpolated from.
//
// For a fine column (i, j) the x and y steps on one coarse plane involve the
// coarse cells (I, J), (I + sx, J), (I, J + sy), (I + sx, J + sy) of that
// plane (sx, sy: side of the fine cell within its parent); they give the
// plane value Y and whether the plane's cell (I, J) takes part (active and
// inside the box).  The z step then combines the planes K and K +- 1.
// The plane value from the four coarse values, whether each cell takes part
// (a00 already includes in_plane, a01 in_plane and iny) and the boundary
// face coefficients cfx0, cfx1 (x faces on the fine cell's side, rows 0 and
// 1) and cfy (y face on its side, row 0).
template <class C>
__device__ __forceinline__ void plane_value(C e00, C e10, C e01, C e11, bool a00, bool a10,
                                            bool a01, bool a11, C cfx0, C cfx1, C cfy, bool inx,
                                            bool iny, C& Y, bool& act) {
  const C w3 = (C)0.75, w1 = (C)0.25;
  const C nb0 = inx ? (a10 ? e10 : e00) : ((C)1 - cfx0) * e00;
  const C X0 = a00 ? w3 * e00 + w1 * nb0 : (C)0;
  const C nb1 = inx ? (a11 ? e11 : e01) : ((C)1 - cfx1) * e01;
  const C X1 = a01 ? w3 * e01 + w1 * nb1 : (C)0;
  const C yn = iny ? (a01 ? X1 : X0) : ((C)1 - cfy) * X0;
  Y = a00 ? w3 * X0 + w1 * yn : (C)0;
  act = a00;
}

template <class C, class SC>
__device__ __forceinline__ void plane_rules(const LevelView& Cl, const SC* __restrict__ e, int Q,
                                            int sx, int oy, bool in_plane, bool inx, bool iny,
                                            C& Y, bool& act) {
  // every index lies in the padded array (one ghost layer around the box)
  const C e00 = St<SC, C>::ld(e + Q), e10 = St<SC, C>::ld(e + Q + sx);
  const C e01 = St<SC, C>::ld(e + Q + oy), e11 = St<SC, C>::ld(e + Q + oy + sx);
  const bool a00 = in_plane && Cl.cls[Q] != MG_INACTIVE;
  const bool a10 = Cl.cls[Q + sx] != MG_INACTIVE;
  const bool a01 = iny && in_plane && Cl.cls[Q + oy] != MG_INACTIVE;
  const bool a11 = Cl.cls[Q + oy + sx] != MG_INACTIVE;
  const C cfx0 = (C)Cl.cf0[sx > 0 ? Q + 1 : Q];
  const C cfx1 = (C)Cl.cf0[sx > 0 ? Q + oy + 1 : Q + oy];
  const C cfy = (C)Cl.cf1[oy > 0 ? Q + oy : Q];
  plane_value<C>(e00, e10, e01, e11, a00, a10, a01, a11, cfx0, cfx1, cfy, inx, iny, Y, act);
}

// The same plane value when the four cells are active and inside the box.
template <class C, class SC>
__device__ __forceinline__ C plane_interior(const SC* __restrict__ e, int Q, int sx, int oy) {
  const C w3 = (C)0.75, w1 = (C)0.25;
  const C e00 = St<SC, C>::ld(e + Q), e10 = St<SC, C>::ld(e + Q + sx);
  const C e01 = St<SC, C>::ld(e + Q + oy), e11 = St<SC, C>::ld(e + Q + oy + sx);
  const C X0 = w3 * e00 + w1 * e10;
  const C X1 = w3 * e01 + w1 * e11;
  return w3 * X0 + w1 * X1;
}

// One thread per fine column (i, j) walking the coarse planes K of its tile,
// with the plane values of K - 1, K and K + 1 in registers (two fine cells
// per coarse plane).  Per plane the wave takes one of two forms: when the
// coarse cells under all its columns have their 26 neighbours active and
// inside the box (`full`), the next plane costs four coarse loads and the
// rules reduce to plain weights; otherwise every lane evaluates all rules
// from the plane's values, flags and face coefficients.  The choice is
// uniform over the wave, so no lane waits for another's path, and both forms
// give the same value where both apply.
template <class S, class C, class SC>
struct ProlongArgs {
  LevelView F;
  Tiles T;  // fine columns, coarse planes
  S* x;
  LevelView Cl;
  const SC* e;
  const double* ctl;
};

template <class S, class C, class SC>
__device__ __forceinline__ void prolong_body(const ProlongArgs<S, C, SC>& a, const TileCtx& c,
                                             bool) {
  // the stopping flag is read with the first loads and tested before the
  // first store (no barrier in this kernel)
  const bool done = a.ctl[S_DONE] != 0.0;
  const LevelView& F = a.F;
  const LevelView& Cl = a.Cl;
  S* __restrict__ x = a.x;
  const SC* __restrict__ e = a.e;
  const int i = c.tx * MBX + threadIdx.x, j = c.ty * MBY + threadIdx.y;
  if (i >= F.g.nx || j >= F.g.ny) return;
  const Geom& cg = Cl.g;
  const bool d3 = cg.dim == 3;
  const int K0 = c.tz * a.T.cz, K1 = min(cg.nz, K0 + a.T.cz);
  const int I = i >> 1, J = j >> 1;
  const int sx = (i & 1) ? 1 : -1, oy = (j & 1) ? cg.sx : -cg.sx;
  const bool inx = (unsigned)(I + sx) < (unsigned)cg.nx;
  const bool iny = (unsigned)(J + ((j & 1) ? 1 : -1)) < (unsigned)cg.ny;
  const C w3 = (C)0.75, w1 = (C)0.25;
  int PC = cg.idx(I, J, K0);
  C ym = 0, yc;
  bool am = false, ac;
  plane_rules<C, SC>(Cl, e, PC, sx, oy, true, inx, iny, yc, ac);
  if (d3) plane_rules<C, SC>(Cl, e, PC - cg.sxy, sx, oy, K0 > 0, inx, iny, ym, am);
  int P = F.g.idx(i, j, d3 ? 2 * K0 : 0);
  // small coarse levels take the full rule set on every plane, with all its
  // loads issued at once (one memory round per plane); larger ones take the
  // interior form where the whole wave can (fewer loads)
  const bool ceager = cg.cells() <= NBHD_EAGER_CELLS;
  bool full = d3 && !ceager && Cl.full[PC] != 0;
  for (int K = K0; K < K1; ++K, PC += cg.sxy) {
    // the fine cells' loads and the next plane's flag go out first: they do
    // not depend on the coarse values
    const uint8_t fc0 = F.cls[P];
    const S x0 = x[P];
    uint8_t fc1 = MG_INACTIVE;
    S x1 = x0;
    bool full_next = false;
    if (d3) {
      fc1 = F.cls[P + F.g.sxy];
      x1 = x[P + F.g.sxy];
      full_next = !ceager && K + 1 < K1 && Cl.full[PC + cg.sxy] != 0;
    }
    C yp = 0, cz_lo = 0, cz_hi = 0;
    bool ap = false;
    if (d3) {
      if (ceager) {
        plane_rules<C, SC>(Cl, e, PC + cg.sxy, sx, oy, K + 1 < cg.nz, inx, iny, yp, ap);
        cz_lo = (C)Cl.cf2[PC];
        cz_hi = (C)Cl.cf2[PC + cg.sxy];
      } else if (__all(full)) {
        yp = plane_interior<C, SC>(e, PC + cg.sxy, sx, oy);
        ap = true;
      } else {
        plane_rules<C, SC>(Cl, e, PC + cg.sxy, sx, oy, K + 1 < cg.nz, inx, iny, yp, ap);
        cz_lo = (C)Cl.cf2[PC];
        cz_hi = (C)Cl.cf2[PC + cg.sxy];
      }
    }
    if (done) return;
    if (fc0 != MG_INACTIVE) {
      C Z = yc;
      if (d3) {
        const C zn = K > 0 ? (am ? ym : yc) : ((C)1 - cz_lo) * yc;
        Z = w3 * yc + w1 * zn;
      }
      St<S, C>::st(x + P, St<S, C>::ld(&x0) + Z);
    }
    if (d3 && fc1 != MG_INACTIVE) {
      const C zn = K + 1 < cg.nz ? (ap ? yp : yc) : ((C)1 - cz_hi) * yc;
      St<S, C>::st(x + P + F.g.sxy, St<S, C>::ld(&x1) + (w3 * yc + w1 * zn));
    }
    P += d3 ? 2 * F.g.sxy : 0;
    full = full_next;
    ym = yc;
    am = ac;
    yc = yp;
    ac = ap;
  }
}
NFVM_TILE_KERNELS(k_prolong, prolong_body, ProlongArgs, (S, C, SC), (class S, class C, class SC),
                  (S, C, SC), MBS, false)

// Level 0 with nx a multiple of 4: one thread per four fine columns, the
// children of coarse cells I0 and I0 + 1 (I0 even), walking the coarse
// planes.  Per plane the coarse cells I0 - 1 .. I0 + 2 of the two rows the
// rules need (values, class bytes, face coefficients) are loaded once for
// the four columns, and each column's value is plane_value's, so the results
// are prolong_body's; the fine values and class bytes go in four-wide loads.
// Inactive fine cells are written back unchanged.
template <class C, class SC>
__device__ __forceinline__ void plane4(const LevelView& Cl, const SC* __restrict__ e, int Q, int oy,
                                       bool in_plane, bool iny, const bool (&inx)[4], C (&Y)[4],
                                       bool (&act)[4]) {
  // every index lies in the padded array: I0 - 1 >= -1 and I0 + 2 <= nx
  C r0[4], r1[4];
  bool c0[4], c1[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    r0[m] = St<SC, C>::ld(e + Q - 1 + m);
    r1[m] = St<SC, C>::ld(e + Q + oy - 1 + m);
    c0[m] = Cl.cls[Q - 1 + m] != MG_INACTIVE;
    c1[m] = Cl.cls[Q + oy - 1 + m] != MG_INACTIVE;
  }
  // x faces of cells I0, I0 + 1 (the low face at the cell's index) and the
  // y faces between the two rows
  C f0[3], f1[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    f0[m] = (C)Cl.cf0[Q + m];
    f1[m] = (C)Cl.cf0[Q + oy + m];
  }
  const int qy = oy > 0 ? Q + oy : Q;
  const C fy[2] = {(C)Cl.cf1[qy], (C)Cl.cf1[qy + 1]};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int h = q >> 1, sx = (q & 1) ? 1 : -1, m = 1 + h;
    plane_value<C>(r0[m], r0[m + sx], r1[m], r1[m + sx], in_plane && c0[m], c0[m + sx],
                   iny && in_plane && c1[m], c1[m + sx], sx > 0 ? f0[h + 1] : f0[h],
                   sx > 0 ? f1[h + 1] : f1[h], fy[h], inx[q], iny, Y[q], act[q]);
  }
}

template <class S, class C, class SC>
__device__ __forceinline__ void prolong4_body(const ProlongArgs<S, C, SC>& a, const TileCtx& c,
                                              bool) {
  typedef typename Quad<S>::V V4;
  const bool done = a.ctl[S_DONE] != 0.0;
  const LevelView& F = a.F;
  const LevelView& Cl = a.Cl;
  S* __restrict__ x = a.x;
  const SC* __restrict__ e = a.e;
  const int i0 = 4 * (c.tx * MBX + threadIdx.x), j = c.ty * MBY + threadIdx.y;
  if (i0 >= F.g.nx || j >= F.g.ny) return;
  const Geom& cg = Cl.g;
  const bool d3 = cg.dim == 3;
  const int K0 = c.tz * a.T.cz, K1 = min(cg.nz, K0 + a.T.cz);
  const int I0 = i0 >> 1, J = j >> 1;
  const int oy = (j & 1) ? cg.sx : -cg.sx;
  const bool iny = (unsigned)(J + ((j & 1) ? 1 : -1)) < (unsigned)cg.ny;
  bool inx[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    inx[q] = (unsigned)(I0 + (q >> 1) + ((q & 1) ? 1 : -1)) < (unsigned)cg.nx;
  const C w3 = (C)0.75, w1 = (C)0.25;
  int PC = cg.idx(I0, J, K0);
  C ym[4] = {0, 0, 0, 0}, yc[4];
  bool am[4] = {false, false, false, false}, ac[4];
  plane4<C, SC>(Cl, e, PC, oy, true, iny, inx, yc, ac);
  if (d3) plane4<C, SC>(Cl, e, PC - cg.sxy, oy, K0 > 0, iny, inx, ym, am);
  int P = F.g.idx(i0, j, d3 ? 2 * K0 : 0);
  for (int K = K0; K < K1; ++K, PC += cg.sxy) {
    const uchar4 fc0 = *(const uchar4*)(F.cls + P);
    const V4 x0 = *(const V4*)(x + P);
    uchar4 fc1 = fc0;
    V4 x1 = x0;
    C yp[4] = {0, 0, 0, 0}, czl[2] = {0, 0}, czh[2] = {0, 0};
    bool ap[4] = {false, false, false, false};
    if (d3) {
      fc1 = *(const uchar4*)(F.cls + P + F.g.sxy);
      x1 = *(const V4*)(x + P + F.g.sxy);
      plane4<C, SC>(Cl, e, PC + cg.sxy, oy, K + 1 < cg.nz, iny, inx, yp, ap);
      czl[0] = (C)Cl.cf2[PC];
      czl[1] = (C)Cl.cf2[PC + 1];
      czh[0] = (C)Cl.cf2[PC + cg.sxy];
      czh[1] = (C)Cl.cf2[PC + cg.sxy + 1];
    }
    if (done) return;
    const uint8_t f0[4] = {fc0.x, fc0.y, fc0.z, fc0.w}, f1[4] = {fc1.x, fc1.y, fc1.z, fc1.w};
    V4 o0 = x0, o1 = x1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int h = q >> 1;
      if (f0[q] != MG_INACTIVE) {
        C Z = yc[q];
        if (d3) {
          const C zn = K > 0 ? (am[q] ? ym[q] : yc[q]) : ((C)1 - czl[h]) * yc[q];
          Z = w3 * yc[q] + w1 * zn;
        }
        const S xs = x0[q];
        S v;
        St<S, C>::st(&v, St<S, C>::ld(&xs) + Z);
        o0[q] = v;
      }
      if (d3 && f1[q] != MG_INACTIVE) {
        const C zn = K + 1 < cg.nz ? (ap[q] ? yp[q] : yc[q]) : ((C)1 - czh[h]) * yc[q];
        const S xs = x1[q];
        S v;
        St<S, C>::st(&v, St<S, C>::ld(&xs) + (w3 * yc[q] + w1 * zn));
        o1[q] = v;
      }
    }
    *(V4*)(x + P) = o0;
    if (d3) *(V4*)(x + P + F.g.sxy) = o1;
    P += d3 ? 2 * F.g.sxy : 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ym[q] = yc[q];
      am[q] = ac[q];
      yc[q] = yp[q];
      ac[q] = ap[q];
    }
  }
}
NFVM_TILE_KERNELS(k_prolong4, prolong4_body, ProlongArgs, (S, C, SC),
                  (class S, class C, class SC), (S, C, SC), MBS, false)

// Nearest (piecewise-constant) upsampling, the plainest reading of
// Algorithm 1's upsampling: every active fine cell adds its parent's
// correction (the parent of an active cell is active).  One thread per fine
// column walking the coarse planes of its tile, two fine cells per plane in
// 3D; the same tiles as the linear kernel.
template <class S, class C, class SC>
__device__ __forceinline__ void prolong_nearest_body(const ProlongArgs<S, C, SC>& a,
                                                     const TileCtx& c, bool) {
  const bool done = a.ctl[S_DONE] != 0.0;
  const LevelView& F = a.F;
  const Geom& cg = a.Cl.g;
  S* __restrict__ x = a.x;
  const int i = c.tx * MBX + threadIdx.x, j = c.ty * MBY + threadIdx.y;
  if (i >= F.g.nx || j >= F.g.ny) return;
  const bool d3 = cg.dim == 3;
  const int K0 = c.tz * a.T.cz, K1 = min(cg.nz, K0 + a.T.cz);
  int PC = cg.idx(i >> 1, j >> 1, K0);
  int P = F.g.idx(i, j, d3 ? 2 * K0 : 0);
  for (int K = K0; K < K1; ++K, PC += cg.sxy) {
    const C e = St<SC, C>::ld(a.e + PC);
    const uint8_t fc0 = F.cls[P];
    const S x0 = x[P];
    uint8_t fc1 = MG_INACTIVE;
    S x1 = x0;
    if (d3) {
      fc1 = F.cls[P + F.g.sxy];
      x1 = x[P + F.g.sxy];
    }
    if (done) return;
    if (fc0 != MG_INACTIVE) St<S, C>::st(x + P, St<S, C>::ld(&x0) + e);
    if (d3 && fc1 != MG_INACTIVE) St<S, C>::st(x + P + F.g.sxy, St<S, C>::ld(&x1) + e);
    P += d3 ? 2 * F.g.sxy : 0;
  }
}
NFVM_TILE_KERNELS(k_prolong_nearest, prolong_nearest_body, ProlongArgs, (S, C, SC),
                  (class S, class C, class SC), (S, C, SC), MBS, false)

// Whether the prolongation to fine level f takes the four-column kernel.
__host__ inline bool prolong_quad(const Level& f) {
  return f.code && f.g.nx % 4 == 0 && !f.nearest;
}

template <class S, class C, class SC>
ProlongArgs<S, C, SC> prolong_args(const Level& f, const Level& c, const double* ctl) {
  // tiles over fine columns (groups of four with the four-column kernel) and
  // coarse planes
  return ProlongArgs<S, C, SC>{
      view(f),
      make_tiles(prolong_quad(f) ? f.g.nx / 4 : f.g.nx, f.g.ny, c.g.nz, f.tt[TK_PROLONG]),
      (S*)f.x[f.cur], view(c), (const SC*)c.x[c.cur], ctl};
}

template <class S, class C, class SC>
void launch_prolong(const Level& f, const Level& c, const double* ctl, hipStream_t s) {
  const ProlongArgs<S, C, SC> a = prolong_args<S, C, SC>(f, c, ctl);
  if (f.nearest) {
    NFVM_LAUNCH((k_prolong_nearest<S, C, SC>), dim3(a.T.grid), dim3(MBX, MBY), 0, s, a);
  } else if (prolong_quad(f)) {
    if constexpr (has_quad<S>)
      NFVM_LAUNCH((k_prolong4<S, C, SC>), dim3(a.T.grid), dim3(MBX, MBY), 0, s, a);
  } else {
    NFVM_LAUNCH((k_prolong<S, C, SC>), dim3(a.T.grid), dim3(MBX, MBY), 0, s, a);
  }
}

// ---- coarsest level: x = A^-1 b with the dense inverse, one workgroup -------------
template <class SC, class C>
struct CoarseArgs {
  const SC* b;
  SC* x;
  const int* cmap;
  const int* ncount;
  const double* ainv;
  int max_n;
  const double* ctl;
};

template <class SC, class C>
__device__ __forceinline__ void coarse_body(const CoarseArgs<SC, C>& A) {
  if (A.ctl[S_DONE] != 0.0) return;
  __shared__ C bs[512];
  const int n = *A.ncount;
  if (n > A.max_n) return;
  for (int a = threadIdx.x; a < n; a += blockDim.x) bs[a] = St<SC, C>::ld(A.b + A.cmap[a]);
  __syncthreads();
  for (int a = threadIdx.x; a < n; a += blockDim.x) {
    C s = 0;
    const double* row = A.ainv + (size_t)a * n;
    for (int q = 0; q < n; ++q) s += (C)row[q] * bs[q];
    St<SC, C>::st(A.x + A.cmap[a], s);
  }
}
template <class SC, class C>
__global__ __launch_bounds__(256) void k_coarse_solve(CoarseArgs<SC, C> a) {
  coarse_body<SC, C>(a);
}
template <class SC, class C>
__global__ __launch_bounds__(256) void k_coarse_solve_batch(Pack<CoarseArgs<SC, C>> p) {
  coarse_body<SC, C>(p.a[blockIdx.x]);
}

template <class SC, class C>
CoarseArgs<SC, C> coarse_args(const Level& c, const int* cmap, const int* ncount,
                              const double* ainv, int max_n, const double* ctl) {
  return CoarseArgs<SC, C>{(const SC*)c.b, (SC*)c.x[c.cur], cmap, ncount, ainv, max_n, ctl};
}

template <class SC, class C>
void launch_coarse_solve(const Level& c, const int* cmap, const int* ncount, const double* ainv,
                         int max_n, const double* ctl, hipStream_t s) {
  NFVM_LAUNCH((k_coarse_solve<SC, C>), dim3(1), dim3(256), 0, s,
                     coarse_args<SC, C>(c, cmap, ncount, ainv, max_n, ctl));
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
  NFVM_LAUNCH(k_fill_zero<S>, lvl_grid(l.g), dim3(MBX, MBY), 0, s, l.g, (S*)x, ctl);
}

// ---- flexible conjugate gradient on level 0 ---------------------------------------
// Vectors x (phi), r, p (two buffers, alternating by iteration parity), q in
// the outer precision O; z is the V-cycle result in the level-0 storage S; the
// level-0 right-hand side of the next V-cycle is r rounded to S.  Scalars and
// the stopping state live in red.out (ctl).  Every kernel walks column tiles
// and writes one partial per workgroup (tiles outside the grid write zeros).

// r = b - A x0 (x0 = 0 unless given), x = x0 on active cells, 0 elsewhere.
// With z0 set, also the first sweep of the next V-cycle from zero on level 0:
// z0 = wj b0 / D (C: level-0 arithmetic type).
// (level-0 arithmetic is done in the level-0 storage type S)
template <class O, class S>
__device__ __forceinline__ void zero_sweep(const LevelView& L, int P, uint32_t cd, O rP,
                                           S* __restrict__ b0, S* __restrict__ z0, S wj) {
  S bs;
  St<S, O>::st(&bs, rP);
  b0[P] = bs;
  if (z0) z0[P] = wj * bs / diag_code<S>(L.g, cd);
}

template <class O, class S>
__global__ __launch_bounds__(MBS) void k_fcg_start(LevelView L, Tiles T, const O* __restrict__ b,
                                                   const O* __restrict__ x0, O* __restrict__ r,
                                                   O* __restrict__ x, S* __restrict__ b0,
                                                   S* __restrict__ z0, S wj, int have_x0,
                                                   RedBuf red) {
  int tx, ty, tz;
  double bb = 0.0, rr = 0.0;
  if (tile_of(T, tx, ty, tz)) {
    const Geom& g = L.g;
    const int i = tx * MBX + threadIdx.x, j = ty * MBY + threadIdx.y;
    if (i < g.nx && j < g.ny) {
      const int k0 = tz * T.cz, k1 = min(g.nz, k0 + T.cz);
      for (int k = k0; k < k1; ++k) {
        const int P = g.idx(i, j, k);
        const uint32_t cd = L.code[P];
        if (cd == FACE_CODE_INACTIVE) continue;
        const O bP = b[P];
        O rP = bP, xP = 0;
        if (have_x0) {
          xP = x0[P];
          const O xm = g.dim == 3 ? x0[P - g.sxy] : (O)0, xp = g.dim == 3 ? x0[P + g.sxy] : (O)0;
          O Ax, D;
          apply_code<O, O>(g, cd, x0, P, xP, xm, xp, Ax, D);
          rP = bP - Ax;
        }
        r[P] = rP;
        if (x) x[P] = xP;  // null: x is x0 (warm start in place)
        zero_sweep<O, S>(L, P, cd, rP, b0, z0, wj);
        bb += (double)bP * (double)bP;
        rr += (double)rP * (double)rP;
      }
    }
  }
  double vv[2] = {bb, rr};
  block_partial<2, R_SUM, MBS>(vv, red);
}

// Copy slots of red.out to the host-coherent mirror (one thread) and make
// the stores visible to the host before the kernel ends.
__device__ __forceinline__ void publish(const RedBuf& red, int s0, int s1 = -1, int s2 = -1,
                                        int s3 = -1) {
  if (!red.mirror) return;
  red.mirror[s0] = red.out[s0];
  if (s1 >= 0) red.mirror[s1] = red.out[s1];
  if (s2 >= 0) red.mirror[s2] = red.out[s2];
  if (s3 >= 0) red.mirror[s3] = red.out[s3];
  __threadfence_system();
}

// Stopping rule, evaluated by one thread after ||r||^2 is known.
__device__ __forceinline__ void fcg_stop_rule(double* ctl) {
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
    fcg_stop_rule(red.out);
    publish(red, S_BB, S_RR, S_ITER, S_DONE);
  }
}

template <class O, class S>
void launch_fcg_start(const Level& l0, const O* b, const O* x0, O* r, O* x, const RedBuf& red,
                      bool have_x0, double tol, int max_cycles, int forced, hipStream_t s,
                      bool fin, void* z0, double wj) {
  const Tiles T = lvl_tiles(l0, TK_START);
  check_partials(red, T.grid, 2);
  NFVM_LAUNCH((k_fcg_start<O, S>), dim3(T.grid), dim3(MBX, MBY), 0, s, view(l0), T, b, x0,
                     r, (have_x0 && x0 == x) ? nullptr : x, (S*)l0.b, (S*)z0, (S)wj,
                     have_x0 ? 1 : 0, red);
  if (fin)
    NFVM_LAUNCH_FIN(k_fin_start, dim3(1), dim3(FIN), 0, s, red, T.grid, tol * tol,
                       (double)max_cycles, (double)forced);
}

// The search directions live in the level-0 storage type S, in two buffers
// that alternate between iterations: iteration it (the count of finished
// iterations, S_ITER) reads the previous direction from p[it & 1] and writes
// its own to p[(it + 1) & 1], so the update pass can read the previous
// direction at a cell's neighbours while other workgroups write the new one.
// The parity comes from the device-side count, so a captured iteration and a
// batch whose grids are at different iterations need no host bookkeeping.
template <class S>
__device__ __forceinline__ const S* dir_prev(S* const (&p)[2], const double* ctl) {
  return p[(int)ctl[S_ITER] & 1];
}
template <class S>
__device__ __forceinline__ S* dir_next(S* const (&p)[2], const double* ctl) {
  return p[((int)ctl[S_ITER] + 1) & 1];
}

// The new direction at one cell, p = z + beta p_prev rounded to the storage
// type (as one fused multiply-add, so that every thread that forms it, the
// cell's own and its neighbours', gets the same stored value).
template <class O, class S>
__device__ __forceinline__ S dir_at(S z, S pprev, O be) {
  S v;
  St<S, O>::st(&v, fma(be, St<S, O>::ld(&pprev), St<S, O>::ld(&z)));
  return v;
}

// The dot products (z, r), (w, p_prev), (z, w) with w = A z (not stored).
// A is symmetric, so (w, p_prev) = (z, A p_prev) = (z, q_prev) with q_prev
// the previous direction's image, which is therefore not stored either.
// With beta = -(z, q_prev) / (p_prev, q_prev), the new direction
// p = z + beta p_prev has (p, A p) = (z, w) + 2 beta (z, q_prev) +
// beta^2 (p_prev, q_prev): the step length follows without A p.
template <class O, class S>
struct ApplyArgs {
  LevelView L;
  Tiles T;
  const S* z;
  const O* r;
  S* p[2];
  RedBuf red;
};

template <class O, class S>
__device__ __forceinline__ void apply_body(const ApplyArgs<O, S>& a, const TileCtx& c,
                                           bool valid) {
  const RedBuf& red = a.red;
  if (red.out[S_DONE] != 0.0) return;
  const LevelView& L = a.L;
  const S* __restrict__ z = a.z;
  const O* __restrict__ r = a.r;
  const bool first = red.out[S_ITER] == 0.0;
  const S* __restrict__ pp = dir_prev<S>(a.p, red.out);
  double zr = 0.0, zq = 0.0, zw = 0.0;
  if (valid) {
    const Geom& g = L.g;
    const int i = c.tx * MBX + threadIdx.x, j = c.ty * MBY + threadIdx.y;
    if (i < g.nx && j < g.ny) {
      const bool d3 = g.dim == 3;
      const int k0 = c.tz * a.T.cz, k1 = min(g.nz, k0 + a.T.cz);
      int P = g.idx(i, j, k0);
      O zm = d3 ? St<S, O>::ld(z + P - g.sxy) : (O)0, zc = St<S, O>::ld(z + P);
      for (int k = k0; k < k1; ++k, P += g.sxy) {
        const O zp = d3 ? St<S, O>::ld(z + P + g.sxy) : (O)0;
        const uint32_t cd = L.code[P];
        if (cd != FACE_CODE_INACTIVE) {
          O Az, D;
          apply_code<S, O>(g, cd, z, P, zc, zm, zp, Az, D);
          zr += (double)zc * (double)r[P];
          if (!first) zq += (double)Az * (double)St<S, O>::ld(pp + P);
          zw += (double)zc * (double)Az;
        }
        zm = zc;
        zc = zp;
      }
    }
  }
  double vv[3] = {zr, zq, zw};
  block_partial<3, R_SUM, MBS>(vv, red, c.pb);
}
NFVM_TILE_KERNELS(k_fcg_apply, apply_body, ApplyArgs, (O, S), (class O, class S), (O, S), MBS,
                  true)

// The same over four consecutive x cells per thread (nx a multiple of 4),
// with four-wide loads as in k_smooth_code4.
template <class O, class S>
__device__ __forceinline__ void apply4_body(const ApplyArgs<O, S>& a, const TileCtx& c,
                                            bool valid) {
  typedef typename Quad<S>::V S4;
  typedef typename Quad<O>::V O4;
  const RedBuf& red = a.red;
  if (red.out[S_DONE] != 0.0) return;
  const LevelView& L = a.L;
  const S* __restrict__ z = a.z;
  const O* __restrict__ r = a.r;
  const bool first = red.out[S_ITER] == 0.0;
  const S* __restrict__ pp = dir_prev<S>(a.p, red.out);
  double zr = 0.0, zq = 0.0, zw = 0.0;
  if (valid) {
    const Geom& g = L.g;
    const int i0 = 4 * (c.tx * MBX + threadIdx.x), j = c.ty * MBY + threadIdx.y;
    if (i0 < g.nx && j < g.ny) {
      const bool d3 = g.dim == 3;
      const int k0 = c.tz * a.T.cz, k1 = min(g.nz, k0 + a.T.cz);
      int P = g.idx(i0, j, k0);
      S4 zc = *(const S4*)(z + P);
      S4 zm = d3 ? *(const S4*)(z + P - g.sxy) : S4(0);
      for (int k = k0; k < k1; ++k, P += g.sxy) {
        const S4 zp = d3 ? *(const S4*)(z + P + g.sxy) : S4(0);
        const S4 zs = *(const S4*)(z + P - g.sx), zn = *(const S4*)(z + P + g.sx);
        const O zl = St<S, O>::ld(z + P - 1), zh = St<S, O>::ld(z + P + 4);
        const uint2 cw = *(const uint2*)(L.code + P);
        const O4 rv = *(const O4*)(r + P);
        const S4 pv = first ? S4(0) : *(const S4*)(pp + P);
        const uint32_t cd[4] = {cw.x & 0xFFFFu, cw.x >> 16, cw.y & 0xFFFFu, cw.y >> 16};
        const O zv[6] = {zl, (O)zc[0], (O)zc[1], (O)zc[2], (O)zc[3], zh};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (cd[e] != FACE_CODE_INACTIVE) {
            O Az, D;
            apply_code_v<O>(g, cd[e], zv[e + 1], zv[e], zv[e + 2], (O)zs[e], (O)zn[e], (O)zm[e],
                            (O)zp[e], Az, D);
            zr += (double)zv[e + 1] * (double)rv[e];
            zq += (double)Az * (double)(O)pv[e];
            zw += (double)zv[e + 1] * (double)Az;
          }
        }
        zm = zc;
        zc = zp;
      }
    }
  }
  double vv[3] = {zr, zq, zw};
  block_partial<3, R_SUM, MBS>(vv, red, c.pb);
}
NFVM_TILE_KERNELS(k_fcg_apply4, apply4_body, ApplyArgs, (O, S), (class O, class S), (O, S), MBS,
                  true)

// Whether the level-0 CG passes take their four-cells-per-thread kernels.
__host__ inline bool cg_quad(const Level& l0) { return l0.code && l0.g.nx % 4 == 0; }

constexpr int FIN_NV3 = 3;

// Smallest (p, A p) / (z, A z) kept before the CG direction restarts.
constexpr double CG_RESTART = 1e-12;

// Arguments of the one-workgroup finalising kernels (one workgroup per grid
// in a batched launch).
struct FinArgs {
  RedBuf red;
  int nb;
};

// (z, r), (z, q_prev), (z, w); beta, (p, q) and alpha of this iteration.
__device__ __forceinline__ void fin_apply_body(const FinArgs& f) {
  const RedBuf& red = f.red;
  if (red.out[S_DONE] != 0.0) return;
  double acc[FIN_NV3];
  fin_sum<FIN_NV3>(red, f.nb, acc);
  if (threadIdx.x == 0) {
    const double zr = acc[0], zq = acc[1], zw = acc[2];
    const bool first = red.out[S_ITER] == 0.0;
    const double pq_prev = red.out[S_PQ];
    double beta = first ? 0.0 : -zq / pq_prev;
    double pq = first ? zw : zw + 2.0 * beta * zq + beta * beta * pq_prev;
    // (p, A p) = (z, A z) sin^2 of the A-angle between z and p_prev: when the
    // two are (nearly) A-parallel it cancels to rounding noise, so the
    // direction restarts from z (beta = 0); z = 0 takes no step
    if (!first && !(pq > CG_RESTART * zw)) {
      beta = 0.0;
      pq = zw;
    }
    red.out[S_ZR] = zr;
    red.out[S_ZQ] = zq;
    red.out[S_ZW] = zw;
    red.out[S_BETA] = beta;
    red.out[S_PQ] = pq;
    red.out[S_APREV] = first ? 0.0 : red.out[S_ALPHA];
    red.out[S_ALPHA] = pq > 0.0 ? zr / pq : 0.0;
  }
}
__global__ __launch_bounds__(FIN) void k_fin_apply(FinArgs f) { fin_apply_body(f); }
__global__ __launch_bounds__(FIN) void k_fin_apply_batch(Pack<FinArgs> f) {
  fin_apply_body(f.a[blockIdx.x]);
}

template <class O, class S>
ApplyArgs<O, S> apply_args(const Level& l0, const O* r, void* const* dir, const RedBuf& red) {
  const Tiles T = cg_quad(l0) ? make_tiles(l0.g.nx / 4, l0.g.ny, l0.g.nz, l0.tt[TK_APPLY])
                              : lvl_tiles(l0, TK_APPLY);
  return ApplyArgs<O, S>{view(l0), T, (const S*)l0.x[l0.cur], r, {(S*)dir[0], (S*)dir[1]}, red};
}

template <class O, class S>
void launch_fcg_apply(const Level& l0, const O* r, void* const* dir, const RedBuf& red,
                      hipStream_t s, bool fin) {
  const ApplyArgs<O, S> a = apply_args<O, S>(l0, r, dir, red);
  check_partials(red, a.T.grid, 3);
  if (cg_quad(l0))
    NFVM_LAUNCH((k_fcg_apply4<O, S>), dim3(a.T.grid), dim3(MBX, MBY), 0, s, a);
  else
    NFVM_LAUNCH((k_fcg_apply<O, S>), dim3(a.T.grid), dim3(MBX, MBY), 0, s, a);
  if (fin) NFVM_LAUNCH_FIN(k_fin_apply, dim3(1), dim3(FIN), 0, s, FinArgs{red, a.T.grid});
}

// p = z + beta p_prev (stored in S), x += alpha p, r -= alpha A p, ||r||^2,
// the next V-cycle's right-hand side (and first level-0 sweep).  A p is
// formed from the stored p, which every thread forms at a cell's neighbours
// as the cell's own thread does (dir_at), so x and r take the same direction
// and r stays b - A x up to the FP64 rounding of the updates whatever the
// storage type of p.  No image q = A p is stored or read.  Nothing in the
// iteration reads x, so an iteration with an even index leaves its x update
// to the next one, which adds alpha_prev p_prev (the direction it reads
// anyway) and then its own alpha p, the same two updates in the same order:
// x is read and written every other iteration (launch_fcg_flush adds an
// update left pending when the solve stops).
template <class O, class S>
struct UpdateArgs {
  LevelView L;
  Tiles T;
  O* x;
  O* r;
  S* p[2];
  const S* z;
  S* b0;
  S* z0;
  S wj;
  RedBuf red;
};

template <class O, class S>
__device__ __forceinline__ void update_body(const UpdateArgs<O, S>& A, const TileCtx& c,
                                            bool valid) {
  const RedBuf& red = A.red;
  if (red.out[S_DONE] != 0.0) return;
  const LevelView& L = A.L;
  O* __restrict__ x = A.x;
  O* __restrict__ r = A.r;
  const S* __restrict__ pp = dir_prev<S>(A.p, red.out);
  S* __restrict__ pn = dir_next<S>(A.p, red.out);
  const S* __restrict__ z = A.z;
  const bool first = red.out[S_ITER] == 0.0;
  const bool xnow = ((int)red.out[S_ITER] & 1) != 0;  // x updated for this and the previous
  const O a = (O)red.out[S_ALPHA], be = (O)red.out[S_BETA], ap = (O)red.out[S_APREV];
  double rr = 0.0;
  // the new direction at padded index Q
  auto dir = [&](int Q) -> S { return first ? z[Q] : dir_at<O, S>(z[Q], pp[Q], be); };
  if (valid) {
    const Geom& g = L.g;
    const int i = c.tx * MBX + threadIdx.x, j = c.ty * MBY + threadIdx.y;
    if (i < g.nx && j < g.ny) {
      const bool d3 = g.dim == 3;
      const int k0 = c.tz * A.T.cz, k1 = min(g.nz, k0 + A.T.cz);
      int P = g.idx(i, j, k0);
      S qm = d3 ? dir(P - g.sxy) : S(0), qc = dir(P);
      for (int k = k0; k < k1; ++k, P += g.sxy) {
        const S qp = d3 ? dir(P + g.sxy) : S(0);
        const uint32_t cd = L.code[P];
        const S qP = qc, qB = qm;
        qm = qc;
        qc = qp;
        pn[P] = qP;
        if (cd == FACE_CODE_INACTIVE) continue;
        O Ap, D;
        apply_code_v<O>(g, cd, (O)qP, (O)dir(P - 1), (O)dir(P + 1), (O)dir(P - g.sx),
                        (O)dir(P + g.sx), (O)qB, (O)qp, Ap, D);
        if (xnow) {
          O xP = x[P];
          xP += ap * St<S, O>::ld(pp + P);
          xP += a * (O)qP;
          x[P] = xP;
        }
        const O rP = r[P] - a * Ap;
        r[P] = rP;
        zero_sweep<O, S>(L, P, cd, rP, A.b0, A.z0, A.wj);
        rr += (double)rP * (double)rP;
      }
    }
  }
  double vv[1] = {rr};
  block_partial<1, R_SUM, MBS>(vv, red, c.pb);
}
NFVM_TILE_KERNELS(k_fcg_update, update_body, UpdateArgs, (O, S), (class O, class S), (O, S), MBS,
                  true)

// The same over four consecutive x cells per thread (nx a multiple of 4);
// inactive cells keep x and r (written back as read), their direction is
// stored as formed (z and the previous direction are 0 there) and the
// right-hand side and first sweep written as 0, the value they hold.
template <class O, class S>
__device__ __forceinline__ void update4_body(const UpdateArgs<O, S>& A, const TileCtx& c,
                                             bool valid) {
  typedef typename Quad<S>::V S4;
  typedef typename Quad<O>::V O4;
  const RedBuf& red = A.red;
  if (red.out[S_DONE] != 0.0) return;
  const LevelView& L = A.L;
  O* __restrict__ x = A.x;
  O* __restrict__ r = A.r;
  const S* __restrict__ pp = dir_prev<S>(A.p, red.out);
  S* __restrict__ pn = dir_next<S>(A.p, red.out);
  const S* __restrict__ z = A.z;
  const bool first = red.out[S_ITER] == 0.0;
  const bool xnow = ((int)red.out[S_ITER] & 1) != 0;  // x updated for this and the previous
  const O a = (O)red.out[S_ALPHA], be = (O)red.out[S_BETA], ap = (O)red.out[S_APREV];
  double rr = 0.0;
  // the new direction of four cells from index Q, and of one cell
  auto dir4 = [&](int Q) -> S4 {
    const S4 zq = *(const S4*)(z + Q);
    if (first) return zq;
    const S4 pq = *(const S4*)(pp + Q);
    S4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = dir_at<O, S>(zq[e], pq[e], be);
    return v;
  };
  auto dir1 = [&](int Q) -> O {
    return (O)(first ? z[Q] : dir_at<O, S>(z[Q], pp[Q], be));
  };
  if (valid) {
    const Geom& g = L.g;
    const int i0 = 4 * (c.tx * MBX + threadIdx.x), j = c.ty * MBY + threadIdx.y;
    if (i0 < g.nx && j < g.ny) {
      const bool d3 = g.dim == 3;
      const int k0 = c.tz * A.T.cz, k1 = min(g.nz, k0 + A.T.cz);
      int P = g.idx(i0, j, k0);
      S4 qc = dir4(P);
      S4 qm = d3 ? dir4(P - g.sxy) : S4(0);
      for (int k = k0; k < k1; ++k, P += g.sxy) {
        // the operator of apply4_body, on the new direction
        const S4 qp = d3 ? dir4(P + g.sxy) : S4(0);
        const S4 qs = dir4(P - g.sx), qn = dir4(P + g.sx);
        const O ql = dir1(P - 1), qh = dir1(P + 4);
        const uint2 cw = *(const uint2*)(L.code + P);
        O4 xv = xnow ? *(const O4*)(x + P) : O4(0);
        const S4 pv = xnow ? *(const S4*)(pp + P) : S4(0);
        O4 rv = *(const O4*)(r + P);
        const uint32_t cd[4] = {cw.x & 0xFFFFu, cw.x >> 16, cw.y & 0xFFFFu, cw.y >> 16};
        const O qv[6] = {ql, (O)qc[0], (O)qc[1], (O)qc[2], (O)qc[3], qh};
        S4 b0v = S4(0), z0v = S4(0);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (cd[e] == FACE_CODE_INACTIVE) continue;
          O Ap, D;
          apply_code_v<O>(g, cd[e], qv[e + 1], qv[e], qv[e + 2], (O)qs[e], (O)qn[e], (O)qm[e],
                          (O)qp[e], Ap, D);
          xv[e] += ap * (O)pv[e];
          xv[e] += a * qv[e + 1];
          const O rP = rv[e] - a * Ap;
          rv[e] = rP;
          S bs;
          St<S, O>::st(&bs, rP);
          b0v[e] = bs;
          if (A.z0) z0v[e] = A.wj * bs / diag_code<S>(g, cd[e]);
          rr += (double)rP * (double)rP;
        }
        *(S4*)(pn + P) = qc;
        if (xnow) *(O4*)(x + P) = xv;
        *(O4*)(r + P) = rv;
        *(S4*)(A.b0 + P) = b0v;
        if (A.z0) *(S4*)(A.z0 + P) = z0v;
        qm = qc;
        qc = qp;
      }
    }
  }
  double vv[1] = {rr};
  block_partial<1, R_SUM, MBS>(vv, red, c.pb);
}
NFVM_TILE_KERNELS(k_fcg_update4, update4_body, UpdateArgs, (O, S), (class O, class S), (O, S),
                  MBS, true)

// ||r||^2, one more iteration done, stopping rule
__device__ __forceinline__ void fin_update_body(const FinArgs& f) {
  const RedBuf& red = f.red;
  if (red.out[S_DONE] != 0.0) return;
  double acc[1];
  fin_sum<1>(red, f.nb, acc);
  if (threadIdx.x == 0) {
    red.out[S_RR] = acc[0];
    red.out[S_ITER] += 1.0;
    fcg_stop_rule(red.out);
    publish(red, S_RR, S_ITER, S_DONE);
  }
}
__global__ __launch_bounds__(FIN) void k_fin_update(FinArgs f) { fin_update_body(f); }
__global__ __launch_bounds__(FIN) void k_fin_update_batch(Pack<FinArgs> f) {
  fin_update_body(f.a[blockIdx.x]);
}

template <class O, class S>
UpdateArgs<O, S> update_args(const Level& l0, O* x, O* r, void* const* dir, const RedBuf& red,
                             void* z0, double wj) {
  const Tiles T = cg_quad(l0) ? make_tiles(l0.g.nx / 4, l0.g.ny, l0.g.nz, l0.tt[TK_UPDATE])
                              : lvl_tiles(l0, TK_UPDATE);
  return UpdateArgs<O, S>{view(l0), T, x, r, {(S*)dir[0], (S*)dir[1]}, (const S*)l0.x[l0.cur],
                          (S*)l0.b, (S*)z0, (S)wj, red};
}

template <class O, class S>
void launch_fcg_update(const Level& l0, O* x, O* r, void* const* dir, const RedBuf& red,
                       hipStream_t s, bool fin, void* z0, double wj) {
  const UpdateArgs<O, S> a = update_args<O, S>(l0, x, r, dir, red, z0, wj);
  check_partials(red, a.T.grid, 1);
  if (cg_quad(l0))
    NFVM_LAUNCH((k_fcg_update4<O, S>), dim3(a.T.grid), dim3(MBX, MBY), 0, s, a);
  else
    NFVM_LAUNCH((k_fcg_update<O, S>), dim3(a.T.grid), dim3(MBX, MBY), 0, s, a);
  if (fin) NFVM_LAUNCH_FIN(k_fin_update, dim3(1), dim3(FIN), 0, s, FinArgs{red, a.T.grid});
}

// ---- Algorithm 1's plain iteration: x += z, then r = b - A x --------------------
// (the outer loop of the literal mode; the residual is formed again every
// iteration, and its norm goes through the CG update's finaliser, which
// counts the iteration and applies the stopping rule)
template <class O, class S>
__global__ __launch_bounds__(MBS) void k_plain_correct(Geom g, Tiles T, const uint16_t* __restrict__ code,
                                                       O* __restrict__ x, const S* __restrict__ z,
                                                       const double* __restrict__ ctl) {
  if (ctl[S_DONE] != 0.0) return;
  int tx, ty, tz;
  if (!tile_of(T, tx, ty, tz)) return;
  const int i = tx * MBX + threadIdx.x, j = ty * MBY + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const int k0 = tz * T.cz, k1 = min(g.nz, k0 + T.cz);
  for (int k = k0; k < k1; ++k) {
    const int P = g.idx(i, j, k);
    if (code[P] != FACE_CODE_INACTIVE) x[P] += St<S, O>::ld(z + P);
  }
}

template <class O, class S>
__global__ __launch_bounds__(MBS) void k_plain_residual(LevelView L, Tiles T, const O* __restrict__ x,
                                                        const O* __restrict__ b, S* __restrict__ b0,
                                                        RedBuf red) {
  if (red.out[S_DONE] != 0.0) return;  // (uniform: the finaliser returns too)
  int tx, ty, tz;
  double rr = 0.0;
  if (tile_of(T, tx, ty, tz)) {
    const Geom& g = L.g;
    const int i = tx * MBX + threadIdx.x, j = ty * MBY + threadIdx.y;
    if (i < g.nx && j < g.ny) {
      const int k0 = tz * T.cz, k1 = min(g.nz, k0 + T.cz);
      for (int k = k0; k < k1; ++k) {
        const int P = g.idx(i, j, k);
        const uint32_t cd = L.code[P];
        if (cd == FACE_CODE_INACTIVE) continue;
        const O xP = x[P];
        const O xm = g.dim == 3 ? x[P - g.sxy] : (O)0, xp = g.dim == 3 ? x[P + g.sxy] : (O)0;
        O Ax, D;
        apply_code<O, O>(g, cd, x, P, xP, xm, xp, Ax, D);
        const O rP = b[P] - Ax;
        St<S, O>::st(b0 + P, rP);
        rr += (double)rP * (double)rP;
      }
    }
  }
  double vv[1] = {rr};
  block_partial<1, R_SUM, MBS>(vv, red);
}

template <class O, class S>
void launch_plain_update(const Level& l0, O* x, const O* b, const RedBuf& red, hipStream_t s) {
  const Tiles T = lvl_tiles(l0, TK_UPDATE);
  check_partials(red, T.grid, 1);
  NFVM_LAUNCH((k_plain_correct<O, S>), dim3(T.grid), dim3(MBX, MBY), 0, s, l0.g, T, l0.code, x,
              (const S*)l0.x[l0.cur], red.out);
  hipLaunchKernelGGL((k_plain_residual<O, S>), dim3(T.grid), dim3(MBX, MBY), 0, s, view(l0), T, x,
                     b, (S*)l0.b, red);
  NFVM_LAUNCH_FIN(k_fin_update, dim3(1), dim3(FIN), 0, s, FinArgs{red, T.grid});
}
template void launch_plain_update<double, double>(const Level&, double*, const double*,
                                                  const RedBuf&, hipStream_t);
template void launch_plain_update<float, float>(const Level&, float*, const float*, const RedBuf&,
                                                hipStream_t);
template void launch_plain_update<double, float>(const Level&, double*, const double*,
                                                 const RedBuf&, hipStream_t);

// The x update a solve's last iteration left pending.  After an odd count of
// iterations the last one had an even index and deferred x += alpha p; its
// direction sits in p[1] (iteration it writes p[(it + 1) & 1]) and its step
// length in S_ALPHA.  After an even count (zero included) x is complete.
template <class O, class S>
__global__ __launch_bounds__(MBS) void k_fcg_flush(Geom g, Tiles T, const uint16_t* __restrict__ code,
                                                   O* __restrict__ x, const S* __restrict__ p,
                                                   const double* __restrict__ ctl) {
  if (((int)ctl[S_ITER] & 1) == 0) return;
  int tx, ty, tz;
  if (!tile_of(T, tx, ty, tz)) return;
  const int i = tx * MBX + threadIdx.x, j = ty * MBY + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const O a = (O)ctl[S_ALPHA];
  const int k0 = tz * T.cz, k1 = min(g.nz, k0 + T.cz);
  for (int k = k0; k < k1; ++k) {
    const int P = g.idx(i, j, k);
    if (code[P] != FACE_CODE_INACTIVE) x[P] += a * St<S, O>::ld(p + P);
  }
}

template <class O, class S>
void launch_fcg_flush(const Level& l0, O* x, void* const* dir, const double* ctl,
                      hipStream_t s) {
  const Tiles T = lvl_tiles(l0, TK_UPDATE);
  NFVM_LAUNCH((k_fcg_flush<O, S>), dim3(T.grid), dim3(MBX, MBY), 0, s, l0.g, T, l0.code, x,
              (const S*)dir[1], ctl);
}
template void launch_fcg_flush<double, double>(const Level&, double*, void* const*,
                                               const double*, hipStream_t);
template void launch_fcg_flush<float, float>(const Level&, float*, void* const*, const double*,
                                             hipStream_t);
template void launch_fcg_flush<double, float>(const Level&, double*, void* const*,
                                              const double*, hipStream_t);

int fcg_max_blocks(const Level& l0) {
  const Tiles ts = lvl_tiles(l0, TK_START);
  const Tiles ta = cg_quad(l0) ? make_tiles(l0.g.nx / 4, l0.g.ny, l0.g.nz, l0.tt[TK_APPLY])
                               : lvl_tiles(l0, TK_APPLY);
  const Tiles tu = cg_quad(l0) ? make_tiles(l0.g.nx / 4, l0.g.ny, l0.g.nz, l0.tt[TK_UPDATE])
                               : lvl_tiles(l0, TK_UPDATE);
  return std::max(ts.grid, std::max(ta.grid, tu.grid));
}

__global__ void k_fill_f64(double* __restrict__ x, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

void launch_fill_f64(double* x, int n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_f64, dim3((n + 255) / 256), dim3(256), 0, s, x, n, v);
}

// ---- deterministic finalisation of block partials ---------------------------------
template <int NV, int OP>
__global__ __launch_bounds__(256) void k_finalize(RedBuf red, const double* __restrict__ part,
                                                  int nb, int s0, int s1) {
  __shared__ double sh[NV][256];
  double acc[NV];
  for (int q = 0; q < NV; ++q) acc[q] = rid<OP>();
  for (int i = threadIdx.x; i < nb; i += 256)
    for (int q = 0; q < NV; ++q) acc[q] = rop<OP>(acc[q], part[(size_t)i * NV + q]);
  block_tree<NV, OP, 256>(acc, sh);
  if (threadIdx.x == 0) {
    red.out[s0] = acc[0];
    if (NV > 1) red.out[s1] = acc[NV - 1];
    publish(red, s0, NV > 1 ? s1 : -1);
  }
}

// Partials one folding workgroup reduces.  A launch over a large grid leaves
// hundreds of thousands of partials, which one workgroup reads at the rate
// of one compute unit; folding them first in fixed chunks over many
// workgroups keeps the order fixed and the finaliser short.
constexpr int FOLD = 1024;

template <int NV, int OP>
__global__ __launch_bounds__(256) void k_fold(const double* __restrict__ part, int nb,
                                              double* __restrict__ out) {
  __shared__ double sh[NV][256];
  double acc[NV];
  for (int q = 0; q < NV; ++q) acc[q] = rid<OP>();
  const int base = blockIdx.x * FOLD;
  for (int i = threadIdx.x; i < FOLD; i += 256) {
    const int b = base + i;
    if (b < nb)
      for (int q = 0; q < NV; ++q) acc[q] = rop<OP>(acc[q], part[(size_t)b * NV + q]);
  }
  block_tree<NV, OP, 256>(acc, sh);
  if (threadIdx.x == 0)
    for (int q = 0; q < NV; ++q) out[(size_t)blockIdx.x * NV + q] = acc[q];
}

template <int NV, int OP>
void finalize_as(const RedBuf& red, int nb, int slot0, int slot1, hipStream_t s) {
  const int nf = (nb + FOLD - 1) / FOLD;
  // the folded values go after the partials, in the same buffer
  const bool fold = nb > 2 * FOLD && (size_t)(nb + nf) * NV <= (size_t)red.max_blocks * RED_MAX_NV;
  if (!fold) {
    NFVM_LAUNCH_FIN((k_finalize<NV, OP>), dim3(1), dim3(256), 0, s, red, red.partial, nb, slot0,
                    slot1);
    return;
  }
  double* folded = red.partial + (size_t)nb * NV;
  // (timed as one finaliser: both launches between the pair of events; a
  // failed record shows when the profiler reads the pair)
  hipEvent_t e0 = t_launch_ev.fstart, e1 = t_launch_ev.fstop;
  t_launch_ev.fstart = t_launch_ev.fstop = nullptr;
  if (e0) (void)hipEventRecord(e0, s);
  hipLaunchKernelGGL((k_fold<NV, OP>), dim3(nf), dim3(256), 0, s, red.partial, nb, folded);
  hipLaunchKernelGGL((k_finalize<NV, OP>), dim3(1), dim3(256), 0, s, red, folded, nf, slot0,
                     slot1);
  if (e1) (void)hipEventRecord(e1, s);
}

void launch_finalize(int nv, int op, const RedBuf& red, int nblocks, int slot0, int slot1,
                     hipStream_t s) {
  if (nv == 1 && op == R_SUM)
    finalize_as<1, R_SUM>(red, nblocks, slot0, slot1, s);
  else if (nv == 1 && op == R_MAX)
    finalize_as<1, R_MAX>(red, nblocks, slot0, slot1, s);
  else if (nv == 2 && op == R_SUM)
    finalize_as<2, R_SUM>(red, nblocks, slot0, slot1, s);
  else
    finalize_as<2, R_MIN>(red, nblocks, slot0, slot1, s);
}

// ---- LDS bottom solver ----------------------------------------------------------------
// The same operators as the per-level kernels on compact LDS arrays (cell
// index (k ny + j) nx + i).  Everything a phase reads lives in LDS: iterates,
// right-hand side, class bytes and the face coefficients (x faces
// (nx+1) ny nz, y faces nx (ny+1) nz, z faces nx ny (nz+1), low face of cell
// c at its own index, high face one row/plane further).  Neighbours outside
// the box read as 0 and inactive cells hold 0, as in global memory.
// The workgroup's dynamic LDS.  Level arrays are addressed as byte offsets
// from it (pointers kept in memory would lose the LDS address space and
// turn every access into a flat one).
extern __shared__ __align__(16) unsigned char bot_lds[];

template <class C>
struct LdsLevel {
  int n, nx, ny, nz, d3;
  float inx, inxy;
  C ih2x, ih2y, ih2z;
  int ox0, ox1, ob, ofx, ofy, ofz, owd, ocl;  // byte offsets in bot_lds
  __device__ C* x0() const { return (C*)(bot_lds + ox0); }
  __device__ C* x1() const { return (C*)(bot_lds + ox1); }
  __device__ C* b() const { return (C*)(bot_lds + ob); }
  __device__ const float* fx() const { return (const float*)(bot_lds + ofx); }
  __device__ const float* fy() const { return (const float*)(bot_lds + ofy); }
  __device__ const float* fz() const { return (const float*)(bot_lds + ofz); }
  __device__ const C* wd() const { return (const C*)(bot_lds + owd); }
  __device__ const uint8_t* cls() const { return bot_lds + ocl; }
};

template <class C>
__device__ __forceinline__ LdsLevel<C> lds_level(const BottomLevel& L) {
  LdsLevel<C> v;
  v.n = L.n;
  v.nx = L.g.nx;
  v.ny = L.g.ny;
  v.nz = L.g.nz;
  v.d3 = L.g.dim == 3;
  v.ih2x = (C)(1.0 / (L.g.hx * L.g.hx));
  v.ih2y = (C)(1.0 / (L.g.hy * L.g.hy));
  v.ih2z = (C)(1.0 / (L.g.hz * L.g.hz));
  v.ox0 = L.bx0;
  v.ox1 = L.bx1;
  v.ob = L.bb;
  v.ofx = L.bfx;
  v.ofy = L.bfy;
  v.ofz = L.bfz;
  v.owd = L.bwd;
  v.ocl = L.bcl;
  v.inx = L.inx;
  v.inxy = L.inxy;
  return v;
}

// A x at compact cell c = (i, j, k).
template <class C>
__device__ __forceinline__ C lds_apply(const LdsLevel<C>& L, const C* x, int c, int i, int j,
                                       int k, C xP) {
  const int nxy = L.nx * L.ny;
  const int fxl = (k * L.ny + j) * (L.nx + 1) + i;
  const float* fx = L.fx();
  const C cxl = (C)fx[fxl], cxh = (C)fx[fxl + 1];
  const C xw = i > 0 ? x[c - 1] : (C)0, xe = i < L.nx - 1 ? x[c + 1] : (C)0;
  C s = (cxl * (xP - xw) + cxh * (xP - xe)) * L.ih2x;
  const int fyl = (k * (L.ny + 1) + j) * L.nx + i;
  const float* fy = L.fy();
  const C cyl = (C)fy[fyl], cyh = (C)fy[fyl + L.nx];
  const C xs = j > 0 ? x[c - L.nx] : (C)0, xn = j < L.ny - 1 ? x[c + L.nx] : (C)0;
  s += (cyl * (xP - xs) + cyh * (xP - xn)) * L.ih2y;
  if (L.d3) {
    const float* fz = L.fz();
    const C czl = (C)fz[c], czh = (C)fz[c + nxy];
    const C xb = k > 0 ? x[c - nxy] : (C)0, xt = k < L.nz - 1 ? x[c + nxy] : (C)0;
    s += (czl * (xP - xb) + czh * (xP - xt)) * L.ih2z;
  }
  return s;
}

// q = n / d for 0 <= n < 2^22 from a float reciprocal of d, corrected to the
// exact integer quotient.
__device__ __forceinline__ int qdiv(int n, int d, float inv) {
  int q = (int)((float)n * inv);
  const int r = n - q * d;
  q += (r >= d) - (r < 0);
  return q;
}

template <class C>
__device__ __forceinline__ void lds_ijk(const LdsLevel<C>& L, int c, int& i, int& j, int& k) {
  k = qdiv(c, L.nx * L.ny, L.inxy);
  const int r = c - k * L.nx * L.ny;
  j = qdiv(r, L.nx, L.inx);
  i = r - j * L.nx;
}

__device__ __forceinline__ void lds_cell(int nx, int ny, int c, int& i, int& j, int& k) {
  i = c % nx;
  j = (c / nx) % ny;
  k = c / (nx * ny);
}

// Builds the constant part of the bottom solver's LDS image (everything
// from byte zero_bytes on) in global memory, once per grid.
template <class C>
__global__ __launch_bounds__(1024) void k_bottom_image(Bottom B, unsigned char* __restrict__ img) {
  const int t = threadIdx.x, NT = blockDim.x;
  unsigned char* base = img - B.zero_bytes;  // LDS byte offsets index img + (off - zero_bytes)
  const int nl = B.nlev;
  for (int l = 0; l < nl; ++l) {
    const BottomLevel& G = B.lv[l];
    const Geom& g = G.g;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    uint8_t* cls = base + G.bcl;
    float* fx = (float*)(base + G.bfx);
    float* fy = (float*)(base + G.bfy);
    float* fz = (float*)(base + G.bfz);
    C* wd = (C*)(base + G.bwd);
    const double ih2x = 1.0 / (g.hx * g.hx), ih2y = 1.0 / (g.hy * g.hy),
                 ih2z = 1.0 / (g.hz * g.hz);
    for (int c = t; c < G.n; c += NT) {
      int i, j, k;
      lds_cell(nx, ny, c, i, j, k);
      const int P = g.idx(i, j, k);
      cls[c] = G.cls[P];
      // the diagonal in the level's arithmetic type, as the sweep kernels form it
      C d = ((C)G.cf0[P] + (C)G.cf0[P + 1]) * (C)ih2x + ((C)G.cf1[P] + (C)G.cf1[P + g.sx]) * (C)ih2y;
      if (g.dim == 3) d += ((C)G.cf2[P] + (C)G.cf2[P + g.sxy]) * (C)ih2z;
      wd[c] = G.cls[P] == MG_INACTIVE ? (C)0 : (C)B.wj / d;
    }
    const int nfx = (nx + 1) * ny * nz;
    for (int e = t; e < nfx; e += NT) {
      const int i = e % (nx + 1), j = (e / (nx + 1)) % ny, k = e / ((nx + 1) * ny);
      fx[e] = G.cf0[g.idx(i, j, k)];
    }
    const int nfy = nx * (ny + 1) * nz;
    for (int e = t; e < nfy; e += NT) {
      const int i = e % nx, j = (e / nx) % (ny + 1), k = e / (nx * (ny + 1));
      fy[e] = G.cf1[g.idx(i, j, k)];
    }
    if (g.dim == 3) {
      const int nfz = nx * ny * (nz + 1);
      for (int e = t; e < nfz; e += NT) {
        const int i = e % nx, j = (e / nx) % ny, k = e / (nx * ny);
        fz[e] = G.cf2[g.idx(i, j, k)];
      }
    }
  }
  int* cidx = (int*)(base + B.bcidx);
  const int nco = *B.ncount;
  const BottomLevel& G = B.lv[nl - 1];
  if (nco <= B.max_n)
    for (int a = t; a < nco; a += NT) {
      const int P = B.cmap[a] - G.g.off;
      const int kk = P / G.g.sxy, jj = (P % G.g.sxy) / G.g.sx, ii = P % G.g.sx;
      cidx[a] = (kk * G.g.ny + jj) * G.g.nx + ii;
    }
}

template <class C>
void launch_bottom_image(const Bottom& B, void* img, hipStream_t s) {
  hipLaunchKernelGGL(k_bottom_image<C>, dim3(1), dim3(1024), 0, s, B, (unsigned char*)img);
}
template void launch_bottom_image<double>(const Bottom&, void*, hipStream_t);
template void launch_bottom_image<float>(const Bottom&, void*, hipStream_t);

template <class SC, class C>
__device__ __forceinline__ void bottom_body(const Bottom& B, const SC* __restrict__ btop,
                                            SC* __restrict__ xtop,
                                            const double* __restrict__ ctl) {
  // the stopping flag is read with the image and tested after phase 0,
  // which writes only LDS
  const bool done = ctl[S_DONE] != 0.0;
  const int t = threadIdx.x, NT = blockDim.x;
  const int nl = B.nlev;
  const bool pre = B.nu1 > 0;
  // level descriptors, read from LDS by every phase (not from the kernel
  // arguments, whose scalar loads would stall each phase)
  __shared__ LdsLevel<C> lvs[BOTTOM_MAX_LEVELS];
  if (t < nl) lvs[t] = lds_level<C>(B.lv[t]);
  // ---- phase 0: constant image, cleared iterates, the top level's
  // right-hand side and its first sweep from zero (disjoint LDS ranges)
  {
    const uint4* __restrict__ src = (const uint4*)B.img;
    uint4* dst = (uint4*)(bot_lds + B.zero_bytes);
    const int n16 = (int)((B.lds_bytes - (size_t)B.zero_bytes) / 16);
    for (int e0 = t; e0 < n16; e0 += 4 * NT) {
      // indices past the end re-read the last element (kept in registers)
      const uint4 v0 = src[e0], v1 = src[min(e0 + NT, n16 - 1)];
      const uint4 v2 = src[min(e0 + 2 * NT, n16 - 1)], v3 = src[min(e0 + 3 * NT, n16 - 1)];
      dst[e0] = v0;
      if (e0 + NT < n16) dst[e0 + NT] = v1;
      if (e0 + 2 * NT < n16) dst[e0 + 2 * NT] = v2;
      if (e0 + 3 * NT < n16) dst[e0 + 3 * NT] = v3;
    }
    const BottomLevel& G = B.lv[0];
    // top level: x0 [bx0, bx1), x1 [bx1, bb), b [bb, ...): clear x1 and
    // every later level's iterates and right-hand side
    for (int e = G.bx1 / 4 + t; e < G.bb / 4; e += NT) ((float*)bot_lds)[e] = 0.f;
    const int z1 = (int)((G.bb + (size_t)G.n * sizeof(C) + 15) & ~(size_t)15);
    for (int e = z1 / 4 + t; e < B.zero_bytes / 4; e += NT) ((float*)bot_lds)[e] = 0.f;
    // class bytes and wj / D of the top level straight from the image in
    // global memory (the LDS copy is not complete before the barrier)
    const uint8_t* gcl = (const uint8_t*)B.img + (G.bcl - B.zero_bytes);
    const C* gwd = (const C*)((const uint8_t*)B.img + (G.bwd - B.zero_bytes));
    C* x0 = (C*)(bot_lds + G.bx0);
    C* bt = (C*)(bot_lds + G.bb);
    const LdsLevel<C> L = lds_level<C>(G);
    for (int c = t; c < G.n; c += NT) {
      int i, j, k;
      lds_ijk(L, c, i, j, k);
      const C v = St<SC, C>::ld(btop + G.g.idx(i, j, k));
      const bool act = gcl[c] != MG_INACTIVE;
      bt[c] = v;
      x0[c] = (pre && act) ? v * gwd[c] : (C)0;
    }
  }
  int* cidx = (int*)(bot_lds + B.bcidx);
  const int nco = *B.ncount;
  __syncthreads();
  if (done) return;  // uniform over the workgroup
  // current iterate buffer of every level, one bit per level (a bit mask
  // rather than an array keeps it in a register); x0 holds the first sweep
  unsigned curm = 0;
  auto cur_of = [&](int l) -> int { return (int)((curm >> l) & 1u); };
  // one damped-Jacobi sweep on level l (to global memory: the last sweep of
  // the top level)
  auto sweep = [&](int l, bool to_global) {
    const LdsLevel<C> L = lvs[l];
    const C* xin = cur_of(l) ? L.x1() : L.x0();
    C* xout = cur_of(l) ? L.x0() : L.x1();
    const uint8_t* cls = L.cls();
    const C* bb = L.b();
    const C* wd = L.wd();
    for (int c = t; c < L.n; c += NT) {
      if (cls[c] == MG_INACTIVE) continue;
      int i, j, k;
      lds_ijk(L, c, i, j, k);
      const C xP = xin[c];
      const C v = xP + (bb[c] - lds_apply<C>(L, xin, c, i, j, k, xP)) * wd[c];
      if (to_global)
        St<SC, C>::st(xtop + B.lv[0].g.idx(i, j, k), v);
      else
        xout[c] = v;
    }
    curm ^= 1u << l;
    __syncthreads();
  };
  // ---- down the hierarchy
  for (int l = 0; l < nl - 1; ++l) {
    for (int s = 1; s < B.nu1; ++s) sweep(l, false);
    // residual and restriction in one phase: 8 consecutive lanes take the 8
    // children of one coarse cell and sum their residuals by lane exchange;
    // the coarse level's first sweep from zero follows at once
    const LdsLevel<C> F = lvs[l];
    const LdsLevel<C> Cc = lvs[l + 1];
    const C* x = cur_of(l) ? F.x1() : F.x0();
    const uint8_t* fcls = F.cls();
    const uint8_t* ccls = Cc.cls();
    const int kz = Cc.d3 ? 2 : 1;
    const int ncl8 = Cc.n * 8;
    for (int base = 0; base < ncl8; base += NT) {  // uniform trip count
      const int q = base + t;
      const int c = q >> 3, ch = q & 7;
      C r = 0;
      const bool cact = q < ncl8 && ccls[c] != MG_INACTIVE;
      int I = 0, J = 0, K = 0;
      if (cact) lds_ijk(Cc, c, I, J, K);
      const int a = ch & 1, bj = (ch >> 1) & 1, cc = ch >> 2;
      if (cact && cc < kz) {
        const int i = 2 * I + a, j = 2 * J + bj, k = kz * K + cc;
        const int fc = (k * F.ny + j) * F.nx + i;
        if (fcls[fc] != MG_INACTIVE) r = F.b()[fc] - lds_apply<C>(F, x, fc, i, j, k, x[fc]);
      }
      r += __shfl_xor(r, 1);
      r += __shfl_xor(r, 2);
      r += __shfl_xor(r, 4);
      if (cact && ch == 0) {
        const C bc = r * (C)(kz == 2 ? 0.125 : 0.25);
        Cc.b()[c] = bc;
        Cc.x0()[c] = pre ? bc * Cc.wd()[c] : (C)0;
      }
    }
    __syncthreads();
  }
  // ---- coarsest level: dense inverse
  {
    const LdsLevel<C> L = lvs[nl - 1];
    curm &= ~(1u << (nl - 1));
    if (nco <= B.max_n) {
      for (int a = t; a < nco; a += NT) {
        C s = 0;
        const double* row = B.ainv + (size_t)a * nco;
        for (int q = 0; q < nco; ++q) s += (C)row[q] * L.b()[cidx[q]];
        L.x0()[cidx[a]] = s;
      }
    }
    __syncthreads();
  }
  // ---- up the hierarchy: prolongation and post-smoothing
  for (int l = nl - 2; l >= 0; --l) {
    const LdsLevel<C> F = lvs[l];
    const LdsLevel<C> Cc = lvs[l + 1];
    C* x = cur_of(l) ? F.x1() : F.x0();
    const C* e = cur_of(l + 1) ? Cc.x1() : Cc.x0();
    const bool d3 = Cc.d3;
    const int cnx = Cc.nx, cny = Cc.ny, cnz = Cc.nz;
    const uint8_t* ccls = Cc.cls();
    const float* cfxa = Cc.fx();
    const float* cfya = Cc.fy();
    const float* cfza = Cc.fz();
    auto cc_of = [&](int I, int J, int K) { return (K * cny + J) * cnx + I; };
    const int nf = F.n;
    const uint8_t* fcls = F.cls();
    const bool direct = l == 0 && B.nu2 == 0;  // no post-sweep: write out here
    for (int c = t; c < nf; c += NT) {
      if (fcls[c] == MG_INACTIVE) continue;
      int i, j, k;
      lds_ijk(F, c, i, j, k);
      // the prolongation rules (plane_rules, then the z step) on the compact
      // arrays: indices outside the box are clamped to the cell itself and
      // their values masked
      const int I = i >> 1, J = j >> 1, K = d3 ? (k >> 1) : 0;
      const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
      const C w3 = (C)0.75, w1 = (C)0.25;
      const bool inx = (unsigned)(I + sx) < (unsigned)cnx;
      const bool iny = (unsigned)(J + sy) < (unsigned)cny;
      const bool inz = d3 && (unsigned)(K + sz) < (unsigned)cnz;
      const int In = inx ? I + sx : I, Jn = iny ? J + sy : J, Kn = inz ? K + sz : K;
      const int Jq[4] = {J, Jn, J, Jn}, Kq[4] = {K, K, Kn, Kn};
      C ev[4], en[4], cfx[4];
      bool ac[4], an[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int Q = cc_of(I, Jq[q], Kq[q]), Qn = cc_of(In, Jq[q], Kq[q]);
        ev[q] = e[Q];
        en[q] = e[Qn];
        ac[q] = ccls[Q] != MG_INACTIVE;
        an[q] = ccls[Qn] != MG_INACTIVE;
        cfx[q] = (C)cfxa[(Kq[q] * cny + Jq[q]) * (cnx + 1) + I + (sx > 0 ? 1 : 0)];
      }
      const C cfy0 = (C)cfya[(K * (cny + 1) + J + (sy > 0 ? 1 : 0)) * cnx + I];
      const C cfy1 = (C)cfya[(Kn * (cny + 1) + J + (sy > 0 ? 1 : 0)) * cnx + I];
      const C cfz = d3 ? (C)cfza[((K + (sz > 0 ? 1 : 0)) * cny + J) * cnx + I] : (C)0;
      const bool act[4] = {ac[0], iny && ac[1], inz && ac[2], iny && inz && ac[3]};
      C X[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const C nb = inx ? (an[q] ? en[q] : ev[q]) : ((C)1 - cfx[q]) * ev[q];
        X[q] = act[q] ? w3 * ev[q] + w1 * nb : (C)0;
      }
      const C yn0 = iny ? (act[1] ? X[1] : X[0]) : ((C)1 - cfy0) * X[0];
      const C Y0 = act[0] ? w3 * X[0] + w1 * yn0 : (C)0;
      C Z = Y0;
      if (d3) {
        const C yn1 = iny ? (act[3] ? X[3] : X[2]) : ((C)1 - cfy1) * X[2];
        const C Y1 = act[2] ? w3 * X[2] + w1 * yn1 : (C)0;
        const C zn = inz ? (act[2] ? Y1 : Y0) : ((C)1 - cfz) * Y0;
        Z = w3 * Y0 + w1 * zn;
      }
      const C v = x[c] + Z;
      if (direct)
        St<SC, C>::st(xtop + B.lv[0].g.idx(i, j, k), v);
      else
        x[c] = v;
    }
    __syncthreads();
    for (int s = 0; s < B.nu2; ++s) sweep(l, l == 0 && s == B.nu2 - 1);
  }
}

// One bottom solve per workgroup: the single launch takes the descriptor as a
// kernel argument, the batched launch one descriptor per workgroup.
struct BottomArgsBase {
  Bottom B;
  const void* btop;
  void* xtop;
  const double* ctl;
};

template <class SC, class C>
__global__ __launch_bounds__(1024) void k_bottom(Bottom B, const SC* __restrict__ btop,
                                                 SC* __restrict__ xtop,
                                                 const double* __restrict__ ctl) {
  bottom_body<SC, C>(B, btop, xtop, ctl);
}

template <class SC, class C>
__global__ __launch_bounds__(1024) void k_bottom_batch(const BottomArgsBase* __restrict__ a) {
  const BottomArgsBase& e = a[blockIdx.x];
  bottom_body<SC, C>(e.B, (const SC*)e.btop, (SC*)e.xtop, e.ctl);
}

// Dynamic LDS bytes one bottom workgroup may use on the current device: the
// device's LDS per workgroup less the kernel's static LDS (its level table);
// dynamic LDS above 64 KiB is enabled per kernel where the device has it.
template <class SC, class C>
size_t bottom_lds_limit() {
  int dev = 0, lim = 0;
  hipFuncAttributes fa;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
      hipFuncGetAttributes(&fa, (const void*)k_bottom<SC, C>) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  const int stat = (int)fa.sharedSizeBytes;
  const int dyn = lim - stat;
  if (dyn <= 0) return 0;
  if (lim > 64 * 1024 &&
      (hipFuncSetAttribute((const void*)k_bottom<SC, C>,
                           hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess ||
       hipFuncSetAttribute((const void*)k_bottom_batch<SC, C>,
                           hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess)) {
    (void)hipGetLastError();
    return (size_t)(64 * 1024 - stat);
  }
  return (size_t)dyn;
}
template size_t bottom_lds_limit<double, double>();
template size_t bottom_lds_limit<float, float>();
template size_t bottom_lds_limit<bf16, float>();

template <class SC, class C>
void launch_bottom(const Bottom& B, const void* btop, void* xtop, const double* ctl,
                   hipStream_t s) {
  NFVM_LAUNCH((k_bottom<SC, C>), dim3(1), dim3(1024), B.lds_bytes, s, B, (const SC*)btop,
                     (SC*)xtop, ctl);
}
template void launch_bottom<double, double>(const Bottom&, const void*, void*, const double*,
                                            hipStream_t);
template void launch_bottom<float, float>(const Bottom&, const void*, void*, const double*,
                                          hipStream_t);
template void launch_bottom<bf16, float>(const Bottom&, const void*, void*, const double*,
                                         hipStream_t);

// ---- batched iteration plan ---------------------------------------------------------
namespace {

size_t al16(size_t v) { return (v + 15) & ~(size_t)15; }

// Argument structs of one kernel for the grids of one batched launch.
template <class A>
using Group = std::vector<A>;

template <class V>
size_t put(BatchOps& o, const std::vector<V>& v) {
  const size_t off = al16(o.blob.size());
  o.blob.resize(off + v.size() * sizeof(V));
  if (!v.empty()) memcpy(o.blob.data() + off, v.data(), v.size() * sizeof(V));
  return off;
}

// Tile kernels: one grid takes the single kernel (T.grid blocks); more grids
// take the batched kernel, MAXB grids per launch, ceil(blocks / 8) * 8
// workgroups.  With pad, a grid's padding tiles are part of its range (its
// reduction partials are all written).
template <class A, class K1, class KB>
void emit_tiles(BatchOps& o, const Group<A>& g, K1 single, KB batched, bool pad) {
  if (g.size() == 1) {
    const A a = g[0];
    o.ops.push_back([=](const unsigned char*, hipStream_t s) {
      hipLaunchKernelGGL(single, dim3(a.T.grid), dim3(MBX, MBY), 0, s, a);
    });
    return;
  }
  for (size_t i0 = 0; i0 < g.size(); i0 += MAXB) {
    Pack<A> p;
    memset(&p, 0, sizeof p);
    p.n = (int)std::min(g.size() - i0, (size_t)MAXB);
    p.start[0] = 0;
    for (int i = 0; i < p.n; ++i) {
      p.a[i] = g[i0 + i];
      p.start[i + 1] = p.start[i] + (pad ? p.a[i].T.grid : p.a[i].T.total);
    }
    const int blocks = (p.start[p.n] + 7) / 8 * 8;
    o.ops.push_back([=](const unsigned char*, hipStream_t s) {
      hipLaunchKernelGGL(batched, dim3(blocks), dim3(MBX, MBY), 0, s, p);
    });
  }
}

// One workgroup per grid, arguments by value (MAXB grids per launch).
template <class A, class KB>
void emit_packed_blocks(BatchOps& o, const Group<A>& g, KB kern, int threads) {
  for (size_t i0 = 0; i0 < g.size(); i0 += MAXB) {
    Pack<A> p;
    memset(&p, 0, sizeof p);
    p.n = (int)std::min(g.size() - i0, (size_t)MAXB);
    for (int i = 0; i < p.n; ++i) p.a[i] = g[i0 + i];
    const int n = p.n;
    o.ops.push_back([=](const unsigned char*, hipStream_t s) {
      hipLaunchKernelGGL(kern, dim3(n), dim3(threads), 0, s, p);
    });
  }
}

// One workgroup per grid, arguments in the plan's device memory (the bottom
// solver's descriptors are too large for the kernel-argument segment).
template <class A, class K>
void emit_blocks(BatchOps& o, const std::vector<A>& args, K kern, int threads, size_t lds) {
  if (args.empty()) return;
  const size_t ao = put(o, args);
  const int n = (int)args.size();
  o.ops.push_back([=](const unsigned char* base, hipStream_t s) {
    hipLaunchKernelGGL(kern, dim3(n), dim3(threads), lds, s, (const A*)(base + ao));
  });
}

// Sweep groups of one level, by kernel: face-code or class-byte sweep, from
// zero or not.
template <class S, class C>
struct SweepGroups {
  // [class bytes, face codes, face codes four cells per thread, class bytes
  // four cells per thread][from zero]
  Group<SmoothArgs<S, C>> g[4][2];
  void add(const Level& l, double wj, bool zero, const double* ctl) {
    const void* xin = zero ? nullptr : l.x[l.cur];
    void* xout = zero ? l.x[0] : l.x[l.cur ^ 1];
    const int kind = sweep_quad(l, zero)         ? 2
                     : coarse_quad<S>(l, zero) ? 3
                     : l.code != nullptr       ? 1
                                               : 0;
    g[kind][zero].push_back(smooth_args<S, C>(l, xin, xout, wj, zero, ctl));
  }
  void emit(BatchOps& o) const {
    emit_tiles(o, g[0][0], k_smooth<S, C, false>, k_smooth_batch<S, C, false>, false);
    emit_tiles(o, g[0][1], k_smooth<S, C, true>, k_smooth_batch<S, C, true>, false);
    emit_tiles(o, g[1][0], k_smooth_code<S, C, false>, k_smooth_code_batch<S, C, false>, false);
    emit_tiles(o, g[1][1], k_smooth_code<S, C, true>, k_smooth_code_batch<S, C, true>, false);
    if constexpr (has_quad<S>) {
      emit_tiles(o, g[2][0], k_smooth_code4<S, C>, k_smooth_code4_batch<S, C>, false);
      emit_tiles(o, g[3][0], k_smooth4<S, C>, k_smooth4_batch<S, C>, false);
    }
  }
};

// Levels below the top whose V-cycle step is a regular one (not the
// bottom solver's or the coarsest solve's).
int stop_level(const MgGridDesc& d) { return d.bottom_top >= 0 ? d.bottom_top : d.L - 1; }

// Pre- and post-smoothing sweeps of grid d on level l.
int pre_of(const MgGridDesc& d, int l) { return l > 0 ? d.nu1c : d.nu1; }
int post_of(const MgGridDesc& d, int l) { return l > 0 ? d.nu2c : d.nu2; }

// Sweep number s on level l of grid d (the same order as one grid's
// recursive V-cycle): pre-smoothing when `pre`.
template <class S, class C>
void add_sweep(SweepGroups<S, C>& sg, MgGridDesc& d, int l, int s, bool pre) {
  Level& v = d.lv[l];
  const double* ctl = d.red.out;
  if (pre) {
    if (pre_of(d, l) == 0) return;
    if (s == 0) {
      if (d.zero[l]) {
        v.cur = 0;  // written by the kernel that formed this level's right-hand side
      } else {
        sg.add(v, d.wj, true, ctl);
        v.cur = 0;
      }
      return;
    }
    if (s >= pre_of(d, l)) return;
  } else if (s >= post_of(d, l)) {
    return;
  }
  sg.add(v, d.wj, false, ctl);
  v.cur ^= 1;
}

// Whether level l of grid d is held in the level-0 storage type.
bool wide_of(const MgGridDesc& d, int l) { return l == 0 || d.lv[l].wide; }

// The bottom solves of grids whose bottom solver's top level is held in type
// T: the single kernel for one grid, else one workgroup per grid.
template <class T, class C>
void emit_bottoms(BatchOps& o, const std::vector<BottomArgsBase>& bo, size_t lds) {
  if (bo.size() == 1) {
    const BottomArgsBase e = bo[0];
    o.ops.push_back([=](const unsigned char*, hipStream_t s) {
      hipLaunchKernelGGL((k_bottom<T, C>), dim3(1), dim3(1024), e.B.lds_bytes, s, e.B,
                         (const T*)e.btop, (T*)e.xtop, e.ctl);
    });
  } else {
    emit_blocks(o, bo, k_bottom_batch<T, C>, 1024, lds);
  }
}

// Restrictions from a level of type A to one of type B, by kernel.
template <class A, class B, class C>
struct RestrictSet {
  Group<RestrictArgs<A, C, B>> plain, quad;
  void add(const MgGridDesc& d, int l) {
    (restrict_quad(d.lv[l]) ? quad : plain)
        .push_back(restrict_args<A, C, B>(d.lv[l], d.lv[l + 1], d.red.out, d.zero[l + 1], d.wj));
  }
  void emit(BatchOps& o) const {
    emit_tiles(o, plain, k_resid_restrict<A, C, B>, k_resid_restrict_batch<A, C, B>, false);
    if constexpr (has_quad<A>)
      emit_tiles(o, quad, k_resid_restrict4<A, C, B>, k_resid_restrict4_batch<A, C, B>, false);
  }
};

// Prolongations to a level of type A from one of type B, by kernel.
template <class A, class B, class C>
struct ProlongSet {
  Group<ProlongArgs<A, C, B>> plain, quad, nearest;
  void add(const MgGridDesc& d, int l) {
    (d.lv[l].nearest ? nearest : prolong_quad(d.lv[l]) ? quad : plain)
        .push_back(prolong_args<A, C, B>(d.lv[l], d.lv[l + 1], d.red.out));
  }
  void emit(BatchOps& o) const {
    emit_tiles(o, plain, k_prolong<A, C, B>, k_prolong_batch<A, C, B>, false);
    if constexpr (has_quad<A>)
      emit_tiles(o, quad, k_prolong4<A, C, B>, k_prolong4_batch<A, C, B>, false);
    emit_tiles(o, nearest, k_prolong_nearest<A, C, B>, k_prolong_nearest_batch<A, C, B>, false);
  }
};

// The four pairings of the two storage types (wide = the level-0 type W,
// narrow = the coarse type N) between a level and the next coarser one.
template <template <class, class, class> class Set, class W, class N, class C>
struct TypePairs {
  Set<W, W, C> ww;
  Set<W, N, C> wn;
  Set<N, N, C> nn;
  Set<N, W, C> nw;
  void add(const MgGridDesc& d, int l) {
    const bool a = wide_of(d, l), b = wide_of(d, l + 1);
    if (a && b)
      ww.add(d, l);
    else if (a)
      wn.add(d, l);
    else if (b)
      nw.add(d, l);
    else
      nn.add(d, l);
  }
  void emit(BatchOps& o) const {
    ww.emit(o);
    wn.emit(o);
    nn.emit(o);
    nw.emit(o);
  }
};

}  // namespace

template <class O, class S0, class SC, class C>
void plan_fcg_iteration(MgGridDesc* G, int n, BatchOps& o) {
  int top = 0;
  for (int i = 0; i < n; ++i) top = std::max(top, stop_level(G[i]));
  // the most sweeps any grid takes on level l
  auto max_pre = [&](int l) {
    int m = 0;
    for (int i = 0; i < n; ++i) m = std::max(m, pre_of(G[i], l));
    return m;
  };
  auto max_post = [&](int l) {
    int m = 0;
    for (int i = 0; i < n; ++i) m = std::max(m, post_of(G[i], l));
    return m;
  };
  // zero-filled levels (no pre-smoothing): one launch per grid, not batched
  auto fill = [&](MgGridDesc& d, int l) {
    Level& v = d.lv[l];
    v.cur = 0;
    const Level lv = v;
    const double* ctl = d.red.out;
    o.ops.push_back([=](const unsigned char*, hipStream_t s) {
      if (l == 0 || lv.wide)
        launch_fill_zero<S0>(lv, lv.x[0], ctl, s);
      else
        launch_fill_zero<SC>(lv, lv.x[0], ctl, s);
    });
  };
  // down: pre-smoothing and restriction, level by level
  for (int l = 0; l < top; ++l) {
    for (int s = 0; s < std::max(max_pre(l), 1); ++s) {
      SweepGroups<S0, C> g0;
      SweepGroups<SC, C> gc;
      for (int i = 0; i < n; ++i) {
        if (l >= stop_level(G[i])) continue;
        if (pre_of(G[i], l) == 0) {
          if (s == 0) fill(G[i], l);
          continue;
        }
        if (wide_of(G[i], l))
          add_sweep(g0, G[i], l, s, true);
        else
          add_sweep(gc, G[i], l, s, true);
      }
      g0.emit(o);
      gc.emit(o);
    }
    TypePairs<RestrictSet, S0, SC, C> rs;
    for (int i = 0; i < n; ++i)
      if (l < stop_level(G[i])) rs.add(G[i], l);
    rs.emit(o);
  }
  // bottom solver or coarsest solve of every grid
  {
    // [bottom top level held in the coarse type, in the level-0 type]
    std::vector<BottomArgsBase> bo[2];
    size_t lds[2] = {0, 0};
    Group<CoarseArgs<S0, C>> c0;
    Group<CoarseArgs<SC, C>> cc;
    for (int i = 0; i < n; ++i) {
      MgGridDesc& d = G[i];
      if (d.bottom_top >= 0) {
        Level& v = d.lv[d.bottom_top];
        v.cur = 0;
        const int w = wide_of(d, d.bottom_top) ? 1 : 0;
        bo[w].push_back(BottomArgsBase{*d.bot, v.b, v.x[0], d.red.out});
        lds[w] = std::max(lds[w], d.bot->lds_bytes);
      } else {
        Level& v = d.lv[d.L - 1];
        v.cur = 0;
        if (wide_of(d, d.L - 1))
          c0.push_back(coarse_args<S0, C>(v, d.cmap, d.ncount, d.ainv, d.coarse_max, d.red.out));
        else
          cc.push_back(coarse_args<SC, C>(v, d.cmap, d.ncount, d.ainv, d.coarse_max, d.red.out));
      }
    }
    emit_bottoms<SC, C>(o, bo[0], lds[0]);
    emit_bottoms<S0, C>(o, bo[1], lds[1]);
    emit_packed_blocks(o, c0, k_coarse_solve_batch<S0, C>, 256);
    emit_packed_blocks(o, cc, k_coarse_solve_batch<SC, C>, 256);
  }
  // up: prolongation and post-smoothing
  for (int l = top - 1; l >= 0; --l) {
    TypePairs<ProlongSet, S0, SC, C> ps;
    for (int i = 0; i < n; ++i)
      if (l < stop_level(G[i])) ps.add(G[i], l);
    ps.emit(o);
    for (int s = 0; s < max_post(l); ++s) {
      SweepGroups<S0, C> g0;
      SweepGroups<SC, C> gc;
      for (int i = 0; i < n; ++i) {
        if (l >= stop_level(G[i])) continue;
        if (wide_of(G[i], l))
          add_sweep(g0, G[i], l, s, false);
        else
          add_sweep(gc, G[i], l, s, false);
      }
      g0.emit(o);
      gc.emit(o);
    }
  }
  // CG: the dot products with w = A z, then the vector update
  Group<ApplyArgs<O, S0>> ap[2];  // [one cell, four cells per thread]
  Group<UpdateArgs<O, S0>> up[2];
  Group<FinArgs> fa, fu;
  for (int i = 0; i < n; ++i) {
    MgGridDesc& d = G[i];
    const auto a = apply_args<O, S0>(d.lv[0], (const O*)d.r, d.dir, d.red);
    check_partials(d.red, a.T.grid, 3);
    ap[cg_quad(d.lv[0])].push_back(a);
    fa.push_back(FinArgs{d.red, a.T.grid});
  }
  for (int i = 0; i < n; ++i) {
    MgGridDesc& d = G[i];
    const auto a = update_args<O, S0>(d.lv[0], (O*)d.x, (O*)d.r, d.dir, d.red,
                                      d.zero[0], d.wj);
    check_partials(d.red, a.T.grid, 1);
    up[cg_quad(d.lv[0])].push_back(a);
    fu.push_back(FinArgs{d.red, a.T.grid});
  }
  emit_tiles(o, ap[0], k_fcg_apply<O, S0>, k_fcg_apply_batch<O, S0>, true);
  emit_tiles(o, ap[1], k_fcg_apply4<O, S0>, k_fcg_apply4_batch<O, S0>, true);
  if (n == 1)
    o.ops.push_back([f = fa[0]](const unsigned char*, hipStream_t s) {
      hipLaunchKernelGGL(k_fin_apply, dim3(1), dim3(FIN), 0, s, f);
    });
  else
    emit_packed_blocks(o, fa, k_fin_apply_batch, FIN);
  emit_tiles(o, up[0], k_fcg_update<O, S0>, k_fcg_update_batch<O, S0>, true);
  emit_tiles(o, up[1], k_fcg_update4<O, S0>, k_fcg_update4_batch<O, S0>, true);
  if (n == 1)
    o.ops.push_back([f = fu[0]](const unsigned char*, hipStream_t s) {
      hipLaunchKernelGGL(k_fin_update, dim3(1), dim3(FIN), 0, s, f);
    });
  else
    emit_packed_blocks(o, fu, k_fin_update_batch, FIN);
}
template void plan_fcg_iteration<double, double, double, double>(MgGridDesc*, int, BatchOps&);
template void plan_fcg_iteration<float, float, float, float>(MgGridDesc*, int, BatchOps&);
template void plan_fcg_iteration<double, float, bf16, float>(MgGridDesc*, int, BatchOps&);

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
template void launch_smooth2<double, double>(const Level&, const void*, void*, double,
                                             const double*, hipStream_t);
template void launch_smooth2<float, float>(const Level&, const void*, void*, double,
                                           const double*, hipStream_t);

#define INST_PAIR(S, C, SC)                                                                 \
  template void launch_resid_restrict<S, C, SC>(const Level&, const Level&, const double*,   \
                                                hipStream_t, void*, double);                  \
  template void launch_prolong<S, C, SC>(const Level&, const Level&, const double*,          \
                                         hipStream_t);
INST_PAIR(double, double, double)
INST_PAIR(float, float, float)
INST_PAIR(float, float, bf16)
INST_PAIR(bf16, float, bf16)
INST_PAIR(bf16, float, float)

template void launch_coarse_solve<double, double>(const Level&, const int*, const int*,
                                                  const double*, int, const double*, hipStream_t);
template void launch_coarse_solve<float, float>(const Level&, const int*, const int*,
                                                const double*, int, const double*, hipStream_t);
template void launch_coarse_solve<bf16, float>(const Level&, const int*, const int*,
                                               const double*, int, const double*, hipStream_t);

#define INST_FCG(O, S)                                                                          \
  template void launch_fcg_start<O, S>(const Level&, const O*, const O*, O*, O*, const RedBuf&, \
                                       bool, double, int, int, hipStream_t, bool, void*, double); \
  template void launch_fcg_apply<O, S>(const Level&, const O*, void* const*, const RedBuf&,     \
                                       hipStream_t, bool);                                      \
  template void launch_fcg_update<O, S>(const Level&, O*, O*, void* const*, const RedBuf&,      \
                                        hipStream_t, bool, void*, double);
INST_FCG(double, double)
INST_FCG(float, float)
INST_FCG(double, float)

}  // namespace nfvm
