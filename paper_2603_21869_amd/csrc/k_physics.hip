// Physics kernels of one time step: semi-implicit k-omega destruction
// (Sec. 2.5, Algorithm 3), the explicit finite-volume update of the rest terms
// (Sec. 2.3, Algorithms 2 and 4, eqs. ko_mom to ko_temp), the Poisson
// right-hand side (eq. pc_residual) and the projection (Sec. 2.4).
//
// Layout: one thread per cell, 64 x 4 cells per workgroup (x fastest, so a
// wavefront reads 64 consecutive values of a row), one z plane per grid
// slice.  Face neighbours come from the padded arrays; a non-fluid neighbour
// is replaced by the ghost value of its boundary patch.
#include <hip/hip_runtime.h>

#include "nfvm_device.hpp"

namespace nfvm {

constexpr int BX = 64, BY = 4, BS = BX * BY;

__host__ inline dim3 cell_grid(const Geom& g) {
  return dim3((g.nx + BX - 1) / BX, (g.ny + BY - 1) / BY, g.nz);
}

// column tiles (see Tiles): a few workgroups per compute unit, each thread
// walking a chunk of planes
__host__ inline Tiles cell_tiles(const Geom& g, int tt) { return make_tiles(g.nx, g.ny, g.nz, tt); }

// LDS planes of the stencil kernels that stage a tile: the 64 x 4 cells and
// their one-cell rim on the four sides (corners unused).  The rim is loaded
// by the threads of the first and last rows (the rows outside) and by 2 x 4
// threads of the second row (the columns outside).
constexpr int PL_W = BX + 2, PL_N = PL_W * (BY + 2);

// slot of tile cell (a, b), a in [-1, BX], b in [-1, BY]
__device__ __forceinline__ int pl_slot(int a, int b) { return (b + 1) * PL_W + a + 1; }

// The rim cell (a, b) relative to the tile that thread (x, y) stages, if any.
__device__ __forceinline__ bool pl_rim(int x, int y, int& a, int& b) {
  if (y == 0) {
    a = x, b = -1;
  } else if (y == BY - 1) {
    a = x, b = BY;
  } else if (y == 1 && x < 2 * BY) {
    a = x < BY ? -1 : BX;
    b = x < BY ? x : x - BY;
  } else {
    a = b = 0;
    return false;
  }
  return true;
}

// ---- dense <-> padded copies ------------------------------------------------
// padded = dense - offset (rounded to F) and back
template <class F>
__global__ void k_pack(Geom g, const double* __restrict__ d, F* __restrict__ p, double off) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  p[g.idx(i, j, k)] = (F)(d[((size_t)k * g.ny + j) * g.nx + i] - off);
}
template <class F>
__global__ void k_unpack(Geom g, const F* __restrict__ p, double* __restrict__ d, double off) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  d[((size_t)k * g.ny + j) * g.nx + i] = (double)p[g.idx(i, j, k)] + off;
}
template <class F>
void launch_pack(const Geom& g, const double* dense, F* padded, double off, hipStream_t s) {
  hipLaunchKernelGGL(k_pack<F>, cell_grid(g), dim3(BX, BY), 0, s, g, dense, padded, off);
}
template <class F>
void launch_unpack(const Geom& g, const F* padded, double* dense, double off, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack<F>, cell_grid(g), dim3(BX, BY), 0, s, g, padded, dense, off);
}
template void launch_pack<double>(const Geom&, const double*, double*, double, hipStream_t);
template void launch_pack<float>(const Geom&, const double*, float*, double, hipStream_t);
template void launch_unpack<double>(const Geom&, const double*, double*, double, hipStream_t);
template void launch_unpack<float>(const Geom&, const float*, double*, double, hipStream_t);

// ---- semi-implicit destruction ---------------------------------------------
// k_new = k / (1 + tau beta* f_beta* omega), omega_new = omega / (1 + tau beta
// f_beta omega) with cell-centred central gradients (face derivative D, then
// average L) feeding chi_k and chi_omega; every right-hand side uses the
// input k and omega.  Fixed wall cells keep omega.
// The values a cell's gradients read from one neighbour (loaded whatever the
// neighbour's kind; every index lies in the padded arrays).
template <class R>
struct DestroyNb {
  uint8_t t;
  R u[3], k, w;
};

// Each workgroup walks the planes of a 64 x 4 column tile, one cell per
// thread.  A plane's values (u, v, w, k, omega at the arithmetic type) and
// kind bytes go to LDS for the tile and its rim, so a cell takes its four
// in-plane neighbours from there; the cells below and above stay in the
// thread's registers (the cell above, loaded with the next plane's rim while
// the plane is computed, becomes the next centre).  Two LDS planes
// alternate, so one barrier per plane suffices.  The vortex stretching
// Omega_ij Omega_jk S_ki is tr(W W S) with W the antisymmetric part of the
// gradient; for W = [a]x (the cross-product matrix of a), W W = a a^T -
// |a|^2 I, so it is a^T S a - |a|^2 tr S.
template <class V, class F, bool RED>
__global__ __launch_bounds__(BS) void k_destroy(Geom g, Phys ph, const uint8_t* __restrict__ type,
                                                const DevPatch* __restrict__ pt,
                                                const V* __restrict__ u, const V* __restrict__ v,
                                                const V* __restrict__ w, const F* __restrict__ kk,
                                                const F* __restrict__ om, V tau,
                                                F* __restrict__ k_out, F* __restrict__ om_out,
                                                F* __restrict__ nut_out, RedBuf red, Tiles T) {
  typedef V R;
  __shared__ R lv[2][5][PL_N];
  __shared__ uint8_t lt[2][PL_N];
  int tx = 0, ty = 0, tz = 0;
  const bool tile = tile_of(T, tx, ty, tz);  // (whole workgroup)
  const int a = threadIdx.x, b = threadIdx.y;
  const int i0 = tx * BX, j0 = ty * BY;
  const int i = i0 + a, j = j0 + b;
  const int kb = tz * T.cz, ke = tile ? min(g.nz, kb + T.cz) : kb;
  const bool d3 = g.dim == 3;
  const bool valid = i < g.nx && j < g.ny;
  double mk = INFINITY, mw = INFINITY;
  auto load = [&](int N) {
    DestroyNb<R> c;
    c.t = type[N];
    c.u[0] = u[N];
    c.u[1] = v[N];
    c.u[2] = w[N];
    c.k = kk[N];
    c.w = om[N];
    return c;
  };
  auto stage = [&](R (*L)[PL_N], uint8_t* T8, int sl, const DestroyNb<R>& c) {
    L[0][sl] = c.u[0];
    L[1][sl] = c.u[1];
    L[2][sl] = c.u[2];
    L[3][sl] = c.k;
    L[4][sl] = c.w;
    T8[sl] = c.t;
  };
  const R inu = (R)(1.0 / ph.nu);
  const bool own = i <= g.nx && j <= g.ny;
  int ha, hb;
  const bool rim = pl_rim(a, b, ha, hb) && i0 + ha <= g.nx && j0 + hb <= g.ny;
  const int so = pl_slot(a, b), sh = pl_slot(ha, hb);
  int P = g.idx(i, j, kb), H = g.idx(i0 + ha, j0 + hb, kb);
  DestroyNb<R> cm, cc, ch;
  if (tile && own) {
    cc = load(P);
    if (d3) cm = load(P - g.sxy);
  }
  if (tile && rim) ch = load(H);
  for (int k = kb, buf = 0; k < ke; ++k, P += g.sxy, H += g.sxy, buf ^= 1) {
    R(*L)[PL_N] = lv[buf];
    if (own) stage(L, lt[buf], so, cc);
    if (rim) stage(L, lt[buf], sh, ch);
    DestroyNb<R> cp;
    if (d3 && own) cp = load(P + g.sxy);
    if (rim && k + 1 < ke) ch = load(H + g.sxy);
    __syncthreads();
    const uint8_t tp = cc.t;
    const R kP = cc.k, wP = cc.w;
    R kn = kP, wn = wP;
    if (valid && is_fluid(tp)) {
      R G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      R gk[3] = {0, 0, 0}, gw[3] = {0, 0, 0};
      const R ih2[3] = {(R)(0.5 / g.hx), (R)(0.5 / g.hy), (R)(0.5 / g.hz)};
      // constant trip counts keep G, gk and gw in registers
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int s = -1; s <= 1; s += 2) {
          if (d >= g.dim) continue;
          DestroyNb<R> n;
          if (d == 2) {
            n = s < 0 ? cm : cp;
          } else {
            const int sl = d == 0 ? pl_slot(a + s, b) : pl_slot(a, b + s);
            n.u[0] = L[0][sl];
            n.u[1] = L[1][sl];
            n.u[2] = L[2][sl];
            n.k = L[3][sl];
            n.w = L[4][sl];
            n.t = lt[buf][sl];
          }
          if (!is_fluid(n.t)) {
            const DevPatch& pp = pt[n.t & 0x7f];
            for (int c = 0; c < 3; ++c) n.u[c] = ghost<R>(pp, G_U + c, cc.u[c], ph.komega);
            n.k = ghost<R>(pp, G_K, kP, ph.komega);
            n.w = ghost<R>(pp, G_OM, wP, ph.komega);
          }
          const R sc = (R)s * ih2[d];
#pragma unroll
          for (int c = 0; c < 3; ++c)
            if (c < g.dim) G[c][d] += sc * n.u[c];
          gk[d] += sc * n.k;
          gw[d] += sc * n.w;
        }
      const R oh = omhat(wP);
      const R ioh = (R)1 / oh;
      const R ioh3 = ioh * ioh * ioh;
      const R dkdw = gk[0] * gw[0] + gk[1] * gw[1] + gk[2] * gw[2];
      const R chik = dkdw * ioh3;
      const R fbs = chik <= (R)0 ? (R)1
                                 : ((R)1 + (R)680 * chik * chik) / ((R)1 + (R)400 * chik * chik);
      const R ret = kP * ioh * inu;
      const R x = ret * (R)(1.0 / C_R_BETA);
      const R x2 = x * x;
      const R x4 = x2 * x2;
      // 0.09 (4/15 + x^4)/(1 + x^4), written so that x^4 = inf gives 0.09
      const R bst = (R)C_BSTAR * ((R)1 - (R)(11.0 / 15.0) / ((R)1 + x4));
      kn = kP / ((R)1 + tau * bst * fbs * wP);
      if (!(tp & FIXED_BIT)) {
        const R a0 = (R)0.5 * (G[2][1] - G[1][2]), a1 = (R)0.5 * (G[0][2] - G[2][0]),
                a2 = (R)0.5 * (G[1][0] - G[0][1]);
        const R s01 = (R)0.5 * (G[0][1] + G[1][0]), s02 = (R)0.5 * (G[0][2] + G[2][0]),
                s12 = (R)0.5 * (G[1][2] + G[2][1]);
        const R aSa = a0 * a0 * G[0][0] + a1 * a1 * G[1][1] + a2 * a2 * G[2][2] +
                      (R)2 * (a0 * a1 * s01 + a0 * a2 * s02 + a1 * a2 * s12);
        const R X = aSa - (a0 * a0 + a1 * a1 + a2 * a2) * (G[0][0] + G[1][1] + G[2][2]);
        const R chiw = fabs(X) * ioh3 * (R)(1.0 / (C_BSTAR * C_BSTAR * C_BSTAR));
        const R fb = ((R)1 + (R)70 * chiw) / ((R)1 + (R)80 * chiw);
        wn = wP / ((R)1 + tau * (R)C_BETA_I * fb * wP);
      }
      mk = fmin(mk, (double)kn);
      mw = fmin(mw, (double)wn);
      // eddy viscosity of the stored k, omega, for the explicit step
      if (nut_out) nut_out[P] = (F)eddy_visc<R>((R)ph.nu, (R)(F)kn, (R)(F)wn);
    }
    if (valid) {
      k_out[P] = (F)kn;
      om_out[P] = (F)wn;
    }
    cm = cc;
    cc = cp;
  }
  if (RED) {
    double vv[2] = {mk, mw};
    block_partial<2, R_MIN, BS>(vv, red);
  }
}

template <class V, class F>
void launch_destroy(const Geom& g, const Phys& ph, const uint8_t* type, const DevPatch* pt,
                    const V* u, const V* v, const V* w, const F* k, const F* om, double tau,
                    F* k_out, F* om_out, F* nut_out, const RedBuf* red, int tt, hipStream_t s) {
  const Tiles T = cell_tiles(g, tt);
  if (red) {
    check_partials(*red, T.grid, 2);
    NFVM_LAUNCH((k_destroy<V, F, true>), dim3(T.grid), dim3(BX, BY), 0, s, g, ph, type, pt,
                       u, v, w, k, om, (V)tau, k_out, om_out, nut_out, *red, T);
    launch_finalize(2, R_MIN, *red, T.grid, S_MINK, S_MINW, s);
  } else
    NFVM_LAUNCH((k_destroy<V, F, false>), dim3(T.grid), dim3(BX, BY), 0, s, g, ph, type,
                       pt, u, v, w, k, om, (V)tau, k_out, om_out, nut_out, RedBuf{}, T);
}
#define INST_DESTROY(V, F)                                                                      \
  template void launch_destroy<V, F>(const Geom&, const Phys&, const uint8_t*, const DevPatch*, \
                                     const V*, const V*, const V*, const F*, const F*, double,  \
                                     F*, F*, F*, const RedBuf*, int, hipStream_t);
INST_DESTROY(double, double)
INST_DESTROY(float, float)
INST_DESTROY(double, float)

// ---- explicit step of the rest terms -----------------------------------------
// For each transported field phi: face flux F = -U_f phi_up + Gamma_f D(phi)
// (upwind value from the lower cell when U_f >= 0), with -(p + 2/3 k)_f on the
// faces normal to a momentum component; RHS = sum_d (F_+ - F_-)/h_d plus
// sources (buoyancy, G_k = nu_t S^2, G_omega = alpha_inf (alpha_0 +
// Re_t/R_w)/(1 + Re_t/R_w) S^2); one forward-Euler step; k, omega >= eps.
// Values of one cell that the face fluxes need.
template <class R>
struct CellVals {
  R v[6];  // u v w T k omega
  R p, nut;
};

template <class V, class F, class P, class R>
__device__ __forceinline__ void load_cell(const FieldSet<V, F>& in, const P* __restrict__ p,
                                          const F* __restrict__ nut, int N, int komega,
                                          CellVals<R>& c) {
  c.v[0] = (R)in.u[N];
  c.v[1] = (R)in.v[N];
  c.v[2] = (R)in.w[N];
  c.v[3] = (R)in.T[N];
  c.v[4] = (R)in.k[N];
  c.v[5] = (R)in.om[N];
  c.p = (R)p[N];
  c.nut = komega ? (R)nut[N] : (R)0;
}

// Ghost values across a face to a non-fluid neighbour of cell P.
template <class R>
__device__ __forceinline__ void ghost_cell(const DevPatch& pp, const CellVals<R>& P, int komega,
                                           CellVals<R>& c) {
  for (int a = 0; a < 3; ++a) c.v[a] = ghost<R>(pp, G_U + a, P.v[a], komega);
  c.v[3] = ghost<R>(pp, G_T, P.v[3], komega);
  c.v[4] = ghost<R>(pp, G_K, P.v[4], komega);
  c.v[5] = ghost<R>(pp, G_OM, P.v[5], komega);
  c.p = ghost<R>(pp, G_P, P.p, komega);
  c.nut = ghost<R>(pp, G_NUT, P.nut, komega);
}

// Fluxes of the six fields through the face between P and N along axis d
// (s = -1: N below, +1: N above) and the face velocity.  The value depends
// only on the lower and upper cell, so the two cells of a face get the same
// numbers.
template <class R>
__device__ __forceinline__ void face_flux(const Phys& ph, const CellVals<R>& P,
                                          const CellVals<R>& N, int d, int s, R ihd,
                                          R (&Ff)[6], R& Uf) {
  const int komega = ph.komega;
  const R nu = (R)ph.nu;
  const R gam0[6] = {nu, nu, nu, (R)ph.alpha_T, nu, nu};
  const R isig[6] = {(R)1, (R)1, (R)1, (R)ph.inv_Pr_t, (R)ph.inv_sigma_k, (R)ph.inv_sigma_w};
  Uf = (R)0.5 * (P.v[d] + N.v[d]);
  const R nutf = (R)0.5 * (P.nut + N.nut);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const R lower = s < 0 ? N.v[f] : P.v[f];
    const R upper = s < 0 ? P.v[f] : N.v[f];
    const R up = Uf >= (R)0 ? lower : upper;
    const R gam = gam0[f] + nutf * isig[f];
    R F_ = -Uf * up + gam * (upper - lower) * ihd;
    if (f == d) {
      const R pf = (R)0.5 * (P.p + N.p);
      const R kf = komega ? (R)0.5 * (P.v[4] + N.v[4]) : (R)0;
      F_ -= pf + (R)(2.0 / 3.0) * kf;
    }
    Ff[f] = F_;
  }
}

// Each workgroup walks cz planes of a 64 x 4 column tile, one cell per
// thread.  A plane's values (u, v, w, T, k, omega, p, nu_t at the arithmetic
// type) and kind bytes go to LDS for the tile and its one-cell rim on the
// four sides, so a cell takes its four in-plane neighbours from LDS instead
// of loading them (the rim is loaded by the threads of the edge rows and 2 x 4
// threads of the second row).  The cell above is loaded by the cell's own
// thread with the next plane's rim while the plane is computed, and becomes
// the next centre; the flux through the face between them is kept, so a cell
// computes five face fluxes instead of six.  Two LDS planes alternate, so one
// barrier per plane suffices: a wave that writes plane k + 1 has passed the
// barrier of plane k, which every wave reaches only after computing plane
// k - 1, the last reader of that buffer.  The sums are formed in the same
// order as face by face.
template <class V, class F, class P>
__global__ __launch_bounds__(BS, 3) void k_explicit(Geom g, Phys ph, const uint8_t* __restrict__ type,
                                                 const DevPatch* __restrict__ pt,
                                                 FieldSet<V, F> in, const P* __restrict__ p,
                                                 const F* __restrict__ nut, FieldSet<V, F> out,
                                                 Tiles T) {
  typedef V R;
  __shared__ R lv[2][8][PL_N];
  __shared__ uint8_t lt[2][PL_N];
  int tx = 0, ty = 0, tz = 0;
  if (!tile_of(T, tx, ty, tz)) return;  // (whole workgroup)
  const int a = threadIdx.x, b = threadIdx.y;
  const int i0 = tx * BX, j0 = ty * BY;
  const int i = i0 + a, j = j0 + b;
  const int kb = tz * T.cz, ke = min(g.nz, kb + T.cz);
  const bool valid = i < g.nx && j < g.ny;
  const R nu = (R)ph.nu;
  const int komega = ph.komega;
  const bool d3 = g.dim == 3;
  const R ih[3] = {(R)(1.0 / g.hx), (R)(1.0 / g.hy), (R)(1.0 / g.hz)};
  const R dt = (R)ph.dt;
  // the cell this thread stages (its own, when it lies in the padded plane)
  // and its rim cell, if any
  const bool own = i <= g.nx && j <= g.ny;
  int ha, hb;
  const bool rim = pl_rim(a, b, ha, hb) && i0 + ha <= g.nx && j0 + hb <= g.ny;
  const int so = pl_slot(a, b), sh = pl_slot(ha, hb);
  int C0 = g.idx(i, j, kb), H0 = g.idx(i0 + ha, j0 + hb, kb);
  CellVals<R> cP, cH;
  uint8_t tp = 0, th = 0;
  if (own) {
    tp = type[C0];
    load_cell<V, F, P, R>(in, p, nut, C0, komega, cP);
  }
  if (rim) {
    th = type[H0];
    load_cell<V, F, P, R>(in, p, nut, H0, komega, cH);
  }
  // the face below the centre: its flux when the cell below was a fluid
  // centre of this walk
  bool have_lo = false;
  R Flo[6], Ulo = 0;
  R vlo[3] = {0, 0, 0};  // velocities of the fluid cell below
  for (int k = kb, buf = 0; k < ke; ++k, C0 += g.sxy, H0 += g.sxy, buf ^= 1) {
    R(*L)[PL_N] = lv[buf];
    if (own) {
#pragma unroll
      for (int f = 0; f < 6; ++f) L[f][so] = cP.v[f];
      L[6][so] = cP.p;
      L[7][so] = cP.nut;
      lt[buf][so] = tp;
    }
    if (rim) {
#pragma unroll
      for (int f = 0; f < 6; ++f) L[f][sh] = cH.v[f];
      L[6][sh] = cH.p;
      L[7][sh] = cH.nut;
      lt[buf][sh] = th;
    }
    // the cell above (loaded whatever its kind: every index lies in the
    // padded arrays) and the next plane's rim cell
    const int Nz = C0 + g.sxy;
    uint8_t tz_ = 1;
    CellVals<R> cU;
    if (d3 && own) {
      tz_ = type[Nz];
      load_cell<V, F, P, R>(in, p, nut, Nz, komega, cU);
    }
    if (rim && k + 1 < ke) {
      th = type[H0 + g.sxy];
      load_cell<V, F, P, R>(in, p, nut, H0 + g.sxy, komega, cH);
    }
    __syncthreads();
    bool next_have = false;
    R Fhi[6], Uhi = 0;
    if (valid && !is_fluid(tp)) {
      out.u[C0] = (V)cP.v[0];
      out.v[C0] = (V)cP.v[1];
      out.w[C0] = (V)cP.v[2];
      out.T[C0] = (F)cP.v[3];
      out.k[C0] = (F)cP.v[4];
      out.om[C0] = (F)cP.v[5];
    } else if (valid) {
      R rhs[6] = {0, 0, 0, 0, 0, 0};
      R G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      R divU = 0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int s = -1; s <= 1; s += 2) {
          if (d >= g.dim) continue;
          R Ff[6], Uf;
          R vN[3];
          if (d == 2 && s < 0 && have_lo) {
            for (int f = 0; f < 6; ++f) Ff[f] = Flo[f];
            Uf = Ulo;
            for (int a2 = 0; a2 < 3; ++a2) vN[a2] = vlo[a2];
          } else {
            CellVals<R> cN;
            uint8_t tn;
            if (d == 2) {
              if (s > 0) {
                cN = cU;
                tn = tz_;
              } else {  // the first plane of the walk, or below a non-fluid cell
                tn = type[C0 - g.sxy];
                load_cell<V, F, P, R>(in, p, nut, C0 - g.sxy, komega, cN);
              }
            } else {
              const int sl = d == 0 ? pl_slot(a + s, b) : pl_slot(a, b + s);
              tn = lt[buf][sl];
#pragma unroll
              for (int f = 0; f < 6; ++f) cN.v[f] = L[f][sl];
              cN.p = L[6][sl];
              cN.nut = L[7][sl];
            }
            if (!is_fluid(tn)) ghost_cell<R>(pt[tn & 0x7f], cP, komega, cN);
            face_flux<R>(ph, cP, cN, d, s, ih[d], Ff, Uf);
            for (int a2 = 0; a2 < 3; ++a2) vN[a2] = cN.v[a2];
            if (d == 2 && s > 0 && is_fluid(tn)) {
              next_have = true;
              for (int f = 0; f < 6; ++f) Fhi[f] = Ff[f];
              Uhi = Uf;
            }
          }
          const R sc = (R)s * ih[d];
          divU += sc * Uf;
          const R hg = (R)s * (R)0.5 * ih[d];
#pragma unroll
          for (int a2 = 0; a2 < 3; ++a2)
            if (a2 < g.dim) G[a2][d] += hg * vN[a2];
#pragma unroll
          for (int f = 0; f < 6; ++f) rhs[f] += sc * Ff[f];
        }
      }
      // temperature is stored as theta = T - T_ref: the convective flux of the
      // constant T_ref adds -T_ref div(U_f), which keeps the update identical to
      // the one of T itself
      rhs[3] -= (R)ph.T_ref * divU;
      R o[6];
#pragma unroll
      for (int a2 = 0; a2 < 3; ++a2) {
        R src = 0;
        if (ph.buoyancy) src = -(R)ph.beta_T * cP.v[3] * (R)ph.g[a2];
        o[a2] = a2 < g.dim ? cP.v[a2] + dt * (rhs[a2] + src) : cP.v[a2];
      }
      o[3] = ph.energy ? cP.v[3] + dt * rhs[3] : cP.v[3];
      o[4] = cP.v[4];
      o[5] = cP.v[5];
      if (komega) {
        R S2 = 0;
#pragma unroll
        for (int a2 = 0; a2 < 3; ++a2)
#pragma unroll
          for (int b2 = 0; b2 < 3; ++b2) {
            const R sab = (R)0.5 * (G[a2][b2] + G[b2][a2]);
            S2 += sab * sab;
          }
        S2 *= (R)2;
        const R ret = cP.v[4] / (nu * omhat(cP.v[5]));
        const R xr = ret * (R)(1.0 / C_R_W);
        const R Gk = cP.nut * S2;
        const R Gw = (R)C_A_INF * ((R)C_A0 + xr) / ((R)1 + xr) * S2;
        const R kn = cP.v[4] + dt * (rhs[4] + Gk);
        o[4] = kn > (R)C_EPS ? kn : (R)C_EPS;
        if (!(tp & FIXED_BIT)) {
          const R wn = cP.v[5] + dt * (rhs[5] + Gw);
          o[5] = wn > (R)C_EPS ? wn : (R)C_EPS;
        }
      }
      out.u[C0] = (V)o[0];
      out.v[C0] = (V)o[1];
      out.w[C0] = (V)o[2];
      out.T[C0] = (F)o[3];
      out.k[C0] = (F)o[4];
      out.om[C0] = (F)o[5];
    }
    // shift: the cell above becomes the centre
    have_lo = next_have;
    if (next_have) {
      for (int f = 0; f < 6; ++f) Flo[f] = Fhi[f];
      Ulo = Uhi;
      for (int a2 = 0; a2 < 3; ++a2) vlo[a2] = cP.v[a2];
    }
    if (d3) {
      tp = tz_;
      cP = cU;
    }
  }
}

template <class V, class F, class P>
void launch_explicit(const Geom& g, const Phys& ph, const uint8_t* type, const DevPatch* pt,
                     FieldSet<V, F> in, const P* p, const F* nut, FieldSet<V, F> out, int tt,
                     hipStream_t s) {
  const Tiles T = cell_tiles(g, tt);
  NFVM_LAUNCH((k_explicit<V, F, P>), dim3(T.grid), dim3(BX, BY), 0, s, g, ph, type, pt, in,
                     p, nut, out, T);
}
#define INST_EXPLICIT(V, F, P)                                                                 \
  template void launch_explicit<V, F, P>(const Geom&, const Phys&, const uint8_t*,             \
                                         const DevPatch*, FieldSet<V, F>, const P*, const F*,  \
                                         FieldSet<V, F>, int, hipStream_t);
INST_EXPLICIT(double, double, double)
INST_EXPLICIT(float, float, float)
INST_EXPLICIT(double, float, double)

// ---- second-order explicit stage (option): Heun's method in its
// strong-stability-preserving form, U* = (U + E(E(U))) / 2 with E the Euler
// step above; the second step takes nu_t from the first stage's k and omega
template <class V, class F>
__global__ __launch_bounds__(BS) void k_nut(Geom g, Phys ph, const uint8_t* __restrict__ type,
                                            const F* __restrict__ kk, const F* __restrict__ om,
                                            F* __restrict__ nut, Tiles T) {
  typedef V R;
  int tx = 0, ty = 0, tz = 0;
  const bool tile = tile_of(T, tx, ty, tz);
  const int i = tx * BX + threadIdx.x, j = ty * BY + threadIdx.y;
  const int kb = tz * T.cz, ke = min(g.nz, kb + T.cz);
  if (!tile || i >= g.nx || j >= g.ny) return;
  for (int k = kb; k < ke; ++k) {
    const int P = g.idx(i, j, k);
    if (is_fluid(type[P])) nut[P] = (F)eddy_visc<R>((R)ph.nu, (R)kk[P], (R)om[P]);
  }
}

// out = (a + c) / 2 on every cell of the box (cells the Euler step leaves
// alone hold the same value in a and c, which the average keeps exactly)
template <class V, class F>
__global__ __launch_bounds__(BS) void k_rk2_average(Geom g, FieldSet<V, F> a, FieldSet<V, F> c,
                                                    FieldSet<V, F> out, Tiles T) {
  typedef V R;
  int tx = 0, ty = 0, tz = 0;
  const bool tile = tile_of(T, tx, ty, tz);
  const int i = tx * BX + threadIdx.x, j = ty * BY + threadIdx.y;
  const int kb = tz * T.cz, ke = min(g.nz, kb + T.cz);
  if (!tile || i >= g.nx || j >= g.ny) return;
  const R h = (R)0.5;
  for (int k = kb; k < ke; ++k) {
    const int P = g.idx(i, j, k);
    out.u[P] = (V)(((R)a.u[P] + (R)c.u[P]) * h);
    out.v[P] = (V)(((R)a.v[P] + (R)c.v[P]) * h);
    out.w[P] = (V)(((R)a.w[P] + (R)c.w[P]) * h);
    out.T[P] = (F)(((R)a.T[P] + (R)c.T[P]) * h);
    out.k[P] = (F)(((R)a.k[P] + (R)c.k[P]) * h);
    out.om[P] = (F)(((R)a.om[P] + (R)c.om[P]) * h);
  }
}

template <class V, class F>
void launch_nut(const Geom& g, const Phys& ph, const uint8_t* type, const F* k, const F* om,
                F* nut, hipStream_t s) {
  const Tiles T = cell_tiles(g, TILE_DEFAULT);
  NFVM_LAUNCH((k_nut<V, F>), dim3(T.grid), dim3(BX, BY), 0, s, g, ph, type, k, om, nut, T);
}

template <class V, class F>
void launch_rk2_average(const Geom& g, FieldSet<V, F> a, FieldSet<V, F> c, FieldSet<V, F> out,
                        hipStream_t s) {
  const Tiles T = cell_tiles(g, TILE_DEFAULT);
  NFVM_LAUNCH((k_rk2_average<V, F>), dim3(T.grid), dim3(BX, BY), 0, s, g, a, c, out, T);
}
#define INST_RK2(V, F)                                                                        \
  template void launch_nut<V, F>(const Geom&, const Phys&, const uint8_t*, const F*, const F*, \
                                 F*, hipStream_t);                                            \
  template void launch_rk2_average<V, F>(const Geom&, FieldSet<V, F>, FieldSet<V, F>,          \
                                         FieldSet<V, F>, hipStream_t);
INST_RK2(double, double)
INST_RK2(float, float)
INST_RK2(double, float)

// ---- Poisson right-hand side: b = -(1/dt) sum_d D_d L_d BC_d(u*_d) ------------
// Each workgroup walks the planes of a 64 x 4 column tile; per plane u, v and
// the kind bytes of its cells and their rim go to one of two alternating LDS
// planes (one barrier per plane), and the column's w and kind below and
// above stay in registers.
template <class F, class O>
__global__ __launch_bounds__(BS) void k_rhs_b(Geom g, Phys ph, const uint8_t* __restrict__ type,
                                              const DevPatch* __restrict__ pt,
                                              const F* __restrict__ u, const F* __restrict__ v,
                                              const F* __restrict__ w, O* __restrict__ b,
                                              RedBuf red, Tiles T) {
  __shared__ O lu[2][PL_N], lv[2][PL_N];
  __shared__ uint8_t lt[2][PL_N];
  int tx = 0, ty = 0, tz = 0;
  const bool tile = tile_of(T, tx, ty, tz);  // (whole workgroup)
  const int a = threadIdx.x, bq = threadIdx.y;
  const int i0 = tx * BX, j0 = ty * BY;
  const int i = i0 + a, j = j0 + bq;
  const int kb = tz * T.cz, ke = tile ? min(g.nz, kb + T.cz) : kb;
  const bool valid = i < g.nx && j < g.ny;
  const bool own = i <= g.nx && j <= g.ny;
  int ha, hb;
  const bool rim = pl_rim(a, bq, ha, hb) && i0 + ha <= g.nx && j0 + hb <= g.ny;
  const int so = pl_slot(a, bq), sh = pl_slot(ha, hb);
  const bool d3 = g.dim == 3;
  const O ih[3] = {(O)(1.0 / g.hx), (O)(1.0 / g.hy), (O)(1.0 / g.hz)};
  double acc = 0.0;
  int C0 = g.idx(i, j, kb), H0 = g.idx(i0 + ha, j0 + hb, kb);
  O uc = 0, vc = 0, wc = 0, wm = 0, uh = 0, vh = 0;
  uint8_t tc = 0, tm = 0, th = 0;
  if (tile && own) {
    uc = (O)u[C0];
    vc = (O)v[C0];
    wc = (O)w[C0];
    tc = type[C0];
    if (d3) {
      wm = (O)w[C0 - g.sxy];
      tm = type[C0 - g.sxy];
    }
  }
  if (tile && rim) {
    uh = (O)u[H0];
    vh = (O)v[H0];
    th = type[H0];
  }
  for (int k = kb, buf = 0; k < ke; ++k, C0 += g.sxy, H0 += g.sxy, buf ^= 1) {
    if (own) {
      lu[buf][so] = uc;
      lv[buf][so] = vc;
      lt[buf][so] = tc;
    }
    if (rim) {
      lu[buf][sh] = uh;
      lv[buf][sh] = vh;
      lt[buf][sh] = th;
    }
    O up_ = 0, vp_ = 0, wp = 0;
    uint8_t tq = 0;
    if (d3 && own) {
      const int N = C0 + g.sxy;
      up_ = (O)u[N];
      vp_ = (O)v[N];
      wp = (O)w[N];
      tq = type[N];
    }
    if (rim && k + 1 < ke) {
      uh = (O)u[H0 + g.sxy];
      vh = (O)v[H0 + g.sxy];
      th = type[H0 + g.sxy];
    }
    __syncthreads();
    if (valid) {
      O bv = 0;
      if (is_fluid(tc)) {
        const O vc3[3] = {uc, vc, wc};
        O div = 0;
        for (int d = 0; d < g.dim; ++d) {
          const O vp = vc3[d];
          O fl[2];
          for (int s = -1; s <= 1; s += 2) {
            O vf;
            uint8_t tn;
            if (d == 2) {
              vf = s < 0 ? wm : wp;
              tn = s < 0 ? tm : tq;
            } else {
              const int sl = d == 0 ? pl_slot(a + s, bq) : pl_slot(a, bq + s);
              vf = d == 0 ? lu[buf][sl] : lv[buf][sl];
              tn = lt[buf][sl];
            }
            const O vn = is_fluid(tn) ? vf : ghost<O>(pt[tn & 0x7f], G_U + d, vp, ph.komega);
            fl[s > 0] = (O)0.5 * (vp + vn);
          }
          div += (fl[1] - fl[0]) * ih[d];
        }
        bv = -div / (O)ph.dt;
      }
      b[C0] = bv;
      acc += (double)bv * (double)bv;
    }
    wm = wc;
    tm = tc;
    uc = up_;
    vc = vp_;
    wc = wp;
    tc = tq;
  }
  double vv[1] = {acc};
  block_partial<1, R_SUM, BS>(vv, red);
}

template <class F, class O>
void launch_rhs_b(const Geom& g, const Phys& ph, const uint8_t* type, const DevPatch* pt,
                  const F* u, const F* v, const F* w, O* b, const RedBuf& red, int tt,
                  hipStream_t s) {
  const Tiles T = cell_tiles(g, tt);
  check_partials(red, T.grid, 1);
  NFVM_LAUNCH((k_rhs_b<F, O>), dim3(T.grid), dim3(BX, BY), 0, s, g, ph, type, pt, u, v, w,
                     b, red, T);
  launch_finalize(1, R_SUM, red, T.grid, S_BB, S_BB, s);
}
template void launch_rhs_b<double, double>(const Geom&, const Phys&, const uint8_t*,
                                           const DevPatch*, const double*, const double*,
                                           const double*, double*, const RedBuf&, int, hipStream_t);
template void launch_rhs_b<float, float>(const Geom&, const Phys&, const uint8_t*,
                                         const DevPatch*, const float*, const float*, const float*,
                                         float*, const RedBuf&, int, hipStream_t);


// ---- projection ----------------------------------------------------------------
// p += phi; u_d = u*_d - dt (phi_E - phi_W)/(2 h_d) with pressure ghosts;
// corrected face fluxes F = L(u*) - dt c_f D(phi) give the cell divergence
// (max reduced into S_DIV).  Arithmetic in the outer precision O.
// Each workgroup walks the planes of a 64 x 4 column tile; per plane phi, u,
// v (the x- and y-face velocities) and the kind bytes of its cells and their
// rim go to one of two alternating LDS planes (one barrier per plane), and
// the column's phi, w and kind below and above stay in registers.
template <class F, class P, class O>
__global__ __launch_bounds__(BS) void k_project(Geom g, Phys ph, const uint8_t* __restrict__ type,
                                                const DevPatch* __restrict__ pt,
                                                O* __restrict__ phi, const F* __restrict__ u,
                                                const F* __restrict__ v, const F* __restrict__ w,
                                                F* __restrict__ uo, F* __restrict__ vo,
                                                F* __restrict__ wo, P* __restrict__ p,
                                                RedBuf red, Tiles T) {
  __shared__ O lphi[2][PL_N], lu[2][PL_N], lv[2][PL_N];
  __shared__ uint8_t lt[2][PL_N];
  int tx = 0, ty = 0, tz = 0;
  const bool tile = tile_of(T, tx, ty, tz);  // (whole workgroup)
  const int a = threadIdx.x, b = threadIdx.y;
  const int i0 = tx * BX, j0 = ty * BY;
  const int i = i0 + a, j = j0 + b;
  const int kb = tz * T.cz, ke = tile ? min(g.nz, kb + T.cz) : kb;
  const bool valid = i < g.nx && j < g.ny;
  const bool own = i <= g.nx && j <= g.ny;
  int ha, hb;
  const bool rim = pl_rim(a, b, ha, hb) && i0 + ha <= g.nx && j0 + hb <= g.ny;
  const int so = pl_slot(a, b), sh = pl_slot(ha, hb);
  const bool d3 = g.dim == 3;
  double mdiv = 0.0;
  // b = 0: the increment is 0 whatever the solve started from; it is taken
  // as 0 here and cleared, so the next step does not start from it
  const bool zero_inc = red.out[S_BB] == 0.0;
  auto ldphi = [&](int N) -> O { return zero_inc ? (O)0 : phi[N]; };
  const O ih[3] = {(O)(1.0 / g.hx), (O)(1.0 / g.hy), (O)(1.0 / g.hz)};
  const O dt = (O)ph.dt;
  int C0 = g.idx(i, j, kb), H0 = g.idx(i0 + ha, j0 + hb, kb);
  // this column at planes k - 1 (m) and k (c); the rim cell at plane k (h)
  O fc = 0, uc = 0, vc = 0, wc = 0, fm = 0, wm = 0, fh = 0, uh = 0, vh = 0;
  uint8_t tc = 0, tm = 0, th = 0;
  if (tile && own) {
    fc = ldphi(C0);
    uc = (O)u[C0];
    vc = (O)v[C0];
    wc = (O)w[C0];
    tc = type[C0];
    if (d3) {
      fm = ldphi(C0 - g.sxy);
      wm = (O)w[C0 - g.sxy];
      tm = type[C0 - g.sxy];
    }
  }
  if (tile && rim) {
    fh = ldphi(H0);
    uh = (O)u[H0];
    vh = (O)v[H0];
    th = type[H0];
  }
  for (int k = kb, buf = 0; k < ke; ++k, C0 += g.sxy, H0 += g.sxy, buf ^= 1) {
    if (own) {
      lphi[buf][so] = fc;
      lu[buf][so] = uc;
      lv[buf][so] = vc;
      lt[buf][so] = tc;
    }
    if (rim) {
      lphi[buf][sh] = fh;
      lu[buf][sh] = uh;
      lv[buf][sh] = vh;
      lt[buf][sh] = th;
    }
    // the plane above (loaded whatever its kind) and the next rim cell
    O fp = 0, up_ = 0, vp_ = 0, wp = 0;
    uint8_t tq = 0;
    if (d3 && own) {
      const int N = C0 + g.sxy;
      fp = ldphi(N);
      up_ = (O)u[N];
      vp_ = (O)v[N];
      wp = (O)w[N];
      tq = type[N];
    }
    if (rim && k + 1 < ke) {
      fh = ldphi(H0 + g.sxy);
      uh = (O)u[H0 + g.sxy];
      vh = (O)v[H0 + g.sxy];
      th = type[H0 + g.sxy];
    }
    __syncthreads();
    if (valid) {
      const F* vel[3] = {u, v, w};
      F* vout[3] = {uo, vo, wo};
      const O vc3[3] = {uc, vc, wc};
      if (!is_fluid(tc)) {
        for (int d = 0; d < 3; ++d) vout[d][C0] = (F)vc3[d];
      } else {
        const O fP = fc;
        if (zero_inc) phi[C0] = (O)0;
        O div = 0;
        O unew[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          if (d >= g.dim) continue;
          const O vp = vc3[d];
          O grad = 0;
          O fl[2];
#pragma unroll
          for (int s = -1; s <= 1; s += 2) {
            O vf, ff;
            uint8_t tn;
            if (d == 2) {
              vf = s < 0 ? wm : wp;
              ff = s < 0 ? fm : fp;
              tn = s < 0 ? tm : tq;
            } else {
              const int sl = d == 0 ? pl_slot(a + s, b) : pl_slot(a, b + s);
              vf = d == 0 ? lu[buf][sl] : lv[buf][sl];
              ff = lphi[buf][sl];
              tn = lt[buf][sl];
            }
            O vn, fN_ghost, fN_face, c;
            if (is_fluid(tn)) {
              vn = vf;
              fN_ghost = ff;
              fN_face = fN_ghost;
              c = 1;
            } else {
              const DevPatch& pp = pt[tn & 0x7f];
              vn = ghost<O>(pp, G_U + d, vp, ph.komega);
              fN_ghost = ghost<O>(pp, G_P, fP, ph.komega);
              c = pp.kind == K_OUTLET ? (O)2 : (O)0;
              fN_face = 0;
            }
            grad += (O)s * fN_ghost;
            const O dphi = s > 0 ? (fN_face - fP) : (fP - fN_face);
            fl[s > 0] = (O)0.5 * (vp + vn) - dt * c * dphi * ih[d];
          }
          unew[d] = vp - dt * grad * (O)0.5 * ih[d];
          div += (fl[1] - fl[0]) * ih[d];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) vout[d][C0] = d < g.dim ? (F)unew[d] : vel[d][C0];
        p[C0] = (P)((O)p[C0] + fP);
        mdiv = fmax(mdiv, fabs((double)div));
      }
    }
    // shift: the plane above becomes the centre
    fm = fc;
    wm = wc;
    tm = tc;
    fc = fp;
    uc = up_;
    vc = vp_;
    wc = wp;
    tc = tq;
  }
  double vv[1] = {mdiv};
  block_partial<1, R_MAX, BS>(vv, red);
}

template <class F, class P, class O>
void launch_project(const Geom& g, const Phys& ph, const uint8_t* type, const DevPatch* pt,
                    O* phi, const F* u, const F* v, const F* w, F* uo, F* vo, F* wo, P* p,
                    const RedBuf& red, int tt, hipStream_t s) {
  const Tiles T = cell_tiles(g, tt);
  check_partials(red, T.grid, 1);
  NFVM_LAUNCH((k_project<F, P, O>), dim3(T.grid), dim3(BX, BY), 0, s, g, ph, type, pt, phi,
                     u, v, w, uo, vo, wo, p, red, T);
  launch_finalize(1, R_MAX, red, T.grid, S_DIV, S_DIV, s);
}
template void launch_project<double, double, double>(const Geom&, const Phys&, const uint8_t*,
                                                     const DevPatch*, double*,
                                                     const double*, const double*, const double*,
                                                     double*, double*, double*, double*,
                                                     const RedBuf&, int, hipStream_t);
template void launch_project<float, float, float>(const Geom&, const Phys&, const uint8_t*,
                                                  const DevPatch*, float*, const float*,
                                                  const float*, const float*, float*, float*,
                                                  float*, float*, const RedBuf&, int, hipStream_t);

// ---- reverse mode of the pressure step ------------------------------------------
// The step (Sec. 2.4) maps u* to u = u* - dt G(phi), p = p^n + phi with
// phi = A^-1 b and b = -(1/dt) sum_d D_d L_d BC_d(u*_d) (eq. pc_residual);
// it is affine in u*.  Its transposed Jacobian, written as gathers over the
// cells whose forward formulas read a cell: each fluid cell's face average and
// central difference read its fluid neighbours directly and its own value
// through the slope of a ghost rule (ghost = s v_P + const, s = ghost(1) -
// ghost(0)).  Inputs and outputs are dense FP64 [nz][ny][nx]; the solve's
// right-hand side and solution are the grid's padded vectors.
__device__ __forceinline__ double ghost_slope(const DevPatch& pp, int fld, int komega) {
  return ghost<double>(pp, fld, 1.0, komega) - ghost<double>(pp, fld, 0.0, komega);
}

// phibar = pbar - dt G^T ubar on fluid cells (0 elsewhere), into the solve's
// right-hand side
template <class O>
__global__ __launch_bounds__(BS) void k_adj_phibar(Geom g, Phys ph, const uint8_t* __restrict__ type,
                                                   const DevPatch* __restrict__ pt,
                                                   const double* __restrict__ ub,
                                                   const double* __restrict__ vb,
                                                   const double* __restrict__ wb,
                                                   const double* __restrict__ pb,
                                                   O* __restrict__ rhs) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const int C0 = g.idx(i, j, k);
  const long long n = ((long long)k * g.ny + j) * g.nx + i;
  if (!is_fluid(type[C0])) {
    rhs[C0] = (O)0;
    return;
  }
  const double* bar[3] = {ub, vb, wb};
  const int st[3] = {1, g.sx, g.sxy};
  const long long sd[3] = {1, g.nx, (long long)g.nx * g.ny};
  const double h[3] = {g.hx, g.hy, g.hz};
  double acc = pb[n];
  for (int d = 0; d < g.dim; ++d) {
    const double f = ph.dt / (2.0 * h[d]);
    const uint8_t tl = type[C0 - st[d]], th = type[C0 + st[d]];
    const double uP = bar[d][n];
    if (is_fluid(tl))
      acc -= f * bar[d][n - sd[d]];
    else
      acc += f * uP * ghost_slope(pt[tl & 0x7f], G_P, ph.komega);
    if (is_fluid(th))
      acc += f * bar[d][n + sd[d]];
    else
      acc -= f * uP * ghost_slope(pt[th & 0x7f], G_P, ph.komega);
  }
  rhs[C0] = (O)acc;
}

// usbar = ubar + (d b / d u*)^T lambda (fluid cells; ubar elsewhere)
template <class O>
__global__ __launch_bounds__(BS) void k_adj_velocity(Geom g, Phys ph, const uint8_t* __restrict__ type,
                                                     const DevPatch* __restrict__ pt,
                                                     const O* __restrict__ lam,
                                                     const double* __restrict__ ub,
                                                     const double* __restrict__ vb,
                                                     const double* __restrict__ wb,
                                                     double* __restrict__ usb,
                                                     double* __restrict__ vsb,
                                                     double* __restrict__ wsb) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const int C0 = g.idx(i, j, k);
  const long long n = ((long long)k * g.ny + j) * g.nx + i;
  const double* bar[3] = {ub, vb, wb};
  double* out[3] = {usb, vsb, wsb};
  const bool fl = is_fluid(type[C0]);
  const int st[3] = {1, g.sx, g.sxy};
  const double h[3] = {g.hx, g.hy, g.hz};
  for (int d = 0; d < 3; ++d) {
    double acc = bar[d][n];
    if (fl && d < g.dim) {
      // s_Y = -lambda_Y / (dt h_d): d b_Y / d (face average) of a face of Y
      const double c = -1.0 / (ph.dt * h[d]);
      const double sP = c * (double)lam[C0];
      const uint8_t tl = type[C0 - st[d]], th = type[C0 + st[d]];
      if (is_fluid(tl))
        acc += 0.5 * c * (double)lam[C0 - st[d]];
      else
        acc -= 0.5 * sP * ghost_slope(pt[tl & 0x7f], G_U + d, ph.komega);
      if (is_fluid(th))
        acc -= 0.5 * c * (double)lam[C0 + st[d]];
      else
        acc += 0.5 * sP * ghost_slope(pt[th & 0x7f], G_U + d, ph.komega);
    }
    out[d][n] = acc;
  }
}

template <class O>
void launch_adj_phibar(const Geom& g, const Phys& ph, const uint8_t* type, const DevPatch* pt,
                       const double* ub, const double* vb, const double* wb, const double* pb,
                       O* rhs, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_phibar<O>, cell_grid(g), dim3(BX, BY), 0, s, g, ph, type, pt, ub, vb,
                     wb, pb, rhs);
}
template <class O>
void launch_adj_velocity(const Geom& g, const Phys& ph, const uint8_t* type, const DevPatch* pt,
                         const O* lam, const double* ub, const double* vb, const double* wb,
                         double* usb, double* vsb, double* wsb, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_velocity<O>, cell_grid(g), dim3(BX, BY), 0, s, g, ph, type, pt, lam,
                     ub, vb, wb, usb, vsb, wsb);
}
#define INST_ADJ(O)                                                                             \
  template void launch_adj_phibar<O>(const Geom&, const Phys&, const uint8_t*, const DevPatch*, \
                                     const double*, const double*, const double*, const double*, \
                                     O*, hipStream_t);                                          \
  template void launch_adj_velocity<O>(const Geom&, const Phys&, const uint8_t*,                \
                                       const DevPatch*, const O*, const double*, const double*, \
                                       const double*, double*, double*, double*, hipStream_t);
INST_ADJ(double)
INST_ADJ(float)

}  // namespace nfvm

