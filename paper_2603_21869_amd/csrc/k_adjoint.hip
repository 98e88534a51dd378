// Reverse mode of the explicit stage and of the destruction step.
//
// Explicit stage (Sec. 2.3, Algorithms 2 and 4, eqs. ko_mom, ko_temp, ko_k,
// ko_o; the solver's differentiability, Sec. 1 and 4):
// the adjoints of the stage's inputs u, v, w, p, T, k, omega from those of its
// outputs u, v, w, T, k, omega, at a given input state, with nu_t the closure
// of the input k and omega (eqs. a_star, ko_turb_diff), so that its adjoint
// is folded into theirs.
//
// The stage updates every fluid cell by dt times a sum of face fluxes, each a
// function of the two cells of the face (a boundary face's outer values being
// affine ghost rules of the inner cell, Sec. 2.7), plus cell sources that
// read the central velocity gradient.  The transposed Jacobian is formed as
// a gather, one thread per input cell, in two passes over padded FP64 arrays:
//   1. per output cell: the weights dt * ybar of the outputs that the fluxes
//      feed (zero where an output is not updated or is clamped at eps), the
//      factor by which each output passes its own input (1, or 0 where k or
//      omega is clamped), and 4 Lambda S_ab with Lambda = W_k nu_t + W_omega
//      alpha, the weight of the strain-rate sources;
//   2. per input cell: its own pass terms, then each face's flux derivatives
//      with respect to this cell's values times the difference of the two
//      cells' weights, the production terms of its own and of its
//      neighbours' strain rates, buoyancy, and the closure chain rule.
// Arithmetic in FP64 throughout.
#include <hip/hip_runtime.h>

#include "nfvm_device.hpp"

namespace nfvm {

namespace {
constexpr int ABX = 64, ABY = 4;

// transported fields in flux order and their ghost-rule codes
constexpr int NF = 6;  // u v w theta k omega
__device__ __forceinline__ int ghost_code(int f) {
  return f < 3 ? G_U + f : (f == 3 ? G_T : (f == 4 ? G_K : G_OM));
}

// The cell of this thread.  The launch is one-dimensional, 8 * per
// workgroups of ABX x ABY threads over the list of (column tile, plane)
// entries, planes fastest; workgroup b runs on XCD b % 8 and takes entry
// (b % 8) * per + b / 8, so the workgroups in flight on one XCD hold
// consecutive planes of the same column tiles and the planes above and below
// that each cell reads are in that XCD's L2.
__device__ __forceinline__ bool adj_cell(const Geom& g, int& i, int& j, int& k) {
  const int ntx = (g.nx + ABX - 1) / ABX, nty = (g.ny + ABY - 1) / ABY;
  const long long total = (long long)ntx * nty * g.nz;
  const long long per = gridDim.x >> 3;
  const long long t = (long long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (t >= total) return false;
  k = (int)(t % g.nz);
  const long long c = t / g.nz;
  i = (int)(c % ntx) * ABX + threadIdx.x;
  j = (int)(c / ntx) * ABY + threadIdx.y;
  return i < g.nx && j < g.ny;
}

// workgroups of the launches that use adj_cell (a multiple of 8)
inline dim3 adj_grid(const Geom& g) {
  const long long total =
      (long long)((g.nx + ABX - 1) / ABX) * ((g.ny + ABY - 1) / ABY) * g.nz;
  return dim3((unsigned)(8 * ((total + 7) / 8)));
}

struct AdjCell {
  double v[NF], nu;
  uint8_t t;
};

// nu_t = alpha*(Re_t) k / omega-hat and its partial derivatives in k and
// omega (eqs. a_star and Re_t with alpha*_inf = 1, alpha*_0 = beta_i / 3)
__device__ __forceinline__ void closure_grad(double nu, double k, double w, double& nt,
                                             double& dk, double& dw) {
  const bool live = w > C_EPS;
  const double oh = live ? w : C_EPS;
  const double ret = k / (nu * oh);
  const double x = ret * (1.0 / C_R_K);
  const double a0 = C_BETA_I / 3.0;
  const double as = (a0 + x) / (1.0 + x);
  const double das = (1.0 - a0) * (1.0 / C_R_K) / ((1.0 + x) * (1.0 + x));  // d as / d ret
  nt = as * k / oh;
  dk = das * (1.0 / (nu * oh)) * k / oh + as / oh;
  dw = live ? das * (-ret / oh) * k / oh - as * k / (oh * oh) : 0.0;
}

// alpha of the omega production (eq. a with eqs. k_gen, o_gen) and its
// derivatives in k and omega
__device__ __forceinline__ void alpha_grad(double nu, double k, double w, double& al,
                                           double& dk, double& dw) {
  const bool live = w > C_EPS;
  const double oh = live ? w : C_EPS;
  const double ret = k / (nu * oh);
  const double xr = ret * (1.0 / C_R_W);
  al = C_A_INF * (C_A0 + xr) / (1.0 + xr);
  const double da = C_A_INF * (1.0 - C_A0) * (1.0 / C_R_W) / ((1.0 + xr) * (1.0 + xr));
  dk = da / (nu * oh);
  dw = live ? da * (-ret / oh) : 0.0;
}

// (the stage's Jacobian does not depend on p: it enters the momentum
// update linearly, so the state's p is not read)
struct AdjState {
  const double *u, *v, *w, *T, *k, *om;  // padded; T as T - T_ref
  const double* nu;  // nu_t of the fluid cells (k-omega only), padded
};

__device__ __forceinline__ AdjCell load_adj(const AdjState& S, const uint8_t* type, int N,
                                            const Phys& ph) {
  AdjCell c;
  c.t = type[N];
  c.v[0] = S.u[N];
  c.v[1] = S.v[N];
  c.v[2] = S.w[N];
  c.v[3] = S.T[N];
  c.v[4] = S.k[N];
  c.v[5] = S.om[N];
  c.nu = ph.komega && is_fluid(c.t) ? S.nu[N] : 0.0;
  return c;
}

// values across a boundary face, from the fluid cell P
__device__ __forceinline__ AdjCell ghost_adj(const DevPatch& pp, const AdjCell& P, int komega,
                                             uint8_t t) {
  AdjCell g;
  for (int f = 0; f < NF; ++f) g.v[f] = ghost<double>(pp, ghost_code(f), P.v[f], komega);
  g.nu = ghost<double>(pp, G_NUT, P.nu, komega);
  g.t = t;
  return g;
}

__device__ __forceinline__ double slope(const DevPatch& pp, int code, int komega) {
  return ghost<double>(pp, code, 1.0, komega) - ghost<double>(pp, code, 0.0, komega);
}

__device__ __forceinline__ void field_coef(const Phys& ph, double (&g0)[NF], double (&is)[NF]) {
  g0[0] = g0[1] = g0[2] = ph.nu;
  g0[3] = ph.alpha_T;
  g0[4] = g0[5] = ph.nu;
  is[0] = is[1] = is[2] = 1.0;
  is[3] = ph.inv_Pr_t;
  is[4] = ph.inv_sigma_k;
  is[5] = ph.inv_sigma_w;
}

// central velocity gradient G[a][b] = d u_a / d x_b at fluid cell P with
// boundary ghosts; N[b][s] are the neighbours (s = 0: -, 1: +)
__device__ __forceinline__ void adj_gradient(const Geom& g, const AdjCell& P,
                                             const AdjCell (&N)[3][2], double (&G)[3][3]) {
  const double ih2[3] = {0.5 / g.hx, 0.5 / g.hy, 0.5 / g.hz};
  #pragma unroll
  for (int a = 0; a < 3; ++a)
    #pragma unroll
    for (int b = 0; b < 3; ++b)
      G[a][b] = (a < g.dim && b < g.dim) ? (N[b][1].v[a] - N[b][0].v[a]) * ih2[b] : 0.0;
}

// the six neighbours of fluid cell P, ghosts substituted
__device__ __forceinline__ void adj_neighbours(const Geom& g, const Phys& ph, const AdjState& S,
                                               const uint8_t* type, const DevPatch* pt, int P,
                                               const AdjCell& c, AdjCell (&N)[3][2]) {
  const int st[3] = {1, g.sx, g.sxy};
  #pragma unroll
  for (int d = 0; d < 3; ++d)
    #pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (d >= g.dim) {
        N[d][s] = c;
        continue;
      }
      const int Q = P + (s ? 1 : -1) * st[d];
      const uint8_t tq = type[Q];
      N[d][s] = is_fluid(tq) ? load_adj(S, type, Q, ph) : ghost_adj(pt[tq & 0x7f], c, ph.komega, tq);
    }
}

// neighbour s (0: -, 1: +) of fluid cell P along d < dim, ghost substituted
// (one element of adj_neighbours, loaded where it is used)
__device__ __forceinline__ AdjCell adj_neighbour(const Geom& g, const Phys& ph, const AdjState& S,
                                                 const uint8_t* type, const DevPatch* pt, int P,
                                                 const AdjCell& c, int d, int s) {
  const int Q = P + (s ? 1 : -1) * (d == 0 ? 1 : (d == 1 ? g.sx : g.sxy));
  const uint8_t tq = type[Q];
  return is_fluid(tq) ? load_adj(S, type, Q, ph) : ghost_adj(pt[tq & 0x7f], c, ph.komega, tq);
}

// the central velocity gradient of adj_gradient, from the neighbours'
// velocities alone
__device__ __forceinline__ void adj_gradient_at(const Geom& g, const Phys& ph, const AdjState& S,
                                                const uint8_t* type, const DevPatch* pt, int P,
                                                const AdjCell& c, double (&G)[3][3]) {
  const double ih2[3] = {0.5 / g.hx, 0.5 / g.hy, 0.5 / g.hz};
  const double* vel[3] = {S.u, S.v, S.w};
  #pragma unroll
  for (int a = 0; a < 3; ++a)
    #pragma unroll
    for (int b = 0; b < 3; ++b) G[a][b] = 0.0;
  #pragma unroll
  for (int b = 0; b < 3; ++b) {
    if (b >= g.dim) continue;
    double vn[2][3];
    #pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int Q = P + (s ? 1 : -1) * (b == 0 ? 1 : (b == 1 ? g.sx : g.sxy));
      const uint8_t tq = type[Q];
      #pragma unroll
      for (int a = 0; a < 3; ++a)
        vn[s][a] = is_fluid(tq) ? vel[a][Q]
                                : ghost<double>(pt[tq & 0x7f], G_U + a, c.v[a], ph.komega);
    }
    #pragma unroll
    for (int a = 0; a < 3; ++a)
      if (a < g.dim) G[a][b] = (vn[1][a] - vn[0][a]) * ih2[b];
  }
}
}  // namespace

// nu_t of every fluid cell (the closure of its k and omega), read by both
// passes at a cell and its six neighbours instead of being formed there.
__global__ __launch_bounds__(ABX* ABY) void k_adj_nut(Geom g, Phys ph,
                                                     const uint8_t* __restrict__ type,
                                                     const double* __restrict__ kk,
                                                     const double* __restrict__ om,
                                                     double* __restrict__ nu) {
  int i, j, k;
  if (!adj_cell(g, i, j, k)) return;
  const int P = g.idx(i, j, k);
  double nt = 0.0, dk, dw;
  if (is_fluid(type[P])) closure_grad(ph.nu, kk[P], om[P], nt, dk, dw);
  nu[P] = nt;
}

// Pass 1: weights of each output cell.  W: six padded arrays (u v w theta k
// omega), pass: two (k, omega), L4S: six (S00 S11 S22 S01 S02 S12 times
// 4 Lambda).  ybar: dense [nz][ny][nx] adjoints of the six outputs.
__global__ __launch_bounds__(ABX* ABY) void k_adj_ex_weights(
    Geom g, Phys ph, const uint8_t* __restrict__ type, const DevPatch* __restrict__ pt,
    AdjState S, const double* __restrict__ ybu, const double* __restrict__ ybv,
    const double* __restrict__ ybw, const double* __restrict__ ybT,
    const double* __restrict__ ybk, const double* __restrict__ ybo, double* __restrict__ W,
    double* __restrict__ pass, double* __restrict__ L4S) {
  int i, j, k;
  if (!adj_cell(g, i, j, k)) return;
  const int P = g.idx(i, j, k);
  const size_t D = ((size_t)k * g.ny + j) * g.nx + i;
  const size_t T = (size_t)g.total;
  const uint8_t tp = type[P];
  // formed in registers and stored once (zero weights and pass 1 where the
  // cell is not fluid)
  double Wv[NF] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, Lv[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double ps[2] = {1.0, 1.0};
  [&]() {
    if (!is_fluid(tp)) return;
    const double dt = ph.dt;
    const double yb[NF] = {ybu[D], ybv[D], ybw[D], ybT[D], ybk[D], ybo[D]};
    #pragma unroll
    for (int a = 0; a < 3; ++a) Wv[a] = a < g.dim ? dt * yb[a] : 0.0;
    Wv[3] = ph.energy ? dt * yb[3] : 0.0;
    if (!ph.komega) return;
    const AdjCell c = load_adj(S, type, P, ph);
    AdjCell N[3][2];
    adj_neighbours(g, ph, S, type, pt, P, c, N);
    double g0[NF], is[NF];
    field_coef(ph, g0, is);
    const double ih[3] = {1.0 / g.hx, 1.0 / g.hy, 1.0 / g.hz};
    double rk = 0.0, rw = 0.0;
    #pragma unroll
    for (int d = 0; d < 3; ++d)
      #pragma unroll
      for (int s = 0; s < 2; ++s) {
        if (d >= g.dim) continue;
        const AdjCell& n = N[d][s];
        const double sg = s ? 1.0 : -1.0;
        const double Uf = 0.5 * (c.v[d] + n.v[d]);
        const double nutf = 0.5 * (c.nu + n.nu);
        #pragma unroll
        for (int f = 4; f < 6; ++f) {
          const double lower = s ? c.v[f] : n.v[f], upper = s ? n.v[f] : c.v[f];
          const double up = Uf >= 0.0 ? lower : upper;
          const double F = -Uf * up + (g0[f] + nutf * is[f]) * (upper - lower) * ih[d];
          (f == 4 ? rk : rw) += sg * F * ih[d];
        }
      }
    double G[3][3];
    adj_gradient(g, c, N, G);
    double Sab[6];
    Sab[0] = G[0][0];
    Sab[1] = G[1][1];
    Sab[2] = G[2][2];
    Sab[3] = 0.5 * (G[0][1] + G[1][0]);
    Sab[4] = 0.5 * (G[0][2] + G[2][0]);
    Sab[5] = 0.5 * (G[1][2] + G[2][1]);
    const double S2 = 2.0 * (Sab[0] * Sab[0] + Sab[1] * Sab[1] + Sab[2] * Sab[2] +
                             2.0 * (Sab[3] * Sab[3] + Sab[4] * Sab[4] + Sab[5] * Sab[5]));
    double al, dak, daw;
    alpha_grad(ph.nu, c.v[4], c.v[5], al, dak, daw);
    const double kn = c.v[4] + dt * (rk + c.nu * S2);
    const double wn = c.v[5] + dt * (rw + al * S2);
    const bool pk = kn > C_EPS;
    const bool fixed = (tp & FIXED_BIT) != 0;
    const bool pw = fixed || wn > C_EPS;
    const double Wk = pk ? dt * yb[4] : 0.0;
    const double Ww = (!fixed && pw) ? dt * yb[5] : 0.0;
    Wv[4] = Wk;
    Wv[5] = Ww;
    ps[0] = pk ? 1.0 : 0.0;
    ps[1] = pw ? 1.0 : 0.0;
    const double lam4 = 4.0 * (Wk * c.nu + Ww * al);
    #pragma unroll
    for (int q = 0; q < 6; ++q) Lv[q] = lam4 * Sab[q];
  }();
  #pragma unroll
  for (int f = 0; f < NF; ++f) {
    W[f * T + P] = Wv[f];
    L4S[f * T + P] = Lv[f];
  }
  pass[P] = ps[0];
  pass[T + P] = ps[1];
}

// Pass 2: the adjoints of the inputs, dense [nz][ny][nx]: xb = {u v w p T k omega}.
__global__ __launch_bounds__(ABX* ABY) void k_adj_ex_gather(
    Geom g, Phys ph, const uint8_t* __restrict__ type, const DevPatch* __restrict__ pt,
    AdjState S, const double* __restrict__ ybu, const double* __restrict__ ybv,
    const double* __restrict__ ybw, const double* __restrict__ ybT,
    const double* __restrict__ ybk, const double* __restrict__ ybo,
    const double* __restrict__ W, const double* __restrict__ pass,
    const double* __restrict__ L4S, double* __restrict__ xu, double* __restrict__ xv,
    double* __restrict__ xw, double* __restrict__ xp, double* __restrict__ xT,
    double* __restrict__ xk, double* __restrict__ xo) {
  int i, j, k;
  if (!adj_cell(g, i, j, k)) return;
  const int P = g.idx(i, j, k);
  const size_t D = ((size_t)k * g.ny + j) * g.nx + i;
  const size_t T = (size_t)g.total;
  const uint8_t tp = type[P];
  // each output passes its own input (k and omega unless clamped)
  double xb[NF] = {ybu[D], ybv[D], ybw[D], ybT[D], ybk[D] * pass[P], ybo[D] * pass[T + P]};
  double pb = 0.0, nb = 0.0;  // adjoints of p and of nu_t at this cell
  if (is_fluid(tp)) {
    const AdjCell c = load_adj(S, type, P, ph);
    double g0[NF], is[NF];
    field_coef(ph, g0, is);
    const int st[3] = {1, g.sx, g.sxy};
    const double ih[3] = {1.0 / g.hx, 1.0 / g.hy, 1.0 / g.hz};
    double Wc[NF];
    #pragma unroll
    for (int f = 0; f < NF; ++f) Wc[f] = W[f * T + P];
    const int komega = ph.komega;
    // faces
    #pragma unroll
    for (int d = 0; d < 3; ++d)
      #pragma unroll
      for (int s = 0; s < 2; ++s) {
        if (d >= g.dim) continue;
        const AdjCell n = adj_neighbour(g, ph, S, type, pt, P, c, d, s);
        const double sg = s ? 1.0 : -1.0;
        const bool nf = is_fluid(n.t);
        const int Q = P + (s ? 1 : -1) * st[d];
        // d(outer value) / d(own value) across this face
        double gs[NF], gp = 0.0, gn = 0.0;
        double wf[NF];
        if (nf) {
          #pragma unroll
          for (int f = 0; f < NF; ++f) {
            gs[f] = 0.0;
            wf[f] = sg * ih[d] * (Wc[f] - W[f * T + Q]);
          }
        } else {
          const DevPatch& pp = pt[n.t & 0x7f];
          #pragma unroll
          for (int f = 0; f < NF; ++f) {
            gs[f] = slope(pp, ghost_code(f), komega);
            wf[f] = sg * ih[d] * Wc[f];
          }
          gp = slope(pp, G_P, komega);
          gn = slope(pp, G_NUT, komega);
        }
        const double Uf = 0.5 * (c.v[d] + n.v[d]);
        const double nutf = 0.5 * (c.nu + n.nu);
        // the upwind value is this cell's when the face velocity points away
        // from it (lower cell for Uf >= 0)
        const bool own_up = (Uf >= 0.0) == (s == 1);
        double dUf = 0.0, dnut = 0.0;
        #pragma unroll
        for (int f = 0; f < NF; ++f) {
          const double lower = s ? c.v[f] : n.v[f], upper = s ? n.v[f] : c.v[f];
          const double up = Uf >= 0.0 ? lower : upper;
          const double gam = g0[f] + nutf * is[f];
          const double dup = own_up ? 1.0 : gs[f];
          // d F / d phi_own, d F / d U_f, d F / d nut_f
          xb[f] += wf[f] * (-Uf * dup + gam * sg * (gs[f] - 1.0) * ih[d]);
          dUf += wf[f] * (-up - (f == 3 ? ph.T_ref : 0.0));
          dnut += wf[f] * is[f] * (upper - lower) * ih[d];
        }
        xb[d] += dUf * 0.5 * (1.0 + gs[d]);
        nb += dnut * 0.5 * (1.0 + gn);
        // -(p + 2/3 k)_f on the faces normal to momentum component d
        pb += wf[d] * -0.5 * (1.0 + (nf ? 0.0 : gp));
        if (komega) xb[4] += wf[d] * (-1.0 / 3.0) * (1.0 + gs[4]);
      }
    // buoyancy -beta_T theta g_a
    if (ph.buoyancy)
      #pragma unroll
      for (int a = 0; a < 3; ++a)
        if (a < g.dim) xb[3] += Wc[a] * -ph.beta_T * ph.g[a];
    if (komega) {
      // production nu_t S^2 and alpha S^2 at this cell
      double G[3][3];
      adj_gradient_at(g, ph, S, type, pt, P, c, G);
      double S2 = 0.0;
      #pragma unroll
      for (int a = 0; a < 3; ++a)
        #pragma unroll
        for (int b = 0; b < 3; ++b) {
          const double sab = 0.5 * (G[a][b] + G[b][a]);
          S2 += sab * sab;
        }
      S2 *= 2.0;
      double al, dak, daw;
      alpha_grad(ph.nu, c.v[4], c.v[5], al, dak, daw);
      nb += Wc[4] * S2;
      xb[4] += Wc[5] * S2 * dak;
      xb[5] += Wc[5] * S2 * daw;
      // strain rates that read this cell's velocity: a neighbour's across the
      // face (its own 4 Lambda S_ab), or this cell's own through a ghost
      const double ih2[3] = {0.5 / g.hx, 0.5 / g.hy, 0.5 / g.hz};
      const int sidx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
      #pragma unroll
      for (int b = 0; b < 3; ++b)
        #pragma unroll
        for (int s = 0; s < 2; ++s) {
          if (b >= g.dim) continue;
          const double sg = s ? 1.0 : -1.0;
          const int Q = P + (s ? 1 : -1) * st[b];
          const uint8_t tq = type[Q];
          if (is_fluid(tq)) {
            // this cell is the neighbour of Q on Q's side -sg along b
            #pragma unroll
            for (int a = 0; a < 3; ++a)
              if (a < g.dim) xb[a] += L4S[sidx[a][b] * T + Q] * -sg * ih2[b];
          } else {
            const DevPatch& pp = pt[tq & 0x7f];
            #pragma unroll
            for (int a = 0; a < 3; ++a)
              if (a < g.dim)
                xb[a] += L4S[sidx[a][b] * T + P] * sg * ih2[b] * slope(pp, G_U + a, komega);
          }
        }
      // nu_t is the closure of this cell's k and omega
      double nt, dk, dw;
      closure_grad(ph.nu, c.v[4], c.v[5], nt, dk, dw);
      xb[4] += nb * dk;
      xb[5] += nb * dw;
    }
  }
  xu[D] = xb[0];
  xv[D] = xb[1];
  xw[D] = xb[2];
  xp[D] = pb;
  xT[D] = xb[3];
  xk[D] = xb[4];
  xo[D] = xb[5];
}

void launch_explicit_adjoint(const Geom& g, const Phys& ph, const uint8_t* type,
                             const DevPatch* pt, const double* const st[7],
                             const double* const yb[6], double* W, double* pass, double* L4S,
                             double* nu, double* const xb[7], hipStream_t s) {
  const AdjState S{st[0], st[1], st[2], st[4], st[5], st[6], nu};
  const dim3 G = adj_grid(g), B(ABX, ABY);
  if (ph.komega) hipLaunchKernelGGL(k_adj_nut, G, B, 0, s, g, ph, type, st[5], st[6], nu);
  hipLaunchKernelGGL(k_adj_ex_weights, G, B, 0, s, g, ph, type, pt, S, yb[0], yb[1], yb[2],
                     yb[3], yb[4], yb[5], W, pass, L4S);
  hipLaunchKernelGGL(k_adj_ex_gather, G, B, 0, s, g, ph, type, pt, S, yb[0], yb[1], yb[2],
                     yb[3], yb[4], yb[5], W, pass, L4S, xb[0], xb[1], xb[2], xb[3], xb[4],
                     xb[5], xb[6]);
}

// ---- destruction step (Sec. 2.5, Algorithm 3, eqs. k_des_step, o_des_step,
// beta_star, o_des) ------------------------------------------------------------
// k' = k / Dk, Dk = 1 + tau beta*(Re_t) f_beta*(chi_k) omega, chi_k = (grad k .
// grad omega) / omega-hat^3; omega' = omega / Dw, Dw = 1 + tau beta_i
// f_beta(chi_omega) omega, chi_omega = |X| / (beta*_inf omega-hat)^3 with X
// the vortex stretching a^T S a - |a|^2 tr S (a the axial vector of the
// antisymmetric part of the velocity gradient, S its symmetric part); fixed
// cells keep omega, non-fluid cells keep both.  Pass 1 stores per output cell
// the adjoints of its gradients: of grad k and grad omega (E, six values) and
// of the velocity gradient G (M, nine values); pass 2 gathers, per input
// cell, its own terms and those of the gradients that read it.
namespace {
struct DesLocal {
  double kn, wn;           // outputs
  double dkn_k, dkn_w;     // d k' / d (own k, own omega), gradients held
  double dwn_w;            // d omega' / d own omega, gradient held
  double lam_k;            // d k' / d (grad k . grad omega)
  double lam_w;            // d omega' / d X
};

// The destruction at one fluid cell from its k, omega, the gradients of k
// and omega and the velocity gradient, with the partial derivatives the
// reverse mode needs.
__device__ __forceinline__ DesLocal des_local(const Phys& ph, double tau, double kP, double wP,
                                              const double (&gk)[3], const double (&gw)[3],
                                              const double (&G)[3][3], bool fixed) {
  DesLocal r;
  const bool live = wP > C_EPS;
  const double oh = live ? wP : C_EPS;
  const double ioh = 1.0 / oh, ioh3 = ioh * ioh * ioh;
  const double dkdw = gk[0] * gw[0] + gk[1] * gw[1] + gk[2] * gw[2];
  const double chik = dkdw * ioh3;
  const double q = 1.0 + 400.0 * chik * chik;
  const double fbs = chik <= 0.0 ? 1.0 : (1.0 + 680.0 * chik * chik) / q;
  const double dfbs = chik <= 0.0 ? 0.0 : 560.0 * chik / (q * q);  // d fbs / d chi_k
  const double ret = kP * ioh / ph.nu;
  const double x = ret * (1.0 / C_R_BETA);
  const double x4 = x * x * x * x;
  const double bst = C_BSTAR * (1.0 - (11.0 / 15.0) / (1.0 + x4));
  const double dbst = C_BSTAR * (11.0 / 15.0) / ((1.0 + x4) * (1.0 + x4)) * 4.0 * x * x * x *
                      (1.0 / C_R_BETA);  // d bst / d ret
  const double Dk = 1.0 + tau * bst * fbs * wP;
  r.kn = kP / Dk;
  const double dDk = -kP / (Dk * Dk);  // d k' / d Dk
  const double dret_k = ioh / ph.nu, dret_w = live ? -ret * ioh : 0.0;
  const double dchik_w = live ? -3.0 * chik * ioh : 0.0;
  r.dkn_k = 1.0 / Dk + dDk * tau * fbs * wP * dbst * dret_k;
  r.dkn_w = dDk * tau * (bst * fbs + fbs * wP * dbst * dret_w + bst * wP * dfbs * dchik_w);
  r.lam_k = dDk * tau * bst * wP * dfbs * ioh3;
  r.wn = wP;
  r.dwn_w = 1.0;
  r.lam_w = 0.0;
  if (!fixed) {
    const double a0 = 0.5 * (G[2][1] - G[1][2]), a1 = 0.5 * (G[0][2] - G[2][0]),
                 a2 = 0.5 * (G[1][0] - G[0][1]);
    const double s01 = 0.5 * (G[0][1] + G[1][0]), s02 = 0.5 * (G[0][2] + G[2][0]),
                 s12 = 0.5 * (G[1][2] + G[2][1]);
    const double aSa = a0 * a0 * G[0][0] + a1 * a1 * G[1][1] + a2 * a2 * G[2][2] +
                       2.0 * (a0 * a1 * s01 + a0 * a2 * s02 + a1 * a2 * s12);
    const double X = aSa - (a0 * a0 + a1 * a1 + a2 * a2) * (G[0][0] + G[1][1] + G[2][2]);
    const double c3 = 1.0 / (C_BSTAR * C_BSTAR * C_BSTAR);
    const double chiw = fabs(X) * ioh3 * c3;
    const double fb = (1.0 + 70.0 * chiw) / (1.0 + 80.0 * chiw);
    const double dfb = -10.0 / ((1.0 + 80.0 * chiw) * (1.0 + 80.0 * chiw));
    const double Dw = 1.0 + tau * C_BETA_I * fb * wP;
    r.wn = wP / Dw;
    const double dfbw = -tau * C_BETA_I * wP * wP / (Dw * Dw);  // d omega' / d fb
    r.dwn_w = 1.0 / (Dw * Dw) + dfbw * dfb * (live ? -3.0 * chiw * ioh : 0.0);
    const double sgn = X > 0.0 ? 1.0 : (X < 0.0 ? -1.0 : 0.0);
    r.lam_w = dfbw * dfb * sgn * ioh3 * c3;
  }
  return r;
}

// d X / d G_pq = a_p a_q - |a|^2 delta_pq + the part through a (the axial
// vector), with dX/da = 2 S a - 2 a tr S
__device__ __forceinline__ void stretch_grad(const double (&G)[3][3], double (&dX)[3][3]) {
  const double a[3] = {0.5 * (G[2][1] - G[1][2]), 0.5 * (G[0][2] - G[2][0]),
                       0.5 * (G[1][0] - G[0][1])};
  double S[3][3];
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) S[p][q] = 0.5 * (G[p][q] + G[q][p]);
  const double tr = S[0][0] + S[1][1] + S[2][2];
  const double aa = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
  double ga[3];
  for (int p = 0; p < 3; ++p)
    ga[p] = 2.0 * (S[p][0] * a[0] + S[p][1] * a[1] + S[p][2] * a[2]) - 2.0 * a[p] * tr;
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) dX[p][q] = a[p] * a[q] - (p == q ? aa : 0.0);
  dX[2][1] += 0.5 * ga[0];
  dX[1][2] -= 0.5 * ga[0];
  dX[0][2] += 0.5 * ga[1];
  dX[2][0] -= 0.5 * ga[1];
  dX[1][0] += 0.5 * ga[2];
  dX[0][1] -= 0.5 * ga[2];
}

struct DesState {
  const double *u, *v, *w, *k, *om;  // padded
};

// gradients of k, omega and the velocity at fluid cell P, ghosts substituted
__device__ __forceinline__ void des_gradients(const Geom& g, const Phys& ph, const DesState& S,
                                              const uint8_t* type, const DevPatch* pt, int P,
                                              double (&gk)[3], double (&gw)[3],
                                              double (&G)[3][3]) {
  const int st[3] = {1, g.sx, g.sxy};
  const double ih2[3] = {0.5 / g.hx, 0.5 / g.hy, 0.5 / g.hz};
  const double own[5] = {S.u[P], S.v[P], S.w[P], S.k[P], S.om[P]};
  const int code[5] = {G_U, G_V, G_W, G_K, G_OM};
  for (int d = 0; d < 3; ++d) {
    gk[d] = gw[d] = 0.0;
    for (int a = 0; a < 3; ++a) G[a][d] = 0.0;
  }
  for (int d = 0; d < g.dim; ++d) {
    double val[2][5];
    for (int s = 0; s < 2; ++s) {
      const int Q = P + (s ? 1 : -1) * st[d];
      const uint8_t tq = type[Q];
      if (is_fluid(tq)) {
        val[s][0] = S.u[Q];
        val[s][1] = S.v[Q];
        val[s][2] = S.w[Q];
        val[s][3] = S.k[Q];
        val[s][4] = S.om[Q];
      } else {
        const DevPatch& pp = pt[tq & 0x7f];
        for (int f = 0; f < 5; ++f) val[s][f] = ghost<double>(pp, code[f], own[f], ph.komega);
      }
    }
    for (int a = 0; a < g.dim; ++a) G[a][d] = (val[1][a] - val[0][a]) * ih2[d];
    gk[d] = (val[1][3] - val[0][3]) * ih2[d];
    gw[d] = (val[1][4] - val[0][4]) * ih2[d];
  }
}
}  // namespace

// Pass 1: E (6 padded arrays: d k'/d grad k, d k'/d grad omega, times kbar)
// and M (9: d omega'/d G times wbar) per output cell.
__global__ __launch_bounds__(ABX* ABY) void k_adj_des_weights(
    Geom g, Phys ph, const uint8_t* __restrict__ type, const DevPatch* __restrict__ pt,
    DesState S, double tau, const double* __restrict__ kb, const double* __restrict__ wb,
    double* __restrict__ E, double* __restrict__ M) {
  int i, j, k;
  if (!adj_cell(g, i, j, k)) return;
  const int P = g.idx(i, j, k);
  const size_t D = ((size_t)k * g.ny + j) * g.nx + i;
  const size_t T = (size_t)g.total;
  const uint8_t tp = type[P];
  // formed in registers and stored once (zero where the cell is not fluid)
  double Ev[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double Mv[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (is_fluid(tp)) {
    double gk[3], gw[3], G[3][3];
    des_gradients(g, ph, S, type, pt, P, gk, gw, G);
    const DesLocal r = des_local(ph, tau, S.k[P], S.om[P], gk, gw, G, (tp & FIXED_BIT) != 0);
    const double lk = kb[D] * r.lam_k;
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      Ev[d] = lk * gw[d];
      Ev[3 + d] = lk * gk[d];
    }
    if (r.lam_w != 0.0) {
      double dX[3][3];
      stretch_grad(G, dX);
      const double lw = wb[D] * r.lam_w;
      #pragma unroll
      for (int p = 0; p < 3; ++p)
        #pragma unroll
        for (int q = 0; q < 3; ++q) Mv[3 * p + q] = lw * dX[p][q];
    }
  }
  #pragma unroll
  for (int q = 0; q < 6; ++q) E[q * T + P] = Ev[q];
  #pragma unroll
  for (int q = 0; q < 9; ++q) M[q * T + P] = Mv[q];
}

// Pass 2: the adjoints of the inputs u, v, w, k, omega (dense).
__global__ __launch_bounds__(ABX* ABY) void k_adj_des_gather(
    Geom g, Phys ph, const uint8_t* __restrict__ type, const DevPatch* __restrict__ pt,
    DesState S, double tau, const double* __restrict__ kb, const double* __restrict__ wb,
    const double* __restrict__ E, const double* __restrict__ M, double* __restrict__ xu,
    double* __restrict__ xv, double* __restrict__ xw, double* __restrict__ xk,
    double* __restrict__ xo) {
  int i, j, k;
  if (!adj_cell(g, i, j, k)) return;
  const int P = g.idx(i, j, k);
  const size_t D = ((size_t)k * g.ny + j) * g.nx + i;
  const size_t T = (size_t)g.total;
  const uint8_t tp = type[P];
  double x[5] = {0.0, 0.0, 0.0, kb[D], wb[D]};  // u v w k omega
  if (is_fluid(tp)) {
    double gk[3], gw[3], G[3][3];
    des_gradients(g, ph, S, type, pt, P, gk, gw, G);
    const DesLocal r = des_local(ph, tau, S.k[P], S.om[P], gk, gw, G, (tp & FIXED_BIT) != 0);
    x[3] = kb[D] * r.dkn_k;
    x[4] = kb[D] * r.dkn_w + wb[D] * r.dwn_w;
    const int st[3] = {1, g.sx, g.sxy};
    const double ih2[3] = {0.5 / g.hx, 0.5 / g.hy, 0.5 / g.hz};
    for (int b = 0; b < g.dim; ++b)
      for (int s = 0; s < 2; ++s) {
        const double sg = s ? 1.0 : -1.0;
        const int Q = P + (s ? 1 : -1) * st[b];
        const uint8_t tq = type[Q];
        if (is_fluid(tq)) {
          // this cell is Q's neighbour on Q's side -sg along b
          const double f = -sg * ih2[b];
          x[3] += E[b * T + Q] * f;
          x[4] += E[(3 + b) * T + Q] * f;
          for (int a = 0; a < g.dim; ++a) x[a] += M[(3 * a + b) * T + Q] * f;
        } else {
          // this cell's own gradients read it through the ghost
          const DevPatch& pp = pt[tq & 0x7f];
          const double f = sg * ih2[b];
          x[3] += E[b * T + P] * f * slope(pp, G_K, ph.komega);
          x[4] += E[(3 + b) * T + P] * f * slope(pp, G_OM, ph.komega);
          for (int a = 0; a < g.dim; ++a)
            x[a] += M[(3 * a + b) * T + P] * f * slope(pp, G_U + a, ph.komega);
        }
      }
  }
  xu[D] = x[0];
  xv[D] = x[1];
  xw[D] = x[2];
  xk[D] = x[3];
  xo[D] = x[4];
}

void launch_destroy_adjoint(const Geom& g, const Phys& ph, const uint8_t* type,
                            const DevPatch* pt, const double* const st[5], double tau,
                            const double* kb, const double* wb, double* E, double* M,
                            double* const xb[5], hipStream_t s) {
  const DesState S{st[0], st[1], st[2], st[3], st[4]};
  const dim3 G = adj_grid(g), B(ABX, ABY);
  hipLaunchKernelGGL(k_adj_des_weights, G, B, 0, s, g, ph, type, pt, S, tau, kb, wb, E, M);
  hipLaunchKernelGGL(k_adj_des_gather, G, B, 0, s, g, ph, type, pt, S, tau, kb, wb, E, M, xb[0],
                     xb[1], xb[2], xb[3], xb[4]);
}

// ---- helpers of the whole step's reverse mode ------------------------------------
__global__ void k_dense_add(size_t n, const double* __restrict__ a, const double* __restrict__ b,
                            double* __restrict__ out, double scale) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) out[q] = scale * (a[q] + b[q]);
}
// out = scale (a + b) over n dense values (scale 1 leaves the sum as formed)
void launch_dense_add(size_t n, const double* a, const double* b, double* out, hipStream_t s,
                      double scale) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_dense_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, b,
                     out, scale);
}

__global__ void k_zero_held(Geom g, const uint8_t* __restrict__ type, double* __restrict__ a) {
  const int i = blockIdx.x * ABX + threadIdx.x, j = blockIdx.y * ABY + threadIdx.y,
            k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const uint8_t t = type[g.idx(i, j, k)];
  if (is_fluid(t) && (t & FIXED_BIT)) a[((size_t)k * g.ny + j) * g.nx + i] = 0.0;
}
// zero the dense adjoint a on the wall-adjacent cells whose omega is held
void launch_zero_held(const Geom& g, const uint8_t* type, double* a, hipStream_t s) {
  const dim3 G((g.nx + ABX - 1) / ABX, (g.ny + ABY - 1) / ABY, g.nz), B(ABX, ABY);
  hipLaunchKernelGGL(k_zero_held, G, B, 0, s, g, type, a);
}

}  // namespace nfvm
