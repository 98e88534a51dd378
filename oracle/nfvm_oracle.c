/*
 * Serial FP64 reference for one NeuralFVM time step.  TEST INFRASTRUCTURE
 * ONLY: the product library never calls it.  Plain loops, no blocking, no
 * fusion; each routine names the passage of the paper it writes out.
 *
 * Readings of the paper where it is silent (constants, ghost rules, stage
 * order, multigrid components) are the ones recorded in the design notes;
 * they are repeated next to the code that uses them.
 */
#include "nfvm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- model constants: Sec. 2.1 (eqs. a_star, Re_t, k_gen, o_gen, a,
 *      beta_star, o_des).  R_beta is not printed in the paper; the value 8
 *      is the standard low-Reynolds k-omega constant (reading). ---------- */
#define BETA_I 0.072
#define BSTAR_INF 0.09
#define ASTAR_INF 1.0
#define ASTAR_0 (BETA_I / 3.0)
#define R_K 6.0
#define A_INF 0.52
#define A_0 (1.0 / 9.0)
#define R_W 2.95
#define R_BETA 8.0
#define EPS 1e-10 /* guard in max(omega, eps) and the k/omega clamp (reading) */

enum { F_U = 0, F_V = 1, F_W = 2, F_P, F_T, F_K, F_OM, F_NUT };

static int cidx(const orc_case* c, int i, int j, int k) {
  return (k * c->n[1] + j) * c->n[0] + i;
}
static int ncells(const orc_case* c) { return c->n[0] * c->n[1] * c->n[2]; }
static int is_fluid(const orc_case* c, int id) { return !(c->solid && c->solid[id]); }
static double omhat(double om) { return om > EPS ? om : EPS; }

/* ---------------------------------------------------------------------------
 * Neighbour classification (Sec. 2.7, boundary conditions).  A face of a
 * fluid cell either touches another fluid cell, a solid cell (internal
 * boundary: a wall, held at T_solid), or the outside of the box, where the
 * first patch covering the face decides the kind (default: adiabatic wall).
 * ------------------------------------------------------------------------- */
typedef struct {
  int fluid, idx, kind, solid;
  const orc_patch* patch;
} nbinfo;

static const orc_patch* find_patch(const orc_case* c, int dir, int t0, int t1) {
  for (int q = 0; q < c->n_patches; ++q) {
    const orc_patch* p = &c->patches[q];
    if (p->face == dir && t0 >= p->lo[0] && t0 < p->hi[0] && t1 >= p->lo[1] && t1 < p->hi[1])
      return p;
  }
  return NULL;
}

static nbinfo neighbour(const orc_case* c, int i, int j, int k, int dir) {
  nbinfo r;
  memset(&r, 0, sizeof r);
  int d = dir / 2, s = (dir & 1) ? 1 : -1;
  int q[3] = {i, j, k};
  q[d] += s;
  if (q[d] < 0 || q[d] >= c->n[d]) {
    int t0, t1;
    if (d == 0) { t0 = j; t1 = k; }
    else if (d == 1) { t0 = i; t1 = k; }
    else { t0 = i; t1 = j; }
    r.patch = find_patch(c, dir, t0, t1);
    r.kind = r.patch ? r.patch->kind : ORC_WALL;
    return r;
  }
  int id = cidx(c, q[0], q[1], q[2]);
  if (!is_fluid(c, id)) {
    r.kind = ORC_WALL;
    r.solid = 1;
    return r;
  }
  r.fluid = 1;
  r.idx = id;
  return r;
}

/* closure: eqs. a_star and Re_t, then eq. ko_turb_diff (nu_t = alpha* k / omega) */
static double alpha_star(double Re_t) {
  return ASTAR_INF * (ASTAR_0 + Re_t / R_K) / (1.0 + Re_t / R_K);
}
static double nut_point(double nu, double k, double om) {
  double oh = omhat(om);
  double Re_t = k / (nu * oh);
  return alpha_star(Re_t) * k / oh;
}

void orc_closure_point(double nu, double k, double om, double out[4]) {
  double oh = omhat(om);
  double Re_t = k / (nu * oh);
  double as = alpha_star(Re_t);
  double x4 = pow(Re_t / R_BETA, 4.0);
  out[0] = as;
  out[1] = as * k / oh;
  out[2] = (A_INF / as) * (A_0 + Re_t / R_W) / (1.0 + Re_t / R_W); /* eq. a */
  out[3] = BSTAR_INF * (4.0 / 15.0 + x4) / (1.0 + x4);            /* eq. beta_star */
}

/* Ghost value across a boundary face (Sec. 2.7).  Dirichlet value b on the
 * face: ghost = 2b - phi_P (the face average is b); zero gradient:
 * ghost = phi_P.  Per field:
 *   velocity  wall/solid 0, inlet U, outlet zero-gradient;
 *   pressure  zero-gradient, outlet 0;
 *   T         wall T_wall (adiabatic if NaN), inlet T, outlet zero-gradient;
 *   k, omega  wall zero-gradient (omega fixed in the wall cell), inlet value;
 *   nu_t      wall 0, inlet nu_t(k_in, omega_in), outlet zero-gradient. */
static double ghost(const orc_case* c, const nbinfo* nb, int fld, double vP) {
  const orc_patch* p = nb->patch;
  int kind = nb->kind;
  switch (fld) {
    case F_U: case F_V: case F_W:
      if (kind == ORC_INLET) return 2.0 * p->U[fld - F_U] - vP;
      if (kind == ORC_OUTLET) return vP;
      return -vP;
    case F_P:
      return kind == ORC_OUTLET ? -vP : vP;
    case F_T: {
      if (kind == ORC_INLET) return 2.0 * p->T - vP;
      if (kind == ORC_OUTLET) return vP;
      double Tw = nb->solid ? c->T_solid : (p ? p->T_wall : NAN);
      return isnan(Tw) ? vP : 2.0 * Tw - vP;
    }
    case F_K:
      return kind == ORC_INLET ? 2.0 * p->k - vP : vP;
    case F_OM:
      return kind == ORC_INLET ? 2.0 * p->omega - vP : vP;
    case F_NUT:
      if (!(c->physics & ORC_KOMEGA)) return 0.0;
      if (kind == ORC_INLET) return 2.0 * nut_point(c->nu, p->k, p->omega) - vP;
      if (kind == ORC_OUTLET) return vP;
      return -vP;
  }
  return vP;
}

static double nbval(const orc_case* c, const nbinfo* nb, const double* a, int fld, int P) {
  return nb->fluid ? a[nb->idx] : ghost(c, nb, fld, a[P]);
}

/* Wall treatment (Sec. 2.7): in a fluid cell touching a wall or a solid,
 * omega is held at 6 nu / (beta_i d^2), d = half the cell width normal to
 * that wall (the smallest one when several walls touch the cell). */
void orc_fixed_omega(const orc_case* c, double* omega) {
  if (!(c->physics & ORC_KOMEGA)) return;
  for (int k = 0; k < c->n[2]; ++k)
    for (int j = 0; j < c->n[1]; ++j)
      for (int i = 0; i < c->n[0]; ++i) {
        int P = cidx(c, i, j, k);
        if (!is_fluid(c, P)) continue;
        double dmin = INFINITY;
        for (int dir = 0; dir < 2 * c->dim; ++dir) {
          nbinfo nb = neighbour(c, i, j, k, dir);
          if (!nb.fluid && nb.kind == ORC_WALL) {
            double d = 0.5 * c->h[dir / 2];
            if (d < dmin) dmin = d;
          }
        }
        if (dmin < INFINITY) omega[P] = 6.0 * c->nu / (BETA_I * dmin * dmin);
      }
}

static int is_fixed(const orc_case* c, int i, int j, int k) {
  if (!(c->physics & ORC_KOMEGA)) return 0;
  for (int dir = 0; dir < 2 * c->dim; ++dir) {
    nbinfo nb = neighbour(c, i, j, k, dir);
    if (!nb.fluid && nb.kind == ORC_WALL) return 1;
  }
  return 0;
}

/* The boundary classification of every fluid cell as tables: per cell P
 * and face direction dir (0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+),
 * nidx[6P + dir] is the neighbour's index, or -1 where the face takes a
 * ghost value, whose rule is affine in the cell's own value: ghost =
 * a0 + a1 value_P for field fld (F_U .. F_NUT) at a0/a1[8 (6P + dir) + fld];
 * fixed[P] flags the cells whose omega is held (wall-adjacent).  The
 * reverse mode of the explicit stage is differentiated through these. */
void orc_ghost_table(const orc_case* c, int* nidx, double* a0, double* a1,
                     unsigned char* fixed) {
  for (int k = 0; k < c->n[2]; ++k)
    for (int j = 0; j < c->n[1]; ++j)
      for (int i = 0; i < c->n[0]; ++i) {
        int P = cidx(c, i, j, k);
        fixed[P] = is_fluid(c, P) ? (unsigned char)is_fixed(c, i, j, k) : 0;
        for (int dir = 0; dir < 6; ++dir) {
          int e = 6 * P + dir;
          nidx[e] = -1;
          for (int f = 0; f < 8; ++f) a0[8 * e + f] = a1[8 * e + f] = 0.0;
          if (!is_fluid(c, P) || dir >= 2 * c->dim) continue;
          nbinfo nb = neighbour(c, i, j, k, dir);
          if (nb.fluid) {
            nidx[e] = nb.idx;
            continue;
          }
          for (int f = 0; f < 8; ++f) {
            double g0 = ghost(c, &nb, f, 0.0);
            a0[8 * e + f] = g0;
            a1[8 * e + f] = ghost(c, &nb, f, 1.0) - g0;
          }
        }
      }
}

void orc_nut(const orc_case* c, const double* k, const double* om, double* nut) {
  int N = ncells(c);
  for (int P = 0; P < N; ++P)
    nut[P] = ((c->physics & ORC_KOMEGA) && is_fluid(c, P)) ? nut_point(c->nu, k[P], om[P]) : 0.0;
}

/* Cell-centred gradient of one field: face derivative D then average L
 * (Algorithm 3), i.e. (phi_E - phi_W) / (2 h) with ghosts at boundaries. */
static double cgrad(const orc_case* c, const double* a, int fld, int i, int j, int k, int d) {
  if (d >= c->dim) return 0.0;
  int P = cidx(c, i, j, k);
  nbinfo m = neighbour(c, i, j, k, 2 * d), p = neighbour(c, i, j, k, 2 * d + 1);
  return (nbval(c, &p, a, fld, P) - nbval(c, &m, a, fld, P)) / (2.0 * c->h[d]);
}

/* velocity gradient G[a][b] = d u_a / d x_b */
static void velgrad(const orc_case* c, const double* u, const double* v, const double* w, int i,
                    int j, int k, double G[3][3]) {
  const double* vel[3] = {u, v, w};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      G[a][b] = (a < c->dim) ? cgrad(c, vel[a], F_U + a, i, j, k, b) : 0.0;
}

/* Velocity gradient of every cell, G[a][b] = d u_a / d x_b as nine values
 * per cell (row-major), with the central gradient and boundary ghosts of
 * Algorithm 3; zero on non-fluid cells.  Post-processing input: the lambda2
 * vortex criterion of Sec. 3.2 is formed from it. */
void orc_velocity_gradient(const orc_case* c, const double* u, const double* v,
                           const double* w, double* G9) {
  for (int k = 0; k < c->n[2]; ++k)
    for (int j = 0; j < c->n[1]; ++j)
      for (int i = 0; i < c->n[0]; ++i) {
        int P = cidx(c, i, j, k);
        double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        if (is_fluid(c, P)) velgrad(c, u, v, w, i, j, k, G);
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) G9[9 * (size_t)P + 3 * a + b] = G[a][b];
      }
}

/* S^2 = 2 S_ij S_ij (eqs. strain_rate_magnitude, strain_rate) */
static double strain2(double G[3][3]) {
  double s = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double Sab = 0.5 * (G[a][b] + G[b][a]);
      s += Sab * Sab;
    }
  return 2.0 * s;
}

/* Face-flux divergence of one transported field at cell P (Sec. 2.3,
 * Algorithms 2 and 4): upwind convection with the lower cell taken when the
 * face velocity is >= 0, central diffusion Gamma_f (phi_N - phi_P)/h with
 * Gamma_f = gamma0 + L(nu_t)/sigma, and for momentum component q the face
 * term -(p + 2/3 k)_f on the q-faces (eq. ko_mom); then the divergence
 * theorem (eq. divergence_theorem). */
static double transport(const orc_case* c, const orc_fields* s, const double* nut,
                        const double* phi, int fld, double gamma0, double inv_sigma, int i,
                        int j, int k, int q) {
  const double* vel[3] = {s->u, s->v, s->w};
  int P = cidx(c, i, j, k);
  double rhs = 0.0;
  for (int d = 0; d < c->dim; ++d)
    for (int side = -1; side <= 1; side += 2) {
      int dir = 2 * d + (side > 0);
      nbinfo nb = neighbour(c, i, j, k, dir);
      double Uf = 0.5 * (vel[d][P] + nbval(c, &nb, vel[d], F_U + d, P));
      double phN = nbval(c, &nb, phi, fld, P);
      double lower = side < 0 ? phN : phi[P];
      double upper = side < 0 ? phi[P] : phN;
      double up = Uf >= 0.0 ? lower : upper;
      double nutf = 0.5 * (nut[P] + nbval(c, &nb, nut, F_NUT, P));
      double Gam = gamma0 + nutf * inv_sigma;
      double F = -Uf * up + Gam * (upper - lower) / c->h[d];
      if (q == d) {
        double pf = 0.5 * (s->p[P] + nbval(c, &nb, s->p, F_P, P));
        double kf = (c->physics & ORC_KOMEGA) ? 0.5 * (s->k[P] + nbval(c, &nb, s->k, F_K, P)) : 0.0;
        F -= pf + (2.0 / 3.0) * kf;
      }
      rhs += side * F / c->h[d];
    }
  return rhs;
}

/* Right-hand sides of the explicitly advanced terms ("rest" terms):
 * momentum (eq. ko_mom, plus Boussinesq buoyancy -beta_T (T - T_ref) g),
 * energy (eq. ko_temp), k and omega without destruction (eqs. ko_k, ko_o):
 * G_k = nu_t S^2, G_omega = alpha (omega/k) G_k, which with nu_t = alpha* k/omega
 * equals alpha_inf (alpha_0 + Re_t/R_w)/(1 + Re_t/R_w) S^2 (eqs. k_gen, o_gen, a). */
void orc_explicit_rhs(const orc_case* c, const orc_fields* s, orc_fields* r) {
  int N = ncells(c);
  double* nut = (double*)malloc(sizeof(double) * N);
  orc_nut(c, s->k, s->omega, nut);
  const double* vel[3] = {s->u, s->v, s->w};
  double* rv[3] = {r->u, r->v, r->w};
  int komega = c->physics & ORC_KOMEGA;
  for (int k = 0; k < c->n[2]; ++k)
    for (int j = 0; j < c->n[1]; ++j)
      for (int i = 0; i < c->n[0]; ++i) {
        int P = cidx(c, i, j, k);
        r->u[P] = r->v[P] = r->w[P] = r->p[P] = r->T[P] = r->k[P] = r->omega[P] = 0.0;
        if (!is_fluid(c, P)) continue;
        for (int a = 0; a < c->dim; ++a) {
          double src = 0.0;
          if (c->physics & ORC_BUOYANCY) src = -c->beta_T * (s->T[P] - c->T_ref) * c->gravity[a];
          rv[a][P] = transport(c, s, nut, vel[a], F_U + a, c->nu, 1.0, i, j, k, a) + src;
        }
        if (c->physics & ORC_ENERGY)
          r->T[P] = transport(c, s, nut, s->T, F_T, c->alpha_T, 1.0 / c->Pr_t, i, j, k, -1);
        if (komega) {
          double G[3][3];
          velgrad(c, s->u, s->v, s->w, i, j, k, G);
          double S2 = strain2(G);
          double Re_t = s->k[P] / (c->nu * omhat(s->omega[P]));
          double Gk = nut[P] * S2;
          double Gw = A_INF * (A_0 + Re_t / R_W) / (1.0 + Re_t / R_W) * S2;
          r->k[P] = transport(c, s, nut, s->k, F_K, c->nu, 1.0 / c->sigma_k, i, j, k, -1) + Gk;
          r->omega[P] =
              transport(c, s, nut, s->omega, F_OM, c->nu, 1.0 / c->sigma_w, i, j, k, -1) + Gw;
        }
      }
  free(nut);
}

/* One forward-Euler step of the rest terms (the paper's explicit
 * Runge-Kutta of unstated order, read as first order), with k and omega
 * clamped to stay positive (appendix, explicit time stepping); solid cells and
 * wall-fixed omega cells keep their values. */
static void explicit_euler(const orc_case* c, const orc_fields* s, orc_fields* o) {
  int N = ncells(c);
  orc_fields r;
  double* buf = (double*)malloc(sizeof(double) * 7 * N);
  r.u = buf; r.v = buf + N; r.w = buf + 2 * N; r.p = buf + 3 * N;
  r.T = buf + 4 * N; r.k = buf + 5 * N; r.omega = buf + 6 * N;
  orc_explicit_rhs(c, s, &r);
  double dt = c->dt;
  for (int k = 0; k < c->n[2]; ++k)
    for (int j = 0; j < c->n[1]; ++j)
      for (int i = 0; i < c->n[0]; ++i) {
        int P = cidx(c, i, j, k);
        o->u[P] = s->u[P]; o->v[P] = s->v[P]; o->w[P] = s->w[P]; o->p[P] = s->p[P];
        o->T[P] = s->T[P]; o->k[P] = s->k[P]; o->omega[P] = s->omega[P];
        if (!is_fluid(c, P)) continue;
        o->u[P] = s->u[P] + dt * r.u[P];
        if (c->dim > 1) o->v[P] = s->v[P] + dt * r.v[P];
        if (c->dim > 2) o->w[P] = s->w[P] + dt * r.w[P];
        if (c->physics & ORC_ENERGY) o->T[P] = s->T[P] + dt * r.T[P];
        if (c->physics & ORC_KOMEGA) {
          double kn = s->k[P] + dt * r.k[P];
          o->k[P] = kn > EPS ? kn : EPS;
          if (!is_fixed(c, i, j, k)) {
            double wn = s->omega[P] + dt * r.omega[P];
            o->omega[P] = wn > EPS ? wn : EPS;
          }
        }
      }
  free(buf);
}

/* The explicit stage (Algorithms 2 and 4): one forward-Euler step, or with
 * rk_order = 2 Heun's method written as the average of the start and a
 * second Euler step taken from the first one (nu_t of the second from the
 * first stage's k and omega; each stage clamps k and omega). */
void orc_explicit(const orc_case* c, const orc_fields* s, orc_fields* o) {
  explicit_euler(c, s, o);
  if (c->rk_order != 2) return;
  int N = ncells(c);
  double* buf = (double*)malloc(sizeof(double) * 7 * N);
  orc_fields t;
  t.u = buf; t.v = buf + N; t.w = buf + 2 * N; t.p = buf + 3 * N;
  t.T = buf + 4 * N; t.k = buf + 5 * N; t.omega = buf + 6 * N;
  explicit_euler(c, o, &t);
  for (int P = 0; P < N; ++P) {
    o->u[P] = 0.5 * (s->u[P] + t.u[P]);
    o->v[P] = 0.5 * (s->v[P] + t.v[P]);
    o->w[P] = 0.5 * (s->w[P] + t.w[P]);
    o->T[P] = 0.5 * (s->T[P] + t.T[P]);
    o->k[P] = 0.5 * (s->k[P] + t.k[P]);
    o->omega[P] = 0.5 * (s->omega[P] + t.omega[P]);
  }
  free(buf);
}

/* Semi-implicit destruction over a time tau (Sec. 2.5, eqs. k_des_step and
 * o_des_step, Algorithm 3).  All right-hand sides use the input k and omega.
 * chi_omega uses (beta*_inf max(omega, eps))^3 as in eq. o_des. */
void orc_destroy(const orc_case* c, const double* u, const double* v, const double* w,
                 const double* kk, const double* om, double tau, double* k_out,
                 double* om_out) {
  for (int k = 0; k < c->n[2]; ++k)
    for (int j = 0; j < c->n[1]; ++j)
      for (int i = 0; i < c->n[0]; ++i) {
        int P = cidx(c, i, j, k);
        k_out[P] = kk[P];
        om_out[P] = om[P];
        if (!is_fluid(c, P)) continue;
        double oh = omhat(om[P]);
        double dkdo = 0.0;
        for (int d = 0; d < c->dim; ++d)
          dkdo += cgrad(c, kk, F_K, i, j, k, d) * cgrad(c, om, F_OM, i, j, k, d);
        double chik = dkdo / (oh * oh * oh);
        double fbs = chik <= 0.0 ? 1.0 : (1.0 + 680.0 * chik * chik) / (1.0 + 400.0 * chik * chik);
        double Re_t = kk[P] / (c->nu * oh);
        double x4 = pow(Re_t / R_BETA, 4.0);
        double bstar = BSTAR_INF * (4.0 / 15.0 + x4) / (1.0 + x4);
        k_out[P] = kk[P] / (1.0 + tau * bstar * fbs * om[P]);
        if (is_fixed(c, i, j, k)) continue;
        double G[3][3], S[3][3], W[3][3];
        velgrad(c, u, v, w, i, j, k, G);
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            S[a][b] = 0.5 * (G[a][b] + G[b][a]);
            W[a][b] = 0.5 * (G[a][b] - G[b][a]);
          }
        double X = 0.0; /* Omega_ij Omega_jk S_ki */
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b)
            for (int e = 0; e < 3; ++e) X += W[a][b] * W[b][e] * S[e][a];
        double den = BSTAR_INF * oh;
        double chiw = fabs(X) / (den * den * den);
        double fb = (1.0 + 70.0 * chiw) / (1.0 + 80.0 * chiw);
        om_out[P] = om[P] / (1.0 + tau * BETA_I * fb * om[P]);
      }
}

/* Face velocity of component d on the face between a fluid cell and its
 * neighbour in direction dir: L of the ghost-padded velocity. */
static double face_u(const orc_case* c, const double* a, int d, int i, int j, int k, int dir) {
  int P = cidx(c, i, j, k);
  nbinfo nb = neighbour(c, i, j, k, dir);
  return 0.5 * (a[P] + nbval(c, &nb, a, F_U + d, P));
}

/* Poisson right-hand side b = -(1/dt) sum_d D_d L_d BC_d(u*_d)
 * (eq. pc_residual, Algorithm 1 first lines). */
void orc_rhs_b(const orc_case* c, const double* us, const double* vs, const double* ws,
               double* b) {
  const double* vel[3] = {us, vs, ws};
  for (int k = 0; k < c->n[2]; ++k)
    for (int j = 0; j < c->n[1]; ++j)
      for (int i = 0; i < c->n[0]; ++i) {
        int P = cidx(c, i, j, k);
        b[P] = 0.0;
        if (!is_fluid(c, P)) continue;
        double div = 0.0;
        for (int d = 0; d < c->dim; ++d)
          div += (face_u(c, vel[d], d, i, j, k, 2 * d + 1) - face_u(c, vel[d], d, i, j, k, 2 * d)) /
                 c->h[d];
        b[P] = -div / c->dt;
      }
}

/* Coefficient of the pressure operator on the face of a fluid cell in
 * direction dir: 1 to a fluid neighbour, 0 for zero-gradient faces (walls,
 * inlets, solids), 2 for the zero-value outlet face (ghost -phi_P), whose
 * neighbour value then counts as 0 (eqs. neg_lap_discretize, pc_discretized). */
static double face_coef(const orc_case* c, int i, int j, int k, int dir, int* nidx) {
  nbinfo nb = neighbour(c, i, j, k, dir);
  *nidx = nb.fluid ? nb.idx : -1;
  if (nb.fluid) return 1.0;
  return nb.kind == ORC_OUTLET ? 2.0 : 0.0;
}

/* Projection (Sec. 2.4): p^{n+1} = p^n + phi and u = u* - dt * grad(phi),
 * the gradient being the cell-centred central one used for the pressure
 * term; the face fluxes L(u*) - dt * c_f D(phi) are returned as the largest
 * cell divergence. */
void orc_project(const orc_case* c, const double* phi, const double* us, const double* vs,
                 const double* ws, double* p, double* u, double* v, double* w,
                 double* max_face_div) {
  const double* vs3[3] = {us, vs, ws};
  double* vo[3] = {u, v, w};
  double mdiv = 0.0;
  for (int k = 0; k < c->n[2]; ++k)
    for (int j = 0; j < c->n[1]; ++j)
      for (int i = 0; i < c->n[0]; ++i) {
        int P = cidx(c, i, j, k);
        for (int a = 0; a < 3; ++a) vo[a][P] = vs3[a][P];
        if (!is_fluid(c, P)) continue;
        double div = 0.0;
        for (int d = 0; d < c->dim; ++d) {
          vo[d][P] = vs3[d][P] - c->dt * cgrad(c, phi, F_P, i, j, k, d);
          for (int side = -1; side <= 1; side += 2) {
            int dir = 2 * d + (side > 0), nidx;
            double cf = face_coef(c, i, j, k, dir, &nidx);
            double phN = nidx >= 0 ? phi[nidx] : 0.0;
            double dphi = side > 0 ? (phN - phi[P]) : (phi[P] - phN);
            double F = face_u(c, vs3[d], d, i, j, k, dir) - c->dt * cf * dphi / c->h[d];
            div += side * F / c->h[d];
          }
        }
        p[P] += phi[P];
        if (fabs(div) > mdiv) mdiv = fabs(div);
      }
  if (max_face_div) *max_face_div = mdiv;
}

/* Slope of a ghost rule: the ghost value is affine in the cell's own value,
 * ghost = s phi_P + const, and s = ghost(1) - ghost(0). */
static double ghost_slope(const orc_case* c, const nbinfo* nb, int fld) {
  return ghost(c, nb, fld, 1.0) - ghost(c, nb, fld, 0.0);
}

/* Reverse mode of the pressure step: each forward formula of orc_rhs_b and
 * orc_project is taken term by term and its partial derivative scattered
 * onto the value it reads (a fluid neighbour, or the cell itself through the
 * slope of a ghost rule). */
static int pressure_adjoint_with(const orc_case* c, const orc_mg* mg, const double* ubar,
                                 const double* vbar, const double* wbar, const double* pbar,
                                 double tol, int max_cycles, int forced, double* usbar,
                                 double* vsbar, double* wsbar, double* phibar_out,
                                 double* lambda_out, int* cycles, double* rel) {
  const int N = ncells(c);
  const double* ub[3] = {ubar, vbar, wbar};
  double* usb[3] = {usbar, vsbar, wsbar};
  double* phib = (double*)calloc(N, sizeof(double));
  double* lam = (double*)calloc(N, sizeof(double));
  /* u_d = u*_d - dt (phi~_+ - phi~_-) / (2 h_d) on fluid cells, p += phi:
   * phibar = pbar + d/dphi of the velocity outputs */
  for (int k = 0; k < c->n[2]; ++k)
    for (int j = 0; j < c->n[1]; ++j)
      for (int i = 0; i < c->n[0]; ++i) {
        int P = cidx(c, i, j, k);
        if (!is_fluid(c, P)) continue;
        phib[P] += pbar[P];
        for (int d = 0; d < c->dim; ++d) {
          double g = -c->dt * ub[d][P] / (2.0 * c->h[d]);
          nbinfo hi = neighbour(c, i, j, k, 2 * d + 1), lo = neighbour(c, i, j, k, 2 * d);
          if (hi.fluid) phib[hi.idx] += g;
          else phib[P] += g * ghost_slope(c, &hi, F_P);
          if (lo.fluid) phib[lo.idx] -= g;
          else phib[P] -= g * ghost_slope(c, &lo, F_P);
        }
      }
  /* lambda = A^-T phibar = A^-1 phibar (A symmetric) */
  int st = orc_mg_solve(mg, phib, lam, tol, max_cycles, forced, cycles, rel);
  /* b_P = -(1/dt) sum_d (uf_+ - uf_-) / h_d, uf = (u*_P + u~_N) / 2:
   * usbar = ubar (u = u* + correction) + d/du* of b, weighted by lambda */
  for (int d = 0; d < 3; ++d)
    for (int P = 0; P < N; ++P) usb[d][P] = ub[d][P];
  for (int k = 0; k < c->n[2]; ++k)
    for (int j = 0; j < c->n[1]; ++j)
      for (int i = 0; i < c->n[0]; ++i) {
        int P = cidx(c, i, j, k);
        if (!is_fluid(c, P)) continue;
        for (int d = 0; d < c->dim; ++d) {
          double s = -lam[P] / (c->dt * c->h[d]);
          for (int side = -1; side <= 1; side += 2) {
            nbinfo nb = neighbour(c, i, j, k, 2 * d + (side > 0));
            double gf = side * 0.5 * s; /* d b_P / d uf of this face, times 1/2 */
            usb[d][P] += gf;
            if (nb.fluid) usb[d][nb.idx] += gf;
            else usb[d][P] += gf * ghost_slope(c, &nb, F_U + d);
          }
        }
      }
  if (phibar_out) memcpy(phibar_out, phib, sizeof(double) * N);
  if (lambda_out) memcpy(lambda_out, lam, sizeof(double) * N);
  free(phib);
  free(lam);
  return st;
}

/* ===========================================================================
 * Geometric multigrid for A phi = b (Sec. 2.4, Algorithm 1).
 *
 * Reading of the cycle: a V(nu1, nu2) cycle with damped Jacobi
 * (eq. jacobi_pc with the diagonal of the operator and weight omega_J),
 * restriction RES = mean of the 2^dim children ("pooling"), prolongation PROL
 * = cell-centred (bi/tri)linear interpolation with weights 3/4, 1/4 per axis
 * ("upsampling"), and an exact solve on the coarsest level.  Coarse levels
 * halve every axis; a coarse cell is active when any child is; a coarse face
 * coefficient is the mean of the fine sub-face coefficients it covers.
 * ========================================================================= */
typedef struct {
  int n[3];
  double h[3];
  unsigned char* act;
  double* cf[3]; /* face coefficients, face q along d sits between cells q-1 and q */
} orc_level;

struct orc_mg {
  int dim, L, nu1, nu2, nuc, prolong, literal;
  double wj;
  orc_level lv[24];
  int nc;        /* active cells on the coarsest level */
  int* cmap;     /* their cell indices */
  double* lu;    /* dense LU factors, nc x nc */
  int* piv;
};

static int lcells(const orc_level* l) { return l->n[0] * l->n[1] * l->n[2]; }
static int lidx(const orc_level* l, int i, int j, int k) { return (k * l->n[1] + j) * l->n[0] + i; }
static int fidx(const orc_level* l, int d, int i, int j, int k) {
  int e0 = d == 0, e1 = d == 1;
  return (k * (l->n[1] + e1) + j) * (l->n[0] + e0) + i;
}
static int fcount(const orc_level* l, int d) {
  return (l->n[0] + (d == 0)) * (l->n[1] + (d == 1)) * (l->n[2] + (d == 2));
}

/* operator value contributed by the face in direction dir of cell (i,j,k):
 * coefficient and neighbour index (-1 outside the box) */
static double lface(const orc_level* l, int d, int side, int i, int j, int k, int* nidx) {
  int q[3] = {i, j, k};
  int fq[3] = {i, j, k};
  if (side > 0) fq[d] += 1;
  q[d] += side;
  *nidx = (q[d] >= 0 && q[d] < l->n[d]) ? lidx(l, q[0], q[1], q[2]) : -1;
  return l->cf[d][fidx(l, d, fq[0], fq[1], fq[2])];
}

static double ldiag(const orc_mg* mg, const orc_level* l, int i, int j, int k) {
  double D = 0.0;
  int nidx;
  if (mg->literal) {
    /* eq. jacobi_pc: D replaced by the scalar 6/dx^2 (2 sum_d 1/h_d^2 with
     * unequal spacings), whatever the cell's faces */
    for (int d = 0; d < mg->dim; ++d) D += 2.0 / (l->h[d] * l->h[d]);
    return D;
  }
  for (int d = 0; d < mg->dim; ++d)
    for (int s = -1; s <= 1; s += 2) D += lface(l, d, s, i, j, k, &nidx) / (l->h[d] * l->h[d]);
  return D;
}

void orc_mg_apply(const orc_mg* mg, int li, const double* x, double* y) {
  const orc_level* l = &mg->lv[li];
  for (int k = 0; k < l->n[2]; ++k)
    for (int j = 0; j < l->n[1]; ++j)
      for (int i = 0; i < l->n[0]; ++i) {
        int P = lidx(l, i, j, k);
        y[P] = 0.0;
        if (!l->act[P]) continue;
        double s = 0.0;
        for (int d = 0; d < mg->dim; ++d)
          for (int sd = -1; sd <= 1; sd += 2) {
            int nidx;
            double cf = lface(l, d, sd, i, j, k, &nidx);
            double xn = nidx >= 0 ? x[nidx] : 0.0;
            s += cf * (x[P] - xn) / (l->h[d] * l->h[d]);
          }
        y[P] = s;
      }
}

void orc_mg_smooth(const orc_mg* mg, int li, double* x, const double* b, int sweeps) {
  const orc_level* l = &mg->lv[li];
  int N = lcells(l);
  double* Ax = (double*)malloc(sizeof(double) * N);
  for (int s = 0; s < sweeps; ++s) {
    orc_mg_apply(mg, li, x, Ax);
    for (int k = 0; k < l->n[2]; ++k)
      for (int j = 0; j < l->n[1]; ++j)
        for (int i = 0; i < l->n[0]; ++i) {
          int P = lidx(l, i, j, k);
          if (!l->act[P]) continue;
          x[P] += mg->wj * (b[P] - Ax[P]) / ldiag(mg, l, i, j, k);
        }
  }
  free(Ax);
}

void orc_mg_restrict(const orc_mg* mg, int li, const double* r, double* bc) {
  const orc_level* f = &mg->lv[li];
  const orc_level* c = &mg->lv[li + 1];
  int kz = mg->dim == 3 ? 2 : 1;
  double w = mg->dim == 3 ? 0.125 : 0.25;
  for (int K = 0; K < c->n[2]; ++K)
    for (int J = 0; J < c->n[1]; ++J)
      for (int I = 0; I < c->n[0]; ++I) {
        double s = 0.0;
        for (int c2 = 0; c2 < kz; ++c2)
          for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
              int P = lidx(f, 2 * I + a, 2 * J + b, kz * K + c2);
              if (f->act[P]) s += r[P];
            }
        bc[lidx(c, I, J, K)] = w * s;
      }
}

/* value of the coarse correction one cell beyond cell q along axis d on the
 * side sgn, for the 1D linear interpolation along d: the neighbour's value
 * when it is an active cell, the cell's own value when the neighbour is an
 * inactive (solid) cell (mirror), and the boundary ghost (1 - c_f) v when it
 * lies outside the box (c_f = 0: zero gradient, c_f = 2: zero value on the
 * face, as on the fine level). */
static int in_box(const orc_level* l, const int q[3]) {
  for (int d = 0; d < 3; ++d)
    if (q[d] < 0 || q[d] >= l->n[d]) return 0;
  return 1;
}

/* Prolongation (PROL, eq. prolongation): cell-centred linear interpolation
 * applied axis by axis (x, then y, then z) with weights 3/4 (parent side)
 * and 1/4 (neighbour side); the correction is added to active fine cells.
 * With prolong = 1 the upsampling of Algorithm 1 is read as nearest
 * (piecewise-constant) instead. */
void orc_mg_prolong_add(const orc_mg* mg, int li, const double* e, double* x) {
  const orc_level* f = &mg->lv[li];
  const orc_level* c = &mg->lv[li + 1];
  int dim = mg->dim;
  if (mg->prolong == 1) {
    /* nearest upsampling: an active fine cell takes its parent's value (the
     * parent of an active cell is active) */
    for (int k = 0; k < f->n[2]; ++k)
      for (int j = 0; j < f->n[1]; ++j)
        for (int i = 0; i < f->n[0]; ++i) {
          int P = lidx(f, i, j, k);
          if (f->act[P]) x[P] += e[lidx(c, i / 2, j / 2, dim == 3 ? k / 2 : 0)];
        }
    return;
  }
  for (int k = 0; k < f->n[2]; ++k)
    for (int j = 0; j < f->n[1]; ++j)
      for (int i = 0; i < f->n[0]; ++i) {
        int P = lidx(f, i, j, k);
        if (!f->act[P]) continue;
        int I = i / 2, J = j / 2, K = dim == 3 ? k / 2 : 0;
        int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
        double X[2][2] = {{0, 0}, {0, 0}};
        int nzc = dim == 3 ? 2 : 1;
        /* x pass on the rows (J + b sy, K + cc sz) whose parent column cell is active */
        for (int cc = 0; cc < nzc; ++cc)
          for (int b = 0; b < 2; ++b) {
            int Q[3] = {I, J + b * sy, K + cc * sz};
            if (!in_box(c, Q) || !c->act[lidx(c, Q[0], Q[1], Q[2])]) continue;
            double eq = e[lidx(c, Q[0], Q[1], Q[2])];
            int R[3] = {I + sx, Q[1], Q[2]};
            double en;
            if (!in_box(c, R)) {
              int fq[3] = {Q[0] + (sx > 0), Q[1], Q[2]};
              en = (1.0 - c->cf[0][fidx(c, 0, fq[0], fq[1], fq[2])]) * eq;
            } else {
              int r = lidx(c, R[0], R[1], R[2]);
              en = c->act[r] ? e[r] : eq;
            }
            X[cc][b] = 0.75 * eq + 0.25 * en;
          }
        /* y pass */
        double Y[2] = {0, 0};
        for (int cc = 0; cc < nzc; ++cc) {
          int Q0[3] = {I, J, K + cc * sz};
          if (!in_box(c, Q0) || !c->act[lidx(c, Q0[0], Q0[1], Q0[2])]) continue;
          int Q1[3] = {I, J + sy, K + cc * sz};
          double yn;
          if (!in_box(c, Q1)) {
            int fq[3] = {I, J + (sy > 0), K + cc * sz};
            yn = (1.0 - c->cf[1][fidx(c, 1, fq[0], fq[1], fq[2])]) * X[cc][0];
          } else {
            yn = c->act[lidx(c, Q1[0], Q1[1], Q1[2])] ? X[cc][1] : X[cc][0];
          }
          Y[cc] = 0.75 * X[cc][0] + 0.25 * yn;
        }
        double Z = Y[0];
        if (dim == 3) {
          int Q2[3] = {I, J, K + sz};
          double zn;
          if (!in_box(c, Q2)) {
            int fq[3] = {I, J, K + (sz > 0)};
            zn = (1.0 - c->cf[2][fidx(c, 2, fq[0], fq[1], fq[2])]) * Y[0];
          } else {
            zn = c->act[lidx(c, Q2[0], Q2[1], Q2[2])] ? Y[1] : Y[0];
          }
          Z = 0.75 * Y[0] + 0.25 * zn;
        }
        x[P] += Z;
      }
}

static void coarse_factor(orc_mg* mg) {
  int L = mg->L - 1;
  orc_level* l = &mg->lv[L];
  int N = lcells(l);
  int nc = 0;
  mg->cmap = (int*)malloc(sizeof(int) * (N > 0 ? N : 1));
  int* inv = (int*)malloc(sizeof(int) * (N > 0 ? N : 1));
  for (int P = 0; P < N; ++P) {
    inv[P] = -1;
    if (l->act[P]) { inv[P] = nc; mg->cmap[nc++] = P; }
  }
  mg->nc = nc;
  mg->lu = (double*)calloc((size_t)nc * nc + 1, sizeof(double));
  mg->piv = (int*)malloc(sizeof(int) * (nc + 1));
  /* columns of the dense matrix are A applied to unit vectors */
  double* e = (double*)calloc(N, sizeof(double));
  double* y = (double*)malloc(sizeof(double) * N);
  for (int col = 0; col < nc; ++col) {
    e[mg->cmap[col]] = 1.0;
    orc_mg_apply(mg, L, e, y);
    e[mg->cmap[col]] = 0.0;
    for (int row = 0; row < nc; ++row) mg->lu[(size_t)row * nc + col] = y[mg->cmap[row]];
  }
  free(e); free(y); free(inv);
  /* Gaussian elimination with partial pivoting */
  double* a = mg->lu;
  for (int kk = 0; kk < nc; ++kk) {
    int pr = kk;
    for (int r = kk + 1; r < nc; ++r)
      if (fabs(a[(size_t)r * nc + kk]) > fabs(a[(size_t)pr * nc + kk])) pr = r;
    mg->piv[kk] = pr;
    if (pr != kk)
      for (int q = 0; q < nc; ++q) {
        double t = a[(size_t)kk * nc + q];
        a[(size_t)kk * nc + q] = a[(size_t)pr * nc + q];
        a[(size_t)pr * nc + q] = t;
      }
    double d = a[(size_t)kk * nc + kk];
    for (int r = kk + 1; r < nc; ++r) {
      double m = a[(size_t)r * nc + kk] / d;
      a[(size_t)r * nc + kk] = m;
      for (int q = kk + 1; q < nc; ++q) a[(size_t)r * nc + q] -= m * a[(size_t)kk * nc + q];
    }
  }
}

static void coarse_solve(const orc_mg* mg, double* x, const double* b) {
  int nc = mg->nc;
  const orc_level* l = &mg->lv[mg->L - 1];
  double* y = (double*)malloc(sizeof(double) * (nc + 1));
  for (int r = 0; r < nc; ++r) y[r] = b[mg->cmap[r]];
  for (int kk = 0; kk < nc; ++kk) {
    int pr = mg->piv[kk];
    if (pr != kk) { double t = y[kk]; y[kk] = y[pr]; y[pr] = t; }
    for (int r = kk + 1; r < nc; ++r) y[r] -= mg->lu[(size_t)r * nc + kk] * y[kk];
  }
  for (int r = nc - 1; r >= 0; --r) {
    double s = y[r];
    for (int q = r + 1; q < nc; ++q) s -= mg->lu[(size_t)r * nc + q] * y[q];
    y[r] = s / mg->lu[(size_t)r * nc + r];
  }
  int N = lcells(l);
  for (int P = 0; P < N; ++P) x[P] = 0.0;
  for (int r = 0; r < nc; ++r) x[mg->cmap[r]] = y[r];
  free(y);
}

orc_mg* orc_mg_create(const orc_case* c) {
  if (c->n_levels < 1 || c->n_levels > 24) return NULL;
  orc_mg* mg = (orc_mg*)calloc(1, sizeof(orc_mg));
  mg->dim = c->dim;
  mg->L = c->n_levels;
  mg->nu1 = c->nu1;
  mg->prolong = c->prolong;
  mg->nu2 = c->nu2;
  mg->nuc = c->nu_coarse;
  mg->wj = c->omega_jacobi > 0 ? c->omega_jacobi : (c->dim == 3 ? 6.0 / 7.0 : 4.0 / 5.0);
  mg->literal = c->literal;
  if (mg->literal) {
    /* Algorithm 1: no pre-smoothing, one sweep per level on the way up,
     * undamped, nearest upsampling */
    mg->nu1 = 0;
    mg->nu2 = 1;
    mg->nuc = 0;
    mg->wj = 1.0;
    mg->prolong = 1;
  }
  /* level 0 from the cell classification */
  orc_level* l0 = &mg->lv[0];
  for (int d = 0; d < 3; ++d) { l0->n[d] = c->n[d]; l0->h[d] = c->h[d]; }
  int N = lcells(l0);
  l0->act = (unsigned char*)malloc(N);
  for (int P = 0; P < N; ++P) l0->act[P] = is_fluid(c, P);
  for (int d = 0; d < c->dim; ++d) {
    l0->cf[d] = (double*)calloc(fcount(l0, d), sizeof(double));
    for (int k = 0; k < c->n[2]; ++k)
      for (int j = 0; j < c->n[1]; ++j)
        for (int i = 0; i < c->n[0]; ++i) {
          int P = cidx(c, i, j, k);
          if (!is_fluid(c, P)) continue;
          for (int side = -1; side <= 1; side += 2) {
            int nidx;
            double cf = face_coef(c, i, j, k, 2 * d + (side > 0), &nidx);
            int fq[3] = {i, j, k};
            if (side > 0) fq[d] += 1;
            l0->cf[d][fidx(l0, d, fq[0], fq[1], fq[2])] = cf;
          }
        }
  }
  for (int li = 1; li < mg->L; ++li) {
    orc_level* f = &mg->lv[li - 1];
    orc_level* l = &mg->lv[li];
    for (int d = 0; d < 3; ++d) {
      if (d < c->dim) {
        if (f->n[d] % 2) { orc_mg_free(mg); return NULL; }
        l->n[d] = f->n[d] / 2;
        l->h[d] = 2.0 * f->h[d];
      } else { l->n[d] = 1; l->h[d] = f->h[d]; }
    }
    int Nc = lcells(l);
    l->act = (unsigned char*)calloc(Nc, 1);
    int kz = c->dim == 3 ? 2 : 1;
    for (int K = 0; K < l->n[2]; ++K)
      for (int J = 0; J < l->n[1]; ++J)
        for (int I = 0; I < l->n[0]; ++I)
          for (int cc = 0; cc < kz; ++cc)
            for (int b = 0; b < 2; ++b)
              for (int a = 0; a < 2; ++a)
                if (f->act[lidx(f, 2 * I + a, 2 * J + b, kz * K + cc)]) l->act[lidx(l, I, J, K)] = 1;
    for (int d = 0; d < c->dim; ++d) {
      l->cf[d] = (double*)calloc(fcount(l, d), sizeof(double));
      int ext[3] = {l->n[0] + (d == 0), l->n[1] + (d == 1), l->n[2] + (d == 2)};
      int nsub = c->dim == 3 ? 4 : 2;
      for (int K = 0; K < ext[2]; ++K)
        for (int J = 0; J < ext[1]; ++J)
          for (int I = 0; I < ext[0]; ++I) {
            double s = 0.0;
            int t[3] = {2 * I, 2 * J, kz * K};
            /* the tangential axes each contribute two fine sub-faces */
            for (int u0 = 0; u0 < 2; ++u0)
              for (int u1 = 0; u1 < (c->dim == 3 ? 2 : 1); ++u1) {
                int q[3] = {t[0], t[1], t[2]};
                int ta = (d == 0) ? 1 : 0, tb = (d == 2) ? 1 : 2;
                q[ta] += u0;
                if (c->dim == 3) q[tb] += u1;
                s += f->cf[d][fidx(f, d, q[0], q[1], q[2])];
              }
            l->cf[d][fidx(l, d, I, J, K)] = s / nsub;
          }
    }
  }
  coarse_factor(mg);
  return mg;
}

void orc_mg_free(orc_mg* mg) {
  if (!mg) return;
  for (int li = 0; li < 24; ++li) {
    free(mg->lv[li].act);
    for (int d = 0; d < 3; ++d) free(mg->lv[li].cf[d]);
  }
  free(mg->cmap); free(mg->lu); free(mg->piv);
  free(mg);
}

int orc_mg_levels(const orc_mg* mg) { return mg->L; }

void orc_mg_level_shape(const orc_mg* mg, int l, int n[3], double h[3]) {
  for (int d = 0; d < 3; ++d) { n[d] = mg->lv[l].n[d]; h[d] = mg->lv[l].h[d]; }
}

void orc_mg_level_active(const orc_mg* mg, int l, unsigned char* act) {
  memcpy(act, mg->lv[l].act, lcells(&mg->lv[l]));
}

static void vcycle(const orc_mg* mg, int li, double* x, const double* b) {
  const orc_level* l = &mg->lv[li];
  if (li == mg->L - 1) {
    if (mg->literal) {
      /* Algorithm 1's coarsest level: one Jacobi sweep from w = 0 */
      memset(x, 0, sizeof(double) * lcells(l));
      orc_mg_smooth(mg, li, x, b, 1);
    } else {
      coarse_solve(mg, x, b);
    }
    return;
  }
  int N = lcells(l);
  /* sweeps of this level: nu1 / nu2 on the finest, nu_coarse below it when set */
  const int pre = li > 0 && mg->nuc > 0 ? mg->nuc : mg->nu1;
  const int post = li > 0 && mg->nuc > 0 ? mg->nuc : mg->nu2;
  orc_mg_smooth(mg, li, x, b, pre);
  double* r = (double*)malloc(sizeof(double) * N);
  orc_mg_apply(mg, li, x, r);
  for (int P = 0; P < N; ++P) r[P] = l->act[P] ? b[P] - r[P] : 0.0;
  int Nc = lcells(&mg->lv[li + 1]);
  double* bc = (double*)calloc(Nc, sizeof(double));
  double* ec = (double*)calloc(Nc, sizeof(double));
  orc_mg_restrict(mg, li, r, bc);
  vcycle(mg, li + 1, ec, bc);
  orc_mg_prolong_add(mg, li, ec, x);
  orc_mg_smooth(mg, li, x, b, post);
  free(r); free(bc); free(ec);
}

void orc_mg_vcycle(const orc_mg* mg, double* x, const double* b) { vcycle(mg, 0, x, b); }

int orc_pressure_adjoint(const orc_case* c, const double* ubar, const double* vbar,
                         const double* wbar, const double* pbar, double tol, int max_cycles,
                         int forced_cycles, double* usbar, double* vsbar, double* wsbar,
                         double* phibar, double* lambda, int* cycles, double* rel_residual) {
  orc_mg* mg = orc_mg_create(c);
  if (!mg) return -1;
  int st = pressure_adjoint_with(c, mg, ubar, vbar, wbar, pbar, tol, max_cycles, forced_cycles,
                                 usbar, vsbar, wsbar, phibar, lambda, cycles, rel_residual);
  orc_mg_free(mg);
  return st;
}

/* Smallest (p, A p) / (z, A z) kept before the direction restarts. */
#define CG_RESTART 1e-12

static double dot_active(const orc_level* l, const double* a, const double* b) {
  int N = lcells(l);
  double s = 0.0;
  for (int P = 0; P < N; ++P)
    if (l->act[P]) s += a[P] * b[P];
  return s;
}

/* Outer iteration.  The paper iterates its multigrid cycle a fixed n_iter
 * times (Algorithm 1).  Plain cycling of the re-discretised hierarchy does
 * not converge when the only zero-pressure faces are small vents, so the
 * cycle is used as the preconditioner of a flexible conjugate-gradient
 * iteration (Polak-Ribiere form), stopped when ||r|| <= tol ||b|| or after
 * forced_cycles preconditioner applications when forced_cycles >= 0:
 *   z = V(r);  beta = (z, r - r_prev) / (z_prev, r_prev) = -alpha_prev (z, q_prev) / (z_prev, r_prev)
 *   p = z + beta p;  q = A p;  alpha = (z, r) / (p, q);  x += alpha p;  r -= alpha q.
 * At a breakdown ((p, q) a vanishing fraction of (z, A z)) the direction
 * restarts as p = z, and a zero (p, q) (z = 0) takes no step. */
int orc_mg_solve(const orc_mg* mg, const double* b, double* x, double tol, int max_cycles,
                 int forced, int* cycles, double* relres) {
  const orc_level* l = &mg->lv[0];
  int N = lcells(l);
  double* r = (double*)malloc(sizeof(double) * N);
  double* z = (double*)malloc(sizeof(double) * N);
  double* pv = (double*)calloc(N, sizeof(double));
  double* q = (double*)calloc(N, sizeof(double));
  double bn = sqrt(dot_active(l, b, b));
  /* A x = 0 has the solution 0, whatever the initial guess */
  if (bn == 0.0) memset(x, 0, sizeof(double) * N);
  orc_mg_apply(mg, 0, x, r);
  for (int P = 0; P < N; ++P) r[P] = l->act[P] ? b[P] - r[P] : 0.0;
  int status = ORC_OK, cyc = 0;
  double rel = 0.0, zr_prev = 0.0, alpha_prev = 0.0, pq_prev = 0.0;
  for (;;) {
    double rn = sqrt(dot_active(l, r, r));
    rel = bn > 0.0 ? rn / bn : 0.0;
    if (!isfinite(rn)) { status = ORC_E_DIVERGED; break; }
    if (forced >= 0) {
      if (cyc >= forced) break;
    } else {
      if (bn == 0.0 || rn <= tol * bn) break;
      if (cyc >= max_cycles) { status = ORC_E_NOTCONV; break; }
    }
    memset(z, 0, sizeof(double) * N);
    vcycle(mg, 0, z, r);
    if (mg->literal) {
      /* Algorithm 1's outer loop: p <- p - w with w the cycle's answer for
       * A w = A p - b (here x += z with z for A z = b - A x), then the
       * residual again (read as recomputed every iteration) */
      for (int P = 0; P < N; ++P) x[P] += z[P];
      orc_mg_apply(mg, 0, x, r);
      for (int P = 0; P < N; ++P) r[P] = l->act[P] ? b[P] - r[P] : 0.0;
      ++cyc;
      continue;
    }
    double zr = dot_active(l, z, r);
    double pq;
    if (cyc == 0) {
      memcpy(pv, z, sizeof(double) * N);
      orc_mg_apply(mg, 0, pv, q);
      pq = dot_active(l, pv, q);
    } else {
      double beta = -alpha_prev * dot_active(l, z, q) / zr_prev;
      for (int P = 0; P < N; ++P) pv[P] = z[P] + beta * pv[P];
      orc_mg_apply(mg, 0, pv, q);
      pq = dot_active(l, pv, q);
      /* Breakdown: p A-orthogonal to p_prev gives (z, A z) = (p, A p) +
       * beta^2 (p_prev, A p_prev); when (p, A p) is a vanishing part of it,
       * z and p_prev are A-parallel and the direction restarts from z. */
      if (!(pq > CG_RESTART * (pq + beta * beta * pq_prev))) {
        memcpy(pv, z, sizeof(double) * N);
        orc_mg_apply(mg, 0, pv, q);
        pq = dot_active(l, pv, q);
      }
    }
    /* z = 0 (an exactly solved system): no step */
    double alpha = pq > 0.0 ? zr / pq : 0.0;
    for (int P = 0; P < N; ++P) {
      x[P] += alpha * pv[P];
      r[P] -= alpha * q[P];
    }
    zr_prev = zr;
    alpha_prev = alpha;
    pq_prev = pq;
    ++cyc;
  }
  free(r); free(z); free(pv); free(q);
  if (cycles) *cycles = cyc;
  if (relres) *relres = rel;
  return status;
}

/* One time step (Sec. 2.5-2.6): half-step semi-implicit destruction, one
 * explicit step of the rest terms, projection (b, multigrid, correction),
 * second half-step destruction.  The flow chart of the paper is missing; this
 * order is the reading recorded in the design notes. */
int orc_step(const orc_case* c, orc_fields* s, int n_steps, const int* forced,
             orc_stats* stats, int warm) {
  int N = ncells(c);
  orc_mg* mg = orc_mg_create(c);
  if (!mg) return ORC_E_INVAL;
  double* buf = (double*)calloc((size_t)N * 10, sizeof(double));
  orc_fields t;
  t.u = buf; t.v = buf + N; t.w = buf + 2 * N; t.p = buf + 3 * N; t.T = buf + 4 * N;
  t.k = buf + 5 * N; t.omega = buf + 6 * N;
  double* b = buf + 7 * N;
  double* phi = buf + 8 * N;
  double* k2 = buf + 9 * N;
  double* om2 = (double*)malloc(sizeof(double) * N);
  int status = ORC_OK;
  int komega = c->physics & ORC_KOMEGA;
  for (int st = 0; st < n_steps; ++st) {
    orc_fixed_omega(c, s->omega);
    if (komega) {
      orc_destroy(c, s->u, s->v, s->w, s->k, s->omega, 0.5 * c->dt, k2, om2);
      memcpy(s->k, k2, sizeof(double) * N);
      memcpy(s->omega, om2, sizeof(double) * N);
    }
    orc_explicit(c, s, &t);
    orc_rhs_b(c, t.u, t.v, t.w, b);
    /* initial guess: zero, or with warm the previous step's increment
     * phi = p^{n} - p^{n-1} */
    if (!warm) memset(phi, 0, sizeof(double) * N);
    int cyc = 0;
    double rel = 0.0, mdiv = 0.0;
    int ms = orc_mg_solve(mg, b, phi, c->tol, c->max_cycles, forced ? forced[st] : -1, &cyc, &rel);
    orc_project(c, phi, t.u, t.v, t.w, s->p, s->u, s->v, s->w, &mdiv);
    memcpy(s->T, t.T, sizeof(double) * N);
    if (komega) {
      orc_destroy(c, s->u, s->v, s->w, t.k, t.omega, 0.5 * c->dt, s->k, s->omega);
    } else {
      memcpy(s->k, t.k, sizeof(double) * N);
      memcpy(s->omega, t.omega, sizeof(double) * N);
    }
    double mk = INFINITY, mo = INFINITY;
    int bad = 0;
    for (int P = 0; P < N; ++P) {
      if (!is_fluid(c, P)) continue;
      if (s->k[P] < mk) mk = s->k[P];
      if (s->omega[P] < mo) mo = s->omega[P];
      if (!isfinite(s->u[P]) || !isfinite(s->p[P]) || !isfinite(s->k[P])) bad = 1;
    }
    if (bad) ms = ORC_E_DIVERGED;
    if (stats) {
      stats[st].cycles = cyc;
      stats[st].status = ms;
      stats[st].rel_residual = rel;
      stats[st].max_face_div = mdiv;
      stats[st].min_k = mk;
      stats[st].min_omega = mo;
    }
    if (ms == ORC_E_DIVERGED) { status = ms; break; }
    if (ms != ORC_OK && status == ORC_OK) status = ms;
  }
  free(buf); free(om2);
  orc_mg_free(mg);
  return status;
}
