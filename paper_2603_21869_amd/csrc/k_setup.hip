// Setup kernels: cell classification against boundary patches and solids
// (Sec. 2.7), wall-fixed omega cells, the multigrid hierarchy (face
// coefficients of the pressure operator per level, Sec. 2.4) and the dense
// inverse of the coarsest level.
#include <hip/hip_runtime.h>

#include "nfvm_device.hpp"

namespace nfvm {

Geom make_geom(int dim, int nx, int ny, int nz, double hx, double hy, double hz) {
  Geom g;
  g.dim = dim;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.gz = dim == 3 ? 1 : 0;
  g.sx = ((nx + 2) + 15) / 16 * 16;
  g.sxy = g.sx * (ny + 2);
  const int pad = 16;
  g.off = pad + g.gz * g.sxy + g.sx;  // idx(-1, -1, -gz) == pad - 1
  g.total = pad + (nz + 2 * g.gz) * g.sxy + pad;
  g.hx = hx;
  g.hy = hy;
  g.hz = hz;
  g.sd = 0.0;
  return g;
}

Tiles make_tiles(int nx, int ny, int nz, int target_blocks) {
  Tiles t;
  t.ntx = (nx + 63) / 64;
  t.nty = (ny + 3) / 4;
  const int nxy = t.ntx * t.nty;
  int nzc = (target_blocks + nxy - 1) / nxy;
  if (nzc < 1) nzc = 1;
  if (nzc > nz) nzc = nz;
  t.cz = (nz + nzc - 1) / nzc;
  t.ntz = (nz + t.cz - 1) / t.cz;
  t.total = nxy * t.ntz;
  t.grid = (t.total + 7) / 8 * 8;
  return t;
}

// One thread per padded cell.  patch_rect: per user patch {face, lo0, lo1, hi0, hi1}.
__global__ void k_classify(Geom g, const uint8_t* __restrict__ solid, const int* __restrict__ rect,
                           int npu, DevPatch* patches, double nu, int komega,
                           uint8_t* __restrict__ type) {
  const long long n = (long long)(g.nx + 2) * (g.ny + 2) * (g.nz + 2 * g.gz);
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t == 0 && komega) {
    for (int q = 0; q < MAX_PATCHES; ++q)
      if (patches[q].kind == K_INLET)
        patches[q].nut = eddy_visc<double>(nu, patches[q].k, patches[q].omega);
  }
  if (t >= n) return;
  const int i = (int)(t % (g.nx + 2)) - 1;
  const int j = (int)((t / (g.nx + 2)) % (g.ny + 2)) - 1;
  const int k = (int)(t / ((long long)(g.nx + 2) * (g.ny + 2))) - g.gz;
  const bool oi = i < 0 || i >= g.nx, oj = j < 0 || j >= g.ny, ok = k < 0 || k >= g.nz;
  const int nout = (int)oi + (int)oj + (int)ok;
  uint8_t ty;
  if (nout == 0) {
    const long long d = ((long long)k * g.ny + j) * g.nx + i;
    ty = (solid && solid[d]) ? PID_SOLID : PID_FLUID;
  } else if (nout > 1) {
    ty = PID_SOLID;  // edge and corner ghosts are never a face neighbour
  } else {
    int face, t0, t1;
    if (oi) { face = i < 0 ? 0 : 1; t0 = j; t1 = k; }
    else if (oj) { face = j < 0 ? 2 : 3; t0 = i; t1 = k; }
    else { face = k < 0 ? 4 : 5; t0 = i; t1 = j; }
    ty = (uint8_t)(PID_DEFWALL + face);
    for (int q = 0; q < npu; ++q) {
      const int* r = rect + 5 * q;
      if (r[0] == face && t0 >= r[1] && t1 >= r[2] && t0 < r[3] && t1 < r[4]) {
        ty = (uint8_t)(PID_USER + q);
        break;
      }
    }
  }
  type[g.idx(i, j, k)] = ty;
}

void launch_classify(const Geom& g, const uint8_t* solid, const int* rect, int npu,
                     DevPatch* patches, double nu, int komega, uint8_t* type, hipStream_t s) {
  const long long n = (long long)(g.nx + 2) * (g.ny + 2) * (g.nz + 2 * g.gz);
  const int bs = 256;
  hipLaunchKernelGGL(k_classify, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, g, solid,
                     rect, npu, patches, nu, komega, type);
}

// Mark fluid cells that touch a wall or a solid (Sec. 2.7 wall treatment).
__global__ void k_fix_omega(Geom g, const DevPatch* __restrict__ pt, uint8_t* type) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y,
            k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const int P = g.idx(i, j, k);
  const uint8_t tp = type[P];
  if (!is_fluid(tp)) return;
  const int st[3] = {1, g.sx, g.sxy};
  bool fixed = false;
  for (int d = 0; d < g.dim; ++d)
    for (int s = -1; s <= 1; s += 2) {
      const uint8_t tn = type[P + s * st[d]];
      if (!is_fluid(tn) && pt[tn & 0x7f].kind == K_WALL) fixed = true;
    }
  if (fixed) type[P] = (uint8_t)(tp | FIXED_BIT);
}

void launch_fix_omega(const Geom& g, const DevPatch* pt, uint8_t* type, hipStream_t s) {
  hipLaunchKernelGGL(k_fix_omega, dim3((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz), dim3(64, 4), 0,
                     s, g, pt, type);
}

// omega = 6 nu / (beta_i d^2) in fixed cells, d = half the smallest normal
// width among the cell's wall faces.
template <class F>
__global__ void k_set_omega_wall(Geom g, const DevPatch* __restrict__ pt, double nu,
                                 const uint8_t* __restrict__ type, F* om) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y,
            k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const int P = g.idx(i, j, k);
  const uint8_t tp = type[P];
  if (!(tp & FIXED_BIT)) return;
  const int st[3] = {1, g.sx, g.sxy};
  const double h[3] = {g.hx, g.hy, g.hz};
  double dmin = 1e300;
  for (int d = 0; d < g.dim; ++d)
    for (int s = -1; s <= 1; s += 2) {
      const uint8_t tn = type[P + s * st[d]];
      if (!is_fluid(tn) && pt[tn & 0x7f].kind == K_WALL) dmin = fmin(dmin, 0.5 * h[d]);
    }
  om[P] = (F)(6.0 * nu / (C_BETA_I * dmin * dmin));
}

template <class F>
void launch_set_omega_wall(const Geom& g, const Phys& ph, const DevPatch* pt, const uint8_t* type,
                           F* om, hipStream_t s) {
  hipLaunchKernelGGL(k_set_omega_wall<F>, dim3((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz),
                     dim3(64, 4), 0, s, g, pt, ph.nu, type, om);
}
template void launch_set_omega_wall<double>(const Geom&, const Phys&, const DevPatch*,
                                            const uint8_t*, double*, hipStream_t);
template void launch_set_omega_wall<float>(const Geom&, const Phys&, const DevPatch*,
                                           const uint8_t*, float*, hipStream_t);

// Level 0 of the pressure operator: coefficient 1 between fluid cells, 0 on
// zero-gradient faces (walls, inlets, solids), 2 on outlet faces (the ghost
// is -x_P there, eq. neg_lap_discretize with the boundary padding).
__device__ __forceinline__ float face0(const DevPatch* pt, uint8_t a, uint8_t b) {
  const bool fa = is_fluid(a), fb = is_fluid(b);
  if (fa && fb) return 1.f;
  if (!fa && !fb) return 0.f;
  const uint8_t o = fa ? b : a;
  return pt[o & 0x7f].kind == K_OUTLET ? 2.f : 0.f;
}

__global__ void k_level0(Geom g, const uint8_t* __restrict__ type, const DevPatch* __restrict__ pt,
                         uint8_t* cls, float* cx, float* cy, float* cz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y,
            k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const int P = g.idx(i, j, k);
  const uint8_t tp = type[P];
  float* cf[3] = {cx, cy, cz};
  const int st[3] = {1, g.sx, g.sxy};
  const int pos[3] = {i, j, k};
  const int nn[3] = {g.nx, g.ny, g.nz};
  bool regular = is_fluid(tp);
  for (int d = 0; d < g.dim; ++d) {
    const float lo = face0(pt, type[P - st[d]], tp);
    const float hi = face0(pt, tp, type[P + st[d]]);
    cf[d][P] = lo;
    if (pos[d] == nn[d] - 1) cf[d][P + st[d]] = hi;
    if (lo != 1.f || hi != 1.f || pos[d] == 0 || pos[d] == nn[d] - 1) regular = false;
  }
  cls[P] = !is_fluid(tp) ? MG_INACTIVE : (regular ? MG_REGULAR : MG_IRREGULAR);
}

void launch_level0(const Geom& g, const uint8_t* type, const DevPatch* pt, uint8_t* cls,
                   float* cx, float* cy, float* cz, hipStream_t s) {
  hipLaunchKernelGGL(k_level0, dim3((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz), dim3(64, 4), 0, s,
                     g, type, pt, cls, cx, cy, cz);
}

// Level-0 face codes from the class bytes and face coefficients (which are
// 0, 1 or 2 on level 0).
__global__ void k_face_codes(Geom g, const uint8_t* __restrict__ cls, const float* __restrict__ cx,
                             const float* __restrict__ cy, const float* __restrict__ cz,
                             uint16_t* __restrict__ code) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const int P = g.idx(i, j, k);
  if (cls[P] == MG_INACTIVE) {
    code[P] = (uint16_t)FACE_CODE_INACTIVE;
    return;
  }
  const float f[6] = {cx[P], cx[P + 1], cy[P], cy[P + g.sx], g.dim == 3 ? cz[P] : 0.f,
                      g.dim == 3 ? cz[P + g.sxy] : 0.f};
  uint32_t c = 0;
  for (int q = 0; q < 6; ++q) c |= ((uint32_t)f[q] & 3u) << (2 * q);
  code[P] = (uint16_t)c;
}

void launch_face_codes(const Geom& g, const uint8_t* cls, const float* cx, const float* cy,
                       const float* cz, uint16_t* code, hipStream_t s) {
  hipLaunchKernelGGL(k_face_codes, dim3((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz), dim3(64, 4), 0, s,
                     g, cls, cx, cy, cz, code);
}

// Coarse level: a cell is active when any child is; a face coefficient is the
// mean of the fine sub-face coefficients it covers.
__global__ void k_coarsen(Geom f, const uint8_t* __restrict__ fcls, const float* __restrict__ fx,
                          const float* __restrict__ fy, const float* __restrict__ fz, Geom c,
                          uint8_t* ccls, float* cx, float* cy, float* cz) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x, J = blockIdx.y * blockDim.y + threadIdx.y,
            K = blockIdx.z;
  if (I >= c.nx || J >= c.ny) return;
  const int kz = c.dim == 3 ? 2 : 1;
  bool act = false;
  for (int cc = 0; cc < kz; ++cc)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a)
        if (fcls[f.idx(2 * I + a, 2 * J + b, kz * K + cc)] != MG_INACTIVE) act = true;
  const float* fcf[3] = {fx, fy, fz};
  float* ccf[3] = {cx, cy, cz};
  const int pos[3] = {I, J, K};
  const int nn[3] = {c.nx, c.ny, c.nz};
  const float inv = c.dim == 3 ? 0.25f : 0.5f;
  bool regular = act;
  for (int d = 0; d < c.dim; ++d) {
    for (int side = 0; side < 2; ++side) {
      if (side == 1 && pos[d] != nn[d] - 1) continue;
      int q[3] = {I, J, K};
      q[d] += side;  // coarse face index along d
      float s = 0.f;
      for (int u0 = 0; u0 < 2; ++u0)
        for (int u1 = 0; u1 < (c.dim == 3 ? 2 : 1); ++u1) {
          int fq[3] = {2 * q[0], 2 * q[1], kz * q[2]};
          const int ta = d == 0 ? 1 : 0, tb = d == 2 ? 1 : 2;
          fq[ta] += u0;
          if (c.dim == 3) fq[tb] += u1;
          s += fcf[d][f.idx(fq[0], fq[1], fq[2])];
        }
      ccf[d][c.idx(q[0], q[1], q[2])] = s * inv;
    }
  }
  // regularity needs both faces of every axis at 1 and all neighbours inside
  for (int d = 0; d < c.dim && regular; ++d) {
    int q[3] = {I, J, K};
    const float lo = ccf[d][c.idx(q[0], q[1], q[2])];
    q[d] += 1;
    // the high face of an interior cell belongs to the next cell; recompute it
    float hi;
    if (pos[d] == nn[d] - 1) {
      hi = ccf[d][c.idx(q[0], q[1], q[2])];
    } else {
      float s = 0.f;
      for (int u0 = 0; u0 < 2; ++u0)
        for (int u1 = 0; u1 < (c.dim == 3 ? 2 : 1); ++u1) {
          int fq[3] = {2 * q[0], 2 * q[1], kz * q[2]};
          const int ta = d == 0 ? 1 : 0, tb = d == 2 ? 1 : 2;
          fq[ta] += u0;
          if (c.dim == 3) fq[tb] += u1;
          s += fcf[d][f.idx(fq[0], fq[1], fq[2])];
        }
      hi = s * inv;
    }
    if (lo != 1.f || hi != 1.f || pos[d] == 0 || pos[d] == nn[d] - 1) regular = false;
  }
  ccls[c.idx(I, J, K)] = !act ? MG_INACTIVE : (regular ? MG_REGULAR : MG_IRREGULAR);
}

void launch_coarsen(const Geom& f, const uint8_t* fcls, float* const fcf[3], const Geom& c,
                    uint8_t* ccls, float* ccf[3], hipStream_t s) {
  hipLaunchKernelGGL(k_coarsen, dim3((c.nx + 63) / 64, (c.ny + 3) / 4, c.nz), dim3(64, 4), 0, s,
                     f, fcls, fcf[0], fcf[1], fcf[2], c, ccls, ccf[0], ccf[1], ccf[2]);
}

// Dense inverse of the coarsest operator by Gauss-Jordan elimination with
// partial pivoting, one workgroup.  work: 2 * max_n * max_n doubles; on exit
// the first n*n entries hold the inverse (row-major over active cells, in
// cmap order).
constexpr int GJ_BS = 1024;
__global__ __launch_bounds__(GJ_BS) void k_coarse_factor(Geom g, const uint8_t* __restrict__ cls,
                                                         const float* __restrict__ cx,
                                                         const float* __restrict__ cy,
                                                         const float* __restrict__ cz,
                                                         int* cmap, int* ncount, double* W,
                                                         int max_n) {
  __shared__ int n_sh;
  __shared__ double vmax[GJ_BS];
  __shared__ int imax[GJ_BS];
  const int t = threadIdx.x;
  if (t == 0) {
    int n = 0;
    for (int k = 0; k < g.nz; ++k)
      for (int j = 0; j < g.ny; ++j)
        for (int i = 0; i < g.nx; ++i) {
          const int P = g.idx(i, j, k);
          if (cls[P] != MG_INACTIVE) {
            if (n < max_n) cmap[n] = P;
            ++n;
          }
        }
    *ncount = n;  // the host rejects the grid when n > max_n
    n_sh = n > max_n ? -1 : n;
  }
  __syncthreads();
  const int n = n_sh;
  if (n < 0) return;
  const int w = 2 * n;
  const float* cf[3] = {cx, cy, cz};
  const int st[3] = {1, g.sx, g.sxy};
  const double ih2[3] = {1.0 / (g.hx * g.hx), 1.0 / (g.hy * g.hy), 1.0 / (g.hz * g.hz)};
  for (long long e = t; e < (long long)n * w; e += GJ_BS) W[e] = 0.0;
  __syncthreads();
  for (int a = t; a < n; a += GJ_BS) {
    const int P = cmap[a];
    double D = 0.0;
    for (int d = 0; d < g.dim; ++d) {
      const double clo = cf[d][P], chi = cf[d][P + st[d]];
      D += (clo + chi) * ih2[d];
      for (int s = -1; s <= 1; s += 2) {
        const int N = P + s * st[d];
        const double c = s < 0 ? clo : chi;
        if (c == 0.0) continue;
        for (int b = 0; b < n; ++b)
          if (cmap[b] == N) W[(long long)a * w + b] -= c * ih2[d];
      }
    }
    W[(long long)a * w + a] += D;
    W[(long long)a * w + n + a] = 1.0;
  }
  __syncthreads();
  __shared__ double fac[512];
  for (int col = 0; col < n; ++col) {
    double bv = -1.0;
    int bi = col;
    for (int r = col + t; r < n; r += GJ_BS) {
      const double v = fabs(W[(long long)r * w + col]);
      if (v > bv) { bv = v; bi = r; }
    }
    vmax[t] = bv;
    imax[t] = bi;
    __syncthreads();
    for (int s = GJ_BS / 2; s > 0; s >>= 1) {
      if (t < s && (vmax[t + s] > vmax[t] || (vmax[t + s] == vmax[t] && imax[t + s] < imax[t]))) {
        vmax[t] = vmax[t + s];
        imax[t] = imax[t + s];
      }
      __syncthreads();
    }
    const int pr = imax[0];
    if (pr != col)
      for (int c = t; c < w; c += GJ_BS) {
        const double tmp = W[(long long)col * w + c];
        W[(long long)col * w + c] = W[(long long)pr * w + c];
        W[(long long)pr * w + c] = tmp;
      }
    __syncthreads();
    const double piv = W[(long long)col * w + col];
    __syncthreads();
    for (int c = t; c < w; c += GJ_BS) W[(long long)col * w + c] /= piv;
    for (int r = t; r < n; r += GJ_BS) fac[r] = W[(long long)r * w + col];
    __syncthreads();
    for (long long e = t; e < (long long)n * w; e += GJ_BS) {
      const int r = (int)(e / w), c = (int)(e % w);
      if (r != col) W[e] -= fac[r] * W[(long long)col * w + c];
    }
    __syncthreads();
  }
  // compact the inverse into the first n*n entries; a forward copy never
  // overwrites a source still to be read (source index >= destination)
  if (t == 0) {
    for (long long e = 0; e < (long long)n * n; ++e) {
      const int r = (int)(e / n), c = (int)(e % n);
      W[e] = W[(long long)r * w + n + c];
    }
  }
}

void launch_coarse_factor(const Geom& g, const uint8_t* cls, float* const cf[3], int* cmap,
                          int* ncount, double* work, int max_n, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_factor, dim3(1), dim3(GJ_BS), 0, s, g, cls, cf[0], cf[1],
                     g.dim == 3 ? cf[2] : cf[0], cmap, ncount, work, max_n);
}

}  // namespace nfvm
