// Post-processing kernels: the lambda2 vortex criterion (Sec. 3.2) and the
// line probes (Sec. 3.1).
#include <hip/hip_runtime.h>

#include "nfvm_device.hpp"
#include "post.hpp"

namespace nfvm {

namespace {
constexpr int PBX = 64, PBY = 4;

// One Jacobi rotation of the symmetric 3x3 matrix A that zeroes A[p][q]
// (r is the third index): tan of the angle from the smaller root of
// t^2 + 2 theta t - 1 = 0, theta = (A[q][q] - A[p][p]) / (2 A[p][q]).
template <class R>
__device__ __forceinline__ void jacobi_rotate(R A[3][3], int p, int q, int r) {
  const R apq = A[p][q];
  if (apq == (R)0) return;
  const R theta = (A[q][q] - A[p][p]) / ((R)2 * apq);
  const R at = fabs(theta);
  R t = at > (R)1e15 ? (R)0.5 / theta : (R)1 / (at + sqrt(theta * theta + (R)1));
  if (at <= (R)1e15 && theta < (R)0) t = -t;
  const R c = (R)1 / sqrt(t * t + (R)1), s = t * c;
  A[p][p] -= t * apq;
  A[q][q] += t * apq;
  A[p][q] = A[q][p] = (R)0;
  const R arp = A[r][p], arq = A[r][q];
  A[r][p] = A[p][r] = c * arp - s * arq;
  A[r][q] = A[q][r] = s * arp + c * arq;
}
}  // namespace

// One thread per cell; block (PBX, PBY) over (i, j), grid z over planes.
// Cyclic Jacobi sweeps (the off-diagonal part shrinks quadratically; six
// sweeps bring a 3x3 matrix to rounding level) give the eigenvalues to the
// rounding of the matrix, repeated ones included.
template <class V>
__global__ __launch_bounds__(PBX * PBY) void k_lambda2(Geom g, Phys ph,
                                                       const uint8_t* __restrict__ type,
                                                       const DevPatch* __restrict__ pt,
                                                       const V* __restrict__ u,
                                                       const V* __restrict__ v,
                                                       const V* __restrict__ w,
                                                       double* __restrict__ out) {
  typedef V R;
  const int i = blockIdx.x * PBX + threadIdx.x, j = blockIdx.y * PBY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nx || j >= g.ny || k >= g.nz) return;
  const size_t o = ((size_t)k * g.ny + j) * g.nx + i;
  const int P = g.idx(i, j, k);
  const uint8_t tp = type[P];
  if (!is_fluid(tp)) {
    out[o] = 0.0;
    return;
  }
  const R vel[3] = {u[P], v[P], w[P]};
  const int st[3] = {1, g.sx, g.sxy};
  const R ih2[3] = {(R)(0.5 / g.hx), (R)(0.5 / g.hy), (R)(0.5 / g.hz)};
  R G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int s = -1; s <= 1; s += 2) {
      if (d >= g.dim) continue;
      const int N = P + s * st[d];
      const uint8_t tn = type[N];
      R vn[3] = {(R)u[N], (R)v[N], (R)w[N]};
      if (!is_fluid(tn)) {
        const DevPatch& pp = pt[tn & 0x7f];
        for (int a = 0; a < 3; ++a) vn[a] = ghost<R>(pp, G_U + a, vel[a], ph.komega);
      }
      const R sc = (R)s * ih2[d];
#pragma unroll
      for (int a = 0; a < 3; ++a)
        if (a < g.dim) G[a][d] += sc * vn[a];
    }
  R S[3][3], W[3][3], M[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      S[a][b] = (R)0.5 * (G[a][b] + G[b][a]);
      W[a][b] = (R)0.5 * (G[a][b] - G[b][a]);
    }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      R m = 0;
#pragma unroll
      for (int e = 0; e < 3; ++e) m += S[a][e] * S[e][b] + W[a][e] * W[e][b];
      M[a][b] = m;
    }
  // symmetric by construction up to rounding: use the mean of the pairs
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a + 1; b < 3; ++b) M[a][b] = M[b][a] = (R)0.5 * (M[a][b] + M[b][a]);
  for (int sweep = 0; sweep < 6; ++sweep) {
    jacobi_rotate<R>(M, 0, 1, 2);
    jacobi_rotate<R>(M, 0, 2, 1);
    jacobi_rotate<R>(M, 1, 2, 0);
  }
  const R e0 = M[0][0], e1 = M[1][1], e2 = M[2][2];
  const R lo = fmin(e0, e1), hi = fmax(e0, e1);
  out[o] = (double)fmax(lo, fmin(hi, e2));
}

template <class V>
void launch_lambda2(const Geom& g, const Phys& ph, const uint8_t* type, const DevPatch* pt,
                    const V* u, const V* v, const V* w, double* out, hipStream_t s) {
  const dim3 grid((g.nx + PBX - 1) / PBX, (g.ny + PBY - 1) / PBY, g.nz);
  NFVM_LAUNCH((k_lambda2<V>), grid, dim3(PBX, PBY), 0, s, g, ph, type, pt, u, v, w, out);
}
template void launch_lambda2<double>(const Geom&, const Phys&, const uint8_t*, const DevPatch*,
                                     const double*, const double*, const double*, double*,
                                     hipStream_t);
template void launch_lambda2<float>(const Geom&, const Phys&, const uint8_t*, const DevPatch*,
                                    const float*, const float*, const float*, double*,
                                    hipStream_t);

// One thread per probe point: the eight cells around the point (four in
// 2D) after clamping it into the box of cell centres, trilinear weights,
// non-fluid cells left out and the weights renormalised; the velocity
// magnitude of the interpolated components.  FP64 arithmetic.
template <class V, class F>
__global__ __launch_bounds__(256) void k_probe(Geom g, const uint8_t* __restrict__ type,
                                               const V* __restrict__ u, const V* __restrict__ v,
                                               const V* __restrict__ w, const F* __restrict__ T,
                                               const F* __restrict__ kk,
                                               const F* __restrict__ om, double T_ref,
                                               const double* __restrict__ pts, int n,
                                               double* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int nn[3] = {g.nx, g.ny, g.nz};
  const double hh[3] = {g.hx, g.hy, g.hz};
  int lo[3] = {0, 0, 0};
  double t[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < g.dim; ++d) {
    const double f = fmin(fmax(pts[3 * q + d] / hh[d] - 0.5, 0.0), (double)(nn[d] - 1));
    const int i = min((int)floor(f), max(nn[d] - 2, 0));
    lo[d] = i;
    t[d] = f - i;
  }
  double acc[6] = {0, 0, 0, 0, 0, 0}, wsum = 0.0;
  const int corners = g.dim == 3 ? 8 : 4;
  for (int c = 0; c < corners; ++c) {
    int idx[3] = {0, 0, 0};
    double wt = 1.0;
    for (int d = 0; d < g.dim; ++d) {
      const int bit = (c >> d) & 1;
      idx[d] = min(lo[d] + bit, nn[d] - 1);
      wt *= bit ? t[d] : 1.0 - t[d];
    }
    const int P = g.idx(idx[0], idx[1], idx[2]);
    if (!is_fluid(type[P])) continue;
    wsum += wt;
    acc[0] += wt * (double)u[P];
    acc[1] += wt * (double)v[P];
    acc[2] += wt * (double)w[P];
    acc[3] += wt * ((double)T[P] + T_ref);
    acc[4] += wt * (double)kk[P];
    acc[5] += wt * (double)om[P];
  }
  double* o = out + 4 * q;
  if (wsum > 0.0) {
    double val[6];
    for (int a = 0; a < 6; ++a) val[a] = acc[a] / wsum;
    o[0] = sqrt(val[0] * val[0] + val[1] * val[1] + val[2] * val[2]);
    o[1] = val[3];
    o[2] = val[4];
    o[3] = val[5];
  } else {
    o[0] = o[1] = o[2] = o[3] = __builtin_nan("");
  }
}

template <class V, class F>
void launch_probe(const Geom& g, const uint8_t* type, const V* u, const V* v, const V* w,
                  const F* T, const F* k, const F* om, double T_ref, const double* pts, int n,
                  double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_probe<V, F>), dim3((n + 255) / 256), dim3(256), 0, s, g, type, u, v, w,
                     T, k, om, T_ref, pts, n, out);
}
template void launch_probe<double, double>(const Geom&, const uint8_t*, const double*,
                                           const double*, const double*, const double*,
                                           const double*, const double*, double, const double*,
                                           int, double*, hipStream_t);
template void launch_probe<float, float>(const Geom&, const uint8_t*, const float*, const float*,
                                         const float*, const float*, const float*, const float*,
                                         double, const double*, int, double*, hipStream_t);
template void launch_probe<double, float>(const Geom&, const uint8_t*, const double*,
                                          const double*, const double*, const float*,
                                          const float*, const float*, double, const double*, int,
                                          double*, hipStream_t);

}  // namespace nfvm
