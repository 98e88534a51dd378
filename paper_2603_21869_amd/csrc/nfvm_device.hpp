// Device helpers shared by the kernel files: storage conversions, the
// deterministic device-wide reduction, ghost rules and the k-omega closure.
#pragma once

#include <math.h>

#include "nfvm_internal.hpp"

namespace nfvm {

// ---- storage types ---------------------------------------------------------
// bf16 keeps the top 16 bits of an IEEE float; conversion rounds to nearest even.
__device__ __forceinline__ float bf_to_f(bf16 h) { return __uint_as_float(((uint32_t)h.v) << 16); }
__device__ __forceinline__ bf16 f_to_bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  bf16 r;
  r.v = (uint16_t)(u >> 16);
  return r;
}

template <class S, class C>
struct St;
template <>
struct St<double, double> {
  __device__ static double ld(const double* p) { return *p; }
  __device__ static void st(double* p, double v) { *p = v; }
};
template <>
struct St<float, float> {
  __device__ static float ld(const float* p) { return *p; }
  __device__ static void st(float* p, float v) { *p = v; }
};
template <>
struct St<float, double> {
  __device__ static double ld(const float* p) { return (double)*p; }
  __device__ static void st(float* p, double v) { *p = (float)v; }
};
template <>
struct St<double, float> {
  __device__ static float ld(const double* p) { return (float)*p; }
  __device__ static void st(double* p, float v) { *p = (double)v; }
};
template <>
struct St<bf16, float> {
  __device__ static float ld(const bf16* p) { return bf_to_f(*p); }
  __device__ static void st(bf16* p, float v) { *p = f_to_bf(v); }
};

// ---- reductions --------------------------------------------------------------
enum { R_SUM = 0, R_MAX = 1, R_MIN = 2 };

template <int OP>
__device__ __forceinline__ double rop(double a, double b) {
  if (OP == R_SUM) return a + b;
  if (OP == R_MAX) return a > b ? a : b;
  return a < b ? a : b;
}
template <int OP>
__device__ __forceinline__ double rid() {
  return OP == R_SUM ? 0.0 : (OP == R_MAX ? -INFINITY : INFINITY);
}

// Fixed-order reduction of NV values over a block of BS threads (BS a
// multiple of 64): a butterfly over the 64 lanes of each wave (lane l takes
// l ^ 32, then l ^ 16, ..., l ^ 1; every lane ends with the same value, as
// both operands of each step are the same pair), then every thread combines
// the waves' results in wave order.  One barrier; every thread returns the
// result.
template <int NV, int OP, int BS>
__device__ __forceinline__ void block_tree(double (&v)[NV], double (*sh)[BS]) {
  static_assert(BS % 64 == 0, "block size must be whole waves");
  constexpr int NW = BS / 64;
  const int t = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
#pragma unroll
  for (int q = 0; q < NV; ++q) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[q] = rop<OP>(v[q], __shfl_xor(v[q], off));
  }
  if ((t & 63) == 0)
    for (int q = 0; q < NV; ++q) sh[q][t >> 6] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double acc = sh[q][0];
#pragma unroll
    for (int w = 1; w < NW; ++w) acc = rop<OP>(acc, sh[q][w]);
    v[q] = acc;
  }
}

// Every block stores its partial in red.partial[block * NV + q]; a separate
// one-workgroup kernel (launch_finalize) then reduces the partials in a fixed
// order, so the result does not depend on block scheduling.  Must be called
// by every thread of every block.
// (pb: the partial's index; by default the block's index in its launch)
template <int NV, int OP, int BS>
__device__ __forceinline__ void block_partial(double (&v)[NV], const RedBuf& red, int pb = -1) {
  __shared__ double sh[NV][BS];
  const int t = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int b = pb >= 0 ? pb : blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  block_tree<NV, OP, BS>(v, sh);
  if (t == 0)
    for (int q = 0; q < NV; ++q) red.partial[(size_t)b * NV + q] = v[q];
}

// ---- boundary ghosts (Sec. 2.7) --------------------------------------------
// Field codes for ghost rules.
enum { G_U = 0, G_V = 1, G_W = 2, G_P = 3, G_T = 4, G_K = 5, G_OM = 6, G_NUT = 7 };

__device__ __forceinline__ bool is_fluid(uint8_t t) { return (t & 0x7f) == 0; }

// Value standing in for a non-fluid neighbour across a face: a Dirichlet
// value b on the face gives 2b - vP, a zero gradient gives vP.  The patch
// values are read whatever the patch kind and the rule is chosen by
// selects, so a wave whose lanes see different kinds takes no branches.
template <class R>
__device__ __forceinline__ R ghost(const DevPatch& p, int fld, R vP, int komega) {
  const int kind = p.kind;
  const bool in = kind == K_INLET, out = kind == K_OUTLET;
  switch (fld) {
    case G_U:
    case G_V:
    case G_W: {
      const R b = (R)(2.0 * p.U[fld]) - vP;
      return in ? b : (out ? vP : -vP);
    }
    case G_P:
      return out ? -vP : vP;
    case G_T: {
      const R bi = (R)(2.0 * p.T) - vP, bw = (R)(2.0 * p.T_wall) - vP;
      return in ? bi : ((kind == K_WALL && p.T_dirichlet) ? bw : vP);
    }
    case G_K: {
      const R b = (R)(2.0 * p.k) - vP;
      return in ? b : vP;
    }
    case G_OM: {
      const R b = (R)(2.0 * p.omega) - vP;
      return in ? b : vP;
    }
    default: {  // G_NUT
      const R b = (R)(2.0 * p.nut) - vP;
      if (!komega) return (R)0;
      return in ? b : (out ? vP : -vP);
    }
  }
}

// ---- k-omega closure constants (Sec. 2.1) ------------------------------------
// R_beta is not printed in the paper; 8 is the standard low-Reynolds value.
constexpr double C_BETA_I = 0.072, C_BSTAR = 0.09, C_R_K = 6.0, C_A_INF = 0.52,
                 C_A0 = 1.0 / 9.0, C_R_W = 2.95, C_R_BETA = 8.0, C_EPS = 1e-10;

template <class R>
__device__ __forceinline__ R omhat(R om) {
  return om > (R)C_EPS ? om : (R)C_EPS;
}

// nu_t = alpha* k / omega with alpha* = (beta_i/3 + Re_t/R_k) / (1 + Re_t/R_k)
template <class R>
__device__ __forceinline__ R eddy_visc(R nu, R k, R om) {
  const R oh = omhat(om);
  const R ret = k / (nu * oh);
  const R x = ret * (R)(1.0 / C_R_K);
  const R astar = ((R)(C_BETA_I / 3.0) + x) / ((R)1 + x);
  return astar * k / oh;
}

}  // namespace nfvm
