// Complex128 GEMM on the FP64 matrix cores (v_mfma_f64_16x16x4_f64).
//
// A complex product C = A*B is four real products: Re C = Ar*Br - Ai*Bi,
// Im C = Ar*Bi + Ai*Br (no 3M trick, so rounding matches the plain 4-multiply form).
// Each work-group computes a 64 x 64 complex tile with 4 waves (2 x 2), each wave a
// 32 x 32 tile made of 2 x 2 MFMA tiles of 16 x 16 with four FP64 accumulators
// (rr, ii, ri, ir). K advances 16 complex at a time through LDS, with real and
// imaginary planes stored k-major so the MFMA operand reads are contiguous.
//
// MFMA 16x16x4 f64 lane layout (measured on gfx950): A operand lane l holds
// A[l%16][l/16], B operand lane l holds B[l/16][l%16], accumulator element r of
// lane l is C[4r + l/16][l%16].
//
// Modes (see desc.hpp): 0 plain grouped GEMM for the selected-inverse products,
// 1 transformed pivot rows of a Gauss-Jordan block step, 2 the front update of
// that step, written to the other pool with the step's row permutation applied.
#include "desc.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace clsel {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16;
constexpr int kGemmThreads = 256;

struct GemmCtx {
  double2* fronts;
  int64_t cfg_stride;
  int64_t pool_elems;
  double2* ws;
  int64_t ws_stride;
  const int32_t* iws;
  int64_t iws_stride;
};

__device__ __forceinline__ const double2* pool_ptr(const GemmCtx& g, int b, int pool) {
  if (pool == kPoolWs) return g.ws + b * g.ws_stride;
  return g.fronts + b * g.cfg_stride + (int64_t)pool * g.pool_elems;
}

__device__ __forceinline__ double2 load_a(const GemmDesc& d, const GemmCtx& g, int b, int i, int t) {
  const double2 z = make_double2(0.0, 0.0);
  if (i >= d.M || t >= d.K) return z;
  if (d.mode == 0) return pool_ptr(g, b, d.a_pool)[d.a_off + (int64_t)i * d.lda + t];
  if (d.mode == 1) return (g.ws + b * g.ws_stride)[d.pinv_off + (int64_t)i * d.nbk + t];
  // mode 2: panel columns of the old front, pivot rows replaced by -e_t
  if (i >= d.k && i < d.k + d.nbk) return make_double2(i - d.k == t ? -1.0 : 0.0, 0.0);
  const int src = g.iws[b * g.iws_stride + d.rmap_off + i];
  return (g.fronts + b * g.cfg_stride)[d.x_off + (int64_t)src * d.ld + d.k + t];
}

__device__ __forceinline__ double2 load_b(const GemmDesc& d, const GemmCtx& g, int b, int t, int j) {
  const double2 z = make_double2(0.0, 0.0);
  if (t >= d.K || j >= d.N) return z;
  if (d.mode == 0) return pool_ptr(g, b, d.b_pool)[d.b_off + (int64_t)t * d.ldb + j];
  if (d.mode == 1) {
    if (j >= d.k && j < d.k + d.nbk) return make_double2(j - d.k == t ? 1.0 : 0.0, 0.0);
    const int src = g.iws[b * g.iws_stride + d.piv_off + t];
    return (g.fronts + b * g.cfg_stride)[d.x_off + (int64_t)src * d.ld + j];
  }
  return (g.ws + b * g.ws_stride)[d.rt_off + (int64_t)t * d.N + j];
}

__device__ __forceinline__ void store_c(const GemmDesc& d, const GemmCtx& g, int b, int i, int j,
                                        double2 acc) {
  if (d.mode == 0) {
    double2 v = cscale(acc, d.alpha);
    if (d.has_c0) v = cadd(v, pool_ptr(g, b, d.c0_pool)[d.c0_off + (int64_t)i * d.ldc0 + j]);
    const_cast<double2*>(pool_ptr(g, b, d.c_pool))[d.c_off + (int64_t)i * d.ldc + j] = v;
    return;
  }
  if (d.mode == 1) {
    (g.ws + b * g.ws_stride)[d.rt_off + (int64_t)i * d.N + j] = acc;
    return;
  }
  // mode 2: Y = base - A*Rt, base = X[rmap(i)][j] off the pivot rows and panel columns
  double2* F = g.fronts + b * g.cfg_stride;
  double2 base = make_double2(0.0, 0.0);
  const bool prow = i >= d.k && i < d.k + d.nbk;
  const bool pcol = j >= d.k && j < d.k + d.nbk;
  if (!prow && !pcol) {
    const int src = g.iws[b * g.iws_stride + d.rmap_off + i];
    base = F[d.x_off + (int64_t)src * d.ld + j];
  }
  int oc = j;
  if (d.last && j < d.p) oc = g.iws[b * g.iws_stride + d.rowid_off + j];
  F[d.y_off + (int64_t)i * d.ld + oc] = csub(base, acc);
}

__global__ void __launch_bounds__(kGemmThreads)
k_gemm(const GemmDesc* __restrict__ descs, int ndesc, GemmCtx g) {
  const int b = blockIdx.y;
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile_start <= (int64_t)blockIdx.x) lo = mid; else hi = mid - 1;
  }
  const GemmDesc d = descs[lo];
  const int64_t tile = (int64_t)blockIdx.x - d.tile_start;
  const int row0 = (int)(tile / d.tiles_n) * BM;
  const int col0 = (int)(tile % d.tiles_n) * BN;

  __shared__ double As[2][BK][BM + 1];
  __shared__ double Bs[2][BK][BN + 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, l4 = lane >> 4;

  d4 acc[2][2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[i][j][q] = d4{0.0, 0.0, 0.0, 0.0};

  for (int k0 = 0; k0 < d.K; k0 += BK) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {  // A tile: 64 rows x 16 k
      const int m = (tid >> 4) + 16 * r, kk = tid & 15;
      const double2 v = load_a(d, g, b, row0 + m, k0 + kk);
      As[0][kk][m] = v.x;
      As[1][kk][m] = v.y;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {  // B tile: 16 k x 64 cols
      const int n = tid & 63, kk = (tid >> 6) + 4 * r;
      const double2 v = load_b(d, g, b, k0 + kk, col0 + n);
      Bs[0][kk][n] = v.x;
      Bs[1][kk][n] = v.y;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < BK / 4; ++k4) {
      const int kk = 4 * k4 + l4;
      double ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ar[i] = As[0][kk][wm * 32 + i * 16 + l16];
        ai[i] = As[1][kk][wm * 32 + i * 16 + l16];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        br[j] = Bs[0][kk][wn * 32 + j * 16 + l16];
        bi[j] = Bs[1][kk][wn * 32 + j * 16 + l16];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], acc[i][j][0], 0, 0, 0);
          acc[i][j][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], bi[j], acc[i][j][1], 0, 0, 0);
          acc[i][j][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], acc[i][j][2], 0, 0, 0);
          acc[i][j][3] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], acc[i][j][3], 0, 0, 0);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wm * 32 + i * 16 + 4 * r + l4;
        const int col = col0 + wn * 32 + j * 16 + l16;
        if (row < d.M && col < d.N) {
          const double2 c = make_double2(acc[i][j][0][r] - acc[i][j][1][r],
                                         acc[i][j][2][r] + acc[i][j][3][r]);
          store_c(d, g, b, row, col, c);
        }
      }
}

void launch_gemm(dim3 grid, hipStream_t st, const GemmDesc* descs, int ndesc, double2* fronts,
                 int64_t cfg_stride, int64_t pool_elems, double2* ws, int64_t ws_stride,
                 const int32_t* iws, int64_t iws_stride) {
  GemmCtx g{fronts, cfg_stride, pool_elems, ws, ws_stride, iws, iws_stride};
  hipLaunchKernelGGL(k_gemm, grid, dim3(kGemmThreads), 0, st, descs, ndesc, g);
}

}  // namespace clsel
