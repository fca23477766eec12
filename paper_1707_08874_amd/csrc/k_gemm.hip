// Complex128 GEMM on the FP64 matrix cores (v_mfma_f64_16x16x4_f64).
//
// A complex product C = A*B is four real products: Re C = Ar*Br - Ai*Bi,
// Im C = Ar*Bi + Ai*Br (not Gauss's three products, whose imaginary part, a difference
// of larger sums, rounds worse).
// Each work-group computes a BM x BN complex tile (64 x 64, or 128 x 64 / 128 x 128)
// with 4 waves (2 x 2), each wave a (BM/2) x (BN/2) tile made of TM x TN MFMA tiles of
// 16 x 16 with two FP64 accumulators (real part fed by Ar*Br and (-Ai)*Bi, imaginary
// part by Ar*Bi and Ai*Br). K advances BK complex per stage through LDS, stored k-major
// as complex pairs, so one 16-byte LDS read gives a lane both parts of its operand. Each
// stage's global loads go to registers one stage ahead; with two LDS buffers (the
// 64 x 64 tile, BK = 8) the registers are stored into the idle buffer right after the
// current stage's MFMAs, so there is one barrier per stage and the kernel fits four
// waves per SIMD. In mode 0 (where the launch allows it) each output is summed in chunks
// of kKChunk products (longer where K exceeds kMaxChunks of them) whose partial sums are
// added to a running total kept in C; the accumulation order over k is then the same for
// the 64 x 64 and 128 x 64 tiles, while the 128 x 128 tile sums all of K in one chain.
//
// MFMA 16x16x4 f64 lane layout (measured on gfx950): A operand lane l holds
// A[l%16][l/16], B operand lane l holds B[l/16][l%16], accumulator element r of
// lane l is C[4r + l/16][l%16].
//
// Modes (see desc.hpp): 0 plain grouped GEMM for the selected-inverse products,
// 1 transformed pivot rows of a Gauss-Jordan block step, 2 the front update of
// that step, written to the other pool with the step's row permutation applied (rows
// from row_base on: the pivot rows, or the update rows' pivot columns, which the
// sweep turns into -L^ by elimination).
// Work-group ids are remapped so that each of the 8 XCDs (separate L2 caches) gets a
// contiguous range of tiles, which share operand rows and columns.
#include <type_traits>

#include "desc.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace clsel {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kGemmThreads = 256;
constexpr int kXcds = 8;
constexpr int kGroupRows = 8;  // rows of tiles per group of the mode-0 raster

struct GemmCtx {
  double2* fronts;
  int64_t cfg_stride;
  int64_t pool_elems;
  double2* ws;
  int64_t ws_stride;
  const int32_t* iws;
  int64_t iws_stride;
  double2* rhs;         // right-hand-side workspace of the solves (pool kPoolRhs)
  int64_t rhs_stride;
  const int32_t* inv_maps;  // plan: front row -> child update row (Schur with has_c0 = 2)
  double2* ext;             // a caller's buffer (pool kPoolExt), per-configuration stride
  int64_t ext_stride;
  const int32_t* lim;       // per-configuration count of live right-hand sides (lim_dim)
  int64_t lim_stride;
};

__device__ __forceinline__ double2* pool_ptr(const GemmCtx& g, int b, int pool) {
  if (pool == kPoolWs) return g.ws + b * g.ws_stride;
  if (pool == kPoolRhs) return g.rhs + b * g.rhs_stride;
  if (pool == kPoolExt) return g.ext + b * g.ext_stride;
  return g.fronts + b * g.cfg_stride + (int64_t)pool * g.pool_elems;
}

// Per-thread operand sources, fixed for the whole K loop. In modes 1 and 2 the descriptor
// fields the loads need are copied here once: read through the descriptor in global memory,
// they would be loaded again at every stage (the loop's stores might alias it), each load
// followed by a wait that also holds the stage's LDS reads. Mode 0 reads its one field, the
// leading dimension of B, from the descriptor: it has no registers to spare for it.
template <int MODE, int RA>
struct Operands {
  const double2* arow[RA];  // A rows handled by this thread (nullptr: zero or special)
  int ai[RA];               // A row index (global)
  const double2* bbase;     // B base
  int64_t ldb;              // B leading dimension (mode 2)
  int k, nbk, row_base;     // the step's pivot block and first row (modes 1 and 2)
  int ld;                   // leading dimension of the front (mode 1)
  const int32_t* piv;       // the step's pivot rows (mode 1)
};

template <int MODE, int RA>
__device__ __forceinline__ double2 ld_a(const Operands<MODE, RA>& o, int r, int t, int Mv, int Kv) {
  const double2 z = make_double2(0.0, 0.0);
  if (t >= Kv || o.ai[r] >= Mv) return z;
  if (MODE == 2) {
    const int i = o.ai[r] + o.row_base;
    if (i >= o.k && i < o.k + o.nbk) return make_double2(i - o.k == t ? -1.0 : 0.0, 0.0);
  }
  return o.arow[r][t];
}

__device__ __forceinline__ unsigned xcd_remap(unsigned bid, unsigned G) {
  const unsigned q = G / kXcds, r = G % kXcds;
  const unsigned x = bid % kXcds, local = bid / kXcds;
  return x * q + min(x, r) + local;
}

// SOLVE: the same kernel for the products of the multi-right-hand-side solves (one side
// narrow, one chain of products per output), instantiated apart so that profiles tell
// the two kinds of launch apart.
template <int MODE, int TM, int TN, int BK, int NBUF, bool SOLVE = false>
__global__ void __launch_bounds__(kGemmThreads, (TM * TN > 4) ? 1 : 4)
k_gemm(const GemmDesc* __restrict__ descs, int ndesc, GemmCtx g) {
  constexpr int BM = 32 * TM, BN = 32 * TN;
  constexpr int RA = BM * BK / kGemmThreads, RB = BN * BK / kGemmThreads;  // loads per thread per stage
  static_assert(RA >= 1 && RB >= 1 && kGemmThreads % BK == 0 && BK % 4 == 0, "load mapping");
  static_assert(NBUF == 1 || NBUF == 2, "one or two LDS buffers");
  const int b = blockIdx.y;
  const unsigned bid = xcd_remap(blockIdx.x, gridDim.x);
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile_start <= (int64_t)bid) lo = mid; else hi = mid - 1;
  }
  const GemmDesc& d = descs[lo];
  const int64_t tile = (int64_t)bid - d.tile_start;
  int row0 = (int)(tile / d.tiles_n) * BM;
  int col0 = (int)(tile % d.tiles_n) * BN;
  if constexpr (MODE == 0 && !SOLVE) {
    // grouped raster: consecutive tiles walk down kGroupRows rows of tiles, then across,
    // so that an XCD's contiguous range of tiles touches fewer operand panels (each XCD has
    // its own L2)
    const int tiles_m = (d.M + BM - 1) / BM;
    const int64_t per_group = (int64_t)kGroupRows * d.tiles_n;
    const int first = (int)(tile / per_group) * kGroupRows;
    const int gm = min(tiles_m - first, kGroupRows);
    const int in = (int)(tile % per_group);
    row0 = (first + in % gm) * BM;
    col0 = (in / gm) * BN;
  }
  if constexpr (SOLVE) {
    if (d.lim_dim == 1) {
      // rows past the live count are cut: the tiles run rows fastest, so that the cut ones
      // are spread over every XCD's range of tiles instead of filling the last XCDs' ranges
      const int tiles_m = (d.M + BM - 1) / BM;
      row0 = (int)(tile % tiles_m) * BM;
      col0 = (int)(tile / tiles_m) * BN;
    }
  }
  // the product's extent; in the solves the right-hand sides past this configuration's
  // live count are neither read nor written (their columns or rows of the result stay
  // as they were; the kernels that read them skip them too)
  int Mv = d.M, Nv = d.N, Kv = d.K;
  if constexpr (SOLVE) {
    if (d.lim_dim) {
      const int c = g.lim[b * g.lim_stride];
      if (d.lim_dim == 1) Mv = min(Mv, c); else Nv = min(Nv, c);
      if (d.lim_dim == 3) Kv = min(Kv, c);
      if (row0 >= Mv || col0 >= Nv) return;  // uniform over the work-group
    }
  }

  __shared__ double2 As[NBUF][BK][BM + 1];  // +1: the k-strided stores spread over banks
  __shared__ double2 Bs[NBUF][BK][BN + 1];
  static_assert(BN <= kGemmThreads && kGemmThreads % BN == 0, "B load mapping");

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int a_kk = tid % BK;          // A loads: rows tid / BK + (256/BK) r, k = tid % BK
  const int a_m0 = tid / BK;
  constexpr int a_mstep = kGemmThreads / BK;
  const int b_n = tid % BN;           // B loads: col tid % BN, k rows tid / BN + (256/BN) r
  const int b_kk0 = tid / BN;
  constexpr int b_kstep = kGemmThreads / BN;

  double2* F = g.fronts + b * g.cfg_stride;
  double2* W = g.ws + b * g.ws_stride;
  const int32_t* IW = g.iws + b * g.iws_stride;

  Operands<MODE, RA> o;
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    const int i = row0 + a_m0 + a_mstep * r;
    o.ai[r] = i;
    o.arow[r] = nullptr;
    if (i < Mv) {
      if (MODE == 0) o.arow[r] = pool_ptr(g, b, d.a_pool) + d.a_off + (int64_t)i * d.lda;
      else if (MODE == 1) o.arow[r] = W + d.pinv_off + (int64_t)i * d.nbk;
      else o.arow[r] = F + d.x_off + (int64_t)IW[d.rmap_off + d.row_base + i] * d.ld + d.k;
    }
  }
  const int bcol = col0 + b_n;
  if (MODE == 0) o.bbase = pool_ptr(g, b, d.b_pool) + d.b_off;
  else if (MODE == 1) o.bbase = F + d.x_off;
  else o.bbase = W + d.rt_off;
  if constexpr (MODE != 0) {
    o.ldb = d.ldb;
    o.k = d.k;
    o.nbk = d.nbk;
    o.row_base = d.row_base;
    o.ld = d.ld;
    o.piv = IW + d.piv_off;
  }

  auto ld_b = [&](int t) __attribute__((always_inline)) -> double2 {
    const double2 z = make_double2(0.0, 0.0);
    const int j = bcol;
    if (t >= Kv || j >= Nv) return z;
    if (MODE == 0) return o.bbase[(int64_t)t * d.ldb + j];
    if (MODE == 1) {
      if (j >= o.k && j < o.k + o.nbk) return make_double2(j - o.k == t ? 1.0 : 0.0, 0.0);
      return o.bbase[(int64_t)o.piv[t] * o.ld + j];
    }
    return o.bbase[(int64_t)t * o.ldb + j];
  };

  d4 cr[TM][TN], ci[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      cr[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      ci[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }

  double2 pa[RA], pb[RB];

  // Each wave owns TM x TN accumulator slots of 16 x 16. In an interior tile slot (i, j)
  // is the sub-tile (2 wm + i, 2 wn + j) of the wave's quadrant. A tile on the ragged edge
  // of a front (sizes not multiples of the tile) has only vr x vc sub-tiles inside the
  // product, and skips the MFMAs of the others. In mode 0 (long K) they are dealt
  // round-robin to the four waves (sub-tile s to wave s % 4), so that all four SIMDs get
  // an equal share and the tile finishes sooner; mode 2 (K = one block) keeps the
  // quadrants, whose shared fragments and row pointers suit its short loop. Slots are
  // uniform over a wave (the wave index goes through readfirstlane, so the compiler
  // keeps them in scalar registers and branches on scalars).
  constexpr int kSlots = TM * TN;
  constexpr bool kRoundRobin = MODE == 0;
  const bool interior = row0 + BM <= Mv && col0 + BN <= Nv;
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  const int vr = (min(BM, Mv - row0) + 15) / 16, vc = (min(BN, Nv - col0) + 15) / 16;
  int srow[kSlots], scol[kSlots];
  bool sok[kSlots];
#pragma unroll
  for (int t = 0; t < kSlots; ++t) {
    if (interior || !kRoundRobin) {
      const int qi = (wave_u >> 1) * TM + t / TN, qj = (wave_u & 1) * TN + t % TN;
      srow[t] = qi * 16;
      scol[t] = qj * 16;
      sok[t] = interior || (qi < vr && qj < vc);
    } else {
      const int sub = wave_u + 4 * t;
      sok[t] = sub < vr * vc;
      srow[t] = (sub / vc) * 16;
      scol[t] = (sub % vc) * 16;
    }
  }

  auto load_stage = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < RA; ++r) pa[r] = ld_a<MODE, RA>(o, r, k0 + a_kk, Mv, Kv);
#pragma unroll
    for (int r = 0; r < RB; ++r) pb[r] = ld_b(k0 + b_kk0 + b_kstep * r);
  };
  auto store_stage = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < RA; ++r) As[buf][a_kk][a_m0 + a_mstep * r] = pa[r];
#pragma unroll
    for (int r = 0; r < RB; ++r) Bs[buf][b_kk0 + b_kstep * r][b_n] = pb[r];
  };
  auto mfma_stage = [&](int buf, auto edge) __attribute__((always_inline)) {
    if constexpr (!decltype(edge)::value) {
      // interior: a 2 x 2 block of sub-tiles shares its A and B fragments
#pragma unroll
      for (int k4 = 0; k4 < BK / 4; ++k4) {
        const int kk = 4 * k4 + l4;
        double2 av[TM], bv[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) av[i] = As[buf][kk][wm * (BM / 2) + i * 16 + l16];
#pragma unroll
        for (int j = 0; j < TN; ++j) bv[j] = Bs[buf][kk][wn * (BN / 2) + j * 16 + l16];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x, bv[j].x, cr[i][j], 0, 0, 0);
            ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x, bv[j].y, ci[i][j], 0, 0, 0);
          }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[i].y, bv[j].y, cr[i][j], 0, 0, 0);
            ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].y, bv[j].x, ci[i][j], 0, 0, 0);
          }
      }
    } else if constexpr (!kRoundRobin) {
      // edge, quadrant slots: fragments of sub-tiles outside the product are not read
      bool rv[TM], cv[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) rv[i] = sok[i * TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) cv[j] = (wave_u & 1) * TN + j < vc;
#pragma unroll
      for (int k4 = 0; k4 < BK / 4; ++k4) {
        const int kk = 4 * k4 + l4;
        double2 av[TM], bv[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
          av[i] = rv[i] ? As[buf][kk][wm * (BM / 2) + i * 16 + l16] : make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < TN; ++j)
          bv[j] = cv[j] ? Bs[buf][kk][wn * (BN / 2) + j * 16 + l16] : make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            if (sok[i * TN + j]) {
              cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x, bv[j].x, cr[i][j], 0, 0, 0);
              ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x, bv[j].y, ci[i][j], 0, 0, 0);
            }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            if (sok[i * TN + j]) {
              cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[i].y, bv[j].y, cr[i][j], 0, 0, 0);
              ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].y, bv[j].x, ci[i][j], 0, 0, 0);
            }
      }
    } else {
      // edge, round-robin slots: each owned sub-tile reads its own fragments
#pragma unroll
      for (int k4 = 0; k4 < BK / 4; ++k4) {
        const int kk = 4 * k4 + l4;
#pragma unroll
        for (int t = 0; t < kSlots; ++t) {
          if (!sok[t]) continue;
          const double2 a = As[buf][kk][srow[t] + l16];
          const double2 bb = Bs[buf][kk][scol[t] + l16];
          d4& xr = cr[t / TN][t % TN];
          d4& xi = ci[t / TN][t % TN];
          xr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, bb.x, xr, 0, 0, 0);
          xi = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, bb.y, xi, 0, 0, 0);
          xr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, bb.y, xr, 0, 0, 0);
          xi = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, bb.x, xi, 0, 0, 0);
        }
      }
    }
  };

  const int nst = (Kv + BK - 1) / BK;
  // Blocked summation (mode 0, d.kblock): the accumulators hold the sum over one chunk of
  // kKChunk products; at the end of each chunk but the last, it is added to the running
  // total, which waits in C (each lane reads and writes only its own outputs), and the
  // accumulators restart from zero. A single chain over all of K would add every product
  // to an ever larger partial sum; with chunks the rounding grows with the chunk length
  // plus the number of chunks instead, which matters where the result is much smaller
  // than the products (the selected-inversion and Schur-complement updates).
  constexpr int kStagesPerChunk = kKChunk / BK;
  static_assert(kKChunk % BK == 0, "chunk of whole stages");
  // (the 128 x 128 tile keeps one chain: its accumulators leave no registers for the
  // partial sums, which would spill)
  constexpr bool kChunkable = MODE == 0 && TM * TN <= 8 && !SOLVE;
  // at most kMaxChunks chunks: a longer K gets longer chunks, which bounds the round trips
  // of the running totals (for K <= kMaxChunks * kKChunk the chunk is kKChunk)
  const int chunk_stages = max(kStagesPerChunk, (nst + kMaxChunks - 1) / kMaxChunks);
  const bool chunked = kChunkable && d.kblock && nst > chunk_stages;
  auto flush_chunk = [&](bool first) __attribute__((always_inline)) {
    // the lane coordinates pass through an empty asm, so that the output addresses are
    // formed here and not kept in registers through the whole K loop
    int lr = l4, lc = l16;
    asm volatile("" : "+v"(lr), "+v"(lc));
    double2* C = pool_ptr(g, b, d.c_pool) + d.c_off;
#pragma unroll
    for (int t = 0; t < kSlots; ++t) {
      const int i = t / TN, j = t % TN;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + srow[t] + 4 * r + lr;
        const int col = col0 + scol[t] + lc;
        if (sok[t] && row < Mv && col < Nv) {
          double2* pc = C + (int64_t)row * d.ldc + col;
          double2 v = make_double2(cr[i][j][r], ci[i][j][r]);
          if (!first) v = cadd(v, *pc);
          *pc = v;
        }
      }
      cr[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      ci[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      // one slot's four loads in flight at a time: the accumulators fill the registers
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  auto pipeline = [&](auto edge) __attribute__((always_inline)) {
    load_stage(0);
    if (NBUF == 1) {
      // one buffer: store the prefetched stage, prefetch the next, MFMAs, two barriers
      int left = chunk_stages;
      for (int st = 0; st + 1 < nst; ++st) {
        store_stage(0);
        __syncthreads();
        load_stage((st + 1) * BK);
        mfma_stage(0, edge);
        if constexpr (kChunkable) {
          if (chunked && --left == 0) {
            flush_chunk(st + 1 == chunk_stages);
            left = chunk_stages;
          }
        }
        __syncthreads();
      }
      store_stage(0);
      __syncthreads();
      mfma_stage(0, edge);
    } else {
      // two buffers: stage st+1 goes into the idle buffer after stage st's MFMAs (that
      // buffer was last read in stage st-1, before the previous barrier): one barrier
      store_stage(0);
      __syncthreads();
      if (nst > 1) load_stage(BK);
      int left = chunk_stages;
      for (int st = 0; st + 1 < nst; ++st) {
        mfma_stage(st & 1, edge);
        store_stage((st + 1) & 1);
        if constexpr (kChunkable) {
          if (chunked && --left == 0) {
            flush_chunk(st + 1 == chunk_stages);
            left = chunk_stages;
          }
        }
        if (st + 2 < nst) load_stage((st + 2) * BK);
        __syncthreads();
      }
      mfma_stage((nst - 1) & 1, edge);
    }
  };
  // (mode 1 has at most one pivot block of rows; its edge copy would not fit four waves,
  // and its edge tiles run the interior copy, which computes every sub-tile)
  if constexpr (MODE == 1) pipeline(std::false_type{});
  else if (interior) pipeline(std::false_type{});
  else pipeline(std::true_type{});

#pragma unroll
  for (int i = 0; i < TM; ++i) {
    // mode 2: the subtrahend of this row block of sub-tiles, all loads in flight together
    double2 bs[TN][4];
    if constexpr (MODE == 2) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wm * (BM / 2) + i * 16 + 4 * r + l4;
        const int frow = d.row_base + row;  // row of the front
        const bool rok = row < d.M && !(frow >= d.k && frow < d.k + d.nbk);
        const double2* xr = rok ? F + d.x_off + (int64_t)IW[d.rmap_off + frow] * d.ld : nullptr;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int col = col0 + wn * (BN / 2) + j * 16 + l16;
          const bool ok = rok && col < d.N && !(col >= d.k && col < d.k + d.nbk);
          bs[j][r] = ok ? xr[col] : make_double2(0.0, 0.0);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int t = i * TN + j;
        // mode 1 runs the interior mapping on every tile
        const int row = row0 + (MODE == 1 ? wm * (BM / 2) + i * 16 : srow[t]) + 4 * r + l4;
        const int col = col0 + (MODE == 1 ? wn * (BN / 2) + j * 16 : scol[t]) + l16;
        if ((MODE != 1 && !sok[t]) || row >= Mv || col >= Nv) continue;
        double2 acc = make_double2(cr[i][j][r], ci[i][j][r]);
        if (MODE == 0) {
          if (chunked) acc = cadd(acc, pool_ptr(g, b, d.c_pool)[d.c_off + (int64_t)row * d.ldc + col]);
          double2 v = cscale(acc, d.alpha);
          if (d.has_c0 == 1) {
            v = cadd(v, pool_ptr(g, b, d.c0_pool)[d.c0_off + (int64_t)row * d.ldc0 + col]);
          } else if (d.has_c0 == 2) {
            // A_SS(row, col) = sum of the children's update blocks at the mapped position,
            // summed in child order as the front assembly sums the other entries
            double2 a = make_double2(0.0, 0.0);
            for (int c = 0; c < d.nchild; ++c) {
              const int ii = g.inv_maps[d.inv_off[c] + d.kid_base + row];
              const int jj = g.inv_maps[d.inv_off[c] + d.kid_base + col];
              if (ii >= 0 && jj >= 0) {
                const int cp = d.child_p[c];
                a = cadd(a, F[d.child_off[c] + (int64_t)(cp + ii) * d.child_ld[c] + cp + jj]);
              }
            }
            v = cadd(v, a);
          }
          pool_ptr(g, b, d.c_pool)[d.c_off + (int64_t)row * d.ldc + col] = v;
        } else if (MODE == 1) {
          W[d.rt_off + (int64_t)row * d.N + col] = acc;
        } else {
          // Y = base - A*Rt, base = X[rmap(row)][col] off the pivot rows and panel columns
          int oc = col;
          if (d.last && col < d.p) oc = IW[d.rowid_off + col];
          F[d.y_off + (int64_t)(d.row_base + row) * d.ld + oc] = csub(bs[j][r], acc);
        }
      }
  }
}

void launch_gemm(int mode, int tile, dim3 grid, hipStream_t st, const GemmDesc* descs, int ndesc,
                 double2* fronts, int64_t cfg_stride, int64_t pool_elems, double2* ws,
                 int64_t ws_stride, const int32_t* iws, int64_t iws_stride, double2* rhs,
                 int64_t rhs_stride, const int32_t* inv_maps, double2* ext, int64_t ext_stride,
                 bool solve, const int32_t* lim, int64_t lim_stride) {
  GemmCtx g{fronts, cfg_stride, pool_elems, ws, ws_stride, iws, iws_stride, rhs, rhs_stride, inv_maps,
            ext, ext_stride, lim, lim_stride};
  const dim3 blk(kGemmThreads);
  if (solve) hipLaunchKernelGGL((k_gemm<0, 2, 2, 8, 2, true>), grid, blk, 0, st, descs, ndesc, g);
  else if (mode == 0 && tile == kTile128) hipLaunchKernelGGL((k_gemm<0, 4, 4, 16, 1>), grid, blk, 0, st, descs, ndesc, g);
  else if (mode == 0 && tile == kTile128x64) hipLaunchKernelGGL((k_gemm<0, 4, 2, 16, 1>), grid, blk, 0, st, descs, ndesc, g);
  else if (mode == 0) hipLaunchKernelGGL((k_gemm<0, 2, 2, 8, 2>), grid, blk, 0, st, descs, ndesc, g);
  else if (mode == 1) hipLaunchKernelGGL((k_gemm<1, 2, 2, 8, 2>), grid, blk, 0, st, descs, ndesc, g);
  else hipLaunchKernelGGL((k_gemm<2, 2, 2, 8, 2>), grid, blk, 0, st, descs, ndesc, g);
}

}  // namespace clsel
