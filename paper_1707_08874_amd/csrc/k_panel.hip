// Panel step of the frontal Gauss-Jordan sweep: pivot choice and pivot-block inverse.
//
// For the block of columns [k, k+nbk) of a front whose rows [k, p) are the pivot
// candidates (row pivoting stays inside the supernode's own rows), this kernel
//   phase 1: picks the nbk pivot rows by partial pivoting (largest modulus, lowest
//            row on ties), running an in-place Gauss-Jordan elimination of the
//            candidate rows over the panel columns in register groups of 8 to 16
//            columns, with the remaining groups updated lazily in a workspace copy;
//            per column: a DPP arg-max in each wave, the wave winners' rows through
//            LDS, one barrier, a DPP combine of the eight wave results;
//   phase 2: inverts Pi, the nbk x nbk block of the chosen rows in pivot order, by
//            Gauss-Jordan elimination without further pivoting in LDS;
//   and records the row permutation of the step and the equation held by each
//   pivot row (needed to put the columns of the inverse back in natural order).
// Pivot perturbation: where the chosen pivot's modulus is below `floor` (> 0) it is
// raised to `floor` with its phase kept. Row operations only ever subtract multiples of
// other rows, so adding delta to the current pivot entry is adding delta to the entry
// of D at (the pivot row's equation, the pivot column): the sweep factorises that
// perturbed matrix, consistently in both phases (phase 2 adds the same delta to Pi).
// Each pivot column records its delta (zero if none) and the equation that pivots it;
// the selected inversion undoes the perturbations with a low-rank correction.
// One work-group of 512 threads per (front, configuration).
#include "desc.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace clsel {

constexpr int kPanelThreads = 512;
constexpr int kWaves = kPanelThreads / 64;
constexpr int kPiLd = kMaxNB + 1;
// Registers per thread: RPT rows x G columns of the current group (4 VGPRs per complex
// value) plus RPT x CH accumulators of the lazy update must stay within the 256 VGPRs a
// wave has at two waves per SIMD; narrower groups for more rows per thread keep the
// kernel free of scratch spills.
template <int RPT> struct PanelShape;
template <> struct PanelShape<1> { static constexpr int G = 16, CH = 8; };
template <> struct PanelShape<2> { static constexpr int G = 12, CH = 4; };
template <> struct PanelShape<3> { static constexpr int G = 8, CH = 2; };

// Cross-lane helpers for the pivot search. DPP moves stay in the vector ALU, so a
// wave-wide reduction costs a few instructions per step and no LDS round trip.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, ROWS, 0xF, false);
}
// readlane moves 32 bits: a double goes as its two halves
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// Pivot search key of row r with |a|^2 = a2: the bits of a2 (a non-negative double)
// with the low 11 significand bits replaced by 2047 - r. The largest key is the row of
// largest |a|^2, compared to 41 significand bits, and among rows equal to that precision
// the lowest one. Keys are non-negative finite doubles, which order like their bit
// patterns, so one fmax reduction finds value and row together. A NaN ranks with zero
// (the row stays a valid choice and the non-finite pivot is flagged); +inf becomes the
// largest finite key. Rows out of the search take -1.
static_assert(kMaxPivotRows <= 2048, "pivot keys hold the row in 11 bits");
__device__ __forceinline__ double pivot_key(double a2, int r) {
  unsigned long long u = __builtin_bit_cast(unsigned long long, a2);
  u = (a2 == a2) ? u : 0ull;
  u = u >= 0x7FF0000000000000ull ? 0x7FEFFFFFFFFFFFFFull : u;
  return __builtin_bit_cast(double, (u & ~0x7FFull) | (unsigned long long)(0x7FF - r));
}
__device__ __forceinline__ int key_row(double key) {
  return 0x7FF - (int)(__builtin_bit_cast(unsigned long long, key) & 0x7FFull);
}
// Largest key over the wave, returned to every lane: DPP quad permutes, row rotations
// by 4 and 8, row broadcasts 15 and 31, then lane 63.
__device__ __forceinline__ double wave_max(double m) {
  m = fmax(m, dpp_f64<0xB1, 0xF>(m));
  m = fmax(m, dpp_f64<0x4E, 0xF>(m));
  m = fmax(m, dpp_f64<0x124, 0xF>(m));
  m = fmax(m, dpp_f64<0x128, 0xF>(m));
  m = fmax(m, dpp_f64<0x142, 0xA>(m));
  m = fmax(m, dpp_f64<0x143, 0xC>(m));
  return readlane_f64(m, 63);
}
// The same over the kWaves wave results, lane l holding result l % 8: each group of
// eight lanes ends with the maximum of all eight.
__device__ __forceinline__ double combine_waves(double m) {
  static_assert(kWaves == 8, "three DPP steps combine eight lanes");
  m = fmax(m, dpp_f64<0xB1, 0xF>(m));
  m = fmax(m, dpp_f64<0x4E, 0xF>(m));
  m = fmax(m, dpp_f64<0x124, 0xF>(m));
  return m;
}

template <int RPT>
__global__ void __launch_bounds__(kPanelThreads)
k_panel(const PanelDesc* __restrict__ descs, const double2* __restrict__ fronts, int64_t cfg_stride,
        double2* __restrict__ ws, int64_t ws_stride, int32_t* __restrict__ iws, int64_t iws_stride,
        int32_t* __restrict__ status, double floor) {
  const PanelDesc d = descs[blockIdx.x];
  const int b = blockIdx.y;
  const int tid = threadIdx.x;
  const double2* X = fronts + b * cfg_stride + d.x_off;
  double2* PW = ws + b * ws_stride + d.pw_off;
  double2* Pinv = ws + b * ws_stride + d.pinv_off;
  int32_t* IW = iws + b * iws_stride;
  const int cand = d.p - d.k, nbk = d.nbk, ld = d.ld, k = d.k;
  constexpr int kGroup = PanelShape<RPT>::G;

  __shared__ double2 s_cand[2][kWaves][kGroup];  // each wave's best row, per column parity
  __shared__ double s_key[2][kWaves];
  __shared__ int s_piv[kMaxNB];
  __shared__ double2 s_delta[kMaxNB];  // perturbation of each pivot of the block
  __shared__ int s_flag;
  __shared__ double2 s_pcol[2][kMaxNB];
  __shared__ double2 s_buf[kMaxNB * kPiLd];
  __shared__ int s_at[kMaxPivotRows];
  __shared__ int s_pos[kMaxPivotRows];

  // Column group 0 is read straight from the front; the lazy update after each group
  // writes the later groups of the unused rows to PW, column-major with leading
  // dimension cand (a wave's lanes hold consecutive rows, so its accesses to one column
  // are contiguous), which is where groups >= 1 are read from.
  const double2* Xp = X + (int64_t)k * ld + k;  // candidate row 0, panel column 0
  if (tid == 0) s_flag = 0;
  __syncthreads();

  bool used[RPT];
  double2 cur[RPT][kGroup];
#pragma unroll
  for (int j = 0; j < RPT; ++j) used[j] = false;
  const int lane = tid & 63, wave = tid >> 6;
  // a wave whose first row is past the candidates holds no candidate row at all (its
  // rows are tid + j * kPanelThreads); it only takes part in the barriers
  const bool wave_dead = (tid & ~63) >= cand;

  // ---- phase 1: pivot choice
  for (int g0 = 0; g0 < nbk; g0 += kGroup) {
    const int gw = min(kGroup, nbk - g0);
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int r = tid + j * kPanelThreads;
      const bool live = r < cand && !used[j];
      // element (r, c) of the group: the front (row-major) for group 0, else PW
      const double2* src = g0 == 0 ? Xp + (int64_t)r * ld : PW + (int64_t)g0 * cand + r;
      const int64_t cs = g0 == 0 ? 1 : cand;
#pragma unroll
      for (int c = 0; c < kGroup; ++c)
        cur[j][c] = (live && c < gw) ? src[c * cs] : make_double2(0.0, 0.0);
    }
    // Each column step rotates the row registers by one slot: the column being
    // eliminated is always slot 0, the updated later columns move down one slot and
    // the multiplier goes to the last slot, so every register index is a constant.
    // All kGroup steps run (steps past the group width only rotate), which brings the frame
    // back: slot t then holds the multiplier of the group's pivot t.
    auto column_step = [&](int c) {
      if (c < gw) {
        const int par = c & 1;
        if (!wave_dead) {
          double key = -1.0;
#pragma unroll
          for (int j = 0; j < RPT; ++j) {
            const int r = tid + j * kPanelThreads;
            const double kj = (r < cand && !used[j]) ? pivot_key(cabs2(cur[j][0]), r) : -1.0;
            key = fmax(key, kj);
          }
          key = wave_max(key);
          // the lane holding its wave's best row publishes it: one barrier per column
          const int bi = key >= 0.0 ? key_row(key) : -1;
#pragma unroll
          for (int j = 0; j < RPT; ++j)
            if (tid + j * kPanelThreads == bi) {
#pragma unroll
              for (int cc = 0; cc < kGroup; ++cc) s_cand[par][wave][cc] = cur[j][cc];
            }
          if (lane == 0) s_key[par][wave] = key;
        } else if (lane == 0) {
          s_key[par][wave] = -1.0;
        }
        __syncthreads();
        const double kk = combine_waves(s_key[par][lane & (kWaves - 1)]);
        int pr = kk >= 0.0 ? key_row(kk) : -1;
        const bool found = pr >= 0 && pr < cand;
        if (!found) pr = 0;  // keeps every index in range; flagged below
        const int ww = (pr & (kPanelThreads - 1)) >> 6;  // the wave that owns row pr
        const double2* pv = s_cand[par][ww];
        if (tid == 0) s_piv[g0 + c] = pr;
#pragma unroll
        for (int j = 0; j < RPT; ++j) used[j] = used[j] || (tid + j * kPanelThreads == pr);
        double2 dp = found ? pv[0] : make_double2(0.0, 0.0);
        const bool finite = isfinite(dp.x) && isfinite(dp.y);
        double2 delta = make_double2(0.0, 0.0);
        if (floor > 0.0 && finite && cabs2(dp) < floor * floor) {
          // raise the modulus to floor, keeping the phase (a zero pivot becomes floor)
          const double a = sqrt(cabs2(dp));
          const double2 up = a > 0.0 ? cscale(dp, floor / a) : make_double2(floor, 0.0);
          delta = csub(up, dp);
          dp = up;
        }
        if (tid == 0) {
          s_delta[g0 + c] = delta;
          if (!found || !finite || !(cabs2(dp) > 0.0)) s_flag = 1;
        }
        if (!(cabs2(dp) > 0.0) || !finite) dp = make_double2(1.0, 0.0);
        const double2 invd = crecip(dp);
        // rows out of the elimination (pivots, rows past the candidates, every row of a
        // wave past the candidates) take a zero multiplier and only rotate; their values
        // are not read again
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const bool live = tid + j * kPanelThreads < cand && !used[j];
          const double2 f = cmul(cur[j][0], invd);
          const double2 fi = live ? f : make_double2(0.0, 0.0);
#pragma unroll
          for (int cc = 0; cc + 1 < kGroup; ++cc) cur[j][cc] = cfms(cur[j][cc + 1], fi, pv[cc + 1]);
          cur[j][kGroup - 1] = make_double2(-fi.x, -fi.y);
        }
      } else {
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const double2 t0 = cur[j][0];
#pragma unroll
          for (int cc = 0; cc + 1 < kGroup; ++cc) cur[j][cc] = cur[j][cc + 1];
          cur[j][kGroup - 1] = t0;
        }
      }
    };
    // unrolled by 4 (register renaming makes the rotation free)
#pragma unroll 4
    for (int c = 0; c < kGroup; ++c) column_step(c);
    __syncthreads();  // s_piv of this group
    // lazy update of the later column groups of the still-unused rows:
    // PW(r, cc) += sum_t W_r[t] * R[t][cc], R = group pivot rows at group start
    const int rest0 = g0 + gw, nrest = nbk - rest0;
    if (nrest > 0) {
      for (int e = tid; e < gw * nrest; e += kPanelThreads) {
        const int t = e / nrest, cc = e % nrest;
        const int pr = s_piv[g0 + t];
        s_buf[t * kMaxNB + cc] = g0 == 0 ? Xp[(int64_t)pr * ld + rest0 + cc]
                                         : PW[(int64_t)(rest0 + cc) * cand + pr];
      }
      __syncthreads();
      // Chunks of CH columns of all RPT rows, software-pipelined: the loads of the next
      // chunk are issued before the products of the current one, so that their latency
      // overlaps arithmetic (each chunk's loads otherwise wait a full memory round trip).
      // They read columns the current chunk does not write, except the clamped reads past
      // the last column, whose values are discarded.
      constexpr int kChunk = PanelShape<RPT>::CH;
      // The loads are unconditional (addresses clamped into the panel, values of rows and
      // columns outside it replaced by zero afterwards): no branch around them, so the
      // wait before the products covers only the current chunk's loads.
      auto load_chunk = [&](int c0, double2 (&a)[RPT][kChunk]) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const int r = tid + j * kPanelThreads;
          const bool ok = r < cand && !used[j];
          const int rc = r < cand ? r : 0;
#pragma unroll
          for (int q = 0; q < kChunk; ++q) {
            const int col = rest0 + min(c0 + q, nrest - 1);
            const double2 v = g0 == 0 ? Xp[(int64_t)rc * ld + col] : PW[(int64_t)col * cand + rc];
            a[j][q] = (ok && c0 + q < nrest) ? v : make_double2(0.0, 0.0);
          }
        }
      };
      // products and stores of one chunk (the sum over t runs in the same order for every
      // element; each pivot-row value is read from LDS once and used for all RPT rows)
      auto update_chunk = [&](int c0, double2 (&a)[RPT][kChunk]) __attribute__((always_inline)) {
#pragma unroll
        for (int t = 0; t < kGroup; ++t) {
          if (t < gw) {
            double2 rv[kChunk];
#pragma unroll
            for (int q = 0; q < kChunk; ++q) rv[q] = s_buf[t * kMaxNB + min(c0 + q, nrest - 1)];
#pragma unroll
            for (int q = 0; q < kChunk; ++q)
#pragma unroll
              for (int j = 0; j < RPT; ++j) a[j][q] = cfma(a[j][q], cur[j][t], rv[q]);
          }
        }
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const int r = tid + j * kPanelThreads;
          if (r < cand && !used[j]) {
            double2* dst = PW + (int64_t)(rest0 + c0) * cand + r;
#pragma unroll
            for (int q = 0; q < kChunk; ++q)
              if (c0 + q < nrest) dst[(int64_t)q * cand] = a[j][q];
          }
        }
      };
      // two register buffers in turn: the next chunk's loads are in flight during the
      // current chunk's products
      if (!wave_dead) {
        double2 ca[RPT][kChunk], cb[RPT][kChunk];
        load_chunk(0, ca);
        for (int c0 = 0; c0 < nrest; c0 += 2 * kChunk) {
          load_chunk(c0 + kChunk, cb);
          update_chunk(c0, ca);
          if (c0 + kChunk >= nrest) break;
          load_chunk(c0 + 2 * kChunk, ca);
          update_chunk(c0 + kChunk, cb);
        }
      }
      __syncthreads();
    }
  }

  // ---- phase 2: Pi^{-1} by Gauss-Jordan without pivoting (rows already in pivot order).
  // Thread (t, cg) = (tid / 8, tid % 8) keeps entries (t, 8cg .. 8cg+7) in registers; per
  // column the pivot row and the pivot column go through LDS (double-buffered), one
  // barrier per column.
  __syncthreads();
  {
    const int t = tid >> 3, cg = tid & 7;
    const bool live = t < nbk;
    double2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int cc = cg * 8 + q;
      v[q] = (live && cc < nbk) ? Xp[(int64_t)s_piv[t] * ld + cc] : make_double2(0.0, 0.0);
      if (live && cc == t) v[q] = cadd(v[q], s_delta[t]);  // the perturbed pivot, as in phase 1
    }
    // Columns in blocks of eight, unrolled: column c = cb + qc is entry qc of the threads
    // with cg = cb / 8, so every register index below is a constant.
    for (int cb = 0; cb < nbk; cb += 8) {
      const bool own = cg == (cb >> 3);  // this thread holds column c of its row
#pragma unroll
      for (int qc = 0; qc < 8; ++qc) {
        const int c = cb + qc;
        if (c < nbk) {  // uniform over the work-group
          const int par = qc & 1;
          if (live && t == c) {
#pragma unroll
            for (int q = 0; q < 8; ++q) s_buf[par * kPiLd + cg * 8 + q] = v[q];
          }
          if (live && own) s_pcol[par][t] = v[qc];
          __syncthreads();
          double2 dp = s_buf[par * kPiLd + c];
          if (!(cabs2(dp) > 0.0) || !isfinite(dp.x) || !isfinite(dp.y)) {
            if (tid == 0) s_flag = 1;
            dp = make_double2(1.0, 0.0);
          }
          const double2 invd = crecip(dp);
          if (live) {
            if (t == c) {
#pragma unroll
              for (int q = 0; q < 8; ++q) v[q] = (own && q == qc) ? invd : cmul(v[q], invd);
            } else {
              const double2 fi = cmul(s_pcol[par][t], invd);
#pragma unroll
              for (int q = 0; q < 8; ++q)
                v[q] = (own && q == qc) ? make_double2(-fi.x, -fi.y)
                                        : cfms(v[q], fi, s_buf[par * kPiLd + cg * 8 + q]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int cc = cg * 8 + q;
      if (live && cc < nbk) Pinv[t * nbk + cc] = v[q];
    }
  }
  __syncthreads();

  // ---- pivot list, perturbation record, row map of this step, equation ids of the pivot rows
  if (tid < nbk) {
    IW[d.piv_off + tid] = k + s_piv[tid];
    ws[b * ws_stride + d.pdelta_off + k + tid] = s_delta[tid];
    IW[d.peq_off + k + tid] = d.pbase + IW[d.rowid_off + k + s_piv[tid]];
  }
  for (int i = tid; i < cand; i += kPanelThreads) { s_at[i] = i; s_pos[i] = i; }
  __syncthreads();
  if (tid == 0) {
    for (int t = 0; t < nbk; ++t) {  // move candidate s_piv[t] to position t
      const int r = s_piv[t], pr = s_pos[r], rt = s_at[t];
      s_at[pr] = rt; s_pos[rt] = pr;
      s_at[t] = r;   s_pos[r] = t;
    }
  }
  __syncthreads();
  for (int i = tid; i < d.H; i += kPanelThreads)
    IW[d.rmap_off + i] = (i >= k && i < d.p) ? k + s_at[i - k] : i;
  int32_t* rowid = IW + d.rowid_off;
  for (int i = tid; i < cand; i += kPanelThreads) s_pos[i] = rowid[k + s_at[i]];
  __syncthreads();
  for (int i = tid; i < cand; i += kPanelThreads) rowid[k + i] = s_pos[i];
  if (tid == 0 && s_flag) atomicMin(&status[b], kStatusSingular);
}

void launch_panel(int rpt, dim3 grid, hipStream_t st, const PanelDesc* descs, const double2* fronts,
                  int64_t cfg_stride, double2* ws, int64_t ws_stride, int32_t* iws,
                  int64_t iws_stride, int32_t* status, double floor) {
  switch (rpt) {
    case 1: hipLaunchKernelGGL(k_panel<1>, grid, dim3(kPanelThreads), 0, st, descs, fronts, cfg_stride, ws, ws_stride, iws, iws_stride, status, floor); break;
    case 2: hipLaunchKernelGGL(k_panel<2>, grid, dim3(kPanelThreads), 0, st, descs, fronts, cfg_stride, ws, ws_stride, iws, iws_stride, status, floor); break;
    default: hipLaunchKernelGGL(k_panel<3>, grid, dim3(kPanelThreads), 0, st, descs, fronts, cfg_stride, ws, ws_stride, iws, iws_stride, status, floor); break;
  }
}

}  // namespace clsel
