// Limits and tile sizes shared by the kernels and the host launch tables.
#pragma once
#include <cstdint>

namespace clsel {

constexpr int kMaxNB = 64;            // widest Gauss-Jordan block
// output tiles of the plain (mode 0) GEMMs
constexpr int kTile64 = 64, kTile128x64 = 12864, kTile128 = 128;
constexpr int kMaxPivotRows = 1536;   // pivot rows per supernode the panel kernel can hold
// K-chunk of the blocked summation of the plain GEMMs: each output sums kKChunk products
// in the matrix-core accumulator, then adds that partial sum to its running total
constexpr int kKChunk = 128;
constexpr int kMaxChunks = 96;        // longer K: chunks of ceil(K / kMaxChunks) products (whole stages);
                                      // K <= 12288 always sums in chunks of kKChunk
// front assembly and Z_SS gather: tile of one 256-thread work-group (one column per thread)
constexpr int kAsmTileRows = 8, kAsmTileCols = 256;
constexpr int kMaxLowRank = 1024;     // columns of the low-rank correction
constexpr int32_t kStatusSingular = -4;
constexpr int32_t kStatusNonFinite = -5;

}  // namespace clsel
