// Launch interface of the shot-major output-format kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace stimgpu {

// Row stride (in uint64) of the shot-major scratch table T: ceil(rows / 64)
// chunks rounded up to a multiple of eight (the transpose writes 64-byte
// pieces of each shot).
inline uint64_t transpose_stride(uint64_t rows) { return ((rows + 63) / 64 + 7) / 8 * 8; }

// table [rows][W] (bit j of word w = shot 64 w + j) -> T [shots][stride]
// (bit i of T[s][c] = row 64 c + i of shot s; rows past the end read as 0).
hipError_t launch_transpose(const uint64_t *table, uint64_t rows, uint64_t W, uint64_t shots, uint64_t *T,
                            hipStream_t stream);
// The b8 format in one pass (the transpose writes the bytes itself); needs
// ceil(rows / 8) a multiple of 4 and a 4-byte aligned `out`.
hipError_t launch_transpose_b8(const uint64_t *table, uint64_t rows, uint64_t W, uint64_t shots, uint8_t *out,
                               hipStream_t stream);
// Dense formats from T: b8 (ceil(rows/8) bytes per shot) or 01 (rows + 1).
hipError_t launch_dense_format(const uint64_t *T, uint64_t rows, uint64_t shots, int b8, uint8_t *out,
                               hipStream_t stream);
// Sparse formats from T (r8 or hits): offs == NULL writes each shot's byte
// count to lens; otherwise writes the bytes of shot s at out + offs[s].
hipError_t launch_sparse_format(const uint64_t *T, uint64_t rows, uint64_t shots, int r8, uint64_t *lens,
                                const uint64_t *offs, uint8_t *out, hipStream_t stream);
// Exclusive prefix sum of n values; `sums` is scratch of kScanBlocks values;
// *total = their sum.
constexpr uint32_t kScanBlocks = 1024;
hipError_t launch_scan(const uint64_t *in, uint64_t n, uint64_t *out, uint64_t *sums, uint64_t *total,
                       hipStream_t stream);

}  // namespace stimgpu
