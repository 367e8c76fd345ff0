// Declarations shared by the scan, top-k and batched translation units.
#pragma once

#include "common.hpp"

namespace bolt {

enum class OutMode { U16, F32, F32T };

// Queries below this count use the few-query scan (tables as 16-byte rows).
constexpr int kSmallQ = 8;

// -1 automatic, 0 generic, 1 few-query, 2 grouped (set by a test hook).
extern int g_force_scan_kernel;

// uint16 scan into out[Q][ldo] on stream s (arguments already validated).
int scan_u16(const uint8_t *codes, int64_t N, int M, const uint8_t *luts, int64_t Q, uint16_t *out,
             int64_t ldo, hipStream_t s);

// Top-k of the rows of a uint16 matrix (arguments already validated).
int topk_u16(const uint16_t *d, int64_t Q, int64_t N, int64_t ldd, int k, int largest,
             uint16_t *vals, int32_t *idx, hipStream_t s);

}  // namespace bolt
