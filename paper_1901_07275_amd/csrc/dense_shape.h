// Shape of a dense (matrix-core) axis pass, shared by the host queue builder
// and the kernels: a block stages R lines of the pass in LDS and computes all
// R x n outputs, so every R lines read the n x n matrix once.
#pragma once

#include <cstddef>

namespace jt {

// Longest axis the dense pass takes.
constexpr int kDenseMax = 1024;
// LDS row stride (elements) of the staged lines: odd, against bank conflicts.
constexpr int dense_ld(int n) { return n | 1; }
// Lines per block: 64, 32 or 16, the most whose staged rows fit `budget`
// bytes of LDS (16 always fit up to kDenseMax in both precisions), but no
// more than the pass's lines need (a one-line pass stages 16 rows, not 64).
constexpr int dense_rows(int n, int elem_bytes, size_t budget, long long lines)
{
    int r = 64;
    while (r > 16 && ((size_t)r * (size_t)dense_ld(n) * (size_t)elem_bytes > budget || r / 2 >= lines)) r /= 2;
    return r;
}
// Dynamic LDS of a dense block of `rows` lines.
constexpr size_t dense_lds_bytes(int n, int rows, int elem_bytes)
{
    return (size_t)rows * (size_t)dense_ld(n) * (size_t)elem_bytes;
}
// LDS budget of the one-pass dense kernel (gfx950: 160 KB per CU).
constexpr size_t kDenseLdsOnePass = 160 * 1024;

}  // namespace jt
