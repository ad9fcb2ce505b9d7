// mixed_fft.h -- index maps of the 16-bit inverse segment transform whose
// butterflies run on the matrix cores (L = 2048 = 16 x 16 x 8).
//
// The inverse transform of the overlap-save product (Alg. 2) is written as
// three passes of small DFTs, each a matrix product over a batch of columns.
// With Z indexed q = k1 + 16 r + 256 s and the output n = j + 128 m,
// j = p + 8 q':
//
//   pass A (radix 8):  c[k1][p][r]    = W128^(p r) sum_s W8^(p s) Z[k1 + 16 r + 256 s]
//   pass B (radix 16): b[k1][p + 8q'] = W2048^(j k1) sum_r W16^(q' r) c[k1][p][r]
//   pass C (radix 16): y[j + 128 m]   = sum_k1 W16^(m k1) b[k1][j]
//
// (W_N^x = exp(+2 pi i x / N): the inverse sign.)  Each matrix product of
// pass A takes the 16 columns k1 of one r, so the twiddle W128^(p r)
// depends only on the row p and is folded into that r's DFT matrix; passes
// B and C then use one and the same DFT16 matrix.  The twiddle W2048^(j k1)
// of pass B's outputs is applied in FP32 by the work-item that holds them.
//
// A complex DFT becomes a real matrix product by interleaving real and
// imaginary parts both along K (inputs) and along the output rows, so every
// lane of every operand holds whole complex numbers.  Operand lane layouts
// (v_mfma_f32_16x16x{16,32}_{f16,bf16}, KPL = K / 4 values per lane):
//   A[i][k]: lane i + 16 (k / KPL), element k % KPL
//   B[k][j]: lane j + 16 (k / KPL), element k % KPL
//   D[i][j]: lane j + 16 (i / 4),   element i % 4
// Each workgroup has 2 waves (128 work-items); wave w, lane l, col = l % 16,
// g = l / 16.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef FDAS_HD
#define FDAS_HD __host__ __device__ __forceinline__
#endif

namespace fdas {
namespace mix {

constexpr int L = 2048;
constexpr int T = 128;          // work-items per transform

// LDS exchanges, in 32-bit words (one complex 16-bit value each).  Both are
// laid out so that every access of the passes below touches distinct banks:
// 4-byte accesses 64 banks per 64 lanes; 16-byte accesses distinct 4-bank
// groups per 16 lanes of 64 banks and per 8 lanes of 32 banks (counters show
// 16-byte accesses served 8 lanes at a time).
//   c[p][k1][r]  at k1 * CK + 16 p + r            (pass A writes, B reads)
//   b[k1][j]     at (j / 4) * BJ + 4 k1 + j % 4   (pass B writes, C reads)
constexpr int CK = 132;         // 128 + 4: consecutive k1 rows move 4 banks
constexpr int BJ = 68;          // 64 + 4
constexpr int CC_WORDS = 16 * CK;
constexpr int BB_WORDS = 32 * BJ;
FDAS_HD int cc_word(int p, int k1, int r) { return k1 * CK + 16 * p + r; }
FDAS_HD int bb_word(int j, int k1) { return (j >> 2) * BJ + 4 * k1 + (j & 3); }

// Power staging of one wave (float words, 16 per output column j' < 64):
// chunk g (rows 2g, 2g + 1, 2g + 8, 2g + 9 of the column, one 16-byte write
// by lane (g, col) of pass C) at 16 j' + 4 ((g + j'/2 + j'/8) mod 4); lane j'
// reads its column's four chunks.  The rotation j'/2 + j'/8 takes all four
// values over the lanes of one parity in any 8 consecutive lanes and over
// the lanes of one residue mod 4 in any 16, so the writes and reads are
// conflict-free under both bank models above.
constexpr int STAGE_WORDS = 64 * 16;
FDAS_HD int stage_word(int jcol, int g) { return 16 * jcol + 4 * ((g + (jcol >> 1) + (jcol >> 3)) & 3); }

// Pass A: group gam of wave w is r = 8 w + gam with columns k1 = col; lane
// (col, g) takes s = 2 g + i (value v = 2 gam + i) and returns p = 2 g, 2 g + 1.
FDAS_HD int zq(int w, int l, int v)
{
    const int gam = v >> 1, i = v & 1;
    return (l & 15) + 16 * (8 * w + gam) + 256 * (2 * (l >> 4) + i);
}
// Pass B: group gam of wave w is p = 4 w + gam, columns k1 = col; lane reads
// r = 4 g .. 4 g + 3 and returns q' = 8 h + 2 g + i for half h.
// Pass C: group gam of wave w is columns j = 16 (4 w + gam) + col; lane reads
// k1 = 4 g .. 4 g + 3 and returns m = 8 h + 2 g + i.

// Angle (in turns) of the complex weight multiplying input `in` for output
// `out` in each pass.
FDAS_HD double turns_A(int r, int p, int s) { return (double)((16 * p * s + p * r) & 127) / 128.0; }
FDAS_HD double turns_D16(int out, int in) { return (double)((out * in) & 15) / 16.0; }

// Real matrix entry for interleaved rows (2 out + a) and columns (2 in + c)
// of the complex weight exp(2 pi i turns): [[cos, -sin], [sin, cos]].
FDAS_HD int entry_sel(int row, int k) { return ((row & 1) << 1) | (k & 1); }  // 0 cos, 1 -sin, 2 sin, 3 cos

}  // namespace mix
}  // namespace fdas
