// kernels.hip - CDNA4 (gfx950) device code of the density-matrix contraction.
//
// One workgroup of 256 threads (4 wave64s) executes one network's op list:
//   OP_GEMM     pairwise contraction as an FP64 GEMM on the matrix cores
//               (v_mfma_f64_16x16x4f64), pipelined over (block, k-chunk) steps with one
//               of six block shapes; operand gathers through index tables fold every
//               mode permutation into the tile loads (split BF16x3 / FP16x3 forms on
//               the 16-bit matrix cores).
//   OP_EIG      symmetric eigensolve of a density matrix (Householder tridiagonal
//               reduction, implicit QL with one wave chasing and three applying the
//               rotations, compact-WY back-transformation of the kept vectors)
//               followed by the keep rule; writes the kept eigenvectors and rank.
//               A learned warm start (subspace iteration from MLP-scored columns with
//               a certificate) may replace the full solve.
// MPS bonds have a runtime extent (the kept rank of the eigensolve that made them):
// tensors keep their static layout and every op touches only the valid box.
//   OP_RESCALE  exact power-of-two normalisation with the exponent summed in int64.
//   OP_SCALAR   ln|z| and sign of a closing scalar.
//   OP_IDENT    identity matrices of the identity insertion.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace tn {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kLdsDoubles = 20000;     // 160,000 bytes of the 160 KiB LDS
constexpr int kTile = 64;
constexpr int kTK = 16;
constexpr int kPitch = kTile + 1;      // padded LDS row of a k-slice

__device__ __forceinline__ int64_t map_off(const int32_t *tab, const IdxMap &m, int32_t i) {
  int32_t h = i / m.lo_n;
  int32_t l = i - h * m.lo_n;
  return int64_t(tab[m.hi + h]) + int64_t(tab[m.lo + l]);
}

// ---------------------------------------------------------------- runtime extents

// The interpreter stages each op in LDS and replaces every Box's slot ids by the
// runtime extents they hold, so these helpers read extents straight from b.id.
__device__ __forceinline__ int32_t box_eff(const Box &b) {
  int32_t n = b.rest;
  for (int d = 0; d < b.nd; ++d) n *= b.id[d];
  return n;
}

// compact index in [0, box_eff) -> static index in the (cap..., rest) layout. With one
// runtime dimension (outermost) the valid box is a prefix of the layout: the identity.
__device__ __forceinline__ int32_t box_conv(const Box &b, int32_t i) {
  if (b.nd <= 1) return i;
  int32_t r = i % b.rest;
  int32_t q = i / b.rest;
  int32_t s = 0, mult = b.rest;
  for (int d = b.nd - 1; d >= 0; --d) {
    const int32_t k = b.id[d];
    s += (q % k) * mult;
    q /= k;
    mult *= b.cap[d];
  }
  return s + r;
}

// ---------------------------------------------------------------- GEMM

constexpr int kKCache = 4096;          // k offsets cached in LDS when K <= kKCache

// Plain tiled GEMM (64x64 output tiles from t_begin in steps of t_step, 16-deep k
// slices): the fallback for ops whose offsets do not fit the pipelined path's caches.
// The k offsets of both operands are cached in LDS when K <= KCACHE (lds holds two
// k-slices, then 2 KCACHE int32). Kept out of line, as one body per cache size.
// With kchunks > 1 (split K, chip-wide only) the work items are (tile, part of K): item w
// takes tile w / kchunks over the kchunks-th share of K and writes its partial tile to
// kpart[(part M + row) N + col] instead of C.
template <int KCACHE>
__device__ __noinline__ void gemm_tiles_k(const Op &op, const double *__restrict__ A, const double *__restrict__ B,
                                          double *__restrict__ C, const int32_t *__restrict__ tab, double *lds,
                                          int t_begin, int t_step, NetScalars *sc, int kchunks = 1,
                                          double *__restrict__ kpart = nullptr) {
  // runtime extents; the output keeps its static row length
  const int M = box_eff(op.bm), N = box_eff(op.bnb), K = box_eff(op.bk_);
  const int NS = op.bn.n;
  if (t_begin == 0 && threadIdx.x == 0) sc->flops += 2LL * M * N * K;
  const int tilesN = (N + kTile - 1) / kTile;
  const int ntiles = ((M + kTile - 1) / kTile) * tilesN;
  double *As = lds;                  // [kTK][kPitch], element (k, m)
  double *Bs = lds + kTK * kPitch;   // [kTK][kPitch], element (k, n)
  int32_t *kA = reinterpret_cast<int32_t *>(lds + 2 * kTK * kPitch);   // A's k offsets
  int32_t *kB = kA + KCACHE;                                           // B's k offsets
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const bool akf = (op.flags & F_A_KFAST) != 0;
  const bool bnf = (op.flags & F_B_NFAST) != 0;
  const bool kcached = K <= KCACHE;
  if (kcached) {
    for (int k = tid; k < K; k += kThreads) {
      const int ks = box_conv(op.bk_, k);
      kA[k] = tab[op.ak + ks];
      kB[k] = tab[op.bk + ks];
    }
    __syncthreads();
  }

  const int kc_len = ((K + kchunks - 1) / kchunks + kTK - 1) / kTK * kTK;   // K per part, whole slices
  for (int w = t_begin; w < ntiles * kchunks; w += t_step) {
    const int tile = w / kchunks, part = w - tile * kchunks;
    const int k_lo = part * kc_len, k_hi = k_lo + kc_len < K ? k_lo + kc_len : K;
    const int m0 = (tile / tilesN) * kTile, n0 = (tile % tilesN) * kTile;
    int64_t aoff[4], boff[4];
    int ai[4], ak_[4], bi[4], bk_[4];
    bool av[4], bv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + kThreads * q;
      ai[q] = akf ? e / kTK : e % kTile;
      ak_[q] = akf ? e % kTK : e / kTile;
      const int m = m0 + ai[q];
      av[q] = m < M;
      aoff[q] = av[q] ? map_off(tab, op.am, box_conv(op.bm, m)) : 0;
      bi[q] = bnf ? e % kTile : e / kTK;
      bk_[q] = bnf ? e / kTile : e % kTK;
      const int n = n0 + bi[q];
      bv[q] = n < N;
      boff[q] = bv[q] ? map_off(tab, op.bn, box_conv(op.bnb, n)) : 0;
    }
    double va[4], vb[4];
    auto load = [&](int k0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + ak_[q];
        double x = 0.0;
        if (av[q] && k < k_hi) x = A[aoff[q] + (kcached ? kA[k] : tab[op.ak + box_conv(op.bk_, k)])];
        va[q] = x;
        const int kb = k0 + bk_[q];
        double y = 0.0;
        if (bv[q] && kb < k_hi) y = B[boff[q] + (kcached ? kB[kb] : tab[op.bk + box_conv(op.bk_, kb)])];
        vb[q] = y;
      }
    };
    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    load(k_lo);
    for (int k0 = k_lo; k0 < k_hi; k0 += kTK) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        As[ak_[q] * kPitch + ai[q]] = va[q];
        Bs[bk_[q] * kPitch + bi[q]] = vb[q];
      }
      __syncthreads();
      if (k0 + kTK < k_hi) load(k0 + kTK);   // next slice in flight during the MFMAs
#pragma unroll
      for (int kk = 0; kk < kTK; kk += 4) {
        const int kr = kk + (lane >> 4);
        double a0 = As[kr * kPitch + wm * 32 + (lane & 15)];
        double a1 = As[kr * kPitch + wm * 32 + 16 + (lane & 15)];
        double b0 = Bs[kr * kPitch + wn * 32 + (lane & 15)];
        double b1 = Bs[kr * kPitch + wn * 32 + 16 + (lane & 15)];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm * 32 + i * 16 + (lane >> 4) + 4 * r;   // D: lane l, reg r = row l/16 + 4r
          const int col = n0 + wn * 32 + j * 16 + (lane & 15);
          if (row < M && col < N) {
            if (kpart) kpart[(int64_t(part) * M + row) * N + col] = acc[i][j][r];
            else C[int64_t(box_conv(op.bm, row)) * NS + box_conv(op.bnb, col)] = acc[i][j][r];
          }
        }
  }
}

// Pipelined GEMM for ops whose row, column and k offsets fit in LDS. The output is
// cut into MB x NB blocks (4 waves, each TM x TN MFMA tiles of 16 x 16) and K into
// chunks of KC; the (block, chunk) steps run as one flat sequence with two LDS
// buffers: while the waves multiply step s out of one buffer, every thread already
// holds its loads of step s+1 (possibly the next block) in registers. Offsets are
// resolved once per op into LDS: kA/kB (k), rA (A row), cB (B column), rC/cC (C).
// GRID: one of many workgroups on a chip-wide op. It takes the blocks [b_begin, b_end)
// (columns fastest) and resolves column offsets on the fly from the index tables
// (cB and cC unused); row and k offsets are still cached in LDS.
template <int MB, int NB, int KC, int TM, int TN, bool GRID = false>
__device__ void gemm_piped(const Op &op, const double *__restrict__ A, const double *__restrict__ B,
                           double *__restrict__ C, double *lds, int M, int N, int K, const int32_t *kA,
                           const int32_t *kB, const int32_t *rA, const int32_t *cB, const int32_t *rC,
                           const int32_t *cC, const int32_t *tab = nullptr, int b_begin = 0, int b_end = -1) {
  constexpr int WN = NB / (16 * TN);               // waves along N
  static_assert((MB / (16 * TM)) * WN == 4, "4 waves per block");
  constexpr int PA = MB + 1, PB = NB + 1;          // LDS pitches of a k row
  constexpr int SA = KC * PA, SB = KC * PB;        // one stage
  constexpr int LA = (MB * KC + kThreads - 1) / kThreads;
  constexpr int LB = (KC * NB + kThreads - 1) / kThreads;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const bool akf = (op.flags & F_A_KFAST) != 0;
  const bool bnf = (op.flags & F_B_NFAST) != 0;
  const int nbm = (M + MB - 1) / MB, nbn = (N + NB - 1) / NB, nch = (K + KC - 1) / KC;
  const int nblk = nbm * nbn;
  const int blk_hi = (b_end < 0 || b_end > nblk) ? nblk : b_end;
  const int s_begin = b_begin * nch;
  const int steps = blk_hi > b_begin ? blk_hi * nch : 0;
  auto colB = [&](int n) -> int64_t {
    if constexpr (GRID) return map_off(tab, op.bn, box_conv(op.bnb, n));
    else return cB[n];
  };
  auto colC = [&](int n) -> int64_t {
    if constexpr (GRID) return box_conv(op.bnb, n);
    else return cC[n];
  };
  double ra[LA], rb[LB];
  auto load = [&](int s) {
    const int blk = s / nch, ch = s - blk * nch;
    const int m0 = (blk / nbn) * MB, n0 = (blk % nbn) * NB, k0 = ch * KC;
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int e = tid + kThreads * q;
      const int i = akf ? e / KC : e % MB, k = akf ? e % KC : e / MB;
      double x = 0.0;
      if (e < MB * KC && m0 + i < M && k0 + k < K) x = A[int64_t(rA[m0 + i]) + kA[k0 + k]];
      ra[q] = x;
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int e = tid + kThreads * q;
      const int j = bnf ? e % NB : e / KC, k = bnf ? e / NB : e % KC;
      double y = 0.0;
      if (e < KC * NB && n0 + j < N && k0 + k < K) y = B[colB(n0 + j) + kB[k0 + k]];
      rb[q] = y;
    }
  };
  auto stash = [&](int buf) {
    double *as = lds + buf * (SA + SB), *bs = as + SA;
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int e = tid + kThreads * q;
      const int i = akf ? e / KC : e % MB, k = akf ? e % KC : e / MB;
      if (e < MB * KC) as[k * PA + i] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int e = tid + kThreads * q;
      const int j = bnf ? e % NB : e / KC, k = bnf ? e / NB : e % KC;
      if (e < KC * NB) bs[k * PB + j] = rb[q];
    }
  };
  v4d acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  if (steps > s_begin) load(s_begin);
  for (int s = s_begin; s < steps; ++s) {
    const int buf = s & 1;
    stash(buf);
    __syncthreads();
    if (s + 1 < steps) load(s + 1);                // in flight during the MFMAs
    const int blk = s / nch, ch = s - blk * nch;
    const int kc = K - ch * KC < KC ? K - ch * KC : KC;
    const double *as = lds + buf * (SA + SB) + wm * TM * 16 + (lane & 15);
    const double *bs = lds + buf * (SA + SB) + SA + wn * TN * 16 + (lane & 15);
    for (int kk = 0; kk < kc; kk += 4) {
      const int kr = kk + (lane >> 4);
      double av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = as[kr * PA + a * 16];
#pragma unroll
      for (int b = 0; b < TN; ++b) bv[b] = bs[kr * PB + b * 16];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (ch == nch - 1) {                           // block done: write it out
      const int m0 = (blk / nbn) * MB, n0 = (blk % nbn) * NB;
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = m0 + wm * TM * 16 + a * 16 + (lane >> 4) + 4 * r;   // D: lane l, reg r = row l/16 + 4r
            const int col = n0 + wn * TN * 16 + b * 16 + (lane & 15);
            if (row < M && col < N) C[int64_t(rC[row]) + colC(col)] = acc[a][b][r];
          }
          acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
        }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- split-precision GEMM
//
// Precision form of a GEMM op: both operands are scaled by exact powers of two
// (max |x| of the op's valid box brought into [1/2, 1)), every value is split into
// three 16-bit floats, each the rounding of what the previous ones leave, and the
// product is the sum of the six part products of order <= 2 (hh, hm, mh, hl, lh, mm)
// on the 16-bit matrix cores, accumulated in FP32 over each 16-deep k chunk and in
// FP64 across chunks. BF16 (8-bit significand, FP32 range): x = h + m + l, one
// accumulator. FP16 (11-bit significand, narrow range): the remainders are scaled up
// before rounding, x = h + 2^-11 m + 2^-22 l, so the parts stay normal, and the
// products of each order get their own accumulator, combined as
// acc0 + 2^-11 acc1 + 2^-22 acc2. The result is scaled back exactly and stored in FP64.

typedef short v4s __attribute__((ext_vector_type(4)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ double bf16_val(unsigned short b) { return double(__uint_as_float((unsigned int)b << 16)); }

template <int SPLIT>
__device__ __forceinline__ void split3(double x, unsigned short &h, unsigned short &m, unsigned short &l) {
  if (SPLIT == 1) {
    h = bf16_rne(float(x));
    const double r1 = x - bf16_val(h);
    m = bf16_rne(float(r1));
    const double r2 = r1 - bf16_val(m);
    l = bf16_rne(float(r2));
  } else {
    const _Float16 hh = _Float16(float(x));
    const double r1 = (x - double(hh)) * 2048.0;             // exact
    const _Float16 mm = _Float16(float(r1));
    const double r2 = (r1 - double(mm)) * 2048.0;
    const _Float16 ll = _Float16(float(r2));
    h = __builtin_bit_cast(unsigned short, hh);
    m = __builtin_bit_cast(unsigned short, mm);
    l = __builtin_bit_cast(unsigned short, ll);
  }
}

template <int SPLIT>
__device__ __forceinline__ v4f mfma16(unsigned long long a, unsigned long long b, v4f c) {
  if (SPLIT == 1)
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(v4s, a), __builtin_bit_cast(v4s, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(v4h, a), __builtin_bit_cast(v4h, b), c, 0, 0, 0);
}

// LDS of one stage: three planes of A (MB rows of KC + 4 parts, k fastest) and three
// planes of B (NB columns of KC + 4 parts, k fastest), as 16-bit words.
constexpr int split_stage_words(int MB, int NB, int KC) { return 3 * (MB + NB) * (KC + 4); }

template <int MB, int NB, int KC, int TM, int TN, int SPLIT>
__device__ void gemm_split(const Op &op, const double *__restrict__ A, const double *__restrict__ B,
                           double *__restrict__ C, double *lds, int M, int N, int K, const int32_t *kA,
                           const int32_t *kB, const int32_t *rA, const int32_t *cB, const int32_t *rC,
                           const int32_t *cC, double sa, double sb) {
  constexpr int WN = NB / (16 * TN);
  static_assert((MB / (16 * TM)) * WN == 4, "4 waves per block");
  static_assert(KC % 16 == 0, "k chunk of whole 16-deep MFMA steps");
  constexpr int P = KC + 4;                        // parts per row / column (8-byte aligned runs of 4)
  constexpr int SW = split_stage_words(MB, NB, KC);
  constexpr int LA = (MB * KC + kThreads - 1) / kThreads;
  constexpr int LB = (KC * NB + kThreads - 1) / kThreads;
  unsigned short *W16 = reinterpret_cast<unsigned short *>(lds);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const bool akf = (op.flags & F_A_KFAST) != 0;
  const bool bnf = (op.flags & F_B_NFAST) != 0;
  const int nbm = (M + MB - 1) / MB, nbn = (N + NB - 1) / NB, nch = (K + KC - 1) / KC;
  const int steps = nbm * nbn * nch;
  double ra[LA], rb[LB];
  auto load = [&](int s) {
    const int blk = s / nch, ch = s - blk * nch;
    const int m0 = (blk / nbn) * MB, n0 = (blk % nbn) * NB, k0 = ch * KC;
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int e = tid + kThreads * q;
      const int i = akf ? e / KC : e % MB, k = akf ? e % KC : e / MB;
      double x = 0.0;
      if (e < MB * KC && m0 + i < M && k0 + k < K) x = A[int64_t(rA[m0 + i]) + kA[k0 + k]];
      ra[q] = x;
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int e = tid + kThreads * q;
      const int j = bnf ? e % NB : e / KC, k = bnf ? e / NB : e % KC;
      double y = 0.0;
      if (e < KC * NB && n0 + j < N && k0 + k < K) y = B[int64_t(cB[n0 + j]) + kB[k0 + k]];
      rb[q] = y;
    }
  };
  auto stash = [&](int buf) {
    unsigned short *a3 = W16 + buf * SW, *b3 = a3 + 3 * MB * P;
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int e = tid + kThreads * q;
      const int i = akf ? e / KC : e % MB, k = akf ? e % KC : e / MB;
      if (e < MB * KC) {
        unsigned short h, m, l;
        split3<SPLIT>(ra[q] * sa, h, m, l);
        a3[i * P + k] = h;
        a3[(MB + i) * P + k] = m;
        a3[(2 * MB + i) * P + k] = l;
      }
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int e = tid + kThreads * q;
      const int j = bnf ? e % NB : e / KC, k = bnf ? e / NB : e % KC;
      if (e < KC * NB) {
        unsigned short h, m, l;
        split3<SPLIT>(rb[q] * sb, h, m, l);
        b3[j * P + k] = h;
        b3[(NB + j) * P + k] = m;
        b3[(2 * NB + j) * P + k] = l;
      }
    }
  };
  const double unscale = 1.0 / (sa * sb);           // exact: a power of two
  constexpr int NACC = SPLIT == 1 ? 1 : 3;          // FP16: one accumulator per order
  v4f acc[NACC][TM][TN];
#pragma unroll
  for (int o = 0; o < NACC; ++o)
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b) acc[o][a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  constexpr int O1 = NACC > 1 ? 1 : 0, O2 = NACC > 1 ? 2 : 0;
  double acc64[TM][TN][4];                         // FP64 sum of the 16-deep FP32 chunk sums
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[a][b][r] = 0.0;
  if (steps > 0) load(0);
  for (int s = 0; s < steps; ++s) {
    const int buf = s & 1;
    stash(buf);
    __syncthreads();
    if (s + 1 < steps) load(s + 1);
    const int blk = s / nch, ch = s - blk * nch;
    const unsigned short *a3 = W16 + buf * SW, *b3 = a3 + 3 * MB * P;
    const int kq = 4 * (lane >> 4);                 // this lane's 4 k values of a 16-deep step
    for (int kk = 0; kk < KC; kk += 16) {
      unsigned long long ah[TM], am[TM], al[TM], bh[TN], bm[TN], bl[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        const int r = wm * TM * 16 + a * 16 + (lane & 15);
        ah[a] = *reinterpret_cast<const unsigned long long *>(a3 + r * P + kk + kq);
        am[a] = *reinterpret_cast<const unsigned long long *>(a3 + (MB + r) * P + kk + kq);
        al[a] = *reinterpret_cast<const unsigned long long *>(a3 + (2 * MB + r) * P + kk + kq);
      }
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int c = wn * TN * 16 + b * 16 + (lane & 15);
        bh[b] = *reinterpret_cast<const unsigned long long *>(b3 + c * P + kk + kq);
        bm[b] = *reinterpret_cast<const unsigned long long *>(b3 + (NB + c) * P + kk + kq);
        bl[b] = *reinterpret_cast<const unsigned long long *>(b3 + (2 * NB + c) * P + kk + kq);
      }
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {               // small terms first
          acc[O2][a][b] = mfma16<SPLIT>(am[a], bm[b], acc[O2][a][b]);
          acc[O2][a][b] = mfma16<SPLIT>(al[a], bh[b], acc[O2][a][b]);
          acc[O2][a][b] = mfma16<SPLIT>(ah[a], bl[b], acc[O2][a][b]);
          acc[O1][a][b] = mfma16<SPLIT>(am[a], bh[b], acc[O1][a][b]);
          acc[O1][a][b] = mfma16<SPLIT>(ah[a], bm[b], acc[O1][a][b]);
          acc[0][a][b] = mfma16<SPLIT>(ah[a], bh[b], acc[0][a][b]);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double v = double(acc[0][a][b][r]);
            if (NACC > 1) v += double(acc[O1][a][b][r]) * 0x1p-11 + double(acc[O2][a][b][r]) * 0x1p-22;
            acc64[a][b][r] += v;
          }
#pragma unroll
          for (int o = 0; o < NACC; ++o) acc[o][a][b] = v4f{0.f, 0.f, 0.f, 0.f};
        }
    }
    if (ch == nch - 1) {
      const int m0 = (blk / nbn) * MB, n0 = (blk % nbn) * NB;
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = m0 + wm * TM * 16 + a * 16 + 4 * (lane >> 4) + r;   // D: lane l, reg r = row 4(l/16) + r
            const int col = n0 + wn * TN * 16 + b * 16 + (lane & 15);
            if (row < M && col < N) C[int64_t(rC[row]) + cC[col]] = acc64[a][b][r] * unscale;
            acc64[a][b][r] = 0.0;
          }
        }
    }
  }
  __syncthreads();
}

__device__ double block_max(double v, double *red);
__device__ __forceinline__ double wave_max(double v);

// 2^-e with e the frexp exponent of max |x| over a valid box (1 for an all-zero box)
__device__ double pow2_scale(double amax) {
  if (!(amax > 0.0)) return 1.0;
  int e;
  frexp(amax, &e);
  return ldexp(1.0, -e);
}

// LDS doubles of the two stages of a gemm_piped configuration
constexpr int piped_stage_doubles(int MB, int NB, int KC) { return 2 * (KC * (MB + 1) + KC * (NB + 1)); }
constexpr int kPipedTiles = piped_stage_doubles(32, 128, 32);   // the largest configuration below
constexpr int64_t kDirectFma = 65536;  // products up to this many multiply-adds skip the pipeline
static_assert(2 * split_stage_words(64, 64, 16) <= 4 * (kPipedTiles - 8), "split stages fit");
static_assert(2 * split_stage_words(32, 128, 16) <= 4 * (kPipedTiles - 8), "split stages fit");
static_assert(2 * split_stage_words(16, 256, 16) <= 4 * (kPipedTiles - 8), "split stages fit");

// Outputs of a small product from LDS: a thread per (R rows, column) item; rows m0..m0+R-1
// of As (k-major, pitch Mp) against column n of Bs, R (or, for R < 4, 2R) independent sums.
template <int R>
__device__ __forceinline__ void gemm_direct_rows(const double *As, const double *Bs, double *__restrict__ C, int M,
                                                 int Mp, int N, int K, const int32_t *rC, const int32_t *cC) {
  constexpr int P = R < 4 ? 2 : 1;                       // partial sums per row
  const int items = (Mp / R) * N;
  for (int e = threadIdx.x; e < items; e += kThreads) {
    const int mb = e / N, n = e - mb * N, m0 = mb * R;
    const double *a = As + m0, *b = Bs + n;
    double s[P][R];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int r = 0; r < R; ++r) s[p][r] = 0.0;
    int k = 0;
    for (; k + P <= K; k += P) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const double bk = b[(k + p) * N];
#pragma unroll
        for (int r = 0; r < R; ++r) s[p][r] = fma(a[(k + p) * Mp + r], bk, s[p][r]);
      }
    }
    if (k < K) {
      const double bk = b[k * N];
#pragma unroll
      for (int r = 0; r < R; ++r) s[0][r] = fma(a[k * Mp + r], bk, s[0][r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (m0 + r < M) C[int64_t(rC[m0 + r]) + cC[n]] = P == 2 ? s[0][r] + s[P - 1][r] : s[0][r];
    }
  }
}

// One GEMM op. Returns false when its offsets do not fit the LDS cache (the caller
// then runs gemm_tiles_k).
__device__ bool gemm_op(const Op &op, const double *__restrict__ A, const double *__restrict__ B,
                        double *__restrict__ C, const int32_t *__restrict__ tab, double *lds, NetScalars *sc,
                        int split, const int *cfgs) {
  const int M = box_eff(op.bm), N = box_eff(op.bnb), K = box_eff(op.bk_);
  const int64_t NS = op.bn.n;
  if (2 * (int64_t(M) + N + K) > 2 * int64_t(kLdsDoubles - kPipedTiles)) return false;
  int32_t *kA = reinterpret_cast<int32_t *>(lds + kPipedTiles);
  int32_t *kB = kA + K, *rA = kB + K, *rC = rA + M, *cB = rC + M, *cC = cB + N;
  const int tid = threadIdx.x;
  if (tid == 0) {
    sc->flops += 2LL * M * N * K;
    if (split) sc->split_flops += 2LL * M * N * K;
  }
  if (K <= kThreads && M <= kThreads && N <= kThreads) {
    // one index of each kind per thread: every table load is issued before the first LDS
    // store, so the offsets cost one memory round trip
    int32_t a0 = 0, b0 = 0, h1 = 0, l1 = 0, h2 = 0, l2 = 0, sm = 0, sn = 0;
    if (tid < K) { const int ks = box_conv(op.bk_, tid); a0 = tab[op.ak + ks]; b0 = tab[op.bk + ks]; }
    if (tid < M) {
      sm = box_conv(op.bm, tid);
      const int32_t h = sm / op.am.lo_n;
      h1 = tab[op.am.hi + h];
      l1 = tab[op.am.lo + (sm - h * op.am.lo_n)];
    }
    if (tid < N) {
      sn = box_conv(op.bnb, tid);
      const int32_t h = sn / op.bn.lo_n;
      h2 = tab[op.bn.hi + h];
      l2 = tab[op.bn.lo + (sn - h * op.bn.lo_n)];
    }
    if (tid < K) { kA[tid] = a0; kB[tid] = b0; }
    if (tid < M) { rA[tid] = int32_t(int64_t(h1) + l1); rC[tid] = int32_t(sm * NS); }
    if (tid < N) { cB[tid] = int32_t(int64_t(h2) + l2); cC[tid] = sn; }
  } else {
    for (int k = tid; k < K; k += kThreads) {
      const int ks = box_conv(op.bk_, k);
      kA[k] = tab[op.ak + ks];
      kB[k] = tab[op.bk + ks];
    }
    for (int m = tid; m < M; m += kThreads) {
      const int sm = box_conv(op.bm, m);
      rA[m] = int32_t(map_off(tab, op.am, sm));
      rC[m] = int32_t(sm * NS);
    }
    for (int n = tid; n < N; n += kThreads) {
      const int sn = box_conv(op.bnb, n);
      cB[n] = int32_t(map_off(tab, op.bn, sn));
      cC[n] = sn;
    }
  }
  __syncthreads();
  if (split) {
    double am = 0.0, bm = 0.0;                   // per-tensor power-of-two scales
    for (int e = tid; e < M * K; e += kThreads) am = fmax(am, fabs(A[int64_t(rA[e / K]) + kA[e % K]]));
    for (int e = tid; e < K * N; e += kThreads) bm = fmax(bm, fabs(B[int64_t(cB[e / K]) + kB[e % K]]));
    const double sa = pow2_scale(block_max(am, lds + kPipedTiles - 8));
    const double sb = pow2_scale(block_max(bm, lds + kPipedTiles - 8));
    if (split == 1) {
      if (M <= 16) gemm_split<16, 256, 16, 1, 4, 1>(op, A, B, C, lds, M, N, K, kA, kB, rA, cB, rC, cC, sa, sb);
      else if (M <= 32) gemm_split<32, 128, 16, 2, 2, 1>(op, A, B, C, lds, M, N, K, kA, kB, rA, cB, rC, cC, sa, sb);
      else gemm_split<64, 64, 16, 2, 2, 1>(op, A, B, C, lds, M, N, K, kA, kB, rA, cB, rC, cC, sa, sb);
    } else {
      if (M <= 16) gemm_split<16, 256, 16, 1, 4, 2>(op, A, B, C, lds, M, N, K, kA, kB, rA, cB, rC, cC, sa, sb);
      else if (M <= 32) gemm_split<32, 128, 16, 2, 2, 2>(op, A, B, C, lds, M, N, K, kA, kB, rA, cB, rC, cC, sa, sb);
      else gemm_split<64, 64, 16, 2, 2, 2>(op, A, B, C, lds, M, N, K, kA, kB, rA, cB, rC, cC, sa, sb);
    }
    return true;
  }
  // a small product (at most kDirectFma multiply-adds, both operands within the stage area):
  // both operands staged in LDS with one round trip, then every output from LDS on the VALU
  // (no k-chunk pipeline, no matrix-core blocks mostly of padding at these sizes). A thread
  // takes R rows of one output column, so each load of B serves R multiply-adds and the R
  // values of A (k-major, rows padded to a multiple of R) are one read shared by the wave.
  if (int64_t(M) * N * K <= kDirectFma) {
    const int R = M >= 4 ? 4 : (M >= 2 ? 2 : 1);
    const int Mp = (M + R - 1) / R * R;
    if (Mp * K + K * N <= kPipedTiles) {
      double *As = lds, *Bs = lds + Mp * K;              // As[k][m] (pitch Mp), Bs[k][n]
      for (int e = tid; e < M * K; e += kThreads) {
        const int m = e / K, k = e - m * K;
        As[k * Mp + m] = A[int64_t(rA[m]) + kA[k]];
      }
      for (int e = tid; e < K * N; e += kThreads) {
        const int k = e / N, n = e - k * N;
        Bs[e] = B[int64_t(cB[n]) + kB[k]];
      }
      __syncthreads();
      if (R == 4) gemm_direct_rows<4>(As, Bs, C, M, Mp, N, K, rC, cC);
      else if (R == 2) gemm_direct_rows<2>(As, Bs, C, M, Mp, N, K, rC, cC);
      else gemm_direct_rows<1>(As, Bs, C, M, Mp, N, K, rC, cC);
      return true;
    }
  }
  // block configuration: the option's choice for this row class, else 16x512 / 32x128 / 64x64
  const int cls = M <= 16 ? 0 : (M <= 32 ? 1 : 2);
  int cfg = cfgs[cls] - 1;
  if (cfg < 0 || cfg >= kGemmConfigs) cfg = cls == 0 ? 0 : (cls == 1 ? 2 : 4);
  switch (cfg) {
    case 0: gemm_piped<16, 512, 8, 1, 8>(op, A, B, C, lds, M, N, K, kA, kB, rA, cB, rC, cC); break;
    case 1: gemm_piped<16, 256, 16, 1, 4>(op, A, B, C, lds, M, N, K, kA, kB, rA, cB, rC, cC); break;
    case 2: gemm_piped<32, 128, 32, 2, 2>(op, A, B, C, lds, M, N, K, kA, kB, rA, cB, rC, cC); break;
    case 3: gemm_piped<32, 128, 16, 2, 2>(op, A, B, C, lds, M, N, K, kA, kB, rA, cB, rC, cC); break;
    case 4: gemm_piped<64, 64, 32, 2, 2>(op, A, B, C, lds, M, N, K, kA, kB, rA, cB, rC, cC); break;
    default: gemm_piped<64, 64, 16, 2, 2>(op, A, B, C, lds, M, N, K, kA, kB, rA, cB, rC, cC); break;
  }
  return true;
}

// ---------------------------------------------------------------- reductions

// Cross-lane moves within a row of 16 lanes run on DPP (a VALU operand modifier) rather
// than through the LDS crossbar that a general shuffle takes; both halves of a double
// move with the same control. Every lane of a group ends with the same bits: each step
// adds a lane's value and its partner's, in the same order on both sides.
// Rows outside ROWS (a 4-bit mask of the wave's four rows of 16) receive 0.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
  return __hiloint2double(hi, lo);
}
constexpr int kDppQuadXor1 = 0xB1;      // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4E;      // quad_perm [2, 3, 0, 1]
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;
constexpr int kDppRowBcast15 = 0x142;   // lane 15 of each row to the next row
constexpr int kDppRowBcast31 = 0x143;   // lane 31 to rows 2 and 3
__device__ __forceinline__ double lane0(double v) {     // lane 0's value, as a uniform scalar
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 0);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 0);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane63(double v) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}
// sum over each aligned group of 4 lanes (all four active), in every lane of the group
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_f64<kDppQuadXor1>(v);
  return v + dpp_f64<kDppQuadXor2>(v);
}
// whole-wave reductions (all lanes active): row results, then rows 1 and 3 take the rows
// before them and row 3 the first two; lane 63's value is read back as a uniform scalar
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64<kDppQuadXor1>(v));
  v = fmax(v, dpp_f64<kDppQuadXor2>(v));
  v = fmax(v, dpp_f64<kDppRowHalfMirror>(v));
  v = fmax(v, dpp_f64<kDppRowMirror>(v));
  v = fmax(v, dpp_f64<kDppRowBcast15, 0xA>(v));
  v = fmax(v, dpp_f64<kDppRowBcast31, 0xC>(v));
  return lane63(v);
}
__device__ __forceinline__ double wave_sum(double v) {
  v = quad_sum(v);
  v += dpp_f64<kDppRowHalfMirror>(v);   // lane i of 8 takes lane 7 - i: the other quad
  v += dpp_f64<kDppRowMirror>(v);       // lane i of 16 takes lane 15 - i: the other half row
  v += dpp_f64<kDppRowBcast15, 0xA>(v); // rows 1, 3: rows 0 + 1, rows 2 + 3
  v += dpp_f64<kDppRowBcast31, 0xC>(v); // row 3: all four rows
  return lane63(v);
}

// block-wide reduction through 4 LDS slots; every thread gets the result
__device__ double block_max(double v, double *red) {
  v = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}
__device__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// ---------------------------------------------------------------- rescale / scalar

// x is stored [rows][ncols]; only the runtime box rows x cols is valid.
__device__ void rescale_wg(const Op &op, double *x, NetScalars *sc, double *red) {
  const bool accum = (op.flags & F_ACCUM) != 0;
  const int32_t R = box_eff(op.bm), Cn = box_eff(op.bnb);
  const int64_t ncols = op.count;
  const int64_t total = int64_t(R) * Cn;
  // up to kCached elements per thread are held in registers between the two passes, so
  // the scaling pass does not read the tensor again
  constexpr int kCached = 16;
  if (total <= int64_t(kCached) * kThreads) {
    double v[kCached];
    int64_t o[kCached];
    double m = 0.0;
#pragma unroll
    for (int q = 0; q < kCached; ++q) {
      const int32_t i = int32_t(threadIdx.x) + q * kThreads;
      o[q] = 0;
      v[q] = 0.0;
      if (i < total) {
        const int32_t r = i / Cn, c = i - r * Cn;
        o[q] = int64_t(box_conv(op.bm, r)) * ncols + box_conv(op.bnb, c);
        v[q] = x[o[q]];
        m = fmax(m, fabs(v[q]));
      }
    }
    m = block_max(m, red);
    if (!(m > 0.0) || !isfinite(m)) {
      if (m == 0.0 && accum && threadIdx.x == 0) sc->zero = 1;
      return;
    }
    int e;
    frexp(m, &e);
#pragma unroll
    for (int q = 0; q < kCached; ++q)
      if (int32_t(threadIdx.x) + q * kThreads < total) x[o[q]] = ldexp(v[q], -e);
    if (accum && threadIdx.x == 0) sc->exp_sum += e;
    return;
  }
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < total; i += kThreads) {
    const int32_t r = int32_t(i / Cn), c = int32_t(i - int64_t(r) * Cn);
    m = fmax(m, fabs(x[int64_t(box_conv(op.bm, r)) * ncols + box_conv(op.bnb, c)]));
  }
  m = block_max(m, red);
  if (!(m > 0.0) || !isfinite(m)) {
    if (m == 0.0 && accum && threadIdx.x == 0) sc->zero = 1;
    return;
  }
  int e;
  frexp(m, &e);
  for (int64_t i = threadIdx.x; i < total; i += kThreads) {
    const int32_t r = int32_t(i / Cn), c = int32_t(i - int64_t(r) * Cn);
    const int64_t o = int64_t(box_conv(op.bm, r)) * ncols + box_conv(op.bnb, c);
    x[o] = ldexp(x[o], -e);
  }
  if (accum && threadIdx.x == 0) sc->exp_sum += e;
}

__device__ void scalar_wg(const double *x, NetScalars *sc) {
  if (threadIdx.x == 0) {
    double z = x[0];
    if (z == 0.0) sc->zero = 1;
    else {
      sc->log_sum += log(fabs(z));
      if (z < 0.0) sc->sign = -sc->sign;
    }
  }
}

__device__ void ident_wg(double *x, int64_t d) {
  for (int64_t i = threadIdx.x; i < d * d; i += kThreads) x[i] = (i / d == i % d) ? 1.0 : 0.0;
}

// ---------------------------------------------------------------- eigensolver

// ---------------------------------------------------------------- dense symmetric eigensolve
//
// Householder reduction to tridiagonal form T = Q^T A Q in LDS (256 threads; the
// reflectors go to global scratch), implicit QL with shifts on T accumulating the
// rotations into Z (every wave runs the sequential recurrence on lane-distributed
// (d, e) registers; each thread rotates its own row of Z), descending order, and a
// back-transformation U = Q Z of only the kept columns.

struct EigWs {          // LDS work area of one solve of order n
  double *A;            // n x pa matrix, then Z (column-major n x n)
  double *vv, *pp, *ww, *dd, *ee, *wsrt;
  int *isrt, *flag;
  double *red;
  double *wq;           // 8n: QL's copy of (d, e) and rotation buffers; then reflector blocks
  double *gw;           // 24: Gram matrix and betas of a reflector block
  double *hv;           // reflectors: v_j at hv[j*n + i], beta_j at hv[n*n + j] (LDS past the
                        // work area when they fit, else the op's global scratch)
  int n, pa;            // pa: odd row pitch of the matrix, and the column pitch of Z (column j
                        // at A[j pa ..]: lanes reading different columns hit different banks)
};

__host__ __device__ constexpr int eig_lds_doubles(int n) { return n * (n + 1) + 14 * n + (n + 1) / 2 + 8 + 24; }
static_assert(eig_lds_doubles(128) <= kLdsDoubles, "a density matrix of order 128 fits LDS");
// Larger density matrices (up to order kMaxEigDim) keep the matrix and Z in the op's global
// scratch and only the solver's vectors in LDS.
static_assert(eig_lds_doubles(kMaxEigDim) - kMaxEigDim * (kMaxEigDim + 1) <= kLdsDoubles,
              "the solver's vectors of the largest density matrix fit LDS");

// Work area of one solve: the matrix at A when given (global scratch), else at the start
// of base; the vectors follow in base.
__device__ EigWs eig_ws(double *base, int n, double *hv, double *A = nullptr) {
  EigWs E;
  E.n = n;
  E.pa = n + 1;                        // odd pitch: conflict-free row access
  E.A = A ? A : base;
  E.vv = A ? base : base + n * E.pa;
  E.pp = E.vv + n;
  E.ww = E.pp + n;
  E.dd = E.ww + n;
  E.ee = E.dd + n;
  E.wsrt = E.ee + n;
  E.isrt = reinterpret_cast<int *>(E.wsrt + n);
  E.flag = E.isrt + n + (n & 1);
  E.red = reinterpret_cast<double *>(E.flag + 4);
  E.wq = E.red + 4;
  E.gw = E.wq + 8 * n;
  E.hv = hv;
  return E;
}

// Tridiagonalise E.A (symmetric, loaded) and diagonalise T by implicit QL.
// On return Z (column j at E.A[j E.pa ..]) overwrites E.A and the eigenvalues are in E.dd.
// (d, e) and (c, s) pairs of the QL solve, 16-byte aligned so that a pair moves in one
// LDS access
struct __attribute__((aligned(16))) Pair { double x, y; };
typedef __attribute__((address_space(3))) Pair lds_pair;

// One sweep of the implicit QL chase, rows mu-1 down to lu of the pairs de = (d_i, e_i),
// run by one wave (every lane computes the same values; lane 0 writes). The (c, s) of
// each rotation go to rb in order. The step carries no branch: an underflow (f = g = 0,
// where T splits) writes the split values and turns the remaining steps into writes to
// the spare pair `spare`, so the chase never waits on a scalar test of a vector result.
// The pointers are taken as LDS pointers, so every access is a ds_ instruction whatever
// the caller's pointer provenance. Returns p and g of the last step, the rotations, and
// whether T split.
struct ChaseOut { double p, g; int cnt, split; };
__device__ __forceinline__ ChaseOut ql_chase(Pair *de_, Pair *rb_, Pair *spare_, int lu_, int mu_, double g,
                                          double di1) {
  lds_pair *de = (lds_pair *)de_, *rb = (lds_pair *)rb_, *spare = (lds_pair *)spare_;   // all in LDS
  const bool lane0 = (threadIdx.x & 63) == 0;
  const int lu = __builtin_amdgcn_readfirstlane(lu_), mu = __builtin_amdgcn_readfirstlane(mu_);
  double s = 1.0, c = 1.0, p = 0.0;
  double nd = de[mu - 1].x, ne = de[mu - 1].y;       // (d[i], e[i]), fetched one step ahead
  asm volatile("" ::"v"(nd), "v"(ne));               // arrived before the loop: no wait inside
  // a step's writes are issued in the next step, after its prefetch, so that waiting for
  // a prefetched pair never waits on writes issued just before it (the first step's
  // pending writes go to the spare pair)
  lds_pair *pd = spare, *pr = spare;
  double pdx = 0.0, pdy = 0.0, prx = 0.0, pry = 0.0;
  int cnt = 0;
  bool live = true;
  auto step = [&](int i) {
    const double ei = ne, di = nd;
    const int nxt = i > lu ? i - 1 : lu;
    nd = de[nxt].x;
    ne = de[nxt].y;
    if (lane0) {
      pd->x = pdx;
      pd->y = pdy;
      pr->x = prx;
      pr->y = pry;
    }
    const double f = s * ei, bb = c * ei;
    const double q = f * f + g * g;
    const bool z = q == 0.0;
    // c = g / sqrt(q), s = f / sqrt(q), r = sqrt(q) from the hardware estimate y0 of
    // 1/sqrt(q) and one correction: with e = 1 - q y0^2, 1/sqrt(q) = y0 (1 + e/2 +
    // 3e^2/8 + O(e^3)), exact to rounding since |e| is below 2^-20; each output is
    // corrected directly, which keeps the step's dependent chain short
    const double y0 = __builtin_amdgcn_rsq(q);
    const double qy = q * y0, gy = g * y0, fy = f * y0;
    const double ey = fma(-qy, y0, 1.0);
    const double pe = fma(ey, 0.375, 0.5);
    c = fma(gy * ey, pe, gy);
    s = fma(fy * ey, pe, fy);
    const double r = fma(qy * ey, pe, qy);
    const double gq = di1 - p;
    const double t = fma(di - gq, s, c * (2.0 * bb));
    p = s * t;
    g = fma(c, t, -bb);
    // the address and data registers of the writes issued at this step's start stay
    // untouched until here, so the step never waits for those writes to reuse them
    asm volatile("" : "+v"(g) : "v"(pdx), "v"(pdy), "v"(prx), "v"(pry), "v"(pd), "v"(pr));
    pd = live ? de + (i + 1) : spare;
    pr = live && !z ? rb + cnt : spare;
    pdx = z ? gq : gq + p;                             // at a split: d[i+1] - p, e[i+1] = 0
    pdy = z ? 0.0 : r;
    prx = c;
    pry = s;
    cnt += live && !z ? 1 : 0;
    live = live && !z;
    di1 = di;
  };
  // two steps per trip: the prefetched pair and the pending writes change registers
  // between the copies instead of being moved at the end of every step
  int i = mu - 1;
  for (; i - 1 >= lu; i -= 2) {
    step(i);
    step(i - 1);
  }
  if (i >= lu) step(i);
  if (lane0) {
    pd->x = pdx;
    pd->y = pdy;
    pr->x = prx;
    pr->y = pry;
  }
  ChaseOut o;
  o.p = p;
  o.g = g;
  o.cnt = __builtin_amdgcn_readfirstlane(cnt);
  o.split = __builtin_amdgcn_readfirstlane(live ? 0 : 1);
  return o;
}

// Householder reduction of an order-n matrix (n <= kWaveReduceMax) by wave 0 alone: lane
// r owns row j+1+r of the trailing block, so no column needs a workgroup barrier. A wave's
// LDS accesses complete in order; the block-scope fences between the phases only keep
// the compiler from moving loads above the stores they read. Same outputs as the
// four-wave reduction: (d, e) in E.dd / E.ee, reflectors and betas in E.hv.
constexpr int kWaveReduceMax = 64;
__device__ void tri_reduce_wave(const EigWs &E) {
  const int n = E.n, pa = E.pa, lane = threadIdx.x & 63;
  double *A = E.A, *vv = E.vv, *pp = E.pp, *dd = E.dd, *ee = E.ee, *hv = E.hv;
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;
    const bool act = lane < m;
    double *row = A + (j + 1 + lane) * pa + j + 1;       // lane's row of the trailing block
    const double x = act ? row[-1] : 0.0;                 // column j below the diagonal
    const double nrm2 = wave_sum(x * x);
    const double x0 = lane0(x);
    if (nrm2 == 0.0) {                                    // column already reduced
      if (lane == 0) { dd[j] = A[j * pa + j]; ee[j] = 0.0; hv[int64_t(n) * n + j] = 0.0; }
      continue;
    }
    const double alpha = -copysign(sqrt(nrm2), x0);
    const double beta = 1.0 / (nrm2 - x0 * alpha);        // 2 / (v^T v)
    const double v = lane == 0 ? x0 - alpha : x;
    if (act) { vv[lane] = v; hv[int64_t(j) * n + lane] = v; }
    if (lane == 0) { dd[j] = A[j * pa + j]; ee[j] = alpha; hv[int64_t(n) * n + j] = beta; }
    __threadfence_block();
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;        // p = beta * A_t v, row by row
    if (act) {
      int k = 0;
      for (; k + 3 < m; k += 4) {
        a0 = fma(row[k], vv[k], a0);
        a1 = fma(row[k + 1], vv[k + 1], a1);
        a2 = fma(row[k + 2], vv[k + 2], a2);
        a3 = fma(row[k + 3], vv[k + 3], a3);
      }
      for (; k < m; ++k) a0 = fma(row[k], vv[k], a0);
    }
    const double p = beta * ((a0 + a1) + (a2 + a3));
    if (act) pp[lane] = p;
    const double K2 = beta * wave_sum(act ? v * p : 0.0);   // 2K = beta v^T p
    __threadfence_block();
    if (act) {                                            // A_t -= v p^T + p v^T - 2K v v^T
      // in chunks of 8: all loads of a chunk are issued before its stores (a store to row[]
      // could alias a later load of pp[] or vv[] as far as the compiler knows, so a plain
      // loop would wait out the LDS latency on every element)
      const double vk = v * K2;
      int b = 0;
      for (; b + 8 <= m; b += 8) {
        double x[8], pb[8], vb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) { x[u] = row[b + u]; pb[u] = pp[b + u]; vb[u] = vv[b + u]; }
#pragma unroll
        for (int u = 0; u < 8; ++u) row[b + u] = x[u] - fma(v, pb[u], fma(p, vb[u], -vk * vb[u]));
      }
      for (; b < m; ++b) row[b] -= fma(v, pp[b], fma(p, vv[b], -vk * vv[b]));
    }
    __threadfence_block();
  }
  if (lane == 0) {
    if (n >= 2) {
      dd[n - 2] = A[(n - 2) * pa + n - 2];
      ee[n - 2] = A[(n - 1) * pa + n - 2];
    }
    dd[n - 1] = A[(n - 1) * pa + n - 1];
    ee[n - 1] = 0.0;
  }
}

// ---------------------------------------------------------------- divide and conquer
//
// Tridiagonal eigensolve by divide and conquer for orders up to kDcMax, used in place of
// QL. Every off-diagonal e_i tears T into diag(T1, T2) + rho v v^T (rho = |e_i|,
// v = e_i + sign(e_i) e_{i+1}), so the leaves are the 1 x 1 blocks d_i - |e_{i-1}| - |e_i|;
// blocks are merged bottom-up, pairs of width S/2 into width S (the first two levels, the
// 4 x 4 blocks, directly by Jacobi rotations). A merge of children with eigenpairs (D1, Q1), (D2, Q2) solves
// D + rho z z^T with z = (last row of Q1, sign * first row of Q2):
//  * deflation: components with rho |z_i| <= tol keep (D_i, column i); pairs of close
//    D (|(D_j - D_i) c s| <= tol after the rotation that moves z_i into z_j) are rotated
//    and one of them deflates; tol = 8 eps max(|D|, rho |z|) of the merge;
//  * each remaining root lam_t of 1 + rho sum z_i^2 / (delta_i - lam) (delta ascending,
//    one root in each (delta_t, delta_t+1), the last below delta_K + rho ||z||^2) is found
//    by a group of lanes, as lam = delta_o + tau with the origin o the nearer pole, so that
//    every delta_i - lam_t is formed without cancellation (dc_root);
//  * the eigenvectors come from z recomputed from the roots (the Loewner formula of Gu
//    and Eisenstat), which keeps them orthogonal to working accuracy:
//    zh_i^2 = prod_t (lam_t - delta_i) / (rho prod_{t != i} (delta_t - delta_i)),
//    u_t = (zh_i / (delta_i - lam_t))_i normalised;
//  * the merged eigenvectors are Q u_t (kept) and the deflated columns of Q.
// Eigenvector blocks alternate between two n x n buffers whose entries outside the
// current blocks stay zero. Up to order kDcLdsMax both buffers and the merge matrices are in
// LDS; up to kDcMax the second buffer and the merge matrices are in the op's global scratch.
constexpr int kDcLdsMax = 64;
constexpr int kDcMax = 128;
__host__ __device__ constexpr int dc_vec_doubles(int n) { return 8 * n + (9 * n + 1) / 2; }
__host__ __device__ constexpr int dc_lds_doubles(int n) { return 2 * n * (n + 1) + dc_vec_doubles(n); }

struct DcBufs {
  double *vec, *zb, *wm;   // per-index vectors (LDS), second eigenvector buffer, merge matrices
};

struct DcWs {
  double *Zb, *W;                                  // second eigenvector buffer; merge matrices
  double *D, *z, *dk, *zk, *tau, *zh, *rc, *rs;    // per index (n each)
  int *perm, *kept, *defl, *org, *rj, *ri, *cnt;   // per index; cnt: K, deflated, rotations at lo
};

__device__ DcWs dc_ws(const DcBufs &b, int n) {
  DcWs W;
  W.Zb = b.zb;                                     // n x (n + 1), as Z
  W.W = b.wm;                                      // n x (n + 1): odd pitch
  double *v = b.vec;
  W.D = v; W.z = v + n; W.dk = v + 2 * n; W.zk = v + 3 * n; W.tau = v + 4 * n; W.zh = v + 5 * n;
  W.rc = v + 6 * n; W.rs = v + 7 * n;
  int *iv = reinterpret_cast<int *>(v + 8 * n);
  W.perm = iv; W.kept = iv + n; W.defl = iv + 2 * n; W.org = iv + 3 * n; W.rj = iv + 4 * n;
  W.ri = iv + 5 * n; W.cnt = iv + 6 * n;             // 3 ints per block start: up to 3n, in 8n doubles' room
  return W;
}

// max over aligned groups of g lanes (g a power of two <= 64)
__device__ __forceinline__ double group_max(double v, int g) {
  if (g >= 2) v = fmax(v, dpp_f64<kDppQuadXor1>(v));       // within rows of 16 on DPP
  if (g >= 4) v = fmax(v, dpp_f64<kDppQuadXor2>(v));
  if (g >= 8) v = fmax(v, dpp_f64<kDppRowHalfMirror>(v));
  if (g >= 16) v = fmax(v, dpp_f64<kDppRowMirror>(v));
  if (g >= 32) v = fmax(v, __shfl_xor(v, 16, 64));          // across rows: two moves
  if (g >= 64) v = fmax(v, __shfl_xor(v, 32, 64));
  return v;
}

// sum and product over aligned groups of L lanes, L in {2, 4, 8, 16} (all lanes of a group
// active); every lane of the group gets the same value
__device__ __forceinline__ double lsum(double v, int L) {
  v += dpp_f64<kDppQuadXor1>(v);
  if (L >= 4) v += dpp_f64<kDppQuadXor2>(v);
  if (L >= 8) v += dpp_f64<kDppRowHalfMirror>(v);
  if (L >= 16) v += dpp_f64<kDppRowMirror>(v);
  return v;
}
__device__ __forceinline__ double lprod(double v, int L) {
  v *= dpp_f64<kDppQuadXor1>(v);
  if (L >= 4) v *= dpp_f64<kDppQuadXor2>(v);
  if (L >= 8) v *= dpp_f64<kDppRowHalfMirror>(v);
  if (L >= 16) v *= dpp_f64<kDppRowMirror>(v);
  return v;
}

// 1/x from the hardware estimate and two Newton steps (within an ulp or two for normal x)
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// Root in (lo, hi) of c + wl / (al - x) + wr / (ar - x) = 0, or lo - 1 if it has none there.
__device__ double dc_quad_root(double c, double al, double ar, double wl, double wr, double lo, double hi) {
  const double b = -(c * (al + ar) + wl + wr), cc = c * al * ar + wl * ar + wr * al;
  if (c != 0.0) {
    const double disc = b * b - 4.0 * c * cc;
    if (disc < 0.0) return lo - 1.0;
    const double q = -0.5 * (b + copysign(sqrt(disc), b));
    const double x1 = q * rcp_nr(c);
    if (lo < x1 && x1 < hi) return x1;
    if (q != 0.0) {
      const double x2 = cc * rcp_nr(q);
      if (lo < x2 && x2 < hi) return x2;
    }
    return lo - 1.0;
  }
  if (b != 0.0) {
    const double x = -cc * rcp_nr(b);
    if (lo < x && x < hi) return x;
  }
  return lo - 1.0;
}

// Root t of 1 + rho sum_i z_i^2 / (delta_i - lam), i < K (delta ascending, rho > 0), by an
// aligned group of L lanes (each sums every L-th term; all of them agree bit for bit). Returns tau with
// lam = delta_o + tau, o in {t, t+1} the nearer pole. The start solves the model with the
// two nearest poles at their exact weights and the others a constant; each step solves the
// model with one pole on each side of the root, weighted to match the derivatives of the
// two partial sums (for the last root: its own pole exact, the others at delta_{K-2}),
// inside a bracket kept by the sign of f.
__device__ double dc_root(const double *dk, const double *zk, int K, int t, double rho, int sub, int L,
                        int *o_out) {
  constexpr double kEps = 2.220446049250313e-16;
  if (K == 1) { *o_out = 0; return rho * zk[0] * zk[0]; }
  const double dt = dk[t];
  int o, pa;
  double lo, hi, tau, rest;
  if (t < K - 1) {
    const double mid = 0.5 * (dk[t + 1] - dt);
    double f = 0.0, two = 0.0;
    for (int i = sub; i < K; i += L) {
      const double term = zk[i] * zk[i] * rcp_nr((dk[i] - dt) - mid);
      f += term;
      two += (i == t || i == t + 1) ? term : 0.0;
    }
    f = lsum(f, L);
    two = lsum(two, L);
    rest = f - two;
    if (1.0 + rho * f >= 0.0) { o = t; lo = 0.0; hi = mid; tau = mid; }
    else { o = t + 1; lo = -mid; hi = 0.0; tau = -mid; }
    pa = t;
  } else {
    double s2 = 0.0, r = 0.0;
    for (int i = sub; i < K; i += L) {
      const double z2 = zk[i] * zk[i];
      s2 += z2;
      r += i + 2 < K ? z2 * rcp_nr(dk[i] - dt) : 0.0;   // the others seen from the origin
    }
    s2 = lsum(s2, L);
    rest = lsum(r, L);
    o = K - 1; lo = 0.0; hi = rho * s2; tau = 0.5 * hi;
    pa = K - 2;
  }
  const double dko = dk[o];
  const double pl = dk[pa] - dko, pr = dk[pa + 1] - dko;   // the two nearest poles
  {
    const double x = dc_quad_root(1.0 + rho * rest, pl, pr, rho * zk[pa] * zk[pa], rho * zk[pa + 1] * zk[pa + 1],
                                  lo, hi);
    if (x >= lo) tau = x;
  }
  const bool last = t == K - 1;
  const double zo2 = zk[o] * zk[o];
  for (int it = 0; it < 64; ++it) {
    double psi = 0.0, phi = 0.0, dpsi = 0.0, dphi = 0.0;
    for (int i = sub; i < K; i += L) {
      const double w = zk[i] * rcp_nr((dk[i] - dko) - tau);
      const double a = zk[i] * w, b = w * w;
      const bool left = i <= t;
      psi += left ? a : 0.0; dpsi += left ? b : 0.0;
      phi += left ? 0.0 : a; dphi += left ? 0.0 : b;
    }
    psi = lsum(psi, L); phi = lsum(phi, L); dpsi = lsum(dpsi, L); dphi = lsum(dphi, L);
    const double f = 1.0 + rho * (psi + phi);
    const double err = kEps * (2.0 + 8.0 * rho * (phi - psi) + 3.0 * rho * fabs(tau) * (dpsi + dphi));   // psi < 0 < phi
    if (f > 0.0) hi = tau;
    else if (f < 0.0) lo = tau;
    if (fabs(f) <= err || hi - lo <= 2.0 * kEps * fmax(fabs(lo), fabs(hi))) break;
    const double al = pl - tau, ar = pr - tau;
    double sl, sr;
    if (!last) { sl = dpsi * al * al; sr = dphi * ar * ar; }
    else { sr = zo2; sl = (dpsi - zo2 * rcp_nr(ar * ar)) * al * al; }
    const double c = f - rho * (sl * rcp_nr(al) + sr * rcp_nr(ar));
    const double eta = dc_quad_root(c, al, ar, rho * sl, rho * sr, lo - tau, hi - tau);
    const double nt = tau + eta;
    if (eta >= lo - tau && lo < nt && nt < hi) {
      if (nt == tau) break;                         // the step no longer moves tau
      tau = nt;
    } else {
      tau = 0.5 * (lo + hi);
    }
  }
  *o_out = o;
  return tau;
}

// Lane groups of width S (one merge each, blocks [lo, lo + S)): gather D and z,
// order D, deflate, rotate the columns of Z the deflation pairs, and list the poles (dk, zk)
// of the remaining secular equation. cnt[3lo] = K roots, cnt[3lo+1] deflated columns.
// tol = 8 eps max(|D|, rho |z|) of the merge: each deflation perturbs the merged block by
// at most that (a tolerance from ||T|| instead would perturb the small eigenvalues of a
// graded matrix far more than a QL solve does).
// Merges of width S <= 64 only: the calling wave takes those whose block starts in
// [64 win, 64 win + 64).
__device__ void dc_deflate(double *Z, const double *dd, const double *ee, const DcWs &W, int n, int S, int win) {
  constexpr double kEps = 2.220446049250313e-16;
  const int zpitch = n + 1;                         // column pitch of Z
  const int lane = threadIdx.x & 63, g = S;
  const int base = (lane / g) * g, lo = 64 * win + (lane / g) * S, t = lane - base;
  const int m = lo + S / 2, hi = lo + S < n ? lo + S : n;
  const bool merge = lo < n && m < hi;
  const int s = merge ? hi - lo : 0, n1 = m - lo;
  const bool act = t < s;
  double rho = 0.0, Dt = 0.0, zt = 0.0;
  if (merge) {
    const double e = ee[m - 1];
    rho = 2.0 * fabs(e);
    if (act) {                                      // z: last row of Q1, first row of Q2
      Dt = dd[lo + t];
      zt = (t < n1 ? Z[(lo + t) * zpitch + (m - 1)] : copysign(1.0, e) * Z[(lo + t) * zpitch + m]) * 0.70710678118654752440;
      W.D[lo + t] = Dt;
      W.z[lo + t] = zt;
    }
  }
  __threadfence_block();
  if (act) {                                        // ascending order, ties by index
    int r = 0;
    for (int u = 0; u < s; ++u) {
      const double du = W.D[lo + u];
      r += (du < Dt) || (du == Dt && u < t);
    }
    W.perm[lo + r] = t;
  }
  const double dmax = group_max(act ? fabs(Dt) : 0.0, g), zmax = group_max(act ? fabs(zt) : 0.0, g);
  const double tol = 8.0 * kEps * fmax(dmax, rho * zmax);
  __threadfence_block();
  // lane = sorted position: small rho |z| deflates; when no neighbouring pair of the others
  // is close enough to rotate, the others are the poles in order
  const int ip = act ? W.perm[lo + t] : 0;
  const double Dp = act ? W.D[lo + ip] : 0.0, zp = act ? W.z[lo + ip] : 0.0;
  const bool big = act && rho > 0.0 && rho * fabs(zp) > tol;
  const unsigned long long gmask = (g == 64 ? ~0ull : ((1ull << g) - 1)) << base;
  const unsigned long long below = (1ull << lane) - 1;
  const unsigned long long nsm = __ballot(big) & gmask;
  const unsigned long long after = nsm & ~below & ~(1ull << lane);
  const int nx = after ? __ffsll((long long)after) - 1 : lane;
  const double Dn = __shfl(Dp, nx, 64), zn = __shfl(zp, nx, 64);
  bool close = false;
  if (big && after) {
    const double tt = hypot(zp, zn);
    close = fabs((Dn - Dp) * (zn / tt) * (zp / tt)) <= tol;
  }
  const unsigned long long closem = __ballot(close) & gmask;
  if (!closem) {
    if (act) {
      if (big) W.kept[lo + __popcll(nsm & below)] = ip;
      else W.defl[lo + __popcll(~nsm & gmask & below)] = ip;
    }
    if (merge && t == 0) {
      const int K = __popcll(nsm);
      W.cnt[3 * lo] = K; W.cnt[3 * lo + 1] = s - K; W.cnt[3 * lo + 2] = 0;
    }
  } else if (merge && t == 0) {                     // rotations needed: one lane per merge
    int K = 0, nd = 0, nr = 0, cand = -1;
    for (int p = 0; p < s; ++p) {
      const int i = W.perm[lo + p];
      const double zi = W.z[lo + i];
      if (rho * fabs(zi) <= tol) { W.defl[lo + nd++] = i; continue; }
      if (cand < 0) { cand = i; continue; }
      const double zc = W.z[lo + cand];
      const double tt = hypot(zc, zi), c = zi / tt, sn = -zc / tt;
      const double dc = W.D[lo + cand], di = W.D[lo + i];
      if (fabs((di - dc) * c * sn) <= tol) {
        W.rj[lo + nr] = cand; W.ri[lo + nr] = i; W.rc[lo + nr] = c; W.rs[lo + nr] = sn; ++nr;
        W.D[lo + cand] = dc * c * c + di * sn * sn;
        W.D[lo + i] = dc * sn * sn + di * c * c;
        W.z[lo + i] = tt;
        W.z[lo + cand] = 0.0;
        W.defl[lo + nd++] = cand;
      } else {
        W.kept[lo + K++] = cand;
      }
      cand = i;
    }
    if (cand >= 0) W.kept[lo + K++] = cand;
    W.cnt[3 * lo] = K; W.cnt[3 * lo + 1] = nd; W.cnt[3 * lo + 2] = nr;
  }
  __threadfence_block();
  const int K = merge ? W.cnt[3 * lo] : 0, nr = merge ? W.cnt[3 * lo + 2] : 0;
  if (act) {                                        // deflation rotations on row lo+t of Q
    const int row = lo + t;
    for (int r = 0; r < nr; ++r) {
      double *qa = Z + (lo + W.rj[lo + r]) * zpitch + row, *qb = Z + (lo + W.ri[lo + r]) * zpitch + row;
      const double c = W.rc[lo + r], sn = W.rs[lo + r], x = *qa, y = *qb;
      *qa = c * x + sn * y;
      *qb = -sn * x + c * y;
    }
  }
  if (t < K) { W.dk[lo + t] = W.D[lo + W.kept[lo + t]]; W.zk[lo + t] = W.z[lo + W.kept[lo + t]]; }
}

// The merge of width 128 (orders 65 to 128): one merge of s = n elements, two per lane of
// the calling wave; the deflation scan runs in one lane.
__device__ __noinline__ void dc_deflate_big(double *Z, const double *dd, const double *ee, const DcWs &W, int n) {
  constexpr double kEps = 2.220446049250313e-16;
  const int zp = n + 1, lane = threadIdx.x & 63, m = 64, s = n;
  const double e = ee[m - 1], rho = 2.0 * fabs(e);
  double dmx = 0.0, zmx = 0.0;
  for (int t = lane; t < s; t += 64) {             // z: last row of Q1, first row of Q2
    const double Dt = dd[t];
    const double zt = (t < m ? Z[t * zp + (m - 1)] : copysign(1.0, e) * Z[t * zp + m]) * 0.70710678118654752440;
    W.D[t] = Dt;
    W.z[t] = zt;
    dmx = fmax(dmx, fabs(Dt));
    zmx = fmax(zmx, fabs(zt));
  }
  const double tol = 8.0 * kEps * fmax(wave_max(dmx), rho * wave_max(zmx));
  __threadfence_block();
  for (int t = lane; t < s; t += 64) {             // ascending order, ties by index
    const double Dt = W.D[t];
    int r = 0;
    for (int u = 0; u < s; ++u) {
      const double du = W.D[u];
      r += (du < Dt) || (du == Dt && u < t);
    }
    W.perm[r] = t;
  }
  __threadfence_block();
  if (lane == 0) {
    int K = 0, nd = 0, nr = 0, cand = -1;
    if (rho == 0.0) {
      for (int p = 0; p < s; ++p) W.defl[nd++] = W.perm[p];
    } else {
      for (int p = 0; p < s; ++p) {
        const int i = W.perm[p];
        const double zi = W.z[i];
        if (rho * fabs(zi) <= tol) { W.defl[nd++] = i; continue; }
        if (cand < 0) { cand = i; continue; }
        const double zc = W.z[cand];
        const double tt = hypot(zc, zi), c = zi / tt, sn = -zc / tt;
        const double dc = W.D[cand], di = W.D[i];
        if (fabs((di - dc) * c * sn) <= tol) {
          W.rj[nr] = cand; W.ri[nr] = i; W.rc[nr] = c; W.rs[nr] = sn; ++nr;
          W.D[cand] = dc * c * c + di * sn * sn;
          W.D[i] = dc * sn * sn + di * c * c;
          W.z[i] = tt;
          W.z[cand] = 0.0;
          W.defl[nd++] = cand;
        } else {
          W.kept[K++] = cand;
        }
        cand = i;
      }
      if (cand >= 0) W.kept[K++] = cand;
    }
    W.cnt[0] = K; W.cnt[1] = nd; W.cnt[2] = nr;
  }
  __threadfence_block();
  const int K = W.cnt[0], nr = W.cnt[2];
  for (int row = lane; row < n; row += 64) {       // deflation rotations on the rows of Q
    for (int r = 0; r < nr; ++r) {
      double *qa = Z + W.rj[r] * zp + row, *qb = Z + W.ri[r] * zp + row;
      const double c = W.rc[r], sn = W.rs[r], x = *qa, y = *qb;
      *qa = c * x + sn * y;
      *qb = -sn * x + c * y;
    }
  }
  for (int t = lane; t < K; t += 64) { W.dk[t] = W.D[W.kept[t]]; W.zk[t] = W.z[W.kept[t]]; }
}

// 1/sqrt(x) from the hardware estimate and two Newton steps (x well inside the normal range)
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

// Jacobi rotation of the symmetric 4 x 4 a (eigenvectors v) that zeroes a[I][J]: with
// d = a_JJ - a_II and t = tan of the angle, the smaller root of t^2 + (d / a_IJ) t - 1 = 0,
// t = sign(d) 2 a_IJ / (|d| + sqrt(d^2 + 4 a_IJ^2)), formed after scaling d and 2 a_IJ by the
// larger of the two (itself first scaled by 2^1000 when below 2^-1000, so that its reciprocal
// stays finite for subnormal entries); then a_II -= t a_IJ, a_JJ += t a_IJ. Entries at or
// below eps (|a_II| + |a_JJ|) / 2 are dropped instead (t = 0).
struct JacRot {
  double t, cs, sn;
  bool rot;
};
template <int I, int J>
__device__ __forceinline__ JacRot jac4_angle(const double (&a)[4][4]) {
  constexpr double kEps = 2.220446049250313e-16;
  JacRot R;
  const double aij = a[I][J];
  R.rot = fabs(aij) > 0.5 * kEps * (fabs(a[I][I]) + fabs(a[J][J]));
  double d = a[J][J] - a[I][I], g = 2.0 * aij, mx = fmax(fabs(d), fabs(g));
  if (mx < 0x1p-1000) {                                  // exactly rescaled: 1/mx must not overflow
    d *= 0x1p1000;
    g *= 0x1p1000;
    mx *= 0x1p1000;
  }
  const double rm = rcp_nr(R.rot ? mx : 1.0);
  const double dn = d * rm, gn = g * rm;
  const double h = fma(dn, dn, gn * gn);                 // in [1, 2]
  const double t = (d >= 0.0 ? gn : -gn) * rcp_nr(fabs(dn) + h * rsq_nr(h));
  R.t = R.rot ? t : 0.0;
  R.cs = R.rot ? rsq_nr(fma(t, t, 1.0)) : 1.0;
  R.sn = R.t * R.cs;
  return R;
}
template <int I, int J>
__device__ __forceinline__ void jac4_apply(double (&a)[4][4], double (&v)[4][4], const JacRot &R) {
  const double aij = a[I][J];
  a[I][I] -= R.t * aij;
  a[J][J] += R.t * aij;
  a[I][J] = 0.0;
  a[J][I] = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (r != I && r != J) {
      const double x = a[r][I], y = a[r][J];
      a[r][I] = a[I][r] = R.cs * x - R.sn * y;
      a[r][J] = a[J][r] = R.sn * x + R.cs * y;
    }
    const double x = v[r][I], y = v[r][J];
    v[r][I] = R.cs * x - R.sn * y;
    v[r][J] = R.sn * x + R.cs * y;
  }
}
// One round of a cyclic sweep: the planes (I, J) and (K, L) are disjoint, so neither angle
// depends on the other rotation and both are formed together. True if either rotated.
template <int I, int J, int K, int L>
__device__ __forceinline__ bool jac4_round(double (&a)[4][4], double (&v)[4][4]) {
  const JacRot r1 = jac4_angle<I, J>(a), r2 = jac4_angle<K, L>(a);
  jac4_apply<I, J>(a, v, r1);
  jac4_apply<K, L>(a, v, r2);
  return r1.rot || r2.rot;
}

// The merge and the position within it that quad q (= index q of the level) stands for.
struct DcPos {
  int lo, t, s, K;
  bool merge;
};
__device__ __forceinline__ DcPos dc_pos(const DcWs &W, int n, int S, int q) {
  DcPos P;
  P.lo = (q / S) * S;
  P.t = q - P.lo;
  const int hi = P.lo + S < n ? P.lo + S : n;
  P.merge = P.lo < n && P.lo + S / 2 < hi;
  P.s = P.merge ? hi - P.lo : 0;
  P.K = P.merge ? W.cnt[3 * P.lo] : 0;
  return P;
}

// Eigenpairs of the tridiagonal (E.dd, E.ee) by divide and conquer: eigenvalues in E.dd
// (unordered), eigenvectors in E.A as Z (column j at E.A[j (n+1) ..]), as the QL solve leaves them.
// Per level: wave 0 (and wave 1 above order 64) deflates every merge; then groups of L lanes (one per index of the
// level) find the roots and write delta_i - lam_t (column t of the merge's block of W, odd
// pitch pw), recompute z, form and normalise the vectors u_t; then the workgroup multiplies.
__device__ void tri_dc(const EigWs &E, const DcBufs &bufs) {
  const int n = E.n, tid = threadIdx.x, wave = tid >> 6;
  const int L = n <= 16 ? 16 : (n <= 32 ? 8 : (n <= 64 ? 4 : 2));   // lanes per index of a level
  const int q = tid / L, sub = tid % L;
  const DcWs W = dc_ws(bufs, n);
  const int pw = n + 1, zp = n + 1;                 // pitches of the merge matrices and of Z
  double *Za = E.A, *Zb = W.Zb;
  for (int e = tid; e < n * zp; e += kThreads) {
    Za[e] = (e / zp == e % zp) ? 1.0 : 0.0;
    Zb[e] = 0.0;
  }
  for (int i = tid; i < n; i += kThreads)           // the tears: leaves d_i - |e_i-1| - |e_i|
    E.dd[i] -= (i > 0 ? fabs(E.ee[i - 1]) : 0.0) + (i + 1 < n ? fabs(E.ee[i]) : 0.0);
  __syncthreads();
  // the first two levels directly: block [4p, 4p + 4) (its inner tears undone) by cyclic
  // Jacobi in one lane, its eigenvectors into the block's columns of Z (jac4_round)
  for (int p = tid; 4 * p < n; p += kThreads) {
    const int i0 = 4 * p, s = n - i0 < 4 ? n - i0 : 4;
    double a[4][4], v[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int c = 0; c < 4; ++c) { a[r][c] = 0.0; v[r][c] = r == c ? 1.0 : 0.0; }
      if (r < s) a[r][r] = E.dd[i0 + r];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      if (r + 1 < s) {
        const double b = E.ee[i0 + r], rb = fabs(b);
        a[r][r] += rb;
        a[r + 1][r + 1] += rb;
        a[r][r + 1] = b;
        a[r + 1][r] = b;
      }
    }
    for (int sweep = 0; sweep < 16; ++sweep) {
      bool rotated = jac4_round<0, 1, 2, 3>(a, v);
      rotated |= jac4_round<0, 2, 1, 3>(a, v);
      rotated |= jac4_round<0, 3, 1, 2>(a, v);
      if (!rotated) break;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c < s) {
        E.dd[i0 + c] = a[c][c];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (r < s) Za[(i0 + c) * zp + i0 + r] = v[r][c];
      }
    }
  }
  __syncthreads();
  double *Zc = Za, *Zn = Zb;
  for (int S = 8; S / 2 < n; S *= 2) {
    if (S <= 64) {
      if (64 * wave < n) dc_deflate(Zc, E.dd, E.ee, W, n, S, wave);
    } else if (wave == 0) {
      dc_deflate_big(Zc, E.dd, E.ee, W, n);
    }
    __syncthreads();
    const DcPos P = dc_pos(W, n, S, q);
    const double *dk = W.dk + P.lo, *zk = W.zk + P.lo;
    double *U = W.W + P.lo * pw + P.lo;             // (delta_i - lam_t), then u: U[t pw + i]
    const double rho = P.merge ? 2.0 * fabs(E.ee[P.lo + S / 2 - 1]) : 0.0;
    if (q < n && P.t < P.K) {                       // root t
      int o;
      const double tau = dc_root(dk, zk, P.K, P.t, rho, sub, L, &o);
      const double dko = dk[o];
      if (sub == 0) W.tau[P.lo + P.t] = dko + tau;
      for (int i = sub; i < P.K; i += L) U[P.t * pw + i] = (dk[i] - dko) - tau;
    }
    __syncthreads();
    if (q < n && P.t < P.K) {                       // zh_t from row t of (delta_i - lam)
      const int t = P.t, K = P.K;
      const double dt = dk[t];
      double p = 1.0;
      for (int u = sub; u < K; u += L) {
        const double num = -U[u * pw + t];
        p *= u == K - 1 ? num / rho : num * rcp_nr((u < t ? dk[u] : dk[u + 1]) - dt);
      }
      p = lprod(p, L);
      if (sub == 0) W.zh[P.lo + t] = copysign(sqrt(p), zk[t]);
    }
    __syncthreads();
    if (q < n && P.t < P.s) {                       // column t of u, normalised; the eigenvalues
      const int t = P.t, K = P.K;
      if (t < K && K <= 16 * L) {                  // at most 16 per lane: kept in registers
        double nrm = 0.0, uv[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const int i = sub + c * L;
          uv[c] = i < K ? W.zh[P.lo + i] * rcp_nr(U[t * pw + i]) : 0.0;
          nrm = fma(uv[c], uv[c], nrm);
        }
        const double sc = 1.0 / sqrt(lsum(nrm, L));
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const int i = sub + c * L;
          if (i < K) U[t * pw + i] = uv[c] * sc;
        }
      } else if (t < K) {
        double nrm = 0.0;
        for (int i = sub; i < K; i += L) {
          const double u = W.zh[P.lo + i] * rcp_nr(U[t * pw + i]);
          U[t * pw + i] = u;
          nrm = fma(u, u, nrm);
        }
        const double sc = 1.0 / sqrt(lsum(nrm, L));
        for (int i = sub; i < K; i += L) U[t * pw + i] *= sc;
      }
      if (sub == 0) E.dd[P.lo + t] = t < K ? W.tau[P.lo + t] : W.D[P.lo + W.defl[P.lo + (t - K)]];
    }
    __syncthreads();
    // Zn's blocks: kept columns Q u_t, then the deflated columns of Q (or the block as it
    // is where nothing merges); 4 columns per thread share each load of Q
    const int nb = (n + S - 1) / S, per = S * ((S + 3) / 4);
    for (int e = tid; e < nb * per; e += kThreads) {
      const int blk = e / per, r = e % per;
      const int lo = blk * S, hi = lo + S < n ? lo + S : n, s = hi - lo;
      const int row = r % S, j0 = (r / S) * 4;
      if (row >= s || j0 >= s) continue;
      const bool merge = lo + S / 2 < hi;
      const int K = merge ? W.cnt[3 * lo] : 0;
      const int jn = j0 < K ? (K - j0 < 4 ? K - j0 : 4) : 0;       // product columns here
      if (jn > 0) {
        const double *Ub = W.W + lo * pw + lo;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        for (int i = 0; i < K; ++i) {
          const double qv = Zc[(lo + W.kept[lo + i]) * zp + lo + row];
          a0 = fma(qv, Ub[j0 * pw + i], a0);
          if (jn > 1) a1 = fma(qv, Ub[(j0 + 1) * pw + i], a1);
          if (jn > 2) a2 = fma(qv, Ub[(j0 + 2) * pw + i], a2);
          if (jn > 3) a3 = fma(qv, Ub[(j0 + 3) * pw + i], a3);
        }
        double *out = Zn + (lo + j0) * zp + lo + row;
        out[0] = a0;
        if (jn > 1) out[zp] = a1;
        if (jn > 2) out[2 * zp] = a2;
        if (jn > 3) out[3 * zp] = a3;
      }
      for (int j = j0 + jn; j < j0 + 4 && j < s; ++j) {          // deflated (or unmerged) columns
        const int src = merge ? lo + W.defl[lo + (j - K)] : lo + j;
        Zn[(lo + j) * zp + lo + row] = Zc[src * zp + lo + row];
      }
    }
    __syncthreads();
    double *tmp = Zc; Zc = Zn; Zn = tmp;
  }
  if (Zc != Za) {
    for (int e = tid; e < n * zp; e += kThreads) Za[e] = Zc[e];
    __syncthreads();
  }
}

// Tridiagonalise E.A and solve T: by divide and conquer in the buffers dcb when use_dc
// (order <= kDcMax), else by implicit QL with the Wilkinson shift (the method of the Handbook
// routine tql2 of Bowdler, Martin, Reinsch and Wilkinson, re-organised for one workgroup).
__device__ void tri_ql(const EigWs &E, NetScalars *sc, bool timed, bool use_dc = false, DcBufs dcb = DcBufs{}) {
  const int n = E.n, pa = E.pa, tid = threadIdx.x, wave = tid >> 6;
  double *A = E.A, *vv = E.vv, *pp = E.pp, *ww = E.ww, *dd = E.dd, *ee = E.ee, *hv = E.hv;
  long long tph = wall_clock64();
  // Householder reduction, three barriers per column. The norm of the next column
  // below the diagonal is summed while the trailing update writes it; the 2-sided
  // update uses w = p - K v without storing w: A -= v p^T + p v^T - 2K v v^T.
  // Matrix-vector products run 4 lanes per row with two partial sums per lane.
  const int lane = tid & 63, sub = tid & 3, grp = tid >> 2;
  double *rs = E.wq, *rs2 = E.wq + 4;                  // per-wave partial sums (free until QL)
  bool have_norm = false;
  if (n <= kWaveReduceMax) {
    if (wave == 0) tri_reduce_wave(E);
  } else {
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;
    double nrm2;
    if (have_norm) {
      nrm2 = (rs[0] + rs[1]) + (rs[2] + rs[3]);
    } else {
      double part = 0.0;
      for (int i = tid; i < m; i += kThreads) {
        const double x = A[(j + 1 + i) * pa + j];
        part += x * x;
      }
      nrm2 = block_sum(part, E.red);
    }
    const double x0 = A[(j + 1) * pa + j];
    if (nrm2 == 0.0) {                     // column already reduced
      if (tid == 0) { dd[j] = A[j * pa + j]; ee[j] = 0.0; hv[int64_t(n) * n + j] = 0.0; }
      have_norm = false;
      __syncthreads();
      continue;
    }
    const double alpha = -copysign(sqrt(nrm2), x0);
    const double beta = 1.0 / (nrm2 - x0 * alpha);       // 2 / (v^T v)
    for (int i = tid; i < m; i += kThreads) {
      const double v = (i == 0) ? x0 - alpha : A[(j + 1 + i) * pa + j];
      vv[i] = v;
      hv[int64_t(j) * n + i] = v;
    }
    if (tid == 0) { dd[j] = A[j * pa + j]; ee[j] = alpha; hv[int64_t(n) * n + j] = beta; }
    __syncthreads();
    double vp = 0.0;
    for (int r = grp; r < m; r += kThreads / 4) {        // p = beta * A_t v
      const double *row = A + (j + 1 + r) * pa + j + 1;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int k = sub;
      for (; k + 12 < m; k += 16) {
        a0 += row[k] * vv[k];
        a1 += row[k + 4] * vv[k + 4];
        a2 += row[k + 8] * vv[k + 8];
        a3 += row[k + 12] * vv[k + 12];
      }
      for (; k < m; k += 4) a0 += row[k] * vv[k];
      const double acc = quad_sum((a0 + a1) + (a2 + a3));
      if (sub == 0) {
        pp[r] = beta * acc;
        vp += vv[r] * (beta * acc);
      }
    }
    vp = wave_sum(vp);
    if (lane == 0) rs2[wave] = vp;
    __syncthreads();
    const double K2 = beta * ((rs2[0] + rs2[1]) + (rs2[2] + rs2[3]));   // 2K
    double nxt = 0.0;
    for (int bh = 0; bh < m; bh += 64) {                 // A_t -= v p^T + p v^T - 2K v v^T
      const int b = bh + lane;
      if (b < m) {
        const double vb = vv[b], pb = pp[b];
        int a = wave;
        for (; a + 12 < m; a += 16) {                    // 4 rows: all loads before the stores
          double va[4], pv[4], x[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            va[u] = vv[a + 4 * u];
            pv[u] = pp[a + 4 * u];
            x[u] = A[(j + 1 + a + 4 * u) * pa + j + 1 + b];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const double val = x[u] - (va[u] * pb + pv[u] * vb - K2 * va[u] * vb);
            A[(j + 1 + a + 4 * u) * pa + j + 1 + b] = val;
            if (b == 0 && a + 4 * u >= 1) nxt += val * val;   // next column, below its diagonal
          }
        }
        for (; a < m; a += kThreads / 64) {
          const double va = vv[a];
          double *x = A + (j + 1 + a) * pa + j + 1 + b;
          const double val = *x - (va * pb + pp[a] * vb - K2 * va * vb);
          *x = val;
          if (b == 0 && a >= 1) nxt += val * val;        // next column, below its diagonal
        }
      }
    }
    nxt = wave_sum(nxt);
    if (lane == 0) rs[wave] = nxt;
    have_norm = true;
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      dd[n - 2] = A[(n - 2) * pa + n - 2];
      ee[n - 2] = A[(n - 1) * pa + n - 2];
    }
    dd[n - 1] = A[(n - 1) * pa + n - 1];
    ee[n - 1] = 0.0;
  }
  }
  __syncthreads();
  if (timed && tid == 0) { const long long t = wall_clock64(); sc->ticks[0] += t - tph; tph = t; }
  if (use_dc) {
    tri_dc(E, dcb);
    if (timed && tid == 0) sc->ticks[6] += wall_clock64() - tph;
    return;
  }

  double *Z = A;
  for (int e = tid; e < n * pa; e += kThreads) Z[e] = (e / pa == e % pa) ? 1.0 : 0.0;
  // Implicit QL, split between a producer and consumers. Wave 0 runs the chase on its
  // own LDS copy of (d, e) (a sweep step reads index i and writes i+1, so the next
  // step's reads are issued one step ahead) and records the (c, s) of every rotation
  // of one QL iteration; after a barrier waves 1-3 apply that iteration's rotations to
  // their rows of Z while wave 0 already chases the next iteration into the other
  // buffer. One barrier per QL iteration; the chase carries no Z traffic.
  // (d_i, e_i) pairs and (c, s) pairs, so that each step of the chase is one 16-byte LDS
  // read and two 16-byte writes; the pair arrays start on a 16-byte boundary (8n doubles
  // at E.wq hold the pairs, both rotation buffers and the spare pair)
  Pair *de = reinterpret_cast<Pair *>(E.wq + ((reinterpret_cast<uintptr_t>(E.wq) >> 3) & 1));
  Pair *rot = de + n;                               // two buffers of n (c, s) pairs
  Pair *spare = rot + 2 * n;                        // write target of the chase after a split
  int *meta = E.flag;                               // per buffer: m, rotations (-1: finished)
  for (int i = tid; i < n; i += kThreads) de[i] = Pair{dd[i], ee[i]};
  __syncthreads();
  constexpr double kEps = 2.220446049250313e-16;
  long long nrot = 0;
  // producer state (wave 0)
  int l = 0, iter = 0;
  double efloor = 0.0;
  if (wave == 0) {
    // absolute deflation floor: an off-diagonal below eps*||T|| is negligible at the
    // absolute accuracy of any backward-stable solver; without it the null space of a
    // rank-deficient density matrix is iterated to full relative precision
    double tn = 0.0;
    for (int i = lane; i < n; i += 64) tn = fmax(tn, fmax(fabs(de[i].x), 2.0 * fabs(de[i].y)));
    efloor = kEps * wave_max(tn);
  }
  const int crow = tid - 64;                        // first consumer row
  for (int b = 0;; b ^= 1) {
    if (wave == 0) {
      int m = -1;
      while (l < n) {
        if (iter >= 64) { ++l; iter = 0; continue; }
        m = n - 1;                                  // first m >= l with a negligible e[m]
        for (int base = l; base < n - 1; base += 64) {
          const int i = base + lane;
          bool small = false;
          if (i < n - 1) {
            const double ei = fabs(de[i].y);
            small = ei <= kEps * (fabs(de[i].x) + fabs(de[i + 1].x)) || ei <= efloor;
          }
          const unsigned long long bl = __ballot(small);
          if (bl) { m = base + __ffsll((long long)bl) - 1; break; }
        }
        if (m != l) break;
        ++l;
        iter = 0;
      }
      if (l >= n) {
        if (lane == 0) { meta[2 * b] = 0; meta[2 * b + 1] = -1; }
      } else {
        ++iter;
        // l and m are the same in every lane: scalar copies keep the chase's loop control,
        // addresses and branches on the scalar unit
        const int lu = __builtin_amdgcn_readfirstlane(l), mu = __builtin_amdgcn_readfirstlane(m);
        Pair *rb = rot + n * b;
        const double dl = de[lu].x, el = de[lu].y;
        const double di1 = de[mu].x;
        // Wilkinson shift d_l - e_l / (g + sign(g) sqrt(g^2 + 1)), g = (d_{l+1} - d_l) / (2 e_l),
        // written as d_l - 2 e_l^2 / (h + sign(h) sqrt(h^2 + 4 e_l^2)) with h = d_{l+1} - d_l: one
        // square root and one reciprocal, both from hardware estimates with one Newton step
        // (a shift only steers convergence, so 2^-46 relative suffices); the exact quotient
        // form where the squares could underflow
        const double h = de[lu + 1].x - dl, w = el + el;
        const double s2 = fma(h, h, w * w);
        double g;
        if (s2 > 1e-280) {
          const double y = __builtin_amdgcn_rsq(s2);
          const double hyp = s2 * y * fma(-0.5 * s2 * y, y, 1.5);
          const double den = h + copysign(hyp, h);
          const double rd = __builtin_amdgcn_rcp(den);
          g = di1 - dl + 2.0 * el * el * (rd * fma(-den, rd, 2.0));
        } else {
          const double g0 = h / w;
          g = di1 - dl + el / (g0 + copysign(sqrt(g0 * g0 + 1.0), g0));
        }
        const ChaseOut co = ql_chase(de, rb, spare, lu, mu, g, di1);
        const int cnt = co.cnt;
        nrot += cnt + co.split;
        if (lane == 0) {
          if (!co.split) de[lu] = Pair{dl - co.p, co.g};
          de[mu].y = 0.0;
          meta[2 * b] = m;
          meta[2 * b + 1] = cnt;
        }
      }
    }
    __syncthreads();
    const int m = meta[2 * b], cnt = meta[2 * b + 1];
    if (cnt < 0) break;
    if (wave > 0 && cnt > 0) {                       // apply the iteration's rotations to rows crow
      const Pair *rb = rot + n * b;
      for (int row = crow; row < n; row += kThreads - 64) {
        double zc = Z[m * pa + row];                 // current value of column i+1
        double zn = Z[(m - 1) * pa + row];           // column i, fetched one step ahead
        for (int j = 0; j < cnt; ++j) {
          const int i = m - 1 - j;
          const double zi = zn;
          if (j + 1 < cnt) zn = Z[(i - 1) * pa + row];
          const Pair cs = rb[j];
          Z[(i + 1) * pa + row] = cs.y * zi + cs.x * zc;
          zc = cs.x * zi - cs.y * zc;
        }
        Z[(m - cnt) * pa + row] = zc;
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += kThreads) dd[i] = de[i].x;   // the eigenvalues
  if (tid == 0) sc->n_rot += nrot;
  __syncthreads();
  if (timed && tid == 0) sc->ticks[6] += wall_clock64() - tph;
}

// descending order of E.dd into E.wsrt / E.isrt (ties by index)
__device__ void order_desc(const EigWs &E) {
  const int n = E.n;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const double wi = E.dd[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double wj = E.dd[j];
      rank += (wj > wi) || (wj == wi && j < i);
    }
    E.wsrt[rank] = wi;
    E.isrt[rank] = i;
  }
  __syncthreads();
}

// The rank rule on descending eigenvalues w[0..navail) of a matrix of order n:
// at most ucols, drop w <= tau_rel*w1 (below what the FP64 solve resolves), and never
// cut where the spectrum does not separate: while w_k - w_{k+1} <= tau_deg*w_k and
// w_{k+1} > floor*w1, the cut moves up (a cut at relative gap g moves the kept subspace
// by about eps/g under the solver's backward error). Returns 0 if nothing survives.
__device__ int keep_rank(const double *w, int navail, int n, int ucols, const KeepParams &kp) {
  const double w1 = w[0];
  int k = ucols < n ? ucols : n;
  if (k > navail) k = navail;
  while (k >= 1 && w[k - 1] <= kp.tau_rel * w1) --k;
  while (k >= 1 && k < navail && w[k] > kp.floor * w1 && w[k - 1] - w[k] <= kp.tau_deg * w[k - 1]) --k;
  return k;
}

// z <- Q z for the k kept columns of Z (E.isrt[0..k)), last reflector first, four
// reflectors at a time in compact WY form: for the block H_lo ... H_hi (H_hi applied
// first), Q_blk = I - V T V^T with V = [v_lo .. v_hi] over rows lo+1..n-1 and T upper
// triangular (T_ii = beta_i, T(1:i-1, i) = -beta_i T(1:i-1, 1:i-1) V(:, 1:i-1)^T v_i).
// Per block: one phase computes w_t = V^T z_t for every kept column (4 lanes per column,
// four partial sums) and the Gram matrix V^T V; the next computes T from it in every
// thread and z_t -= V (T w_t), while the next block's V is staged into the other buffer.
// Two barriers per four reflectors.
constexpr int kWY = 4;
// For up to 64 kept columns: L = 4, 8 or 16 lanes per column (as many as 256 threads give
// the k columns; an aligned group within one wave) each take every L-th row and add their
// dot products across the group, one reflector at a time, so no step waits on a workgroup
// barrier (the groups are independent; the reflectors are read only).
template <int L>
__device__ void back_transform_lanes(const EigWs &E, int k) {
  const int n = E.n, tid = threadIdx.x, sub = tid % L, t = tid / L;
  if (t < k) {                               // every lane of the group takes this branch
    double *z = E.A + E.isrt[t] * E.pa;
    for (int j = n - 3; j >= 0; --j) {
      const double beta = E.hv[int64_t(n) * n + j];
      if (beta == 0.0) continue;             // the same j and beta in every lane
      const int m = n - j - 1;
      const double *v = E.hv + int64_t(j) * n;
      double *zz = z + j + 1;
      double a0 = 0.0, a1 = 0.0;
      int i = sub;
      for (; i + L < m; i += 2 * L) {
        a0 = fma(v[i], zz[i], a0);
        a1 = fma(v[i + L], zz[i + L], a1);
      }
      if (i < m) a0 = fma(v[i], zz[i], a0);
      const double w = beta * lsum(a0 + a1, L);
      int r = sub;                           // loads of 4 rows issued before their stores
      for (; r + 3 * L < m; r += 4 * L) {
        const double v0 = v[r], v1 = v[r + L], v2 = v[r + 2 * L], v3 = v[r + 3 * L];
        const double z0 = zz[r], z1 = zz[r + L], z2 = zz[r + 2 * L], z3 = zz[r + 3 * L];
        zz[r] = fma(-w, v0, z0);
        zz[r + L] = fma(-w, v1, z1);
        zz[r + 2 * L] = fma(-w, v2, z2);
        zz[r + 3 * L] = fma(-w, v3, z3);
      }
      for (; r < m; r += L) zz[r] = fma(-w, v[r], zz[r]);
    }
  }
  __syncthreads();
}
__device__ void back_transform_quads(const EigWs &E, int k) {
  if (k <= kThreads / 16) back_transform_lanes<16>(E, k);
  else if (k <= kThreads / 8) back_transform_lanes<8>(E, k);
  else back_transform_lanes<4>(E, k);
}

__device__ void back_transform(const EigWs &E, int k) {
  const int n = E.n, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, sub = tid & 3, grp = tid >> 2;
  double *Z = E.A;
  double *wbuf = E.vv;                       // k x kWY values of V^T z (vv..ee: 5n doubles)
  double *G = E.gw, *bet = E.gw + 16;        // Gram matrix of the block, its betas
  auto stage = [&](int jhi, double *Vb) {    // V of block jhi .. jlo over rows jlo+1..n-1
    const int jlo = jhi - kWY + 1 > 0 ? jhi - kWY + 1 : 0;
    const int mlo = n - jlo - 1;
    for (int e = tid; e < kWY * n; e += kThreads) {
      const int c = e / n, ip = e % n;       // column c holds v_{jlo+c}, local row ip
      const int j = jlo + c;
      double x = 0.0;
      if (j <= jhi && ip < mlo && ip >= c && E.hv[int64_t(n) * n + j] != 0.0) x = E.hv[int64_t(j) * n + (ip - c)];
      Vb[c * n + ip] = x;
    }
  };
  int cur = 0;
  if (n >= 3) {
    stage(n - 3, E.wq);
    __syncthreads();
  }
  for (int jhi = n - 3; jhi >= 0; jhi -= kWY) {
    const int jlo = jhi - kWY + 1 > 0 ? jhi - kWY + 1 : 0;
    const int b = jhi - jlo + 1;
    const int mlo = n - jlo - 1;
    const double *Vb = E.wq + cur * kWY * n;
    double *Vnext = E.wq + (cur ^ 1) * kWY * n;
    // phase 1: w_t = V^T z_t (tasks t < k) and the Gram entries (tasks k .. k+b-2: v_c . v_l, l < c)
    for (int task = grp; task < k + b - 1; task += kThreads / 4) {
      const double *z = task < k ? Z + E.isrt[task] * E.pa + jlo + 1 : Vb + (task - k + 1) * n;
      double a[kWY] = {0.0, 0.0, 0.0, 0.0};
      for (int i = sub; i < mlo; i += 4) {
        const double zi = z[i];
#pragma unroll
        for (int c = 0; c < kWY; ++c) a[c] += Vb[c * n + i] * zi;
      }
#pragma unroll
      for (int c = 0; c < kWY; ++c) a[c] = quad_sum(a[c]);
      if (sub == 0) {
        if (task < k) {
#pragma unroll
          for (int c = 0; c < kWY; ++c) wbuf[task * kWY + c] = a[c];
        } else {
          const int cc = task - k + 1;       // G[l][cc] = v_l . v_cc for l < cc
#pragma unroll
          for (int l = 0; l < kWY; ++l) if (l < cc) G[l * kWY + cc] = a[l];
        }
      }
    }
    if (tid < kWY) bet[tid] = (jlo + tid <= jhi) ? E.hv[int64_t(n) * n + jlo + tid] : 0.0;
    __syncthreads();
    // phase 2: T from the Gram entries and betas (every thread), z_t -= V (T w_t)
    double T[kWY][kWY];
#pragma unroll
    for (int r = 0; r < kWY; ++r)
#pragma unroll
      for (int c = 0; c < kWY; ++c) T[r][c] = 0.0;
#pragma unroll
    for (int c = 0; c < kWY; ++c) {
      const double bc = c < b ? bet[c] : 0.0;
#pragma unroll
      for (int r = 0; r < kWY; ++r) {
        if (r < c && c < b) {                    // T(r, c) = -beta_c sum_{l=r}^{c-1} T(r, l) G(l, c)
          double acc = 0.0;
#pragma unroll
          for (int l = 0; l < kWY; ++l) if (l >= r && l < c) acc += T[r][l] * G[l * kWY + c];
          T[r][c] = -bc * acc;
        }
      }
      T[c][c] = bc;
    }
    for (int t = wave; t < k; t += kThreads / 64) {
      double w[kWY], u[kWY];
#pragma unroll
      for (int c = 0; c < kWY; ++c) w[c] = wbuf[t * kWY + c];
#pragma unroll
      for (int r = 0; r < kWY; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kWY; ++c) acc += T[r][c] * w[c];
        u[r] = acc;
      }
      double *z = Z + E.isrt[t] * E.pa + jlo + 1;
      for (int i = lane; i < mlo; i += 64) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kWY; ++c) acc += Vb[c * n + i] * u[c];
        z[i] -= acc;
      }
    }
    if (jlo > 0) stage(jlo - 1, Vnext);
    cur ^= 1;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- learned warm start

constexpr int kF = 8, kH1 = 32, kH2 = 32;
constexpr int kNParams = kF * kH1 + kH1 + kH1 * kH2 + kH2 + kH2 + 1;

// Row statistics of L (valid n x n block, row stride ld): diag max, trace, ||L||_F^2.
struct RowStats { double dmax, tr, fro2; };

__device__ RowStats row_stats(const double *L, int ld, int n, double *red) {
  double dm = 0.0, tr = 0.0, f2 = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const double d = L[int64_t(i) * ld + i];
    dm = fmax(dm, d);
    tr += d;
  }
  for (int e = threadIdx.x; e < n * n; e += kThreads) {
    const double v = L[int64_t(e / n) * ld + e % n];
    f2 += v * v;
  }
  RowStats s;
  s.dmax = block_max(dm, red);
  s.tr = block_sum(tr, red);
  s.fro2 = block_sum(f2, red);
  return s;
}

// Bond-local features of row i (same definition as the reference in numpy).
__device__ void row_features(const double *L, int ld, int n, int i, int rest, bool bonded, const RowStats &st,
                             float *f) {
  const double d = L[int64_t(i) * ld + i];
  double rn2 = 0.0;
  for (int j = 0; j < n; ++j) {
    const double v = L[int64_t(i) * ld + j];
    rn2 += v * v;
  }
  const double rel = st.dmax > 0.0 ? d / st.dmax : 0.0;
  f[0] = float(rel);
  f[1] = float(log10(fmax(rel, 1e-30)) / 15.0);
  f[2] = float(st.tr > 0.0 ? d / st.tr : 0.0);
  f[3] = float(st.fro2 > 0.0 ? sqrt(rn2 / st.fro2) : 0.0);
  f[4] = float((d > 0.0 && st.tr > 0.0) ? rn2 / (d * st.tr) : 0.0);
  if (bonded) {
    const int nb = n / rest;
    f[5] = float(double(i / rest) / double(nb > 1 ? nb - 1 : 1));
    f[6] = float(double(i % rest) / double(rest > 1 ? rest - 1 : 1));
  } else {
    f[5] = float(double(i) / double(n > 1 ? n - 1 : 1));
    f[6] = 0.0f;
  }
  f[7] = float(n / 128.0);
}

// MLP 8 -> 32 -> 32 -> 1 (tanh, tanh, logistic); w laid out as W1 (8x32), b1, W2 (32x32), b2, W3, b3.
// Each first-layer unit is folded into the second layer's sums as soon as it is known,
// so only those 32 sums stay live.
__device__ float mlp_score(const float *w, const float *f) {
  const float *W1 = w, *b1 = W1 + kF * kH1, *W2 = b1 + kH1, *b2 = W2 + kH1 * kH2, *W3 = b2 + kH2, *b3 = W3 + kH2;
  float z2[kH2];
#pragma unroll
  for (int j = 0; j < kH2; ++j) z2[j] = b2[j];
  for (int a = 0; a < kH1; ++a) {
    float z = b1[a];
#pragma unroll
    for (int c = 0; c < kF; ++c) z += f[c] * W1[c * kH1 + a];
    const float h = tanhf(z);
#pragma unroll
    for (int j = 0; j < kH2; ++j) z2[j] += h * W2[a * kH2 + j];
  }
  float z = b3[0];
#pragma unroll
  for (int j = 0; j < kH2; ++j) z += tanhf(z2[j]) * W3[j];
  return 1.0f / (1.0f + expf(-z));
}

// Columns of V (n x p, row pitch p, in LDS) orthonormalised in order by classical
// Gram-Schmidt applied twice. A column whose part outside the span of the earlier ones
// has squared norm <= kDropRel times its own (zero columns included) becomes zero: the
// basis keeps its width and the zero directions give Ritz values 0, which the keep
// rule discards. Returns the number of nonzero columns.
constexpr double kDropRel = 1e-26;
__device__ int orth_drop(double *V, int n, int p, double *coef, double *red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int alive = 0;
  for (int j = 0; j < p; ++j) {
    double part = 0.0;
    for (int i = tid; i < n; i += kThreads) { const double v = V[i * p + j]; part += v * v; }
    const double nv2 = block_sum(part, red);
    for (int pass = 0; pass < 2; ++pass) {
      for (int q = wave; q < j; q += kThreads / 64) {   // c_q = V_q . V_j, one wave per q
        double acc = 0.0;
        for (int i = lane; i < n; i += 64) acc += V[i * p + q] * V[i * p + j];
        acc = wave_sum(acc);
        if (lane == 0) coef[q] = acc;
      }
      __syncthreads();
      for (int i = tid; i < n; i += kThreads) {
        double v = V[i * p + j];
        for (int q = 0; q < j; ++q) v -= coef[q] * V[i * p + q];
        V[i * p + j] = v;
      }
      __syncthreads();
    }
    part = 0.0;
    for (int i = tid; i < n; i += kThreads) { const double v = V[i * p + j]; part += v * v; }
    const double nu2 = block_sum(part, red);
    const bool keep = nv2 > 0.0 && nu2 > kDropRel * nv2;
    const double scale = keep ? 1.0 / sqrt(nu2) : 0.0;
    for (int i = tid; i < n; i += kThreads) V[i * p + j] *= scale;
    __syncthreads();
    alive += keep ? 1 : 0;
  }
  return alive;
}

// W = A V (A: n x pa symmetric in LDS, V: n x p)
__device__ void sym_times(const double *A, int pa, const double *V, int n, int p, double *W) {
  for (int e = threadIdx.x; e < n * p; e += kThreads) {
    const int i = e / p, c = e % p;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc += A[i * pa + j] * V[j * p + c];
    W[e] = acc;
  }
  __syncthreads();
}

// Learned warm start. The MLP scores the rows of L; the columns of L at the p best
// scores, orthonormalised (orth_drop), start a subspace iteration V <- orth(L V) with
// Rayleigh-Ritz on H = V^T L V, W = L V. The keep rule runs on the Ritz values. With
// P = V V^T and C = (I-P) L (I-P), the largest eigenvalue of L off span(V) is at most
// b = min(t, f): t = tr(L) - tr(H) = tr(C) (C is PSD when L is), and
// f = sqrt(||L||^2 - 2||W||^2 + ||H||^2 + slack) = ||C||_F (Frobenius identities of
// the 2x2 block split; the slack covers their rounding). The result is accepted when
//  * the weight off span(V) is below the floor of the rank rule, t <= floor * theta_1
//    (so no eigenvalue the exact rule could keep lies outside), or the rank is capped by
//    max_rank and b cannot move that cut (b <= theta_k / 2 and b < (1 - tau_deg) theta_k),
//    and
//  * every kept Ritz pair has ||L x - theta x|| <= residual_tol * theta, relative to its
//    own Ritz value: the smallest kept directions carry weight far below theta_1 and
//    later partitions can amplify them (#CSP networks), so they must be resolved too.
// Returns true with U written and the kept rank set; false leaves everything for the
// exact solve (the reason is counted in sc->rej).
constexpr double kFroSlack = 1e-13;
// Runtime extents (kept ranks) written by this workgroup are also kept in a small LDS cache:
// entry (slot & (kDynCache-1)) holds the slot id, then its value, so staging a later op that
// reads a recent slot needs no memory round trip. dcache may be null (no cache).
constexpr int kDynCache = 256;
__device__ __forceinline__ void set_dyn(int32_t *dyn, int32_t *dcache, int32_t slot, int32_t v) {
  dyn[slot] = v;
  if (dcache) {
    dcache[slot & (kDynCache - 1)] = slot;
    dcache[kDynCache + (slot & (kDynCache - 1))] = v;
  }
}

__device__ bool eig_learned(const Op &op, double *ws, int32_t *dyn, int32_t *dcache, const KeepParams &kp, NetScalars *sc,
                            double *lds, int n, int ld, int ucols) {
  const int tid = threadIdx.x;
  const bool bonded = op.bm.nd > 0;
  const int rest = op.bm.rest;
  const int kprev = bonded ? n / rest : n;
  int p = (bonded && kprev < ucols ? kprev : ucols) + 4;
  if (p > n - 1) p = n - 1;
  const int pa = n + 1;
  // LDS: A (n x pa) | V (n x p) | W (n x p) | G (p x p) | eig of H | weights (floats) | scores, sel
  double *A = lds;
  double *V = A + n * pa;
  double *W = V + n * p;
  double *G = W + n * p;
  double *gd = G + p * p;
  double *Hb = gd + p + 1;
  float *wts = reinterpret_cast<float *>(Hb + eig_lds_doubles(p));
  float *score = wts + kNParams + 1;
  int *sel = reinterpret_cast<int *>(score + n + 1);
  int *flag = sel + n + 1;
  double *red = reinterpret_cast<double *>(flag + 4 + 2);
  const int need = int((reinterpret_cast<char *>(red + 8) - reinterpret_cast<char *>(lds)) / 8);
  if (n < 16 || p < 2 || 4 * p > 3 * n || need > kLdsDoubles) {   // no saving over the full solve
    if (tid == 0) sc->rej[0] += 1;
    return false;
  }
  long long tl = wall_clock64();
  auto lap = [&](int slot) {
    if (tid == 0) { const long long t = wall_clock64(); sc->lticks[slot] += t - tl; tl = t; }
  };
  const double *L = ws + op.a;
  for (int e = tid; e < n * n; e += kThreads) {
    const int i = e / n, j = e % n;
    A[i * pa + j] = 0.5 * (L[int64_t(i) * ld + j] + L[int64_t(j) * ld + i]);
  }
  for (int e = tid; e < kNParams; e += kThreads) wts[e] = kp.model[e];
  const RowStats st = row_stats(L, ld, n, red);
  for (int i = tid; i < n; i += kThreads) {
    float f[kF];
    row_features(L, ld, n, i, rest, bonded, st, f);
    const float sc_i = mlp_score(wts, f);
    score[i] = sc_i == sc_i ? sc_i : -1.0f;              // a NaN score ranks last
  }
  __syncthreads();
  for (int i = tid; i < n; i += kThreads) {              // the p best-scored rows
    const float si = score[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) rank += (score[j] > si) || (score[j] == si && j < i);
    if (rank < p) sel[rank] = i;
  }
  __syncthreads();
  for (int e = tid; e < n * p; e += kThreads) V[e] = A[(e / p) * pa + sel[e % p]];
  __syncthreads();
  const int alive0 = orth_drop(V, n, p, gd, red);
  lap(0);
  if (alive0 == 0) {
    if (tid == 0) sc->rej[1] += 1;
    return false;
  }
  double part = 0.0;
  for (int i = tid; i < n; i += kThreads) part += A[i * pa + i];
  const double trL = block_sum(part, red);
  const double fro2L = st.fro2;
  double *hv2 = ws + op.b + int64_t(n) * n + n;          // reflectors of the p x p solve
  const int kmax = ucols < n ? ucols : n;
  int why = 2;
  for (int it = 0; it < 3; ++it) {
    sym_times(A, pa, V, n, p, W);                        // W = L V
    EigWs E = eig_ws(Hb, p, hv2);
    for (int e = tid; e < p * p; e += kThreads) {        // H = V^T W (symmetrised)
      const int a = e / p, b = e % p;
      double h1 = 0.0, h2 = 0.0;
      for (int i = 0; i < n; ++i) { h1 += V[i * p + a] * W[i * p + b]; h2 += V[i * p + b] * W[i * p + a]; }
      E.A[a * E.pa + b] = 0.5 * (h1 + h2);
    }
    __syncthreads();
    part = 0.0;
    double pw = 0.0, ph = 0.0;
    for (int a = tid; a < p; a += kThreads) part += E.A[a * E.pa + a];
    for (int e = tid; e < n * p; e += kThreads) pw += W[e] * W[e];
    for (int e = tid; e < p * p; e += kThreads) { const double h = E.A[(e / p) * E.pa + e % p]; ph += h * h; }
    const double trH = block_sum(part, red);
    const double fro2W = block_sum(pw, red);
    const double fro2H = block_sum(ph, red);
    lap(1);
    tri_ql(E, sc, false);
    order_desc(E);
    if (tid == 0) flag[2] = keep_rank(E.wsrt, p, n, ucols, kp);
    __syncthreads();
    lap(2);
    const int k = flag[2];
    const double th1 = E.wsrt[0];
    const double tail = fmax(trL - trH, 0.0);
    const double fro = sqrt(fmax(fro2L - 2.0 * fro2W + fro2H, 0.0) + kFroSlack * fro2L);
    const double bnd = fmin(tail, fro);
    bool cut_ok = k >= 1 && th1 > 0.0;
    if (cut_ok) {
      const double thk = E.wsrt[k - 1];
      cut_ok = tail <= kp.floor * th1 || (k == kmax && bnd <= 0.5 * thk && bnd < thk - kp.tau_deg * thk);
    }
    if (cut_ok) {
      back_transform(E, k);                              // Y columns (p x k) in E.A
      // Ritz vectors x_j = V y_j (written to U) and residual norms |W y_j - theta_j x_j|
      for (int j = tid; j < k; j += kThreads) G[j] = 0.0;
      __syncthreads();
      double *U = ws + op.c;
      for (int e = tid; e < n * k; e += kThreads) {
        const int i = e / k, j = e % k;
        const double *y = E.A + E.isrt[j] * E.pa;
        double x = 0.0, wy = 0.0;
        for (int c = 0; c < p; ++c) { x += V[i * p + c] * y[c]; wy += W[i * p + c] * y[c]; }
        const double r = wy - E.wsrt[j] * x;
        atomicAdd(&G[j], r * r);
        U[int64_t(j) * ld + i] = x;
      }
      __syncthreads();
      double rmax = 0.0;                           // largest residual relative to its Ritz value
      for (int j = tid; j < k; j += kThreads) rmax = fmax(rmax, sqrt(G[j]) / E.wsrt[j]);
      rmax = block_max(rmax, red);
      lap(3);
      if (rmax <= kp.residual_tol) {
        if (tid == 0) {
          set_dyn(dyn, dcache, op.out_dyn, k);
          sc->n_learned += 1;
          sc->max_resid = fmax(sc->max_resid, rmax);
          sc->eig_flops += 9LL * p * p * p + 4LL * n * n * p * (it + 1);
        }
        __syncthreads();
        return true;
      }
      why = 3;
    } else {
      why = 2;
    }
    if (it == 2) break;
    __syncthreads();
    for (int e = tid; e < n * p; e += kThreads) V[e] = W[e];   // one more step: V <- orth(L V)
    __syncthreads();
    const int alive = orth_drop(V, n, p, gd, red);
    lap(0);
    if (alive == 0) { why = 1; break; }
  }
  if (tid == 0) sc->rej[why] += 1;
  __syncthreads();
  return false;
}

// Harvest (features, leverage) rows of a solved density matrix for training.
__device__ void harvest_rows(const Op &op, const double *ws, int n, int ld, int k, const KeepParams &kp,
                             double *red, int *slot) {
  const double *L = ws + op.a, *U = ws + op.c;
  const bool bonded = op.bm.nd > 0;
  const int rest = op.bm.rest;
  const RowStats st = row_stats(L, ld, n, red);
  if (threadIdx.x == 0) slot[0] = atomicAdd(kp.hcount, n);
  __syncthreads();
  const long long base = slot[0];
  for (int i = threadIdx.x; i < n; i += kThreads) {
    if (base + i >= kp.hcap) continue;
    float f[kF];
    row_features(L, ld, n, i, rest, bonded, st, f);
    double lev = 0.0;
    for (int j = 0; j < k; ++j) lev += U[int64_t(j) * ld + i] * U[int64_t(j) * ld + i];
    for (int a = 0; a < kF; ++a) kp.hx[(base + i) * kF + a] = f[a];
    kp.hy[base + i] = float(lev);
  }
  __syncthreads();
}

__device__ void eig_keep(const Op &op, double *ws, int32_t *dyn, int32_t *dcache, const KeepParams &kp, NetScalars *sc,
                         double *lds) {
  const int ld = int(op.count);            // static dimension = row stride of L and of U
  const int n = box_eff(op.bm);            // runtime dimension: the valid leading block
  const int ucols = op.K;
  const int tid = threadIdx.x;
  // a matrix too large for LDS (order above about 135) is solved in the op's global
  // scratch: reflectors first (n^2 + n doubles), then the matrix and Z (n (n + 1))
  const bool big = eig_lds_doubles(n) > kLdsDoubles;
  const bool warm = !(op.flags & F_NO_WARM) && !big;
  if (kp.model && warm && eig_learned(op, ws, dyn, dcache, kp, sc, lds, n, ld, ucols)) return;
  // the reflectors stay in LDS when they fit beside the work area (n up to about 90): the
  // reduction's writes and the back-transformation's reads then never wait on memory
  const bool hv_lds = !big && eig_lds_doubles(n) + n * n + n <= kLdsDoubles;
  EigWs E = big ? eig_ws(lds, n, ws + op.b, ws + op.b + (int64_t(n) * n + n))
                : eig_ws(lds, n, hv_lds ? lds + eig_lds_doubles(n) : ws + op.b);
  const double *L = ws + op.a;
  long long t0 = wall_clock64();
  for (int e = tid; e < n * n; e += kThreads) {
    const int i = e / n, j = e % n;
    E.A[i * E.pa + j] = 0.5 * (L[int64_t(i) * ld + j] + L[int64_t(j) * ld + i]);
  }
  __syncthreads();
  // divide and conquer where its work area fits (all in LDS up to order 64; up to 128 with
  // the second eigenvector buffer and the merge matrices in the op's scratch after the
  // reflectors), else QL
  DcBufs dcb{};
  bool dc = false;
  if (!big && !kp.tridiag_ql) {
    double *after = lds + eig_lds_doubles(n) + (hv_lds ? n * n + n : 0);
    if (n <= kDcLdsMax && after + dc_lds_doubles(n) <= lds + kLdsDoubles) {
      dcb = DcBufs{after + 2 * n * (n + 1), after, after + n * (n + 1)};
      dc = true;
    } else if (n <= kDcMax && after + dc_vec_doubles(n) <= lds + kLdsDoubles) {
      double *g0 = ws + op.b + (hv_lds ? 0 : int64_t(n) * n + n);
      dcb = DcBufs{after, g0, g0 + int64_t(n) * (n + 1)};
      dc = true;
    }
  }
  tri_ql(E, sc, true, dc, dcb);
  t0 = wall_clock64();
  order_desc(E);
  if (tid == 0) {
    int k = keep_rank(E.wsrt, n, n, ucols, kp);
    if (k == 0) {
      k = ucols < n ? ucols : n;
      sc->n_fallback += 1;
    }
    E.flag[1] = k;
    set_dyn(dyn, dcache, op.out_dyn, k);
    sc->eig_flops += 9LL * n * n * n;
  }
  __syncthreads();
  const int k = E.flag[1];
  if (k <= kThreads / 4) back_transform_quads(E, k);
  else back_transform(E, k);
  double *U = ws + op.c;                  // U[j][i], j < k kept vectors, i < n components
  for (int e = tid; e < n * k; e += kThreads) {
    const int j = e / n, i = e % n;
    U[int64_t(j) * ld + i] = E.A[E.isrt[j] * E.pa + i];
  }
  __syncthreads();
  if (kp.hx && warm) harvest_rows(op, ws, n, ld, k, kp, E.red, E.flag + 2);
  if (tid == 0) sc->ticks[7] += wall_clock64() - t0;
}

// ---------------------------------------------------------------- QR of the QR-SVD branch
//
// C (m x c valid, read through the op's row and column maps) = Q R by Householder
// reflectors, one workgroup. C sits in LDS (odd pitch); quad t of the workgroup (4 lanes of
// one wave) owns column t (c <= 64). Column j: the quads of the later columns apply
// reflector j, and quad j+1, as soon as its own column is updated, forms reflector j+1 of
// rows j+1..m-1 (beta = 0 for a zero column); one barrier per column. Q's kk = min(m, c)
// columns are then formed as H_0 ... H_t e_t by quad t with no barrier (the reflectors are
// read only). Sums over a column run 4 rows per lane at a time into 4 partial sums, so the
// loads of a chunk are in flight together. Q is written [q][rows], R [q][cols] (zero below
// the diagonal), and kk to the op's slot.
// sum over rows i = i0, i0 + 4, ... < m of x[i * px] y[i * py], 4 rows at a time into 4
// partial sums
__device__ __forceinline__ double quad_col_dot(const double *x, int px, const double *y, int py, int i0, int m) {
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  int i = i0;
  for (; i + 28 < m; i += 32) {                     // 8 rows: 16 loads in flight
    double xv[8], yv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) { xv[u] = x[(i + 4 * u) * px]; yv[u] = y[(i + 4 * u) * py]; }
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u & 3] = fma(xv[u], yv[u], a[u & 3]);
  }
  for (; i + 12 < m; i += 16) {
    double xv[4], yv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) { xv[u] = x[(i + 4 * u) * px]; yv[u] = y[(i + 4 * u) * py]; }
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = fma(xv[u], yv[u], a[u]);
  }
  for (; i < m; i += 4) a[0] = fma(x[i * px], y[i * py], a[0]);
  return (a[0] + a[1]) + (a[2] + a[3]);
}

// Reflector of column j of X (rows j..m-1), by the 4 lanes of one quad: H_j = I - beta v v^T
// with v = (x_j - alpha, x_j+1, ...) maps the column to alpha e_j.
__device__ __forceinline__ void qr_reflector(const double *X, int pitch, int m, int j, int sub, double *vdiag,
                                             double *bet, double *rdiag) {
  const double *col = X + j;
  const double tail = quad_sum(quad_col_dot(col, pitch, col, pitch, j + 1 + sub, m));
  const double x0 = X[j * pitch + j], nrm2 = fma(x0, x0, tail);
  if (sub == 0) {
    if (tail == 0.0) {                               // nothing below the diagonal: H_j = I
      bet[j] = 0.0;
      vdiag[j] = 0.0;
      rdiag[j] = x0;
    } else {
      const double alpha = -copysign(sqrt(nrm2), x0);
      bet[j] = 1.0 / (nrm2 - x0 * alpha);            // 2 / (v^T v)
      vdiag[j] = x0 - alpha;
      rdiag[j] = alpha;
    }
  }
}

constexpr int kQrNb = 8;                            // reflectors per compact-WY block of Q
static_assert(kQrMaxRows * (kQrMaxCols | 1) + kQrMaxCols * (kQrMaxRows | 1) + 3 * kQrMaxCols +
                  (kQrMaxRows + kQrMaxCols) * 3 / 2 + 2 * kQrMaxCols * kQrNb <= kLdsDoubles,
              "the QR of the largest matrix fits LDS");
static_assert(kQrMaxCols % kQrNb == 0 && (kQrMaxCols / kQrNb) * kQrNb <= kThreads, "one lane per row of every T");
__device__ void qr_wg(const Op &op, double *ws, int32_t *dyn, int32_t *dcache, const int32_t *__restrict__ tab, NetScalars *sc,
                      double *lds) {
  const int m = box_eff(op.bm), c = box_eff(op.bnb), kk = m < c ? m : c;
  const int tid = threadIdx.x, sub = tid & 3, t = tid >> 2;
  // odd pitches: the quads of a wave read one row of X, or one row index of their columns
  // of Q, at addresses that spread over the LDS banks (a pitch of m = 128 doubles would put
  // every quad of the wave on the same banks)
  const int pitch = c | 1, mq = m | 1;
  double *X = lds;                                   // m x pitch
  double *Qb = X + m * pitch;                        // kk x mq: column t of Q at Qb[t*mq + i]
  double *vdiag = Qb + kk * mq, *bet = vdiag + kQrMaxCols, *rdiag = bet + kQrMaxCols;
  // offsets resolved once: C's row and column offsets, and where each valid row of Q and
  // column of R is stored (the gathers then need one load per element)
  int64_t *roff = reinterpret_cast<int64_t *>(rdiag + kQrMaxCols), *coff = roff + kQrMaxRows;
  int32_t *qpos = reinterpret_cast<int32_t *>(coff + kQrMaxCols), *rpos = qpos + kQrMaxRows;
  for (int i = tid; i < m; i += kThreads) {
    const int32_t s = box_conv(op.bm, i);
    roff[i] = map_off(tab, op.am, s);
    qpos[i] = s;
  }
  for (int j = tid; j < c; j += kThreads) {
    const int32_t s = box_conv(op.bnb, j);
    coff[j] = map_off(tab, op.bn, s);
    rpos[j] = s;
  }
  __syncthreads();
  const double *Cg = ws + op.a;
  for (int e = tid; e < m * c; e += kThreads) {
    const int i = e / c, j = e % c;
    X[i * pitch + j] = Cg[roff[i] + coff[j]];
  }
  __syncthreads();
  if (t == 0 && kk > 0) qr_reflector(X, pitch, m, 0, sub, vdiag, bet, rdiag);
  __syncthreads();
  for (int j = 0; j < kk; ++j) {
    const double bj = bet[j];
    if (t > j && t < c && bj != 0.0) {               // apply H_j to column t
      const double vj = vdiag[j];
      const double a = quad_sum((sub == 0 ? vj * X[j * pitch + t] : 0.0) +
                                quad_col_dot(X + j, pitch, X + t, pitch, j + 1 + sub, m));
      const double w = bj * a;
      if (sub == 0) X[j * pitch + t] -= w * vj;
      int i = j + 1 + sub;                           // loads of 8 rows issued before their stores
      for (; i + 28 < m; i += 32) {
        double vb[8], xb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) { vb[u] = X[(i + 4 * u) * pitch + j]; xb[u] = X[(i + 4 * u) * pitch + t]; }
#pragma unroll
        for (int u = 0; u < 8; ++u) X[(i + 4 * u) * pitch + t] = fma(-w, vb[u], xb[u]);
      }
      for (; i < m; i += 4) X[i * pitch + t] = fma(-w, X[i * pitch + j], X[i * pitch + t]);
    }
    if (t == j + 1 && j + 1 < kk) {                  // column j+1 is final: its reflector
      __threadfence_block();                         // the quad's stores above, before its loads
      qr_reflector(X, pitch, m, j + 1, sub, vdiag, bet, rdiag);
    }
    __syncthreads();
  }
  // Q's columns from blocks of kQrNb reflectors in compact WY form: H_j0 ... H_j0+nb-1 =
  // I - V T V^T with T upper triangular, T_pp = beta_p and T_lp = -beta_p sum_q T_lq G_qp
  // (G = V^T V of the block). Quads take the blocks' Gram entries, one lane per row of a T
  // builds it; then quad t forms Q e_t = H_0 ... H_t e_t by the blocks that touch it, last
  // block first, with no barrier: p = V^T q, p <- T p, q -= V p.
  const int nblk = (kk + kQrNb - 1) / kQrNb;
  double *Gb = reinterpret_cast<double *>(rpos + kQrMaxCols), *Tb = Gb + kQrMaxCols * kQrNb;
  constexpr int kPairs = kQrNb * (kQrNb - 1) / 2;
  for (int task = t; task < nblk * kPairs; task += kThreads / 4) {
    const int blk = task / kPairs;
    int pr = 0, rr = task % kPairs;                  // pair (pr, qr), pr < qr, of the block
    while (rr >= kQrNb - 1 - pr) { rr -= kQrNb - 1 - pr; ++pr; }
    const int qr = pr + 1 + rr, jp = blk * kQrNb + pr, jq = blk * kQrNb + qr;
    double g = 0.0;
    if (jq < kk)                                     // rows >= jq (v_jq is zero above its diagonal)
      g = quad_sum((sub == 0 ? X[jq * pitch + jp] * vdiag[jq] : 0.0) +
                   quad_col_dot(X + jp, pitch, X + jq, pitch, jq + 1 + sub, m));
    if (sub == 0) Gb[(blk * kQrNb + pr) * kQrNb + qr] = g;
  }
  __syncthreads();
  if (tid < nblk * kQrNb) {
    const int blk = tid / kQrNb, l = tid % kQrNb, j0 = blk * kQrNb;
    double trow[kQrNb];
#pragma unroll
    for (int p = 0; p < kQrNb; ++p) {
      double v = 0.0;
      if (j0 + p < kk) {
        const double bp = bet[j0 + p];
        if (p == l) {
          v = bp;
        } else if (l < p) {
          double s = 0.0;
#pragma unroll
          for (int q = 0; q < p; ++q)
            if (q >= l) s = fma(trow[q], Gb[(j0 + q) * kQrNb + p], s);
          v = -bp * s;
        }
      }
      trow[p] = v;
    }
#pragma unroll
    for (int p = 0; p < kQrNb; ++p) Tb[(j0 + l) * kQrNb + p] = trow[p];
  }
  __syncthreads();
  if (t < kk) {
    double *qc = Qb + t * mq;
    for (int i = sub; i < m; i += 4) qc[i] = i == t ? 1.0 : 0.0;
    for (int blk = t / kQrNb; blk >= 0; --blk) {
      const int j0 = blk * kQrNb, nb = kk - j0 < kQrNb ? kk - j0 : kQrNb;
      // q's rows above j0 are still zero; rows j0 .. j0+7 meet the triangle of V (masked),
      // the rows below read V's row straight from X (all of it in a full block)
      double pv[kQrNb], w[kQrNb];
#pragma unroll
      for (int p = 0; p < kQrNb; ++p) pv[p] = 0.0;
      const int tri = j0 + kQrNb < m ? j0 + kQrNb : m;
      for (int i = j0 + sub; i < tri; i += 4) {
        const double qi = qc[i];
#pragma unroll
        for (int p = 0; p < kQrNb; ++p) {
          const double vip = p < nb && i >= j0 + p ? (i == j0 + p ? vdiag[j0 + p] : X[i * pitch + j0 + p]) : 0.0;
          pv[p] = fma(vip, qi, pv[p]);
        }
      }
      if (nb == kQrNb) {
        int i = tri + ((j0 + sub - tri) & 3);
        for (; i + 4 < m; i += 8) {                  // two rows: their loads in flight together
          const double q0 = qc[i], q1 = qc[i + 4];
          const double *x0 = X + i * pitch + j0, *x1 = x0 + 4 * pitch;
          double r0[kQrNb], r1[kQrNb];
#pragma unroll
          for (int p = 0; p < kQrNb; ++p) { r0[p] = x0[p]; r1[p] = x1[p]; }
#pragma unroll
          for (int p = 0; p < kQrNb; ++p) pv[p] = fma(r1[p], q1, fma(r0[p], q0, pv[p]));
        }
        if (i < m) {
          const double qi = qc[i];
          const double *xr = X + i * pitch + j0;
#pragma unroll
          for (int p = 0; p < kQrNb; ++p) pv[p] = fma(xr[p], qi, pv[p]);
        }
      } else {
        for (int i = tri + ((j0 + sub - tri) & 3); i < m; i += 4) {
          const double qi = qc[i];
          const double *xr = X + i * pitch + j0;
#pragma unroll
          for (int p = 0; p < kQrNb; ++p) pv[p] = fma(p < nb ? xr[p] : 0.0, qi, pv[p]);
        }
      }
#pragma unroll
      for (int p = 0; p < kQrNb; ++p) pv[p] = quad_sum(pv[p]);
#pragma unroll
      for (int l = 0; l < kQrNb; ++l) {
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < kQrNb; ++p)
          if (p >= l) s = fma(Tb[(j0 + l) * kQrNb + p], pv[p], s);
        w[l] = s;
      }
      for (int i = j0 + sub; i < tri; i += 4) {
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < kQrNb; ++p) {
          const double vip = p < nb && i >= j0 + p ? (i == j0 + p ? vdiag[j0 + p] : X[i * pitch + j0 + p]) : 0.0;
          s = fma(vip, w[p], s);
        }
        qc[i] -= s;
      }
      int i = tri + ((j0 + sub - tri) & 3);        // w[p] = 0 for p >= nb
      for (; i + 4 < m; i += 8) {                    // two rows: their loads in flight together
        const double *x0 = X + i * pitch + j0, *x1 = x0 + 4 * pitch;
        double r0[kQrNb], r1[kQrNb];
#pragma unroll
        for (int p = 0; p < kQrNb; ++p) { r0[p] = p < nb ? x0[p] : 0.0; r1[p] = p < nb ? x1[p] : 0.0; }
        const double q0 = qc[i], q1 = qc[i + 4];
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int p = 0; p < kQrNb; ++p) { s0 = fma(r0[p], w[p], s0); s1 = fma(r1[p], w[p], s1); }
        qc[i] = q0 - s0;
        qc[i + 4] = q1 - s1;
      }
      if (i < m) {
        const double *xr = X + i * pitch + j0;
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < kQrNb; ++p) s = fma(p < nb ? xr[p] : 0.0, w[p], s);
        qc[i] -= s;
      }
    }
  }
  __syncthreads();
  double *Q = ws + op.c, *R = ws + op.b;
  const int64_t ldq = op.count, ldr = op.bn.n;
  for (int e = tid; e < kk * m; e += kThreads) {
    const int q = e / m, i = e % m;
    Q[q * ldq + qpos[i]] = Qb[q * mq + i];
  }
  for (int e = tid; e < kk * c; e += kThreads) {
    const int q = e / c, j = e % c;
    R[q * ldr + rpos[j]] = j > q ? X[q * pitch + j] : (j == q ? rdiag[q] : 0.0);
  }
  if (tid == 0) {
    set_dyn(dyn, dcache, op.out_dyn, kk);
    sc->eig_flops += 4LL * m * c * kk;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- interpreter

// Stage op i of a network in LDS with every Box's slot ids replaced by the runtime
// extents they hold (the whole workgroup takes part).
constexpr int kOpWords = int(sizeof(Op) / 4);
static_assert(kOpWords <= kThreads, "Op must be staged by one pass of the workgroup");

// word tid of op i of the network (threads below kOpWords)
__device__ __forceinline__ int32_t op_word(const NetDev &nd, int64_t i) {
  return threadIdx.x < kOpWords ? reinterpret_cast<const int32_t *>(nd.ops + i)[threadIdx.x] : 0;
}

// Stage an op from its words (one per thread) into LDS, then replace its Box slot ids
// by the runtime extents those slots hold.
__device__ void stage_op_words(const NetDev &nd, int32_t w, Op &s_op, const int32_t *dcache = nullptr) {
  const int tid = threadIdx.x;
  if (tid < kOpWords) reinterpret_cast<int32_t *>(&s_op)[tid] = w;
  __syncthreads();
  if (tid < 3 * kMaxDyn) {
    Box *bx = tid < kMaxDyn ? &s_op.bm : (tid < 2 * kMaxDyn ? &s_op.bnb : &s_op.bk_);
    const int d = tid % kMaxDyn;
    if (d < bx->nd) {
      const int32_t id = bx->id[d], e = id & (kDynCache - 1);
      bx->id[d] = dcache && dcache[e] == id ? dcache[kDynCache + e] : nd.dyn[id];
    }
  }
  __syncthreads();
}

__device__ void stage_op(const NetDev &nd, int64_t i, Op &s_op) { stage_op_words(nd, op_word(nd, i), s_op); }

// One workgroup walks ops [first, last) of its network (last < 0: to the end).
__global__ __launch_bounds__(kThreads) void interp_kernel(const NetDev *__restrict__ nets, KeepParams kp,
                                                          int64_t first, int64_t last) {
  __shared__ double lds[kLdsDoubles];
  __shared__ Op s_op;                 // the current op, Box slot ids replaced by extents
  __shared__ NetScalars s_sc;         // the network's scalars while the workgroup runs
  __shared__ int32_t s_dyc[2 * kDynCache];   // recent kept ranks: slot ids, then values
  constexpr int kScWords = int(sizeof(NetScalars) / 8);
  static_assert(kScWords <= kThreads, "NetScalars is copied by one pass of the workgroup");
  NetDev nd = nets[blockIdx.x];
  NetScalars *const g_sc = nd.sc;
  const int tid = threadIdx.x;
  // counters and sums are updated by one thread after most ops; kept in LDS, no update
  // waits on a memory round trip before the next barrier
  if (tid < kScWords) reinterpret_cast<long long *>(&s_sc)[tid] = reinterpret_cast<const long long *>(g_sc)[tid];
  for (int e = tid; e < kDynCache; e += kThreads) s_dyc[e] = -1;   // no slot cached yet
  __syncthreads();
  nd.sc = &s_sc;
  if (first < 0) {                    // a part of a chunked batch: the descriptor's range
    first = nd.op_begin;
    last = nd.op_end;
  }
  const int64_t end = last < 0 ? nd.n_ops : last;
  // the next op's words are loaded while the current op runs: the op arrays are read once
  // per launch, so each descriptor would otherwise cost a full memory round trip
  int32_t w = first < end ? op_word(nd, first) : 0;
  for (int64_t i = first; i < end; ++i) {
    stage_op_words(nd, w, s_op, s_dyc);
    if (i + 1 < end) w = op_word(nd, i + 1);
    const Op &op = s_op;
    const int kind = op.kind;
    const long long t0 = wall_clock64();
    switch (kind) {
      case OP_GEMM: {
        const double *A = ((op.flags & F_A_CONST) ? nd.cst : nd.ws) + op.a;
        const double *B = ((op.flags & F_B_CONST) ? nd.cst : nd.ws) + op.b;
        if (!gemm_op(op, A, B, nd.ws + op.c, nd.tab, lds, nd.sc, op_split(kp, op.flags), kp.gemm_cfg))
          gemm_tiles_k<kKCache>(op, A, B, nd.ws + op.c, nd.tab, lds, 0, 1, nd.sc);
        break;
      }
      case OP_EIG:
        eig_keep(op, nd.ws, nd.dyn, s_dyc, kp, nd.sc, lds);
        break;
      case OP_RESCALE:
        rescale_wg(op, nd.ws + op.c, nd.sc, lds);
        break;
      case OP_SCALAR:
        scalar_wg(nd.ws + op.a, nd.sc);
        break;
      case OP_IDENT:
        ident_wg(nd.ws + op.c, op.count);
        break;
      case OP_QR:
        qr_wg(op, nd.ws, nd.dyn, s_dyc, nd.tab, nd.sc, lds);
        break;
      default:
        break;
    }
    __syncthreads();
    if (tid == 0) {
      if (kind == OP_QR) nd.sc->qr_ticks += wall_clock64() - t0;
      else nd.sc->ticks[kind & 7] += wall_clock64() - t0;
    }
  }
  __syncthreads();
  if (tid < kScWords) reinterpret_cast<long long *>(g_sc)[tid] = reinterpret_cast<const long long *>(&s_sc)[tid];
}

// ---------------------------------------------------------------- grid-wide ops
//
// An op too large for one workgroup (a 3D environment holds up to 10^8 elements) runs
// over the whole chip: every workgroup stages the op, then takes output tiles or
// elements in a stride of the grid.

constexpr int kGridLds = 2 * kTK * kPitch + kKCache;   // gemm_tiles_k<kKCache>: two k-slices and both k caches
constexpr int kGridPipedTiles = piped_stage_doubles(32, 128, 16);   // largest chip-wide piped configuration
constexpr int kGridLdsAll = kGridLds > kGridPipedTiles + kGridOffsetDoubles ? kGridLds : kGridPipedTiles + kGridOffsetDoubles;

// Split-precision chip-wide GEMM in two passes.
// split_operands_kernel: every (row of A, 16-deep k chunk) and every (column of B, chunk)
// becomes one block of three planes of 16 parts (h, m, l as 16-bit words, 96 bytes) and
// the inverse of its power-of-two scale (the block's max |x| into [1/2, 1)). Blocks are
// chunk-major: A's (ch, row) at ch*M + row, then B's (ch, col) at M*nch + ch*N + col; the
// FP64 inverse scales follow all blocks in the same order. Each value is split once.
// gemm_presplit_kernel: 64x64 output tiles in a grid stride, 4 waves of 32x32; every lane
// reads its MFMA operands straight from the planes (no LDS, no barrier), one chunk ahead,
// sums the chunk's six part products in FP32 and adds that sum times its row's and
// column's inverse scales to an FP64 accumulator.
constexpr int kSplitBlockWords = 48;                             // 3 planes x 16 parts
constexpr int kSplitKCache = 2048;                               // k offsets cached in LDS when K <= this

template <int SPLIT>
__global__ __launch_bounds__(kThreads) void split_operands_kernel(const NetDev *__restrict__ ndp, int64_t i,
                                                                  unsigned short *__restrict__ planes) {
  __shared__ int32_t kofs[2 * kSplitKCache];
  __shared__ Op s_op;
  const NetDev nd = *ndp;
  stage_op(nd, i, s_op);
  const Op &op = s_op;
  const double *A = ((op.flags & F_A_CONST) ? nd.cst : nd.ws) + op.a;
  const double *B = ((op.flags & F_B_CONST) ? nd.cst : nd.ws) + op.b;
  const int32_t *tab = nd.tab;
  const int M = box_eff(op.bm), N = box_eff(op.bnb), K = box_eff(op.bk_);
  const int nch = (K + 15) / 16;
  const bool kcached = K <= kSplitKCache;
  if (kcached) {
    for (int k = threadIdx.x; k < K; k += kThreads) {
      const int ks = box_conv(op.bk_, k);
      kofs[k] = tab[op.ak + ks];
      kofs[kSplitKCache + k] = tab[op.bk + ks];
    }
  }
  __syncthreads();
  const int64_t nA = int64_t(M) * nch, total = int64_t(M + N) * nch;
  double *iscale = reinterpret_cast<double *>(planes + total * kSplitBlockWords);
  for (int64_t t = int64_t(blockIdx.x) * kThreads + threadIdx.x; t < total; t += int64_t(gridDim.x) * kThreads) {
    const bool isA = t < nA;
    const int64_t u = isA ? t : t - nA;
    const int n = isA ? M : N;
    const int ch = int(u / n), r = int(u - int64_t(ch) * n);
    const double *X = isA ? A : B;
    const int64_t off = isA ? map_off(tab, op.am, box_conv(op.bm, r)) : map_off(tab, op.bn, box_conv(op.bnb, r));
    const int32_t *kc = kofs + (isA ? 0 : kSplitKCache);
    const int32_t kt = isA ? op.ak : op.bk;
    double x[16];
    double mx = 0.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int k = 16 * ch + j;
      x[j] = k < K ? X[off + (kcached ? kc[k] : tab[kt + box_conv(op.bk_, k)])] : 0.0;
      mx = fmax(mx, fabs(x[j]));
    }
    int e;
    frexp(mx, &e);                                  // 0 for an all-zero block
    unsigned int w[24];                             // planes h, m, l: two parts per word
#pragma unroll
    for (int j = 0; j < 16; j += 2) {
      unsigned short h0, m0, l0, h1, m1, l1;
      split3<SPLIT>(ldexp(x[j], -e), h0, m0, l0);
      split3<SPLIT>(ldexp(x[j + 1], -e), h1, m1, l1);
      w[j / 2] = h0 | (unsigned(h1) << 16);
      w[8 + j / 2] = m0 | (unsigned(m1) << 16);
      w[16 + j / 2] = l0 | (unsigned(l1) << 16);
    }
    uint4 *dst = reinterpret_cast<uint4 *>(planes + t * kSplitBlockWords);
#pragma unroll
    for (int v = 0; v < 6; ++v) dst[v] = make_uint4(w[4 * v], w[4 * v + 1], w[4 * v + 2], w[4 * v + 3]);
    iscale[t] = ldexp(1.0, e);
  }
}

// LDS doubles of one stage of presplit_tiles: the A and B blocks of a tile's chunk in
// 16-byte pieces (96 bytes per block), then one FP64 inverse scale per block
constexpr int presplit_stage_doubles(int MB, int NB) { return 13 * (MB + NB); }
constexpr int kPresplitLds = 2 * presplit_stage_doubles(16, 256);   // the largest configuration below

// MB x NB output tiles in a grid stride; 4 waves of TM x TN 16 x 16 MFMA tiles. Step s
// = (j-th tile of this block, chunk): its pieces are fetched into registers during the
// products of step s - 1 and written to the LDS stage of step s, one barrier per step.
template <int SPLIT, int MB, int NB, int TM, int TN>
__device__ __forceinline__ void presplit_tiles(const Op &op, const unsigned short *__restrict__ planes,
                                               double *__restrict__ C, double *lds, int M, int N, int K) {
  constexpr int WN = NB / (16 * TN);
  static_assert((MB / (16 * TM)) * WN == 4, "4 waves per block");
  constexpr int kPlanePieces = 6 * (MB + NB), kPieces = 7 * (MB + NB);
  constexpr int kStage = presplit_stage_doubles(MB, NB);
  constexpr int NQ = (kPieces + kThreads - 1) / kThreads;
  const int64_t NS = op.bn.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int nch = (K + 15) / 16;
  const int64_t nA = int64_t(M) * nch, total = int64_t(M + N) * nch;
  const unsigned short *Ap = planes, *Bp = planes + nA * kSplitBlockWords;
  const double *sA = reinterpret_cast<const double *>(planes + total * kSplitBlockWords), *sB = sA + nA;
  const int kq = 4 * (lane >> 4);
  const int tilesN = (N + NB - 1) / NB, ntiles = ((M + MB - 1) / MB) * tilesN;
  const int mine = int(blockIdx.x) < ntiles ? (ntiles - 1 - int(blockIdx.x)) / int(gridDim.x) + 1 : 0;
  const int steps = mine * nch;
  constexpr int NACC = SPLIT == 1 ? 1 : 3;
  constexpr int O1 = NACC > 1 ? 1 : 0, O2 = NACC > 1 ? 2 : 0;
  // piece p = tid + 256 q: a 16-byte sixth of an A block (p < 6 MB) or of a B block, or
  // an inverse scale (A's, then B's)
  uint4 pv[NQ];
  auto fetch = [&](int s) {
    const int j = s / nch, ch = s - j * nch;
    const int tile = int(blockIdx.x) + j * int(gridDim.x);
    const int m0 = (tile / tilesN) * MB, n0 = (tile % tilesN) * NB;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int p = tid + kThreads * q;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (p < 6 * MB) {
        const int blk = p / 6;
        if (m0 + blk < M)
          v = *reinterpret_cast<const uint4 *>(Ap + (int64_t(ch) * M + m0 + blk) * kSplitBlockWords + (p - 6 * blk) * 8);
      } else if (p < kPlanePieces) {
        const int pb = p - 6 * MB, blk = pb / 6;
        if (n0 + blk < N)
          v = *reinterpret_cast<const uint4 *>(Bp + (int64_t(ch) * N + n0 + blk) * kSplitBlockWords + (pb - 6 * blk) * 8);
      } else if (p < kPieces) {
        const int r = p - kPlanePieces;
        double d = 0.0;
        if (r < MB) {
          if (m0 + r < M) d = sA[int64_t(ch) * M + m0 + r];
        } else if (n0 + r - MB < N) {
          d = sB[int64_t(ch) * N + n0 + r - MB];
        }
        const unsigned long long u = (unsigned long long)__double_as_longlong(d);
        v.x = unsigned(u);
        v.y = unsigned(u >> 32);
      }
      pv[q] = v;
    }
  };
  auto stash = [&](double *stage) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int p = tid + kThreads * q;
      if (p < kPlanePieces) reinterpret_cast<uint4 *>(stage)[p] = pv[q];
      else if (p < kPieces)
        stage[2 * kPlanePieces + (p - kPlanePieces)] =
            __longlong_as_double((long long)(((unsigned long long)pv[q].y << 32) | pv[q].x));
    }
  };
  double acc64[TM][TN][4];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[a][b][r] = 0.0;
  if (steps > 0) fetch(0);
  for (int s = 0; s < steps; ++s) {
    const int j = s / nch, ch = s - j * nch;
    double *stage = lds + (s & 1) * kStage;
    stash(stage);
    __syncthreads();
    if (s + 1 < steps) fetch(s + 1);               // in flight during the products
    const unsigned short *a3 = reinterpret_cast<const unsigned short *>(stage), *b3 = a3 + MB * kSplitBlockWords;
    const double *ia = stage + 2 * kPlanePieces, *ib = ia + MB;
    unsigned long long av[TM][3], bv[TN][3];
    double rs[TM][4], cs[TN];
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      const int r = wm * 16 * TM + a * 16 + (lane & 15);
#pragma unroll
      for (int pl = 0; pl < 3; ++pl)
        av[a][pl] = *reinterpret_cast<const unsigned long long *>(a3 + r * kSplitBlockWords + 16 * pl + kq);
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4) rs[a][r4] = ia[wm * 16 * TM + a * 16 + kq + r4];
    }
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int c = wn * 16 * TN + b * 16 + (lane & 15);
#pragma unroll
      for (int pl = 0; pl < 3; ++pl)
        bv[b][pl] = *reinterpret_cast<const unsigned long long *>(b3 + c * kSplitBlockWords + 16 * pl + kq);
      cs[b] = ib[c];
    }
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        v4f acc[NACC];
#pragma unroll
        for (int o = 0; o < NACC; ++o) acc[o] = v4f{0.f, 0.f, 0.f, 0.f};
        acc[O2] = mfma16<SPLIT>(av[a][1], bv[b][1], acc[O2]);    // small terms first
        acc[O2] = mfma16<SPLIT>(av[a][2], bv[b][0], acc[O2]);
        acc[O2] = mfma16<SPLIT>(av[a][0], bv[b][2], acc[O2]);
        acc[O1] = mfma16<SPLIT>(av[a][1], bv[b][0], acc[O1]);
        acc[O1] = mfma16<SPLIT>(av[a][0], bv[b][1], acc[O1]);
        acc[0] = mfma16<SPLIT>(av[a][0], bv[b][0], acc[0]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double v = double(acc[0][r]);
          if (NACC > 1) v += double(acc[O1][r]) * 0x1p-11 + double(acc[O2][r]) * 0x1p-22;
          acc64[a][b][r] += v * (rs[a][r] * cs[b]);
        }
      }
    if (ch == nch - 1) {
      const int tile = int(blockIdx.x) + j * int(gridDim.x);
      const int m0 = (tile / tilesN) * MB + wm * 16 * TM, n0 = (tile % tilesN) * NB + wn * 16 * TN;
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = m0 + a * 16 + kq + r;   // D: lane l, reg r = row 4(l/16) + r
            const int col = n0 + b * 16 + (lane & 15);
            if (row < M && col < N) C[int64_t(box_conv(op.bm, row)) * NS + box_conv(op.bnb, col)] = acc64[a][b][r];
            acc64[a][b][r] = 0.0;
          }
    }
  }
}

// the output tile follows the op's runtime row count, as in the FP64 pipelined path
template <int SPLIT>
__global__ __launch_bounds__(kThreads, 2) void gemm_presplit_kernel(const NetDev *__restrict__ ndp, int64_t i,
                                                                    const unsigned short *__restrict__ planes) {
  __shared__ __attribute__((aligned(16))) double lds[kPresplitLds];
  __shared__ Op s_op;
  const NetDev nd = *ndp;
  stage_op(nd, i, s_op);
  const Op &op = s_op;
  const int M = box_eff(op.bm), N = box_eff(op.bnb), K = box_eff(op.bk_);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    nd.sc->flops += 2LL * M * N * K;
    nd.sc->split_flops += 2LL * M * N * K;
  }
  double *C = nd.ws + op.c;
  if (M <= 16) presplit_tiles<SPLIT, 16, 256, 1, 4>(op, planes, C, lds, M, N, K);
  else if (M <= 32) presplit_tiles<SPLIT, 32, 128, 2, 2>(op, planes, C, lds, M, N, K);
  else presplit_tiles<SPLIT, 64, 64, 2, 2>(op, planes, C, lds, M, N, K);
}

// FP64 chip-wide GEMM through the pipelined path: k and row offsets cached in LDS,
// each workgroup a contiguous range of output blocks. False if the caches do not fit.
__device__ __forceinline__ bool gemm_grid_piped(const Op &op, const double *__restrict__ A, const double *__restrict__ B,
                                double *__restrict__ C, const int32_t *__restrict__ tab, double *lds,
                                NetScalars *sc) {
  const int M = box_eff(op.bm), N = box_eff(op.bnb), K = box_eff(op.bk_);
  if (2 * (int64_t(M) + K) > 2 * int64_t(kGridLdsAll - kGridPipedTiles)) return false;
  const int64_t NS = op.bn.n;
  if (int64_t(op.am.n) * NS >= (int64_t(1) << 31)) return false;   // row offsets of C as int32
  int32_t *kA = reinterpret_cast<int32_t *>(lds + kGridPipedTiles);
  int32_t *kB = kA + K, *rA = kB + K, *rC = rA + M;
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && tid == 0) sc->flops += 2LL * M * N * K;
  for (int k = tid; k < K; k += kThreads) {
    const int ks = box_conv(op.bk_, k);
    kA[k] = tab[op.ak + ks];
    kB[k] = tab[op.bk + ks];
  }
  for (int m = tid; m < M; m += kThreads) {
    const int sm = box_conv(op.bm, m);
    rA[m] = int32_t(map_off(tab, op.am, sm));
    rC[m] = int32_t(sm * NS);
  }
  __syncthreads();
  auto range = [&](int nblk, int &b0, int &b1) {
    const int per = (nblk + int(gridDim.x) - 1) / int(gridDim.x);
    b0 = int(blockIdx.x) * per;
    b1 = b0 + per;
  };
  int b0, b1;
  if (M <= 16) {
    range(((N + 255) / 256), b0, b1);
    gemm_piped<16, 256, 8, 1, 4, true>(op, A, B, C, lds, M, N, K, kA, kB, rA, nullptr, rC, nullptr, tab, b0, b1);
  } else if (M <= 32) {
    range(((N + 127) / 128), b0, b1);
    gemm_piped<32, 128, 16, 2, 2, true>(op, A, B, C, lds, M, N, K, kA, kB, rA, nullptr, rC, nullptr, tab, b0, b1);
  } else {
    range(((M + 63) / 64) * ((N + 63) / 64), b0, b1);
    gemm_piped<64, 64, 16, 2, 2, true>(op, A, B, C, lds, M, N, K, kA, kB, rA, nullptr, rC, nullptr, tab, b0, b1);
  }
  return true;
}

// FP64 chip-wide GEMM whose row and k offsets fit LDS (checked on the host from the
// static shapes): a kernel of its own, so its register budget is the pipelined path's
// alone and two workgroups share a CU.
__global__ __launch_bounds__(kThreads, 2) void gemm_grid_piped_kernel(const NetDev *__restrict__ ndp, int64_t i) {
  __shared__ double lds[kGridLdsAll];
  __shared__ Op s_op;
  const NetDev nd = *ndp;
  stage_op(nd, i, s_op);
  const Op &op = s_op;
  const double *A = ((op.flags & F_A_CONST) ? nd.cst : nd.ws) + op.a;
  const double *B = ((op.flags & F_B_CONST) ? nd.cst : nd.ws) + op.b;
  gemm_grid_piped(op, A, B, nd.ws + op.c, nd.tab, lds, nd.sc);
}

// FP64 chip-wide contraction of at most 32 rows and at most KT-deep K over a long N (the
// 3D environments' products with a site tensor): about two flops per byte, so it is bound
// by streaming B (K x N) in and C (M x N) out, not by the matrix cores. A (M x KT) and the
// offsets are staged in LDS; each thread takes CPT columns at a time in a grid stride
// (consecutive threads, consecutive columns), loads their K values of B, and writes M
// outputs per column; every LDS read of A serves CPT columns.
template <int KT, int CPT>
__global__ __launch_bounds__(kThreads) void gemm_stream_kernel(const NetDev *__restrict__ ndp, int64_t i) {
  __shared__ double As[kStreamMaxM * KT];
  __shared__ int32_t kB[KT];
  __shared__ int64_t rC[kStreamMaxM];
  __shared__ Op s_op;
  const NetDev nd = *ndp;
  stage_op(nd, i, s_op);
  const Op &op = s_op;
  const int M = box_eff(op.bm), N = box_eff(op.bnb), K = box_eff(op.bk_);
  const int64_t NS = op.bn.n;
  const double *A = ((op.flags & F_A_CONST) ? nd.cst : nd.ws) + op.a;
  const double *B = ((op.flags & F_B_CONST) ? nd.cst : nd.ws) + op.b;
  double *C = nd.ws + op.c;
  const int32_t *tab = nd.tab;
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && tid == 0) nd.sc->flops += 2LL * M * N * K;
  for (int e = tid; e < kStreamMaxM * KT; e += kThreads) {
    const int m = e / KT, k = e % KT;
    As[e] = (m < M && k < K) ? A[map_off(tab, op.am, box_conv(op.bm, m)) + tab[op.ak + box_conv(op.bk_, k)]] : 0.0;
  }
  for (int k = tid; k < KT; k += kThreads) kB[k] = k < K ? tab[op.bk + box_conv(op.bk_, k)] : 0;
  for (int m = tid; m < kStreamMaxM; m += kThreads) rC[m] = m < M ? int64_t(box_conv(op.bm, m)) * NS : 0;
  __syncthreads();
  const int64_t T = int64_t(gridDim.x) * kThreads;
  for (int64_t n0 = int64_t(blockIdx.x) * kThreads + tid; n0 < N; n0 += T * CPT) {
    int32_t sn[CPT];
    double b[CPT][KT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int64_t n = n0 + c * T;
      sn[c] = n < N ? box_conv(op.bnb, int32_t(n)) : -1;
      const int64_t boff = sn[c] >= 0 ? map_off(tab, op.bn, sn[c]) : 0;
#pragma unroll
      for (int k = 0; k < KT; ++k) b[c][k] = (sn[c] >= 0 && k < K) ? B[boff + kB[k]] : 0.0;
    }
    for (int m = 0; m < M; ++m) {
      double acc[CPT];
#pragma unroll
      for (int c = 0; c < CPT; ++c) acc[c] = 0.0;
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        const double a = As[m * KT + k];
#pragma unroll
        for (int c = 0; c < CPT; ++c) acc[c] = fma(a, b[c][k], acc[c]);
      }
#pragma unroll
      for (int c = 0; c < CPT; ++c)
        if (sn[c] >= 0) C[rC[m] + sn[c]] = acc[c];
    }
  }
}

// FP64 chip-wide GEMM whose offsets do not fit the pipelined path: the tiled GEMM with
// k offsets cached up to K = kGridKCache (the 3D environments contract over K = 8192)
constexpr int kGridKCache = 8192;
constexpr int kGridTilesLds = 2 * kTK * kPitch + kGridKCache;
__global__ __launch_bounds__(kThreads) void gemm_grid_kernel(const NetDev *__restrict__ ndp, int64_t i, int kchunks,
                                                              double *kpart) {
  __shared__ double lds[kGridTilesLds > kGridLdsAll ? kGridTilesLds : kGridLdsAll];
  __shared__ Op s_op;
  const NetDev nd = *ndp;
  stage_op(nd, i, s_op);
  const Op &op = s_op;
  const double *A = ((op.flags & F_A_CONST) ? nd.cst : nd.ws) + op.a;
  const double *B = ((op.flags & F_B_CONST) ? nd.cst : nd.ws) + op.b;
  if (kchunks <= 1 && gemm_grid_piped(op, A, B, nd.ws + op.c, nd.tab, lds, nd.sc)) return;
  gemm_tiles_k<kGridKCache>(op, A, B, nd.ws + op.c, nd.tab, lds, blockIdx.x, gridDim.x, nd.sc, kchunks,
                            kchunks > 1 ? kpart : nullptr);
}

// Second pass of a split-K GEMM: C = the sum of the kchunks partial products, in order.
__global__ __launch_bounds__(kThreads) void gemm_kreduce_kernel(const NetDev *__restrict__ ndp, int64_t i, int kchunks,
                                                                const double *__restrict__ kpart) {
  __shared__ Op s_op;
  const NetDev nd = *ndp;
  stage_op(nd, i, s_op);
  const Op &op = s_op;
  const int M = box_eff(op.bm), N = box_eff(op.bnb);
  const int64_t NS = op.bn.n, MN = int64_t(M) * N;
  double *C = nd.ws + op.c;
  for (int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x; e < MN; e += int64_t(gridDim.x) * kThreads) {
    double s = 0.0;
    for (int p = 0; p < kchunks; ++p) s += kpart[p * MN + e];
    const int row = int(e / N), col = int(e - int64_t(row) * N);
    C[int64_t(box_conv(op.bm, row)) * NS + box_conv(op.bnb, col)] = s;
  }
}

// max |x| over this workgroup's share of the valid box -> partial[blockIdx.x]
__global__ __launch_bounds__(kThreads) void rescale_max_kernel(const NetDev *__restrict__ ndp, int64_t i,
                                                               double *partial) {
  __shared__ double red[8];
  __shared__ Op s_op;
  const NetDev nd = *ndp;
  stage_op(nd, i, s_op);
  const Op &op = s_op;
  const double *x = nd.ws + op.c;
  const int32_t Cn = box_eff(op.bnb);
  const int64_t total = int64_t(box_eff(op.bm)) * Cn, ncols = op.count;
  double m = 0.0;
  for (int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x; e < total; e += int64_t(gridDim.x) * kThreads) {
    const int32_t r = int32_t(e / Cn), c = int32_t(e - int64_t(r) * Cn);
    m = fmax(m, fabs(x[int64_t(box_conv(op.bm, r)) * ncols + box_conv(op.bnb, c)]));
  }
  m = block_max(m, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

// x *= 2^-e with e the frexp exponent of the max over all partials; the exponent is
// added to the log accumulator once (F_ACCUM), a zero max marks Z = 0.
__global__ __launch_bounds__(kThreads) void rescale_apply_kernel(const NetDev *__restrict__ ndp, int64_t i,
                                                                 const double *partial, int nparts) {
  __shared__ double red[8];
  __shared__ Op s_op;
  const NetDev nd = *ndp;
  stage_op(nd, i, s_op);
  const Op &op = s_op;
  double m = 0.0;
  for (int q = threadIdx.x; q < nparts; q += kThreads) m = fmax(m, partial[q]);
  m = block_max(m, red);
  const bool accum = (op.flags & F_ACCUM) != 0;
  if (!(m > 0.0) || !isfinite(m)) {
    if (m == 0.0 && accum && blockIdx.x == 0 && threadIdx.x == 0) nd.sc->zero = 1;
    return;
  }
  int ex;
  frexp(m, &ex);
  double *x = nd.ws + op.c;
  const int32_t Cn = box_eff(op.bnb);
  const int64_t total = int64_t(box_eff(op.bm)) * Cn, ncols = op.count;
  for (int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x; e < total; e += int64_t(gridDim.x) * kThreads) {
    const int32_t r = int32_t(e / Cn), c = int32_t(e - int64_t(r) * Cn);
    const int64_t o = int64_t(box_conv(op.bm, r)) * ncols + box_conv(op.bnb, c);
    x[o] = ldexp(x[o], -ex);
  }
  if (accum && blockIdx.x == 0 && threadIdx.x == 0) nd.sc->exp_sum += ex;
}

hipError_t launch_interp(const NetDev *nets_dev, int n_nets, const KeepParams &kp, hipStream_t stream) {
  hipLaunchKernelGGL(interp_kernel, dim3(n_nets), dim3(kThreads), 0, stream, nets_dev, kp, int64_t(0), int64_t(-1));
  return hipGetLastError();
}

hipError_t launch_interp_parts(const NetDev *nets_dev, int n_nets, const KeepParams &kp, hipStream_t stream) {
  hipLaunchKernelGGL(interp_kernel, dim3(n_nets), dim3(kThreads), 0, stream, nets_dev, kp, int64_t(-1), int64_t(-1));
  return hipGetLastError();
}

hipError_t launch_interp_range(const NetDev *nd_dev, int64_t first, int64_t last, const KeepParams &kp,
                               hipStream_t stream) {
  hipLaunchKernelGGL(interp_kernel, dim3(1), dim3(kThreads), 0, stream, nd_dev, kp, first, last);
  return hipGetLastError();
}

hipError_t launch_gemm_grid(const NetDev *nd_dev, int64_t i, int blocks, int split, bool piped,
                            unsigned short *planes, int split_blocks, int kchunks, double *kpart, int stream_k,
                            hipStream_t stream) {
  if (split == 1 || split == 2) {
    if (!planes || split_blocks < 1) return hipErrorInvalidValue;
    if (split == 1) {
      hipLaunchKernelGGL(split_operands_kernel<1>, dim3(split_blocks), dim3(kThreads), 0, stream, nd_dev, i, planes);
      hipLaunchKernelGGL(gemm_presplit_kernel<1>, dim3(blocks), dim3(kThreads), 0, stream, nd_dev, i,
                         (const unsigned short *)planes);
    } else {
      hipLaunchKernelGGL(split_operands_kernel<2>, dim3(split_blocks), dim3(kThreads), 0, stream, nd_dev, i, planes);
      hipLaunchKernelGGL(gemm_presplit_kernel<2>, dim3(blocks), dim3(kThreads), 0, stream, nd_dev, i,
                         (const unsigned short *)planes);
    }
  } else if (stream_k > 0) {
    switch (stream_k) {
      case 4: hipLaunchKernelGGL((gemm_stream_kernel<4, 8>), dim3(blocks), dim3(kThreads), 0, stream, nd_dev, i); break;
      case 8: hipLaunchKernelGGL((gemm_stream_kernel<8, 4>), dim3(blocks), dim3(kThreads), 0, stream, nd_dev, i); break;
      case 16: hipLaunchKernelGGL((gemm_stream_kernel<16, 2>), dim3(blocks), dim3(kThreads), 0, stream, nd_dev, i); break;
      case 32: hipLaunchKernelGGL((gemm_stream_kernel<32, 1>), dim3(blocks), dim3(kThreads), 0, stream, nd_dev, i); break;
      default: return hipErrorInvalidValue;
    }
  } else if (piped) {
    hipLaunchKernelGGL(gemm_grid_piped_kernel, dim3(blocks), dim3(kThreads), 0, stream, nd_dev, i);
  } else if (kchunks > 1) {
    if (!kpart) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gemm_grid_kernel, dim3(blocks), dim3(kThreads), 0, stream, nd_dev, i, kchunks, kpart);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gemm_kreduce_kernel, dim3(blocks), dim3(kThreads), 0, stream, nd_dev, i, kchunks,
                       (const double *)kpart);
  } else {
    hipLaunchKernelGGL(gemm_grid_kernel, dim3(blocks), dim3(kThreads), 0, stream, nd_dev, i, 1, (double *)nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_rescale_grid(const NetDev *nd_dev, int64_t i, int blocks, double *partial, hipStream_t stream) {
  hipLaunchKernelGGL(rescale_max_kernel, dim3(blocks), dim3(kThreads), 0, stream, nd_dev, i, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rescale_apply_kernel, dim3(blocks), dim3(kThreads), 0, stream, nd_dev, i,
                     (const double *)partial, blocks);
  return hipGetLastError();
}


// ---------------------------------------------------------------- allocation-free scratch
//
// Device memory of the allocation-free entry point: one array per device, held from the
// module's load to the end of the process. Host code must never pass `scratch` itself
// to a kernel or a copy (on the host the name is only a stand-in); it uses the device
// address hipGetSymbolAddress returns, looked up once per device with that device
// current and kept per device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(char **ptr) {
  *ptr = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<char *>(p);
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace tn
