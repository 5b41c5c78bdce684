// kernels.hip - CDNA4 (gfx950) device code of the density-matrix contraction.
//
// One workgroup of 256 threads (4 wave64s) executes one network's op list:
//   OP_GEMM     pairwise contraction as a 64x64-tiled FP64 GEMM on the matrix cores
//               (v_mfma_f64_16x16x4f64); operand gathers through index tables fold
//               every mode permutation into the tile loads.
//   OP_EIG      symmetric eigensolve of a density matrix (Householder tridiagonal
//               reduction, implicit QL, back-transformation of the kept vectors)
//               followed by the keep rule; writes the kept eigenvectors and rank.
// MPS bonds have a runtime extent (the kept rank of the eigensolve that made them):
// tensors keep their static layout and every op touches only the valid box.
//   OP_RESCALE  exact power-of-two normalisation with the exponent summed in int64.
//   OP_SCALAR   ln|z| and sign of a closing scalar.
//   OP_IDENT    identity matrices of the identity insertion.
#include <hip/hip_runtime.h>

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

// compact index in [0, box_eff) -> static index in the (cap..., rest) layout
__device__ __forceinline__ int32_t box_conv(const Box &b, int32_t i) {
  if (b.nd == 0) return i;
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

__device__ void gemm_tiles(const Op &op, const double *__restrict__ A, const double *__restrict__ B,
                           double *__restrict__ C, const int32_t *__restrict__ tab, double *lds,
                           int t_begin, int t_step, NetScalars *sc) {
  // runtime extents; the output keeps its static row length
  const int M = box_eff(op.bm), N = box_eff(op.bnb), K = box_eff(op.bk_);
  const int NS = op.bn.n;
  if (t_begin == 0 && threadIdx.x == 0) sc->flops += 2LL * M * N * K;
  const int tilesN = (N + kTile - 1) / kTile;
  const int ntiles = ((M + kTile - 1) / kTile) * tilesN;
  double *As = lds;                  // [kTK][kPitch], element (k, m)
  double *Bs = lds + kTK * kPitch;   // [kTK][kPitch], element (k, n)
  int32_t *kA = reinterpret_cast<int32_t *>(lds + 2 * kTK * kPitch);   // A's k offsets
  int32_t *kB = kA + kKCache;                                          // B's k offsets
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const bool akf = (op.flags & F_A_KFAST) != 0;
  const bool bnf = (op.flags & F_B_NFAST) != 0;
  const bool kcached = K <= kKCache;
  if (kcached) {
    for (int k = tid; k < K; k += kThreads) {
      const int ks = box_conv(op.bk_, k);
      kA[k] = tab[op.ak + ks];
      kB[k] = tab[op.bk + ks];
    }
    __syncthreads();
  }

  for (int tile = t_begin; tile < ntiles; tile += t_step) {
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
        if (av[q] && k < K) x = A[aoff[q] + (kcached ? kA[k] : tab[op.ak + box_conv(op.bk_, k)])];
        va[q] = x;
        const int kb = k0 + bk_[q];
        double y = 0.0;
        if (bv[q] && kb < K) y = B[boff[q] + (kcached ? kB[kb] : tab[op.bk + box_conv(op.bk_, kb)])];
        vb[q] = y;
      }
    };
    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    load(0);
    for (int k0 = 0; k0 < K; k0 += kTK) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        As[ak_[q] * kPitch + ai[q]] = va[q];
        Bs[bk_[q] * kPitch + bi[q]] = vb[q];
      }
      __syncthreads();
      if (k0 + kTK < K) load(k0 + kTK);   // next slice in flight during the MFMAs
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
          if (row < M && col < N)
            C[int64_t(box_conv(op.bm, row)) * NS + box_conv(op.bnb, col)] = acc[i][j][r];
        }
  }
}

// ---------------------------------------------------------------- lane access

// value of v in lane `src` (src wave-uniform), as a wave-uniform scalar
__device__ __forceinline__ double lane_read(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}
// `old` with lane `dst` replaced by the wave-uniform value x (a per-lane select)
__device__ __forceinline__ double lane_write(double x, int dst, double old) {
  return (int(threadIdx.x & 63) == dst) ? x : old;
}

// 1/sqrt(q) for q > 0: hardware estimate refined by two Newton steps (a few ulps;
// every Givens rotation of the QL sweep needs one, on its critical path)
__device__ __forceinline__ double rsqrt_nr(double q) {
  double y = __builtin_amdgcn_rsq(q);
  const double h = 0.5 * q;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
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

// Symmetric eigensolve of the density matrix and the keep rule.
//  1. Householder reduction to tridiagonal form T = Q^T A Q in LDS (256 threads);
//     the reflectors go to the op's workspace scratch for the back-transformation.
//  2. Implicit QL with shifts on T, accumulating the rotations into Z (T = Z W Z^T).
//     The scalar recurrence is sequential, so every wave runs it on its own copy of
//     (d, e) without barriers and each thread applies the rotations to its row of Z.
//  3. Eigenvalues sorted in descending order, the keep rule picks k, and only the k
//     kept columns of Z are transformed back with the reflectors: U = Q Z_kept.
__device__ void eig_keep(const Op &op, double *ws, int32_t *dyn, const KeepParams &kp, NetScalars *sc,
                         double *lds) {
  const int ld = int(op.count);            // static dimension = row stride of L and of U
  const int n = box_eff(op.bm);            // runtime dimension: the valid leading block
  const int ucols = op.K;
  const int tid = threadIdx.x, wave = tid >> 6;
  const int pa = n + 1;                    // odd LDS pitch of A: conflict-free row access
  double *A = lds;                         // n x pa during the reduction, then Z (column-major n x n)
  double *Z = lds;
  double *vv = lds + n * pa;               // Householder vector of the current step
  double *pp = vv + n;
  double *ww = pp + n;
  double *dd = ww + n;                     // diagonal of T
  double *ee = dd + n;                     // off-diagonal of T (ee[n-1] = 0)
  double *dW = ee + n;                     // per-wave copies of (d, e): 4 x 2n
  double *wsrt = dW + 8 * n;               // eigenvalues, descending
  int *isrt = reinterpret_cast<int *>(wsrt + n);
  int *flag = isrt + n + (n & 1);
  double *red = reinterpret_cast<double *>(flag + 4);
  double *hv = ws + op.b;                  // reflectors: v_j at hv[j*n + i], beta_j at hv[n*n + j]
  const double *L = ws + op.a;

  long long tph = wall_clock64();
  for (int e = tid; e < n * n; e += kThreads) {
    const int i = e / n, j = e % n;
    A[i * pa + j] = 0.5 * (L[int64_t(i) * ld + j] + L[int64_t(j) * ld + i]);
  }
  __syncthreads();

  // 1. tridiagonalisation
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;
    double part = 0.0;
    for (int i = tid; i < m; i += kThreads) {
      const double x = A[(j + 1 + i) * pa + j];
      part += x * x;
    }
    const double nrm2 = block_sum(part, red);
    const double x0 = A[(j + 1) * pa + j];
    if (nrm2 == 0.0) {                     // column already reduced
      if (tid == 0) { dd[j] = A[j * pa + j]; ee[j] = 0.0; hv[int64_t(n) * n + j] = 0.0; }
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
    for (int i = tid; i < m; i += kThreads) {            // p = beta * A_t v
      const double *row = A + (j + 1 + i) * pa + j + 1;
      double acc = 0.0;
      for (int k = 0; k < m; ++k) acc += row[k] * vv[k];
      pp[i] = beta * acc;
    }
    __syncthreads();
    part = 0.0;
    for (int i = tid; i < m; i += kThreads) part += vv[i] * pp[i];
    const double K = 0.5 * beta * block_sum(part, red);
    for (int i = tid; i < m; i += kThreads) ww[i] = pp[i] - K * vv[i];
    __syncthreads();
    for (int e = tid; e < m * m; e += kThreads) {        // A_t -= v w^T + w v^T
      const int a = e / m, b = e % m;
      A[(j + 1 + a) * pa + j + 1 + b] -= vv[a] * ww[b] + ww[a] * vv[b];
    }
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
  __syncthreads();

  if (tid == 0) { const long long t = wall_clock64(); sc->ticks[0] += t - tph; tph = t; }
  // 2. implicit QL on T; Z starts as the identity (A is no longer needed). Every wave
  // holds (d, e) in registers, lane i owning entries i and i + 64, and runs the
  // sequential recurrence with wave-uniform lane reads and writes.
  for (int e = tid; e < n * n; e += kThreads) Z[e] = (e / n == e % n) ? 1.0 : 0.0;
  const int lane = tid & 63;
  double dlo = lane < n ? dd[lane] : 0.0, dhi = lane + 64 < n ? dd[lane + 64] : 0.0;
  double elo = lane < n ? ee[lane] : 0.0, ehi = lane + 64 < n ? ee[lane + 64] : 0.0;
  __syncthreads();
  auto dget = [&](int i) { return i < 64 ? lane_read(dlo, i) : lane_read(dhi, i - 64); };
  auto eget = [&](int i) { return i < 64 ? lane_read(elo, i) : lane_read(ehi, i - 64); };
  auto dset = [&](int i, double v) { if (i < 64) dlo = lane_write(v, i, dlo); else dhi = lane_write(v, i - 64, dhi); };
  auto eset = [&](int i, double v) { if (i < 64) elo = lane_write(v, i, elo); else ehi = lane_write(v, i - 64, ehi); };
  const int row = tid;
  const bool own = row < n;
  constexpr double kEps = 2.220446049250313e-16;
  // absolute deflation floor: an off-diagonal below eps*||T|| is negligible at the
  // absolute accuracy of any backward-stable solver; without it the null space of a
  // rank-deficient density matrix is iterated to full relative precision
  double tn = fmax(fmax(fabs(dlo), fabs(dhi)), 2.0 * fmax(fabs(elo), fabs(ehi)));
  for (int o = 32; o >= 1; o >>= 1) tn = fmax(tn, __shfl_xor(tn, o, 64));
  const double efloor = kEps * tn;
  long long nrot = 0;
  for (int l = 0; l < n; ++l) {
    for (int iter = 0; iter < 64; ++iter) {
      // first m >= l with a negligible e[m] (e[n-1] = 0): one ballot per half
      const double dnl = __shfl_down(dlo, 1, 64), dnh = __shfl_down(dhi, 1, 64);
      const double dlo1 = lane == 63 ? lane_read(dhi, 0) : dnl;
      const bool smlo = lane >= l && lane < n - 1 &&
                        (fabs(elo) <= kEps * (fabs(dlo) + fabs(dlo1)) || fabs(elo) <= efloor);
      const bool smhi = lane + 64 >= l && lane + 64 < n - 1 &&
                        (fabs(ehi) <= kEps * (fabs(dhi) + fabs(dnh)) || fabs(ehi) <= efloor);
      const unsigned long long blo = __ballot(smlo), bhi = __ballot(smhi);
      int m = n - 1;
      if (blo) m = __ffsll((long long)blo) - 1;
      else if (bhi) m = 64 + __ffsll((long long)bhi) - 1;
      if (m == l) break;
      const double dl = dget(l), el = eget(l);
      double g = (dget(l + 1) - dl) / (2.0 * el);
      double r = sqrt(g * g + 1.0);
      g = dget(m) - dl + el / (g + copysign(r, g));
      double s = 1.0, c = 1.0, p = 0.0;
      double zc = own ? Z[m * n + row] : 0.0;           // current value of column i+1
      double zn = own ? Z[(m - 1) * n + row] : 0.0;     // column i, fetched one step ahead
      int i = m - 1;
      bool split = false;
      double di1 = dget(m);
      for (; i >= l; --i) {
        const double ei = eget(i), di = dget(i);
        const double zi = zn;
        if (own && i > l) zn = Z[(i - 1) * n + row];
        ++nrot;
        const double f = s * ei, b = c * ei;
        const double q = f * f + g * g;
        if (q == 0.0) {                                   // underflow: T splits here
          eset(i + 1, 0.0);
          dset(i + 1, di1 - p);
          eset(m, 0.0);
          split = true;
          break;
        }
        const double rr = rsqrt_nr(q);                    // 1/sqrt(f^2 + g^2)
        r = q * rr;
        eset(i + 1, r);
        s = f * rr;
        c = g * rr;
        g = di1 - p;
        r = (di - g) * s + 2.0 * c * b;
        p = s * r;
        dset(i + 1, g + p);
        g = c * r - b;
        di1 = di;
        if (own) {
          Z[(i + 1) * n + row] = s * zi + c * zc;
          zc = c * zi - s * zc;
        }
      }
      if (own) Z[(i + 1) * n + row] = zc;
      if (split) continue;
      dset(l, dl - p);
      eset(l, g);
      eset(m, 0.0);
    }
  }
  if (wave == 0) {                                        // eigenvalues for the ordering
    if (lane < n) dd[lane] = dlo;
    if (lane + 64 < n) dd[lane + 64] = dhi;
    if (lane == 0) sc->n_rot += nrot;                 // rotation count (diagnostic)
  }
  __syncthreads();
  if (tid == 0) { const long long t = wall_clock64(); sc->ticks[6] += t - tph; tph = t; }
  // 3. order, keep rule, back-transformation of the kept columns
  for (int i = tid; i < n; i += kThreads) {
    const double wi = dd[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double wj = dd[j];
      rank += (wj > wi) || (wj == wi && j < i);
    }
    wsrt[rank] = wi;
    isrt[rank] = i;
  }
  __syncthreads();
  if (tid == 0) {
    const double w1 = wsrt[0];
    int k = ucols < n ? ucols : n;
    while (k >= 1 && wsrt[k - 1] <= kp.tau_rel * w1) --k;
    while (k >= 1 && k < n && wsrt[k] > kp.floor * w1 && wsrt[k - 1] - wsrt[k] <= kp.tau_deg * w1) --k;
    if (k == 0) {
      k = ucols < n ? ucols : n;
      sc->n_fallback += 1;
    }
    flag[1] = k;
    dyn[op.out_dyn] = k;
    sc->eig_flops += 9LL * n * n * n;
  }
  __syncthreads();
  const int k = flag[1];
  for (int j = n - 3; j >= 0; --j) {                     // z <- H_j z, last reflector first
    const int m = n - j - 1;
    const double beta = hv[int64_t(n) * n + j];
    if (beta == 0.0) continue;
    for (int i = tid; i < m; i += kThreads) vv[i] = hv[int64_t(j) * n + i];
    __syncthreads();
    for (int t = tid; t < k; t += kThreads) {
      const double *z = Z + isrt[t] * n + j + 1;
      double acc = 0.0;
      for (int i = 0; i < m; ++i) acc += vv[i] * z[i];
      pp[t] = beta * acc;
    }
    __syncthreads();
    for (int e = tid; e < m * k; e += kThreads) {
      const int t = e / m, i = e % m;
      Z[isrt[t] * n + j + 1 + i] -= pp[t] * vv[i];
    }
    __syncthreads();
  }
  double *U = ws + op.c;                  // U[j][i], j < k kept vectors, i < n components
  for (int e = tid; e < n * k; e += kThreads) {
    const int j = e / n, i = e % n;
    U[int64_t(j) * ld + i] = Z[isrt[j] * n + i];
  }
  if (tid == 0) sc->ticks[7] += wall_clock64() - tph;
}

// ---------------------------------------------------------------- interpreter

__global__ __launch_bounds__(kThreads) void interp_kernel(const NetDev *__restrict__ nets, KeepParams kp) {
  __shared__ double lds[kLdsDoubles];
  __shared__ Op s_op;                 // the current op, Box slot ids replaced by extents
  const NetDev nd = nets[blockIdx.x];
  const int tid = threadIdx.x;
  constexpr int kOpWords = int(sizeof(Op) / 4);
  static_assert(kOpWords <= kThreads, "Op must be staged by one pass of the workgroup");
  for (int64_t i = 0; i < nd.n_ops; ++i) {
    if (tid < kOpWords) reinterpret_cast<int32_t *>(&s_op)[tid] = reinterpret_cast<const int32_t *>(nd.ops + i)[tid];
    __syncthreads();
    if (tid < 3 * kMaxDyn) {
      Box *bx = tid < kMaxDyn ? &s_op.bm : (tid < 2 * kMaxDyn ? &s_op.bnb : &s_op.bk_);
      const int d = tid % kMaxDyn;
      if (d < bx->nd) bx->id[d] = nd.dyn[bx->id[d]];
    }
    __syncthreads();
    const Op &op = s_op;
    const int kind = op.kind;
    const long long t0 = wall_clock64();
    switch (kind) {
      case OP_GEMM: {
        const double *A = ((op.flags & F_A_CONST) ? nd.cst : nd.ws) + op.a;
        const double *B = ((op.flags & F_B_CONST) ? nd.cst : nd.ws) + op.b;
        gemm_tiles(op, A, B, nd.ws + op.c, nd.tab, lds, 0, 1, nd.sc);
        break;
      }
      case OP_EIG:
        eig_keep(op, nd.ws, nd.dyn, kp, nd.sc, lds);
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
      default:
        break;
    }
    __syncthreads();
    if (tid == 0) nd.sc->ticks[kind & 7] += wall_clock64() - t0;
  }
}

hipError_t launch_interp(const NetDev *nets_dev, int n_nets, const KeepParams &kp, hipStream_t stream) {
  hipLaunchKernelGGL(interp_kernel, dim3(n_nets), dim3(kThreads), 0, stream, nets_dev, kp);
  return hipGetLastError();
}

}  // namespace tn
