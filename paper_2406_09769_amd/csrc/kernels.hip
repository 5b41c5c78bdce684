// kernels.hip - CDNA4 (gfx950) device code of the density-matrix contraction.
//
// One workgroup of 256 threads (4 wave64s) executes one network's op list:
//   OP_GEMM     pairwise contraction as a 64x64-tiled FP64 GEMM on the matrix cores
//               (v_mfma_f64_16x16x4f64); operand gathers through index tables fold
//               every mode permutation into the tile loads.
//   OP_EIG      symmetric eigensolve of a density matrix (cyclic two-sided Jacobi,
//               round-robin parallel ordering, matrix resident in LDS) followed by the
//               keep rule; writes the kept leading eigenvectors and the kept rank.
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

// Rotation that annihilates a_pq (Golub-Van Loan symmetric Schur step):
// tau = (a_qq - a_pp) / (2 a_pq), t = sgn(tau) / (|tau| + sqrt(1 + tau^2)).
__device__ __forceinline__ void jacobi_rot(double app, double aqq, double apq, double &c, double &s) {
  const double tau = (aqq - app) / (2.0 * apq);
  double t;
  if (fabs(tau) > 1e150) t = 0.5 / tau;
  else t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

__device__ void eig_keep(const Op &op, double *ws, int32_t *dyn, const KeepParams &kp, NetScalars *sc,
                         double *lds) {
  const int ld = int(op.count);            // static dimension = row stride of L and of U
  const int n = box_eff(op.bm);            // runtime dimension: the valid leading block
  const int ucols = op.K;
  const int np = n + (n & 1);
  const int half = np / 2;
  const bool vglob = (op.flags & F_V_GLOBAL) != 0 && (2 * np * np + 4 * np + 16) > kLdsDoubles;
  double *A = lds;                                   // np x np
  double *V = vglob ? ws + op.b : lds + np * np;     // np x np
  double *aux = lds + np * np + (vglob ? 0 : np * np);
  double *cs = aux;                // [half]
  double *sn = aux + half;         // [half]
  double *wsrt = aux + 2 * half;   // [np] sorted eigenvalues
  int *pq = reinterpret_cast<int *>(aux + 2 * half + np);   // [2*half]
  int *isrt = pq + 2 * half;                                 // [np]
  int *flag = isrt + np;                                     // [2]
  double *red = reinterpret_cast<double *>(flag + 4);        // [4]
  const double *L = ws + op.a;
  const int tid = threadIdx.x;

  double fro = 0.0;
  for (int e = tid; e < np * np; e += kThreads) {
    const int i = e / np, j = e % np;
    double v = 0.0;
    if (i < n && j < n) v = 0.5 * (L[int64_t(i) * ld + j] + L[int64_t(j) * ld + i]);
    A[e] = v;
    V[e] = (i == j) ? 1.0 : 0.0;
    fro += v * v;
  }
  fro = sqrt(block_sum(fro, red));
  const double thr = fmax(1e-18 * fro, 1e-300);
  __syncthreads();

  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) flag[0] = 0;
    __syncthreads();
    for (int r = 0; r < np - 1; ++r) {
      if (tid < half) {
        int p, q;
        if (tid == 0) { p = r; q = np - 1; }
        else { p = (r + tid) % (np - 1); q = (r - tid + np - 1) % (np - 1); }
        const double apq = A[p * np + q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > thr) {
          jacobi_rot(A[p * np + p], A[q * np + q], apq, c, s);
          flag[0] = 1;
        }
        pq[2 * tid] = p;
        pq[2 * tid + 1] = q;
        cs[tid] = c;
        sn[tid] = s;
      }
      __syncthreads();
      for (int blk = tid; blk < half * half; blk += kThreads) {
        const int tp = blk / half, tq = blk % half;
        const double c1 = cs[tp], s1 = sn[tp], c2 = cs[tq], s2 = sn[tq];
        if (s1 == 0.0 && s2 == 0.0) continue;
        const int p = pq[2 * tp], q = pq[2 * tp + 1], rr = pq[2 * tq], ss = pq[2 * tq + 1];
        const double apr = A[p * np + rr], aps = A[p * np + ss], aqr = A[q * np + rr], aqs = A[q * np + ss];
        const double xpr = c1 * apr - s1 * aqr, xps = c1 * aps - s1 * aqs;
        const double xqr = s1 * apr + c1 * aqr, xqs = s1 * aps + c1 * aqs;
        A[p * np + rr] = c2 * xpr - s2 * xps;
        A[p * np + ss] = s2 * xpr + c2 * xps;
        A[q * np + rr] = c2 * xqr - s2 * xqs;
        A[q * np + ss] = s2 * xqr + c2 * xqs;
        if (tp == tq) { A[p * np + q] = 0.0; A[q * np + p] = 0.0; }
      }
      for (int e = tid; e < np * half; e += kThreads) {
        const int i = e / half, t = e % half;
        const double s = sn[t];
        if (s == 0.0) continue;
        const double c = cs[t];
        const int p = pq[2 * t], q = pq[2 * t + 1];
        const double vp = V[i * np + p], vq = V[i * np + q];
        V[i * np + p] = c * vp - s * vq;
        V[i * np + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
    const int any = flag[0];
    __syncthreads();
    if (!any) break;
  }

  // descending order of the eigenvalues (ties by index)
  for (int i = tid; i < n; i += kThreads) {
    const double wi = A[i * np + i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double wj = A[j * np + j];
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
  double *U = ws + op.c;                  // U[j][i], j < k kept vectors, i < n components
  for (int e = tid; e < n * k; e += kThreads) {
    const int j = e / n, i = e % n;
    U[int64_t(j) * ld + i] = V[i * np + isrt[j]];
  }
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
