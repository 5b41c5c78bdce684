// program.hpp - the device program a plan compiles to.
//
// A plan turns one (network, path, max_rank, env_size) into a flat list of Ops
// over one network's workspace. The same Op list runs on the device either in the
// persistent interpreter (one workgroup walks every op of one network) or op by
// op with grid-wide launches. Offsets are in elements; int32 index tables live in
// one table pool per plan.
#pragma once
#include <stdint.h>

namespace tn {

enum OpKind : int32_t {
  OP_GEMM = 1,     // C[m*N+n] = sum_k A[am(m)+ak(k)] * B[bk(k)+bn(n)]
  OP_EIG = 2,      // U = kept leading eigenvectors of sym(L), zero-padded to ucols
  OP_RESCALE = 3,  // x *= 2^-e, e = frexp exponent of max|x|; optionally sum e
  OP_SCALAR = 4,   // z = x[0]: add ln|z| and sign(z) to the result
  OP_IDENT = 5,    // x = identity (dim x dim)
  OP_QR = 6,       // C = Q R (Householder) for C read through the row / column maps am / bn
                   // (runtime boxes bm / bnb): Q stored [q][rows] at .c, R [q][cols] at .b,
                   // q = min(rows, cols) written to slot out_dyn
};

// Largest density matrix the eigensolve takes (orders above 128 are solved in global
// scratch, the rest in LDS).
constexpr int32_t kMaxEigDim = 512;

// Largest C the QR-SVD branch factors in one workgroup's LDS: rows x cols.
constexpr int kQrMaxRows = 128;
constexpr int kQrMaxCols = 64;

enum OpFlags : int32_t {
  F_A_CONST = 1,      // A operand lives in the network's input (constant) area
  F_B_CONST = 2,      // B operand lives in the constant area
  F_ACCUM = 4,        // OP_RESCALE: add the exponent to the log accumulator
  F_A_KFAST = 8,      // load A tiles with k varying fastest across threads
  F_B_NFAST = 16,     // load B tiles with n varying fastest across threads
  F_V_GLOBAL = 32,    // OP_EIG: reflector scratch (2 (n*n + n) doubles) at .b
  F_ENV = 64,         // OP_GEMM: builds a right environment or a density matrix; its
                      // rounding only moves the kept subspaces, never the value carried
                      // along the main chain (the split forms may run it in 16-bit parts)
  F_NO_WARM = 128,    // OP_EIG: the small matrix of the QR-SVD branch (rows are not
                      // (bond, leaf) pairs): no learned warm start, no harvested rows
};

// A two-level index map over a row-major multi-index: off(i) = hi[i / lo_n] + lo[i % lo_n]
struct IdxMap {
  int64_t hi;     // table offset of the outer part
  int64_t lo;     // table offset of the inner part
  int32_t lo_n;   // size of the inner part
  int32_t n;      // total (static) extent
};

// Runtime extent of a flattened index group whose leading modes are MPS bonds.
// Static layout: (cap[0], ..., cap[nd-1], rest) row-major. At run time only
// bond indices below the kept rank dyn[id[d]] are valid, so the valid entries
// are the compact range [0, prod(dyn) * rest) mapped back by mixed radix.
constexpr int kMaxDyn = 8;
struct Box {
  int32_t nd;
  int32_t rest;
  int32_t id[kMaxDyn];
  int32_t cap[kMaxDyn];
};

struct Op {
  int32_t kind;
  int32_t flags;
  int64_t c;        // GEMM/EIG/IDENT output offset; RESCALE operand offset
  int64_t a;        // GEMM A; EIG input L; SCALAR operand
  int64_t b;        // GEMM B; EIG scratch (V) when F_V_GLOBAL
  int64_t count;    // IDENT: dim; EIG: static dim of L; RESCALE: static row length; QR: static
                    // rows (row stride of Q; R's row stride is bn.n)
  int32_t K;        // GEMM static contraction extent; EIG: ucols (static kept columns);
                    // QR: static q (min of the static rows and columns)
  int32_t ak;       // GEMM: table offset of A's k offsets
  int32_t bk;       // GEMM: table offset of B's k offsets
  int32_t out_dyn;  // EIG: dyn slot that receives the kept rank
  IdxMap am;        // GEMM: A row map (static extent M)
  IdxMap bn;        // GEMM: B column map (static extent N)
  Box bm, bnb, bk_; // runtime extents of the M, N and K groups (RESCALE: rows, cols)
};

// Scalars each network accumulates on the device.
struct NetScalars {
  double log_sum;     // sum of ln|z| terms
  double max_resid;   // learned eigensolve: largest accepted residual
  long long exp_sum;  // sum of power-of-two exponents (exact)
  long long sign;     // +1 / -1
  long long zero;     // 1 once Z is exactly zero
  long long n_fallback;
  long long n_learned;
  long long flops;      // executed GEMM flops, 2 m n k at the runtime extents
  long long split_flops;  // the part of flops run in 16-bit parts (split forms)
  long long eig_flops;  // 9 n^3 per density matrix at its runtime dimension
  long long n_rot;      // Givens rotations of the QL iterations (diagnostic)
  long long rej[4];     // learned warm starts handed to the exact solve, by reason:
                        // subspace too large for n, lost every column, cut not certified, residual
  long long lticks[4];  // learned warm start, wall-clock ticks: scoring and start basis,
                        // products with L and norms, the small eigensolve, Ritz vectors
  long long ticks[8];   // wall-clock ticks spent per op kind (index = OpKind; the eigensolve also
                        // splits its own time into entries 0, 6 and 7)
  long long qr_ticks;   // wall-clock ticks of the QR factorisations (OP_QR)
};

}  // namespace tn
