// kernels.hpp - launch interface of the device code.
#pragma once
#include <hip/hip_runtime.h>

#include "program.hpp"

namespace tn {

// What one workgroup of the interpreter needs to run one network.
struct NetDev {
  const Op *ops;
  int64_t n_ops;
  const int32_t *tab;
  double *ws;
  const double *cst;
  NetScalars *sc;
  int32_t *dyn;      // kept-rank slots (inside the workspace)
  int64_t op_begin = 0, op_end = -1;   // ops a chunked launch runs (first < 0 in the launch)
};

// Rank rule of the eigensolve: drop w <= tau_rel*w1; never cut where
// w_k - w_{k+1} <= tau_deg*w_k while w_{k+1} exceeds floor*w1 (floor = kClusterFloor*tau_rel).
struct KeepParams {
  double tau_rel;
  double tau_deg;
  double floor;
  double residual_tol;     // learned mode: accepted max ||L x - theta x|| / theta (kept pairs)
  const float *model;      // learned mode: MLP weights, or null for the exact solve
  float *hx, *hy;          // harvest: feature rows (8 floats) and leverage targets, or null
  int *hcount;             // harvest: rows written so far (atomic)
  long long hcap;          // harvest: capacity in rows
  int split;               // contraction precision: 0 FP64, 1 BF16 x3 split, 2 FP16 x3 split
  int split_all;           // split: 0 = only environment and density-matrix GEMMs (F_ENV),
                           // 1 = every GEMM
  int gemm_cfg[3];         // FP64 GEMM block configuration for ops of <= 16, <= 32, > 32 rows:
                           // 0 = built-in choice, k = candidate k-1 of kGemmConfigs
  int tridiag_ql;          // 1: implicit QL for every tridiagonal solve; 0: divide and
                           // conquer where it fits (orders up to 64)
};

// The FP64 pipelined GEMM's candidate block configurations (rows x columns per block,
// k chunk), in the order the options and the autotuner number them.
constexpr int kGemmConfigs = 6;

constexpr double kClusterFloor = 0.1;   // the separation rule acts above kClusterFloor * tau_rel * w1
constexpr int kMlpParams = 8 * 32 + 32 + 32 * 32 + 32 + 32 + 1;   // 8 -> 32 -> 32 -> 1
constexpr int kMlpBatch = 128;                                  // rows per training step (max)

hipError_t launch_mlp_train(float *w, float *m, float *v, const float *X, const float *Y, long long nrows, int steps,
                            int batch, float lr, unsigned long long seed, long long t0, float *loss_out,
                            float *grad_out, hipStream_t stream);

hipError_t launch_interp(const NetDev *nets_dev, int n_nets, const KeepParams &kp, hipStream_t stream);
// The same over each network's ops [op_begin, op_end) of its descriptor (a part of a
// chunked batch; the network's scalars are written back at the end of every part).
hipError_t launch_interp_parts(const NetDev *nets_dev, int n_nets, const KeepParams &kp, hipStream_t stream);

// Precision a GEMM op runs in under kp: kp.split for the ops the split applies to, else 0.
__host__ __device__ inline int op_split(const KeepParams &kp, int32_t op_flags) {
  return (kp.split && (kp.split_all || (op_flags & F_ENV))) ? kp.split : 0;
}

// Large networks, op by op: one workgroup over ops [first, last) of nd_dev's network;
// one GEMM op or one RESCALE op over `blocks` workgroups (partial: blocks doubles of
// device scratch).
constexpr int kGridBlocks = 2048;
hipError_t launch_interp_range(const NetDev *nd_dev, int64_t first, int64_t last, const KeepParams &kp,
                               hipStream_t stream);
// piped: the op's static rows + k fit kGridOffsetDoubles doubles of int32 offset pairs
// and its static output is below 2^31 elements (FP64 runs the pipelined kernel then).
constexpr int kGridOffsetDoubles = 1216;
// split (1, 2): the operands are first split into planes (device scratch of at least
// split_scratch_bytes of the op's static rows, columns and K; split_blocks workgroups),
// then multiplied; hipErrorInvalidValue without them.
inline int64_t split_scratch_bytes(int64_t rows, int64_t cols, int64_t K) {
  return (rows + cols) * ((K + 15) / 16) * (96 + 8);   // three planes of 16 parts + an FP64 scale per block
}
inline int split_grid_blocks(int64_t rows, int64_t cols, int64_t K) {
  const int64_t blocks = ((rows + cols) * ((K + 15) / 16) + 255) / 256;
  return int(blocks < kGridBlocks ? (blocks < 1 ? 1 : blocks) : kGridBlocks);
}
// Split K: an FP64 chip-wide GEMM that does not run pipelined and has too few 64 x 64
// output tiles to fill the chip cuts K into kchunks parts (a power of two, each at least
// 128 deep) so that tiles x kchunks work items reach about 512 (more parts measured slower:
// 382 against 331 us per call with up to 2048); every work item writes its
// partial tile to kpart (kchunks x rows x cols doubles of device scratch at the runtime
// extents), and a second pass adds the parts in a fixed order into C (reproducible).
inline int grid_kchunks(int64_t rows, int64_t cols, int64_t K) {
  const int64_t tiles = ((rows + 63) / 64) * ((cols + 63) / 64);
  int64_t c = 1;
  while (2 * c * tiles <= 512 && K >= 2 * c * 128) c *= 2;
  return int(c);
}
inline int64_t grid_kpart_doubles(int64_t rows, int64_t cols, int64_t K) {
  const int c = grid_kchunks(rows, cols, K);
  return c > 1 ? int64_t(c) * rows * cols : 0;
}
// Streaming: an FP64 chip-wide GEMM of at most kStreamMaxM static rows and at most 32
// static K over at least kStreamMinN columns runs as a VALU kernel streaming B and C
// (stream_k = its K class 4, 8, 16 or 32; 0 = not streamed), over stream_blocks workgroups.
constexpr int kStreamMaxM = 32;
constexpr int64_t kStreamMinN = int64_t(1) << 16;
inline int stream_kclass(int64_t rows, int64_t cols, int64_t K) {
  if (rows > kStreamMaxM || K > 32 || cols < kStreamMinN) return 0;
  return K <= 4 ? 4 : (K <= 8 ? 8 : (K <= 16 ? 16 : 32));
}
inline int stream_blocks(int64_t cols) {
  const int64_t b = (cols + 4 * 256 - 1) / (4 * 256);
  return int(b < kGridBlocks ? (b < 1 ? 1 : b) : kGridBlocks);
}
hipError_t launch_gemm_grid(const NetDev *nd_dev, int64_t i, int blocks, int split, bool piped,
                            unsigned short *planes, int split_blocks, int kchunks, double *kpart, int stream_k,
                            hipStream_t stream);
hipError_t launch_rescale_grid(const NetDev *nd_dev, int64_t i, int blocks, double *partial, hipStream_t stream);

// Scratch of the allocation-free entry point: a static device array of this many bytes
// per device. noalloc_scratch gives its device address on the current device (looked
// up once per device); no device memory is allocated.
constexpr int64_t kNoAllocScratchBytes = int64_t(256) << 20;
hipError_t noalloc_scratch(char **ptr);

}  // namespace tn
