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
};

// Rank rule of the eigensolve: drop w <= tau_rel*w1; never split a cluster with
// gap <= tau_deg*w1 whose lower member exceeds floor*w1.
struct KeepParams {
  double tau_rel;
  double tau_deg;
  double floor;
};

constexpr double kClusterFloor = 1e-10;

hipError_t launch_interp(const NetDev *nets_dev, int n_nets, const KeepParams &kp, hipStream_t stream);

}  // namespace tn
