// planner.hpp - host planner: network structure -> device program.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "program.hpp"

namespace tn {

struct Graph {
  int32_t nt = 0;
  std::vector<std::vector<int64_t>> dims;   // per tensor
  std::vector<int32_t> e_t0, e_m0, e_t1, e_m1;
  // per tensor: incident edges in edge-id order (edge, mode, other endpoint)
  struct Inc { int32_t e, m, other; };
  std::vector<std::vector<Inc>> inc;
  std::vector<int64_t> const_off;           // offset of each tensor in the constant area
  int64_t const_size = 0;
  int64_t edge_dim(int32_t e) const { return dims[e_t0[e]][e_m0[e]]; }
};

// Build the graph; returns "" or an error message (TN_EINVAL).
std::string build_graph(const int64_t *const *dims, const int32_t *orders, int32_t nt,
                        const int32_t *e4, int32_t ne, Graph &g);

struct Plan {
  std::vector<Op> ops;
  std::vector<int32_t> tables;
  int64_t ws_size = 0;       // doubles
  int64_t flops = 0;         // sum 2 m n k over GEMMs
  int64_t eig_flops = 0;     // 9 n^3 per density matrix
  int64_t n_eig = 0;
  int64_t n_qr = 0;          // QR-SVD branches taken
  int32_t max_eig_dim = 0;
  int64_t dyn_off = 0;       // workspace offset (doubles) of the int32 kept-rank slots
  int32_t n_dyn = 0;
  int32_t max_dyn_modes = 0; // most bond modes met in one GEMM index group
  std::string plan_json;     // structural plan (leaf orders and placements)
};

struct PlanArgs {
  std::vector<std::vector<int32_t>> slices;
  int32_t chi = 1;
  int32_t env = 1;
};

// Returns "" or an error message. Structural problems -> TN_EINVAL; a density matrix
// beyond the supported dimension sets *unsupported.
std::string make_plan(const Graph &g, const PlanArgs &a, Plan &out, bool *unsupported);


}  // namespace tn
