// Host-side problem validation and rescaling.
#pragma once
#include <stdint.h>

#include <vector>

#include "pdhcg.h"

namespace pdhcg {

struct Csr {
  int64_t rows = 0, cols = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  int64_t nnz() const { return (int64_t)col.size(); }
};

struct ConeBlock {
  int type, start, dim;
  double alpha;
};

// One problem after validation and rescaling (Section "Problem Rescaling").
struct HostInstance {
  int n = 0, m = 0, r = 0;
  Csr A, AT, P;             // scaled A^, its transpose, scaled P^ (rows==0: absent)
  std::vector<double> R, D; // scaled R^ (r x n) and D^ (r x r)
  std::vector<double> b, c; // scaled (b: the combined row bounds when rows are bounded)
  // implementation form: scaled row bounds (empty: A x = b) and scaled box
  // bounds per coordinate (empty: no box block)
  std::vector<double> rlo, rhi, xlo, xhi;
  std::vector<double> Sx, Sy, qdiag;
  bool resc = false;              // rescaled-cone mode with some SOC/RSOC/EXP/POW block
  double nu_b = 1, nu_c = 1;
  double norm_b = 0, norm_c = 0;  // of the original data
  bool q_diag = true;
  bool p_diag = false;            // P present and diagonal: P u = pdiag * u
  std::vector<double> pdiag;      // diag(P^) when p_diag
  std::vector<ConeBlock> cones;
  // device coordinate order: perm[j] = the caller's index of internal
  // coordinate j (empty: the caller's order).  Either cone blocks are
  // interleaved with the elementwise coordinates, so that contiguous
  // ownership ranges mix both kinds of work, or the coordinates of a
  // cone-free problem are in degree order (see build_instance).
  std::vector<int> perm;
  // degree order: the first `head` coordinates hold the longest A^T rows
  int head = 0;
  // per-coordinate kind and cone work items
  std::vector<uint8_t> ctype;
  std::vector<int> wave_start, wave_dim;
  std::vector<uint8_t> wave_type, wave_euclid;
  std::vector<int> lane_start;
  std::vector<uint8_t> lane_type, lane_euclid;
  std::vector<double> lane_alpha;
};

int build_instance(const pdhcg_problem& p, const pdhcg_settings& s, HostInstance& out);

}  // namespace pdhcg
