// Host-side entry points of the kernels in solver.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace pdhcg {

int block_size();
hipError_t launch_solve(const KArgs& args, int grid, hipStream_t stream);
hipError_t max_coop_grid(int* out);
hipError_t launch_spmv(const int64_t* ptr, const int* col, const double* val, const double* x,
                       double* y, long rows, int Lw, hipStream_t st);
hipError_t launch_norm(const double* x, long n, double* part, double* nrm, hipStream_t st);
hipError_t launch_scale(double* x, long n, const double* nrm, hipStream_t st);
hipError_t launch_fill(double* x, long n, double v, hipStream_t st);

}  // namespace pdhcg
