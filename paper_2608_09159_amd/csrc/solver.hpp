// Host-side entry points of the kernels in solver.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace pdhcg {

int block_size();
hipError_t launch_solve(const KArgs& args, bool fp32, int grid, hipStream_t stream);
// workgroups resident at once for the kernel(s) a solve of this kind runs
hipError_t max_resident_grid_for(bool fp32, bool ext, bool cones, int lds_bytes, int* out);
hipError_t launch_spmv(const int64_t* ptr, const int* col, const double* val, const double* x,
                       double* y, long rows, int Lw, hipStream_t st);
// rows of perm in five length classes (seg[0..5]: class boundaries in perm)
hipError_t launch_spmv_classes(const int64_t* ptr, const int* col, const double* val, const double* x,
                               double* y, const int* perm, const long* seg, hipStream_t st);
hipError_t launch_norm(const double* x, long n, double* part, double* nrm, hipStream_t st);
hipError_t launch_scale(double* x, long n, const double* nrm, hipStream_t st);
hipError_t launch_fill(double* x, long n, double v, hipStream_t st);

// caller-facing vectors: warm starts in (x: S x / nu, inv: v / (nu S)) and
// results out (x: nu v / S with inv, y: nu S v), through the caller order
// perm (nullable); the dual slack s = nu_c S_x (Q^ w + c^ - A^T wy) of the
// original problem into out[perm[i]]; io: IO_DOUBLES doubles of scratch
constexpr int IO_PARTS = 64;
constexpr int IO_DOUBLES = RMAX + IO_PARTS * RMAX;
hipError_t launch_scale_in(const double* src, const int* perm, const double* S, double nu, bool inv, double* dst,
                           long n, hipStream_t st);
hipError_t launch_scale_out(const double* src, const int* perm, const double* S, double nu, bool inv, double* dst,
                            long n, hipStream_t st);
hipError_t launch_dual_slack(const DevProblem& P, const double* w, const double* wy, const int* perm, double* io,
                             double* out, hipStream_t st);

// diagnostics of failed cone root-finding
hipError_t reset_cone_failure(hipStream_t st);
hipError_t read_cone_failure(double rec[8], unsigned* count);

// diagnostic projection of `count` blocks of one cone type (device buffers)
hipError_t launch_project(int type, int dim, long count, const double* alpha, const double* r,
                          const double* m, const unsigned char* euclid, double* out, hipStream_t st);

// batch solve (one workgroup per instance)
int batch_grid_limit(bool cones, bool ext);
hipError_t launch_batch(const BatchArgs& args, bool cones, bool ext, int grid, hipStream_t st);
hipError_t launch_batch_reset(const InstDesc* desc, int count, int* queue, hipStream_t st);
hipError_t launch_batch_power(const InstDesc* desc, int count, int iters, double* out, hipStream_t st);
hipError_t launch_batch_gather(const InstDesc* desc, int count, const long* offx, const long* offy,
                               double* ox, double* oy, int avg, hipStream_t st);

}  // namespace pdhcg
