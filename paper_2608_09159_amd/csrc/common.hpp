// Internal structures shared by the host setup, the driver and the kernels.
#pragma once
#include <stdint.h>

#include "pdhcg.h"

namespace pdhcg {

constexpr int RMAX = 32;          // largest supported rank of the dense factor R
constexpr int MAX_BLOCK = 1024;

// per-coordinate kind used by elementwise passes
enum : uint8_t { CT_FREE = 0, CT_NONNEG = 1, CT_CONE = 2, CT_BOX = 3 };

// reduction slots (each slot holds one double per workgroup)
enum Slot : int {
  SL_DELTA2 = 0,   // ||u_new - u||^2                (inner stop test)
  SL_SJS,          // <s, J s>                       (BB numerator)
  SL_SDG,          // <s, dg>                        (BB denominator)
  SL_SS,           // ||s||^2                        (Euclidean BB numerator)
  SL_DX2,          // ||x - w_x||^2                  (restart metric)
  SL_DY2,          // ||y - w_y||^2
  SL_ADXDY,        // <A(x - w_x), y - w_y>
  SL_XMOV2,        // ||x_new - x||^2                (inner tolerance)
  SL_RP2,          // ||A x - b||^2 (unscaled)
  SL_RD2,          // ||Pi_K(-s)||^2 (unscaled)
  SL_XQX,          // <x, Q x>   (scaled)
  SL_CX,           // <c, x>     (scaled)
  SL_BY,           // <b, y>     (scaled)
  SL_MOVX2,        // ||w_x - a_x||^2                (PID)
  SL_MOVY2,        // ||w_y - a_y||^2
  SL_NAN,          // count of non-finite values
  SL_SPS,          // <s, P s>, diagonal P          (one-sync inner step)
  SL_BOXD,         // sum(lambda+ l^x - lambda- u^x) over box coordinates (scaled)
  SL_H0,           // R u : RMAX slots
  SL_HS0 = SL_H0 + RMAX,   // R s : RMAX slots (one-sync inner step)
  SL_COUNT = SL_HS0 + RMAX
};

struct DevProblem {
  int n, m, r;
  int at_lanes, a_lanes;
  const int64_t* A_ptr;  const int* A_col;  const double* A_val;
  const int64_t* AT_ptr; const int* AT_col; const double* AT_val;
  const int64_t* P_ptr;  const int* P_col;  const double* P_val;  // nullable
  const double* Pd;      // diag(P^) when p_diag (P u is then Pd * u)
  int p_diag;
  const double* R;       // r x n row-major (scaled)
  // FP32 copies of the values of A, A^T, P, R (FP32 mode only; else null)
  const float* A_valf; const float* AT_valf; const float* P_valf; const float* Rf;
  const double* Dm;      // r x r (scaled)
  const double* b;       // m (scaled; the combined row bounds when rows are bounded)
  const double* rlo;     // m scaled row bounds (nullable: A x = b)
  const double* rhi;
  const double* xlo;     // n scaled box bounds (nullable: no box block)
  const double* xhi;
  int ext;               // row bounds, box or fixed-middle EXP blocks present, or the
                         // rescaled-cone mode: the kernel variant compiled with them
                         // (others leave them out)
  int resc;              // rescaled-cone mode: SOC/RSOC/EXP/POW block j is S_j K_j,
                         // S_j = diag(Sx on the block)
  const double* c;       // n (scaled)
  const double* qd;      // n diag(Q^)
  const double* Sx;      // n
  const double* Sy;      // m
  const uint8_t* ctype;  // n
  int n_wave, n_lane;
  const int* wave_start; const int* wave_dim; const uint8_t* wave_type;
  const uint8_t* wave_euclid;
  const int* lane_start; const uint8_t* lane_type; const double* lane_alpha;
  const uint8_t* lane_euclid;
  double nu_b, nu_c, norm_b, norm_c;   // norm_b, norm_c: ||b||, ||c|| of the original data
  double eta, omega0;
  int q_diag;            // Q^ diagonal (includes Q = 0): one metric projection per prox
  // ownership of workgroup w: coordinates [part_c[w], part_c[w+1]), rows
  // [part_r[w], part_r[w+1]), wave items [part_w[w], ...), lane items
  // [part_l[w], ...)
  const long* part_c;
  const long* part_r;
  const int* part_w;
  const int* part_l;
  // A^T rows of each workgroup grouped by length class (skewed row lengths
  // only; else null): at_perm[n], at_seg[(classes + 1) * G]
  const int* at_perm;
  const int* at_seg;
  const unsigned short* part_lanes;  // per workgroup: lanes for A^T/P rows (up to
                                     // 512: the whole workgroup), A rows,
                                    // SOC/RSOC group width, pad
};

struct DevVec {
  double *x, *y, *ax, *ay, *wx, *wy;
  double *Ax, *Aa, *Aw;          // A^ x, A^ a, A^ w_x (m)
  double *v, *u, *up, *g, *gp;   // inner-solve vectors (n)
  double *zb;                    // pre-projection buffer (n)
  double *s;                     // KKT dual slack (n)
  double *t1, *t2;               // SpMV results of the current pass (n)
  double *warm;                  // root-finding warm starts, 2 x (n_wave + n_lane)
  double *xb, *yb, *Axb;         // averaged scheme
  double *partials;              // SL_COUNT x G
};

struct DevSettings {
  double tol;
  long long max_iter;
  int check_every;
  int scheme;
  double rho;
  int avg_epoch;
  int inner;
  int fixed_inner;
  int j_max;
  double eps_in0, gamma_in, eps_min;
  double beta_s, beta_n, beta_a;
  double pid_beta_i, pid_kp, pid_ki, pid_kd;
  int trace_iters;
};

// scalar state persisted in device memory between launches
struct Ctl {
  double omega, eps_in, E0, Eprev, pid_I, e_prev;
  double rel_p, rel_d, rel_gap, pobj, dobj, lastE;
  long long k, ktot, inner_total, restarts;
  int status;       // 0 running, else PDHCG_* status
  int started;
  int resume;       // with started = 0: re-initialise from zb / y, keep counters
  int pad1;
  double hx[RMAX];  // R^ x of the current Halpern primal state
  double hxb[RMAX]; // R^ xbar (averaged scheme)
  unsigned long long pt[16];  // phase timers (wall-clock ticks, workgroup 0)
};

// phase-timer categories
enum : int { PT_INIT = 0, PT_P1, PT_P2, PT_P3, PT_P4, PT_P6, PT_CHECK, PT_HALP, PT_BAR,
             PT_PROJ, PT_WCALL, PT_NCALL, PT_COUNT };

struct TraceBufs {
  int cap;                       // 0 = off
  double *x, *y, *wx, *wy;       // cap*n, cap*m
  double *sc;                    // cap * 8 scalars
};

// grid barrier state: one arrival word per workgroup (64-byte stride) and a
// release word written by workgroup 0
constexpr int BAR_STRIDE = 16;
struct Barrier {
  unsigned gen;
  int abort;
  unsigned pad[BAR_STRIDE - 2];
  unsigned arrive[1];   // really [G * BAR_STRIDE]
};

struct KArgs {
  DevProblem P;
  DevVec V;
  DevSettings S;
  Ctl* ctl;
  Barrier* bar;
  TraceBufs T;
  long long stop_at;   // return to the host when ktot reaches this
  unsigned long long spin_limit;  // grid-barrier wait bound, wall-clock ticks
  double qmax;         // max_i diag(Q^)_i (first Euclidean BB step)
  int lds_bytes;       // dynamic LDS per workgroup (R slice; 0 = none)
  int profile;         // accumulate phase timers in ctl->pt and ptimes
  unsigned long long* ptimes;   // [G][PT_COUNT] per-workgroup timers (profile)
};

// what one solver run reads besides the problem and its vectors
struct Run {
  const DevSettings* S;
  const TraceBufs* T;
  long long stop_at;             // return when ktot reaches this
  double qmax;                   // max_i diag(Q^)_i (first Euclidean BB step)
  unsigned long long deadline;   // wall-clock tick; 0 = none (checked at checks)
  void* lds;                     // dynamic LDS for the workgroup's slice of R (nullable)
  int lds_bytes;
};

// one instance of a batch: its problem, vectors, trace buffers and control
// block, solved by a single workgroup that owns every coordinate and row
struct InstDesc {
  DevProblem P;
  DevVec V;
  TraceBufs T;
  Ctl* ctl;
  double qmax;
  const double* x0;   // scaled warm start (nullable), copied into zb at reset
  const double* y0;   // scaled dual warm start (nullable)
  int la, lr, lg;     // lanes per row of A^T / P and of A, SOC/RSOC group width
  int n_warm;         // root warm-start slots (2 x (wave + lane items))
  const int* perm;    // caller index of each internal coordinate (nullable)
};

struct BatchArgs {
  const InstDesc* desc;
  int count;
  const int* order;        // queue position -> instance (largest first)
  int* queue;              // next queue position (reset to 0 before a launch)
  DevSettings S;
  long long stop_at;       // per-instance iteration cap of this launch
  unsigned long long limit_ticks;   // per-launch wall-clock budget (0 = none)
  unsigned long long* ptimes;       // [grid][PT_COUNT] phase timers, nullable
};

}  // namespace pdhcg
