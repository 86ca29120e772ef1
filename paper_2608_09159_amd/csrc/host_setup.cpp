// Host-side validation, canonicalisation and rescaling of one problem.
//
// Rescaling follows the paper's Section "Problem Rescaling"
// (eq. problem-rescaling, eq. cone-scaling-candidates,
// eq. cone-preserving-scaling) with the defaults of Table practical-defaults:
// Ruiz passes (column candidate sqrt(max_l |A_li|)), one Pock-Chambolle pass
// (column candidate sqrt(sum_l |A_li|^(2-alpha))), rows by the same
// coordinatewise rule (sqrt(max_i |A_li|), sqrt(sum_i |A_li|^alpha)), cone
// blocks sharing one factor (block maximum for Ruiz, block root-mean-square
// for Pock-Chambolle), zero rows and columns keeping factor 1, then
// bound-objective normalisation b^ = b~/(||b~|| + 1), c^ = c~/(||c~|| + 1)
// with Q^ = Q~ (||b~|| + 1)/(||c~|| + 1) so that x^ = x~/nu_b keeps the
// objective proportional.
#include "host_setup.hpp"
#include "common.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <numeric>
#include <system_error>
#include <thread>

namespace pdhcg {

namespace {

// Start f(a, b) on a new thread; false (nothing started) when the system
// refuses one, so that the caller can run the work itself.
template <class F>
bool spawn(std::vector<std::thread>& th, F& f, int64_t a, int64_t b) {
  try {
    th.emplace_back([&f, a, b] { f(a, b); });
    return true;
  } catch (const std::system_error&) {
    return false;
  }
}

// Host threads for the setup loops: the CPUs the system reports, at most 16,
// or fewer when the environment variable PDHCG_HOST_THREADS asks for fewer
// (1 runs every loop on the calling thread).
unsigned host_threads() {
  unsigned t = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (const char* e = std::getenv("PDHCG_HOST_THREADS")) {
    const int k = std::atoi(e);
    if (k >= 1) t = std::min<unsigned>(t, (unsigned)k);
  }
  return t;
}

// Loops over rows run on up to 16 host threads, each thread on one
// contiguous range.  Only work whose result does not depend on the split
// goes through here (per-row work, elementwise updates, maxima), so the
// instance is bit-identical for any thread count.
template <class F>
void par_rows(int64_t rows, F&& f) {
  const unsigned hw = host_threads();
  if (rows < (int64_t(1) << 16) || hw == 1) {
    f(int64_t(0), rows);
    return;
  }
  const int64_t chunk = (rows + hw - 1) / hw;
  std::vector<std::thread> th;
  th.reserve(hw);
  for (unsigned t = 0; t < hw; ++t) {
    const int64_t a = (int64_t)t * chunk, b = std::min(rows, a + chunk);
    if (a >= b) break;
    if (!spawn(th, f, a, b)) {   // no thread to be had: the rest runs here
      f(a, rows);
      break;
    }
  }
  for (auto& x : th) x.join();
}

// The same over the rows of a CSR matrix, split so that every thread gets
// about the same number of nonzeros (rows of very different lengths, such
// as a Fisher market's buyer and good rows, would otherwise leave one
// thread with most of the work).
template <class F>
void par_rows_nnz(const std::vector<int64_t>& ptr, int64_t rows, F&& f) {
  const unsigned hw = host_threads();
  const int64_t nnz = rows > 0 ? ptr[rows] : 0;
  if (nnz < (int64_t(1) << 18) || hw == 1) {
    f(int64_t(0), rows);
    return;
  }
  std::vector<std::thread> th;
  int64_t a = 0;
  for (unsigned t = 1; t <= hw && a < rows; ++t) {
    int64_t b = rows;
    if (t < hw) {
      const int64_t target = nnz / hw * t;
      b = std::upper_bound(ptr.begin(), ptr.begin() + rows + 1, target) - ptr.begin() - 1;
      b = std::max(b, a + 1);
      b = std::min(b, rows);
    }
    if (!spawn(th, f, a, b)) {   // no thread to be had: the rest runs here
      f(a, rows);
      break;
    }
    a = b;
  }
  for (auto& x : th) x.join();
}

// *p = max(*p, v) for the bit patterns of non-negative doubles, which order
// like the values (so the maximum is the same in any order of updates)
inline void atomic_max_bits(uint64_t* p, uint64_t v) {
  uint64_t cur = __atomic_load_n(p, __ATOMIC_RELAXED);
  while (v > cur && !__atomic_compare_exchange_n(p, &cur, v, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
  }
}

inline uint64_t dbits(double v) {
  uint64_t u;
  std::memcpy(&u, &v, sizeof u);
  return u;
}

inline double bitsd(uint64_t u) {
  double v;
  std::memcpy(&v, &u, sizeof v);
  return v;
}

int canon_csr(int64_t rows, int64_t cols, const int64_t* ptr, const int32_t* col,
              const double* val, Csr& out) {
  out.rows = rows;
  out.cols = cols;
  out.ptr.assign(rows + 1, 0);
  if (rows == 0) return PDHCG_OK;
  if (!ptr) return PDHCG_E_ARG;
  if (ptr[0] != 0) return PDHCG_E_CSR;
  for (int64_t i = 0; i < rows; ++i)
    if (ptr[i + 1] < ptr[i]) return PDHCG_E_CSR;
  int64_t nnz = ptr[rows];
  if (nnz > 0 && (!col || !val)) return PDHCG_E_ARG;
  for (int64_t k = 0; k < nnz; ++k)
    if (col[k] < 0 || col[k] >= cols) return PDHCG_E_CSR;
  out.col.reserve(nnz);
  out.val.reserve(nnz);
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t i = 0; i < rows; ++i) {
    row.clear();
    for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) row.emplace_back(col[k], val[k]);
    std::sort(row.begin(), row.end(),
              [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) {
                return a.first < b.first;
              });
    for (size_t k = 0; k < row.size();) {
      int32_t j = row[k].first;
      double acc = 0.0;
      while (k < row.size() && row[k].first == j) acc += row[k++].second;
      out.col.push_back(j);
      out.val.push_back(acc);
    }
    out.ptr[i + 1] = (int64_t)out.col.size();
  }
  return PDHCG_OK;
}

// Transpose of a CSR matrix whose rows are sorted by column.  Each output
// row lists its entries in input-row order, as a serial scatter would; the
// counts are order-free, and each thread fills a range of output rows by
// scanning every input row for the columns of its range (binary search in
// the sorted row), so the result does not depend on the thread count.
Csr transpose(const Csr& a) {
  Csr t;
  t.rows = a.cols;
  t.cols = a.rows;
  t.ptr.assign(t.rows + 1, 0);
  par_rows_nnz(a.ptr, a.rows, [&](int64_t l0, int64_t l1) {
    for (int64_t k = a.ptr[l0]; k < a.ptr[l1]; ++k) __atomic_fetch_add(&t.ptr[a.col[k] + 1], 1, __ATOMIC_RELAXED);
  });
  for (int64_t i = 0; i < t.rows; ++i) t.ptr[i + 1] += t.ptr[i];
  t.col.resize(a.nnz());
  t.val.resize(a.nnz());
  par_rows_nnz(t.ptr, t.rows, [&](int64_t c0, int64_t c1) {
    std::vector<int64_t> pos(t.ptr.begin() + c0, t.ptr.begin() + c1);
    for (int64_t l = 0; l < a.rows; ++l) {
      const int32_t* b0 = a.col.data() + a.ptr[l];
      const int32_t* b1 = a.col.data() + a.ptr[l + 1];
      const int32_t* lo = (c0 == 0) ? b0 : std::lower_bound(b0, b1, (int32_t)c0);
      for (const int32_t* q = lo; q < b1 && *q < c1; ++q) {
        const int64_t d = pos[*q - c0]++;
        t.col[d] = (int32_t)l;
        t.val[d] = a.val[q - a.col.data()];
      }
    }
  });
  return t;
}

double norm2(const std::vector<double>& v) {
  double s = 0.0;
  for (double x : v) s += x * x;
  return std::sqrt(s);
}

// Interleave the cone blocks with the elementwise (FREE / R+) coordinates,
// and the cone types with each other, each in proportion to its count, so
// that contiguous ownership ranges mix projection and elementwise work.
// Renumbers everything indexed by coordinates (columns of A, rows and
// columns of P, columns of R, c, S_x, the cone list) and records the
// permutation; a no-op unless both kinds are present.
void apply_coord_order(HostInstance& H, std::vector<int>& perm, std::vector<ConeBlock>& cones);

void interleave(HostInstance& H) {
  H.perm.clear();
  const int n = H.n;
  struct Unit { int start, dim, type; double alpha; double key; };
  std::vector<Unit> plain, cone;
  for (const auto& cb : H.cones) {
    if (cb.type == PDHCG_CONE_FREE || cb.type == PDHCG_CONE_NONNEG || cb.type == PDHCG_CONE_BOX) {
      for (int i = cb.start; i < cb.start + cb.dim; ++i) plain.push_back({i, 1, cb.type, 0.0, 0.0});
    } else {
      cone.push_back({cb.start, cb.dim, cb.type, cb.alpha, 0.0});
    }
  }
  if (plain.empty() || cone.empty()) return;
  // cone types mixed: key = (rank within the type + 1/2) / count of the type
  int cnt[8] = {0}, seen[8] = {0};
  for (const auto& u : cone) cnt[u.type]++;
  for (auto& u : cone) u.key = (seen[u.type]++ + 0.5) / cnt[u.type];
  std::stable_sort(cone.begin(), cone.end(), [](const Unit& a, const Unit& b) { return a.key < b.key; });
  for (size_t k = 0; k < cone.size(); ++k) cone[k].key = (k + 0.5) / cone.size();
  for (size_t k = 0; k < plain.size(); ++k) plain[k].key = (k + 0.5) / plain.size();
  std::vector<Unit> all;
  all.reserve(plain.size() + cone.size());
  std::merge(plain.begin(), plain.end(), cone.begin(), cone.end(), std::back_inserter(all),
             [](const Unit& a, const Unit& b) { return a.key < b.key; });
  // new order and the renumbered cone list (runs of one elementwise type
  // merge into one block)
  std::vector<int> perm;
  perm.reserve(n);
  std::vector<ConeBlock> cones;
  for (const auto& u : all) {
    const int ns = (int)perm.size();
    for (int j = 0; j < u.dim; ++j) perm.push_back(u.start + j);
    const bool elem = u.type == PDHCG_CONE_FREE || u.type == PDHCG_CONE_NONNEG || u.type == PDHCG_CONE_BOX;
    if (elem && !cones.empty() && cones.back().type == u.type && cones.back().start + cones.back().dim == ns)
      cones.back().dim += 1;
    else
      cones.push_back(ConeBlock{u.type, ns, u.dim, u.alpha});
  }
  apply_coord_order(H, perm, cones);
}

// Renumber everything indexed by coordinates (columns of A, rows and columns
// of P, columns of R, c, S_x, box bounds) to the order perm (perm[j] = the
// current index of new coordinate j), install the renumbered cone list and
// record the permutation.
void apply_coord_order(HostInstance& H, std::vector<int>& perm, std::vector<ConeBlock>& cones) {
  const int n = H.n;
  std::vector<int> inv(n);
  for (int j = 0; j < n; ++j) inv[perm[j]] = j;
  // A: renumber columns, keep rows sorted by column
  {
    Csr& A = H.A;
    par_rows_nnz(A.ptr, A.rows, [&](int64_t l0, int64_t l1) {
      std::vector<std::pair<int32_t, double>> row;
      for (int64_t l = l0; l < l1; ++l) {
        row.clear();
        for (int64_t k = A.ptr[l]; k < A.ptr[l + 1]; ++k) row.emplace_back(inv[A.col[k]], A.val[k]);
        std::sort(row.begin(), row.end(),
                  [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) {
                    return a.first < b.first;
                  });
        int64_t k = A.ptr[l];
        for (const auto& e : row) {
          A.col[k] = e.first;
          A.val[k++] = e.second;
        }
      }
    });
  }
  // P: rows and columns
  if (H.P.rows > 0) {
    Csr Q;
    Q.rows = Q.cols = n;
    Q.ptr.assign(n + 1, 0);
    for (int j = 0; j < n; ++j) Q.ptr[j + 1] = Q.ptr[j] + (H.P.ptr[perm[j] + 1] - H.P.ptr[perm[j]]);
    Q.col.resize(H.P.nnz());
    Q.val.resize(H.P.nnz());
    par_rows(n, [&](int64_t j0, int64_t j1) {
      std::vector<std::pair<int32_t, double>> row;
      for (int64_t j = j0; j < j1; ++j) {
        row.clear();
        const int i = perm[j];
        for (int64_t k = H.P.ptr[i]; k < H.P.ptr[i + 1]; ++k) row.emplace_back(inv[H.P.col[k]], H.P.val[k]);
        std::sort(row.begin(), row.end(),
                  [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) {
                    return a.first < b.first;
                  });
        int64_t k = Q.ptr[j];
        for (const auto& e : row) {
          Q.col[k] = e.first;
          Q.val[k++] = e.second;
        }
      }
    });
    H.P = std::move(Q);
  }
  // R columns, c, S_x
  if (H.r > 0) {
    std::vector<double> R2(H.R.size());
    for (int a = 0; a < H.r; ++a)
      for (int j = 0; j < n; ++j) R2[(size_t)a * n + j] = H.R[(size_t)a * n + perm[j]];
    H.R.swap(R2);
  }
  std::vector<double> c2(n), s2(n);
  for (int j = 0; j < n; ++j) {
    c2[j] = H.c[perm[j]];
    s2[j] = H.Sx[perm[j]];
  }
  H.c.swap(c2);
  H.Sx.swap(s2);
  if (!H.xlo.empty()) {
    std::vector<double> l2(n), h2(n);
    for (int j = 0; j < n; ++j) {
      l2[j] = H.xlo[perm[j]];
      h2[j] = H.xhi[perm[j]];
    }
    H.xlo.swap(l2);
    H.xhi.swap(h2);
  }
  H.cones.swap(cones);
  H.perm.swap(perm);
}

// Degree order of a problem whose coordinates are all elementwise (FREE,
// R+ or box), for A^T rows of skewed length.  Coordinates are sorted by A^T
// row length, longest first.  Rows of at least head_nz nonzeros stay in that
// order at the front (H.head of them; the ownership partition packs that
// head by the work of the A^T phase alone).  The rest are dealt to the
// ranges left of `ranges` (one per workgroup of the partition, less the
// head's) in turn, so that every range holds the same mix of row
// lengths (with a sparse P the inner loop's P rows are then spread evenly
// too) and neighbouring coordinates have similar lengths: a cache line of x
// holds columns of similar degree, and the hot ones stay in L2 during the A
// product.  Returns false (order unchanged) when some block is not
// elementwise.
bool degree_order(HostInstance& H, int ranges, double head_nz) {
  const int n = H.n;
  for (const auto& cb : H.cones)
    if (cb.type != PDHCG_CONE_FREE && cb.type != PDHCG_CONE_NONNEG && cb.type != PDHCG_CONE_BOX) return false;
  std::vector<int> type(n, PDHCG_CONE_FREE);
  for (const auto& cb : H.cones)
    for (int i = cb.start; i < cb.start + cb.dim; ++i) type[i] = cb.type;
  std::vector<int64_t> deg(n, 0);
  for (int64_t k = 0; k < H.A.nnz(); ++k) deg[H.A.col[k]]++;
  // longest first, ties in index order (a counting sort by degree)
  int64_t dmax = 0;
  for (int i = 0; i < n; ++i) dmax = std::max(dmax, deg[i]);
  std::vector<int64_t> start(dmax + 2, 0);
  for (int i = 0; i < n; ++i) start[dmax - deg[i] + 1]++;
  for (int64_t d = 0; d <= dmax; ++d) start[d + 1] += start[d];
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[start[dmax - deg[i]]++] = i;
  int head = 0;
  while (head < n && (double)deg[ord[head]] >= head_nz) ++head;
  std::vector<int> perm;
  perm.reserve(n);
  perm.insert(perm.end(), ord.begin(), ord.begin() + head);
  // the partition packs the head into workgroups of about one range's share
  // of the A^T phase (A^T row plus P row); the rest is dealt over the ranges
  // left, so its ranges line up with the remaining workgroups
  int head_bins = 0;
  {
    auto pnz = [&](int i) { return H.P.rows > 0 ? (double)(H.P.ptr[i + 1] - H.P.ptr[i]) : 0.0; };
    const double share = (double)(H.A.nnz() + (H.P.rows > 0 ? H.P.nnz() : 0)) / std::max(ranges, 1);
    double cur = 0.0;
    for (int k = 0; k < head; ++k) {
      const double z = (double)deg[ord[k]] + pnz(ord[k]);
      if (cur > 0.0 && cur + z > share) {
        ++head_bins;
        cur = 0.0;
      }
      cur += z;
    }
    if (head > 0) ++head_bins;
  }
  const long rest = n - head;
  const int R = (int)std::max<long>(1, std::min<long>(std::max(ranges - head_bins, 1), rest));
  for (int r = 0; r < R; ++r)
    for (long t = r; t < rest; t += R) perm.push_back(ord[head + t]);
  // the cone list: runs of one elementwise type
  std::vector<ConeBlock> cones;
  for (int j = 0; j < n; ++j) {
    const int ty = type[perm[j]];
    if (!cones.empty() && cones.back().type == ty)
      cones.back().dim += 1;
    else
      cones.push_back(ConeBlock{ty, j, 1, 0.0});
  }
  apply_coord_order(H, perm, cones);
  H.head = head;
  return true;
}

// divide entry (l, i) by row[l] * col[i]
void apply_scaling(Csr& a, const std::vector<double>& row, const std::vector<double>& col) {
  par_rows_nnz(a.ptr, a.rows, [&](int64_t l0, int64_t l1) {
    for (int64_t l = l0; l < l1; ++l)
      for (int64_t k = a.ptr[l]; k < a.ptr[l + 1]; ++k) a.val[k] = a.val[k] / (row[l] * col[a.col[k]]);
  });
}

}  // namespace

int build_instance(const pdhcg_problem& p, const pdhcg_settings& s, HostInstance& H) {
  if (p.n < 1 || p.m < 0 || p.r < 0) return PDHCG_E_SHAPE;
  if (p.r > RMAX) return PDHCG_E_SHAPE;
  const bool row_bounds = p.row_lo != nullptr || p.row_hi != nullptr;
  if (row_bounds && (!p.row_lo || !p.row_hi)) return PDHCG_E_ARG;
  if (!p.c || (p.m > 0 && ((!p.b && !row_bounds) || !p.A_rowptr))) return PDHCG_E_ARG;
  if (p.nblocks < 1 || !p.cone_type || !p.cone_start || !p.cone_dim) return PDHCG_E_CONE;
  const int n = p.n, m = p.m;
  H.n = n;
  H.m = m;

  // ---- cones: contiguous tiling of 0..n-1 --------------------------------
  H.cones.clear();
  int pos = 0;
  for (int j = 0; j < p.nblocks; ++j) {
    ConeBlock cb{p.cone_type[j], p.cone_start[j], p.cone_dim[j],
                 p.cone_alpha ? p.cone_alpha[j] : 0.0};
    if (cb.start != pos || cb.dim < 1 || cb.start + cb.dim > n) return PDHCG_E_CONE;
    switch (cb.type) {
      case PDHCG_CONE_FREE:
      case PDHCG_CONE_NONNEG:
      case PDHCG_CONE_SOC:
        break;
      case PDHCG_CONE_BOX:
        if (!p.x_lo || !p.x_hi) return PDHCG_E_ARG;
        for (int i = cb.start; i < cb.start + cb.dim; ++i) {
          const double lo = p.x_lo[i], hi = p.x_hi[i];
          if (std::isnan(lo) || std::isnan(hi) || lo > hi || lo == INFINITY || hi == -INFINITY)
            return PDHCG_E_ARG;
        }
        break;
      case PDHCG_CONE_RSOC:
        if (cb.dim < 2) return PDHCG_E_CONE;
        break;
      case PDHCG_CONE_EXP:
      case PDHCG_CONE_EXP1:
        if (cb.dim != 3) return PDHCG_E_CONE;
        break;
      case PDHCG_CONE_POW:
        if (cb.dim != 3 || !(cb.alpha > 0.0 && cb.alpha < 1.0)) return PDHCG_E_CONE;
        break;
      default:
        return PDHCG_E_CONE;
    }
    H.cones.push_back(cb);
    pos += cb.dim;
  }
  if (pos != n) return PDHCG_E_CONE;

  // ---- matrices ------------------------------------------------------------
  int rc = canon_csr(m, n, p.A_rowptr, p.A_col, p.A_val, H.A);
  if (rc) return rc;
  bool hasP = p.P_rowptr != nullptr;
  if (hasP) {
    rc = canon_csr(n, n, p.P_rowptr, p.P_col, p.P_val, H.P);
    if (rc) return rc;
    // symmetry: P == P^T up to a relative 1e-12 (every entry (i, j) has a
    // mirror (j, i) within the tolerance; rows are sorted, without
    // duplicates)
    double pmax = 0.0;
    for (double v : H.P.val) pmax = std::max(pmax, std::fabs(v));
    const double ptol = 1e-12 * std::max(1.0, pmax);
    const Csr& Pm = H.P;
    int flag = 0;
    par_rows(n, [&](int64_t i0, int64_t i1) {
      bool ok = true;
      for (int64_t i = i0; i < i1 && ok; ++i)
        for (int64_t k = Pm.ptr[i]; k < Pm.ptr[i + 1]; ++k) {
          const int32_t j = Pm.col[k];
          const int32_t* b0 = Pm.col.data() + Pm.ptr[j];
          const int32_t* b1 = Pm.col.data() + Pm.ptr[j + 1];
          const int32_t* it = std::lower_bound(b0, b1, (int32_t)i);
          if (it == b1 || *it != (int32_t)i || std::fabs(Pm.val[it - Pm.col.data()] - Pm.val[k]) > ptol) {
            ok = false;
            break;
          }
        }
      if (!ok) __atomic_store_n(&flag, 1, __ATOMIC_RELAXED);
    });
    if (flag) return PDHCG_E_NONSYM;
  } else {
    H.P = Csr();
  }
  const int r = (p.R != nullptr) ? p.r : 0;
  H.r = r;
  if (r > 0) {
    H.R.assign(p.R, p.R + (size_t)r * n);
    H.D.assign((size_t)r * r, 0.0);
    if (p.D) {
      for (int a = 0; a < r; ++a)
        for (int b2 = 0; b2 < r; ++b2) {
          double dab = p.D[a * r + b2], dba = p.D[b2 * r + a];
          if (std::fabs(dab - dba) > 1e-12 * std::max(1.0, std::fabs(dab))) return PDHCG_E_NONSYM;
          H.D[a * r + b2] = dab;
        }
    } else {
      for (int a = 0; a < r; ++a) H.D[a * r + a] = 1.0;
    }
  }
  H.c.assign(p.c, p.c + n);
  for (double v : H.c) if (!std::isfinite(v)) return PDHCG_E_ARG;
  H.rlo.clear(); H.rhi.clear(); H.xlo.clear(); H.xhi.clear();
  if (row_bounds) {
    // b holds the combined bound of each row: its value for an equality,
    // else the finite endpoint of larger magnitude (0 when neither is
    // finite); it sets the residual normaliser, nu_b and omega_0
    H.rlo.assign(p.row_lo, p.row_lo + m);
    H.rhi.assign(p.row_hi, p.row_hi + m);
    H.b.assign(m, 0.0);
    for (int l = 0; l < m; ++l) {
      const double lo = H.rlo[l], hi = H.rhi[l];
      if (std::isnan(lo) || std::isnan(hi) || lo > hi || lo == INFINITY || hi == -INFINITY) return PDHCG_E_ARG;
      if (lo == hi) H.b[l] = lo;
      else H.b[l] = std::max(std::isfinite(lo) ? std::fabs(lo) : 0.0, std::isfinite(hi) ? std::fabs(hi) : 0.0);
    }
  } else {
    H.b.assign(p.b ? p.b : nullptr, p.b ? p.b + m : nullptr);
    for (double v : H.b) if (!std::isfinite(v)) return PDHCG_E_ARG;
  }
  bool has_box = false;
  for (const auto& cb : H.cones) has_box = has_box || cb.type == PDHCG_CONE_BOX;
  if (has_box) {
    // box bounds per coordinate (unused outside box blocks)
    H.xlo.assign(n, -INFINITY);
    H.xhi.assign(n, INFINITY);
    for (const auto& cb : H.cones)
      if (cb.type == PDHCG_CONE_BOX)
        for (int i = cb.start; i < cb.start + cb.dim; ++i) {
          H.xlo[i] = p.x_lo[i];
          H.xhi[i] = p.x_hi[i];
        }
  }
  H.norm_b = norm2(H.b);
  H.norm_c = norm2(H.c);

  // ---- rescaling -------------------------------------------------------------
  H.Sx.assign(n, 1.0);
  H.Sy.assign(m, 1.0);
  // blocks sharing one factor: every non-elementwise block in the
  // cone-preserving mode; only the EXP1 blocks in the rescaled-cone mode,
  // where SOC/RSOC/EXP/POW coordinates keep their own factors
  std::vector<std::pair<int, int>> blocks;
  const bool resc = s.cone_scaling == PDHCG_SCALE_CONE;
  for (const auto& cb : H.cones) {
    if (cb.type == PDHCG_CONE_FREE || cb.type == PDHCG_CONE_NONNEG || cb.type == PDHCG_CONE_BOX) continue;
    if (resc && cb.type != PDHCG_CONE_EXP1) {
      H.resc = true;
      continue;
    }
    blocks.emplace_back(cb.start, cb.dim);
  }
  Csr& A = H.A;
  if (s.scaling) {
    std::vector<double> row(m), col(n);
    std::vector<uint64_t> colb(n);
    for (int it = 0; it < s.ruiz_iters; ++it) {
      par_rows(n, [&](int64_t i0, int64_t i1) { std::fill(colb.begin() + i0, colb.begin() + i1, dbits(0.0)); });
      par_rows_nnz(A.ptr, m, [&](int64_t l0, int64_t l1) {
        for (int64_t l = l0; l < l1; ++l) {
          double rmax = 0.0;
          for (int64_t k = A.ptr[l]; k < A.ptr[l + 1]; ++k) {
            const double a = std::fabs(A.val[k]);
            if (!(a > 0.0)) continue;   // zeros (and NaN) leave both maxima unchanged
            rmax = std::max(rmax, a);
            atomic_max_bits(&colb[A.col[k]], dbits(a));
          }
          row[l] = rmax;
        }
      });
      par_rows(n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) col[i] = std::sqrt(bitsd(colb[i]));
      });
      par_rows(m, [&](int64_t l0, int64_t l1) {
        for (int64_t l = l0; l < l1; ++l) row[l] = std::sqrt(row[l]);
      });
      for (auto& bk : blocks) {
        double mx = 0.0;
        for (int i = bk.first; i < bk.first + bk.second; ++i) mx = std::max(mx, col[i]);
        for (int i = bk.first; i < bk.first + bk.second; ++i) col[i] = mx;
      }
      par_rows(m, [&](int64_t l0, int64_t l1) {
        for (int64_t l = l0; l < l1; ++l) if (row[l] == 0.0) row[l] = 1.0;
      });
      par_rows(n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) if (col[i] == 0.0) col[i] = 1.0;
      });
      apply_scaling(A, row, col);
      par_rows(m, [&](int64_t l0, int64_t l1) {
        for (int64_t l = l0; l < l1; ++l) H.Sy[l] /= row[l];
      });
      par_rows(n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) H.Sx[i] *= col[i];
      });
    }
    if (s.pock_chambolle) {
      const double al = s.pc_alpha;
      std::fill(row.begin(), row.end(), 0.0);
      std::fill(col.begin(), col.end(), 0.0);
      // sums over the nonzeros (an exponent 0 counts them); the column
      // powers are formed in parallel and summed in row order
      std::vector<double> cpow(A.nnz());
      par_rows_nnz(A.ptr, m, [&](int64_t l0, int64_t l1) {
        for (int64_t l = l0; l < l1; ++l)
          for (int64_t k = A.ptr[l]; k < A.ptr[l + 1]; ++k) {
            const double a = std::fabs(A.val[k]);
            if (a == 0.0) {
              cpow[k] = 0.0;
              continue;
            }
            row[l] += std::pow(a, al);
            cpow[k] = std::pow(a, 2.0 - al);
          }
      });
      for (int64_t l = 0; l < m; ++l)
        for (int64_t k = A.ptr[l]; k < A.ptr[l + 1]; ++k)
          if (A.val[k] != 0.0) col[A.col[k]] += cpow[k];
      for (auto& v : row) v = std::sqrt(v);
      for (auto& v : col) v = std::sqrt(v);
      for (auto& bk : blocks) {
        double ss = 0.0;
        for (int i = bk.first; i < bk.first + bk.second; ++i) ss += col[i] * col[i];
        double rms = std::sqrt(ss / bk.second);
        for (int i = bk.first; i < bk.first + bk.second; ++i) col[i] = rms;
      }
      for (auto& v : row) if (v == 0.0) v = 1.0;
      for (auto& v : col) if (v == 0.0) v = 1.0;
      apply_scaling(A, row, col);
      for (int l = 0; l < m; ++l) H.Sy[l] /= row[l];
      for (int i = 0; i < n; ++i) H.Sx[i] *= col[i];
    }
  }
  // c~ = S_x^-1 c, b~ = S_y b, P~ = S_x^-1 P S_x^-1, R~ = R S_x^-1
  for (int i = 0; i < n; ++i) H.c[i] /= H.Sx[i];
  for (int l = 0; l < m; ++l) H.b[l] *= H.Sy[l];
  for (size_t l = 0; l < H.rlo.size(); ++l) {
    H.rlo[l] *= H.Sy[l];   // infinite endpoints stay infinite
    H.rhi[l] *= H.Sy[l];
  }
  for (size_t i = 0; i < H.xlo.size(); ++i) {
    H.xlo[i] *= H.Sx[i];
    H.xhi[i] *= H.Sx[i];
  }
  if (hasP)
    par_rows(n, [&](int64_t i0, int64_t i1) {
      for (int64_t i = i0; i < i1; ++i)
        for (int64_t k = H.P.ptr[i]; k < H.P.ptr[i + 1]; ++k)
          H.P.val[k] = H.P.val[k] / (H.Sx[i] * H.Sx[H.P.col[k]]);
    });
  for (int a = 0; a < r; ++a)
    for (int i = 0; i < n; ++i) H.R[(size_t)a * n + i] /= H.Sx[i];
  H.nu_b = H.nu_c = 1.0;
  if (s.scaling && s.bound_objective) {
    H.nu_b = norm2(H.b) + 1.0;
    H.nu_c = norm2(H.c) + 1.0;
  }
  for (auto& v : H.b) v /= H.nu_b;
  for (auto& v : H.c) v /= H.nu_c;
  for (auto& v : H.rlo) v /= H.nu_b;
  for (auto& v : H.rhi) v /= H.nu_b;
  for (auto& v : H.xlo) v /= H.nu_b;
  for (auto& v : H.xhi) v /= H.nu_b;
  const double qs = H.nu_b / H.nu_c;
  for (auto& v : H.P.val) v *= qs;
  for (auto& v : H.D) v *= qs;

  // ---- device coordinate order ----------------------------------------------
  // Without cone blocks, skewed A^T rows (the longest at least 64 times the
  // mean) on a large problem (n >= 2^20) get the degree order by default
  // (interleave = 0); interleave = 2 forces it, -1 keeps the caller's order.
  // It is dealt over 512 ranges, the solver's grid for such problems on a
  // 256-CU device (two workgroups per CU); any grid size still gets an even
  // mix.  The head takes the rows of at least 1/8 of a range's share of the
  // A^T and P nonzeros (and at least 4096).
  if (s.interleave == 1) {
    interleave(H);
  } else if (s.interleave == 0 || s.interleave == 2) {
    bool want = s.interleave == 2;
    if (!want && n >= (1 << 20) && A.nnz() > 0) {
      std::vector<int64_t> deg(n, 0);
      for (int64_t k = 0; k < A.nnz(); ++k) deg[A.col[k]]++;
      const int64_t dmax = *std::max_element(deg.begin(), deg.end());
      want = (double)dmax >= 64.0 * (double)A.nnz() / n;
    }
    if (want) {
      const int ranges = 512;
      const double share = (double)(A.nnz() + (hasP ? H.P.nnz() : 0)) / ranges;
      degree_order(H, ranges, std::max(4096.0, share / 8.0));
    }
  }

  // ---- transpose, diagonal of Q^, structure flags -------------------------
  H.AT = transpose(A);
  H.qdiag.assign(n, 0.0);
  H.q_diag = (r == 0);
  bool offdiag = false;
  if (hasP)
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = H.P.ptr[i]; k < H.P.ptr[i + 1]; ++k) {
        if (H.P.col[k] == i) H.qdiag[i] += H.P.val[k];
        else offdiag = true;
      }
  if (offdiag) H.q_diag = false;
  H.p_diag = hasP && !offdiag;
  if (H.p_diag) H.pdiag = H.qdiag;   // R's part is added below
  for (int i = 0; i < n && r > 0; ++i) {
    double acc = 0.0;
    for (int a = 0; a < r; ++a) {
      double ra = H.R[(size_t)a * n + i];
      double t = 0.0;
      for (int b2 = 0; b2 < r; ++b2) t += H.D[a * r + b2] * H.R[(size_t)b2 * n + i];
      acc += ra * t;
    }
    H.qdiag[i] += acc;
  }

  // ---- cone work items ---------------------------------------------------------
  H.ctype.assign(n, CT_CONE);
  H.wave_start.clear(); H.wave_dim.clear(); H.wave_type.clear(); H.wave_euclid.clear();
  H.lane_start.clear(); H.lane_type.clear(); H.lane_euclid.clear(); H.lane_alpha.clear();
  for (const auto& cb : H.cones) {
    // the metric is constant on the block (the Euclidean formulas apply);
    // never for a rescaled cone block, whose metric carries S_j^2
    bool euclid = !(H.resc && cb.type != PDHCG_CONE_EXP1);
    for (int i = cb.start + 1; i < cb.start + cb.dim; ++i)
      if (H.qdiag[i] != H.qdiag[cb.start]) euclid = false;
    switch (cb.type) {
      case PDHCG_CONE_FREE:
        for (int i = cb.start; i < cb.start + cb.dim; ++i) H.ctype[i] = CT_FREE;
        break;
      case PDHCG_CONE_NONNEG:
        for (int i = cb.start; i < cb.start + cb.dim; ++i) H.ctype[i] = CT_NONNEG;
        break;
      case PDHCG_CONE_BOX:
        for (int i = cb.start; i < cb.start + cb.dim; ++i) H.ctype[i] = CT_BOX;
        break;
      case PDHCG_CONE_SOC:
      case PDHCG_CONE_RSOC:
        H.wave_start.push_back(cb.start);
        H.wave_dim.push_back(cb.dim);
        H.wave_type.push_back((uint8_t)cb.type);
        H.wave_euclid.push_back(euclid ? 1 : 0);
        break;
      default:
        H.lane_start.push_back(cb.start);
        H.lane_type.push_back((uint8_t)cb.type);
        H.lane_alpha.push_back(cb.alpha);
        H.lane_euclid.push_back(euclid ? 1 : 0);
        break;
    }
  }
  return PDHCG_OK;
}

}  // namespace pdhcg
