// Host-side probe of the library's problem setup for the CPU tests: reads a
// problem from raw little-endian files, runs pdhcg::build_instance with the
// given settings.interleave, and writes the device coordinate order (perm),
// the head length, the renumbered and rescaled matrices and the scaling.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "host_setup.hpp"

template <class T>
static std::vector<T> read_all(const std::string& path) {
  std::vector<T> v;
  FILE* fp = std::fopen(path.c_str(), "rb");
  if (!fp) return v;
  std::fseek(fp, 0, SEEK_END);
  const long sz = std::ftell(fp);
  std::fseek(fp, 0, SEEK_SET);
  v.resize(sz / sizeof(T));
  if (std::fread(v.data(), sizeof(T), v.size(), fp) != v.size()) v.clear();
  std::fclose(fp);
  return v;
}

template <class T>
static void write_all(const std::string& path, const std::vector<T>& v) {
  FILE* fp = std::fopen(path.c_str(), "wb");
  std::fwrite(v.data(), sizeof(T), v.size(), fp);
  std::fclose(fp);
}

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  const std::string d = argv[1];
  const int order = std::atoi(argv[2]);
  auto Ap = read_all<int64_t>(d + "/A_ptr"), Pp = read_all<int64_t>(d + "/P_ptr");
  auto Ac = read_all<int32_t>(d + "/A_col"), Pc = read_all<int32_t>(d + "/P_col");
  auto Av = read_all<double>(d + "/A_val"), Pv = read_all<double>(d + "/P_val");
  auto b = read_all<double>(d + "/b"), c = read_all<double>(d + "/c");
  auto ct = read_all<int32_t>(d + "/cone_type"), cs = read_all<int32_t>(d + "/cone_start");
  auto cd = read_all<int32_t>(d + "/cone_dim");
  pdhcg_problem p;
  std::memset(&p, 0, sizeof p);
  p.n = (int32_t)c.size();
  p.m = (int32_t)b.size();
  p.A_rowptr = Ap.data(); p.A_col = Ac.data(); p.A_val = Av.data();
  p.b = b.data(); p.c = c.data();
  if (!Pp.empty()) { p.P_rowptr = Pp.data(); p.P_col = Pc.data(); p.P_val = Pv.data(); }
  p.nblocks = (int32_t)ct.size();
  p.cone_type = ct.data(); p.cone_start = cs.data(); p.cone_dim = cd.data();
  pdhcg_settings s;
  std::memset(&s, 0, sizeof s);
  s.scaling = 1; s.ruiz_iters = 10; s.pock_chambolle = 1; s.pc_alpha = 1.0; s.bound_objective = 1;
  s.interleave = order;
  pdhcg::HostInstance H;
  const int rc = pdhcg::build_instance(p, s, H);
  write_all(d + "/perm", H.perm);
  write_all(d + "/A_out_ptr", H.A.ptr);
  write_all(d + "/A_out_col", H.A.col);
  // everything else the setup computes, for the thread-count check
  write_all(d + "/A_out_val", H.A.val);
  write_all(d + "/AT_out_ptr", H.AT.ptr);
  write_all(d + "/AT_out_col", H.AT.col);
  write_all(d + "/AT_out_val", H.AT.val);
  write_all(d + "/P_out_ptr", H.P.ptr);
  write_all(d + "/P_out_col", H.P.col);
  write_all(d + "/P_out_val", H.P.val);
  write_all(d + "/Sx_out", H.Sx);
  write_all(d + "/Sy_out", H.Sy);
  write_all(d + "/b_out", H.b);
  write_all(d + "/c_out", H.c);
  write_all(d + "/qdiag_out", H.qdiag);
  const double nu[2] = {H.nu_b, H.nu_c};
  write_all(d + "/nu_out", std::vector<double>(nu, nu + 2));
  std::printf("%d %d\n", rc, H.head);
  return 0;
}
