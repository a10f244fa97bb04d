// Host-side check of the symbolic and multifrontal analyses, built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py:
// reads one circuit (the binary layout written by that test), runs the
// symbolic analysis, the solve schedules for 256 and 512 threads and the
// multifrontal analysis through the C ABI, and reads every named array back.
// Exit status 0 when every call succeeds (the sanitizers abort otherwise).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../include/expri.h"

namespace {

struct Reader {
  FILE *f;
  template <class T>
  std::vector<T> vec(size_t n) {
    std::vector<T> v(n);
    if (n && fread(v.data(), sizeof(T), n, f) != n) {
      fprintf(stderr, "short read\n");
      exit(2);
    }
    return v;
  }
  template <class T>
  T one() {
    return vec<T>(1)[0];
  }
};

struct Csr {
  std::vector<int32_t> ptr, col;
  std::vector<double> val;
  expri_csr c{};
};

void read_csr(Reader &r, Csr &m) {
  const int32_t rows = r.one<int32_t>(), cols = r.one<int32_t>(), nnz = r.one<int32_t>();
  m.ptr = r.vec<int32_t>(rows + 1);
  m.col = r.vec<int32_t>(nnz);
  m.val = r.vec<double>(nnz);
  m.c = expri_csr{rows, cols, nnz, m.ptr.data(), m.col.data(), m.val.data()};
}

int check(expri_status s, const char *what) {
  if (s != EXPRI_OK) {
    fprintf(stderr, "%s failed: %d\n", what, (int)s);
    exit(3);
  }
  return 0;
}

}  // namespace

int main(int argc, char **argv) {
  if (argc < 2) return 1;
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 1;
  Reader r{f};
  const int32_t n = r.one<int32_t>(), n_src = r.one<int32_t>(), n_dev = r.one<int32_t>();
  Csr G, C, B;
  read_csr(r, G);
  read_csr(r, C);
  read_csr(r, B);
  std::vector<int8_t> type = r.vec<int8_t>(n_dev);
  std::vector<int32_t> d = r.vec<int32_t>(n_dev), g = r.vec<int32_t>(n_dev), s = r.vec<int32_t>(n_dev);
  std::vector<double> kp = r.vec<double>(n_dev), wl = r.vec<double>(n_dev), vth = r.vec<double>(n_dev),
                      lam = r.vec<double>(n_dev);
  std::vector<std::vector<double>> st(n_src), sv(n_src);
  std::vector<expri_pwl> src(n_src);
  for (int q = 0; q < n_src; ++q) {
    const int32_t np = r.one<int32_t>();
    st[q] = r.vec<double>(np);
    sv[q] = r.vec<double>(np);
    src[q] = expri_pwl{np, st[q].data(), sv[q].data()};
  }
  const double vdd = r.one<double>(), T = r.one<double>();
  fclose(f);
  expri_circuit k{};
  k.n = n;
  k.G = G.c;
  k.C = C.c;
  k.B = B.c;
  k.dev = expri_mosfets{n_dev, type.data(), d.data(), g.data(), s.data(), kp.data(), wl.data(), vth.data(),
                        lam.data()};
  k.n_src = n_src;
  k.src = src.data();
  k.vdd = vdd;
  k.T = T;

  const char *sym_names[] = {"perm", "lu_rowptr", "lu_col", "lu_diag", "lev_ptr", "lev_rows", "ulev_ptr",
                             "ulev_rows", "row_grp", "grp_pos", "grp_diag", "grp_ptr", "pair_src", "pair_dst",
                             "lu_gidx", "jac_ptr", "jac_code", "node_ptr", "node_code", "g_rowptr", "g_col",
                             "g_src", "c_rowptr", "c_col", "c_src", "b_rowptr", "b_col", "b_src", "dev_node",
                             "block_of", "lsched", "usched", "slot_pos", "slot_col", "row_of", "pass_code",
                             "c_ell_col"};
  if (argc < 3 || argv[2][0] != 'f') {  // symbolic analysis and schedules
    expri_symbolic *sym = nullptr;
    check(expri_symbolic_create(&sym, &k), "expri_symbolic_create");
    for (int bs : {256, 512}) {
      if (expri_symbolic_schedule(sym, bs, 0) != EXPRI_OK) continue;  // rows too long for this block size
      for (const char *name : sym_names) {
        int64_t len = 0;
        check(expri_symbolic_array(sym, name, nullptr, 0, &len), name);
        std::vector<int32_t> out((size_t)len + 1);
        check(expri_symbolic_array(sym, name, out.data(), len, &len), name);
      }
    }
    expri_symbolic_destroy(sym);
  }
  {  // multifrontal analysis
    const char *fr_names[] = {"perm", "c0", "nc", "fsz", "parent", "height", "r_ptr", "r_idx", "rel", "f_off",
                              "u_off", "owner", "lev_ptr", "lev_front", "ch_ptr", "ch", "ent_pos", "ent_row",
                              "ent_g", "ent_jptr", "ent_jcode", "g_rowptr", "g_col", "g_src", "c_rowptr",
                              "c_col", "c_src", "b_rowptr", "b_col", "b_src", "dev_node", "node_ptr",
                              "node_code"};
    expri_frontal *fr = nullptr;
    check(expri_frontal_create(&fr, &k, 16), "expri_frontal_create");
    double stats[8];
    check(expri_frontal_stats(fr, stats), "expri_frontal_stats");
    for (const char *name : fr_names) {
      int64_t len = 0;
      check(expri_frontal_array(fr, name, nullptr, 0, &len), name);
      std::vector<int64_t> out((size_t)len + 1);
      check(expri_frontal_array(fr, name, out.data(), len, &len), name);
    }
    expri_frontal_destroy(fr);
  }
  printf("ok n=%d\n", n);
  return 0;
}
