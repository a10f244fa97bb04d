// Host-only C entry points exposing the symbolic analysis (diagnostics and
// CPU tests of the schedules the kernels execute).
#include <cstring>
#include <new>
#include <string>

#include "../../include/expri.h"
#include "frontal.hpp"
#include "symbolic.hpp"

struct expri_frontal {
  expri::FrontalSym fs;
};

struct expri_symbolic {
  expri::Symbolic sym;
  // flattened schedules for one block size (expri_symbolic_schedule)
  std::vector<int32_t> lsched, usched, slot_pos, slot_col, row_of, pass_code, c_ell_col;
};

extern "C" {

expri_status expri_symbolic_create(expri_symbolic **out, const expri_circuit *k) {
  if (!out || !k) return EXPRI_EINVAL;
  *out = nullptr;
  expri::PatternInput pin;
  pin.n = k->n;
  if (k->G.n_rows != k->n || k->C.n_rows != k->n || k->B.n_rows != k->n || k->B.n_cols != k->n_src)
    return EXPRI_EINVAL;
  pin.g_rowptr = k->G.rowptr; pin.g_col = k->G.colidx;
  pin.c_rowptr = k->C.rowptr; pin.c_col = k->C.colidx;
  pin.b_rowptr = k->B.rowptr; pin.b_col = k->B.colidx;
  pin.n_src = k->n_src;
  pin.n_dev = k->dev.n;
  pin.dev_d = k->dev.d; pin.dev_g = k->dev.g; pin.dev_s = k->dev.s;
  expri_symbolic *s = new (std::nothrow) expri_symbolic();
  if (!s) return EXPRI_ENOMEM;
  if (!expri::analyse(pin, s->sym)) {
    delete s;
    return EXPRI_EINVAL;
  }
  *out = s;
  return EXPRI_OK;
}

expri_status expri_symbolic_schedule(expri_symbolic *s, int32_t bs, int32_t solve_slots) {
  if (!s || (bs != 256 && bs != 512 && bs != 1024)) return EXPRI_EINVAL;
  if (solve_slots != 0 && solve_slots != 1 && solve_slots != 2 && solve_slots != 4 && solve_slots != 8)
    return EXPRI_EINVAL;
  std::vector<expri::SolveLevel> L, U;
  s->slot_pos.clear();
  s->slot_col.clear();
  s->row_of.clear();
  if (!expri::build_solve_schedule(s->sym, bs, true, L, s->slot_pos, s->slot_col, s->row_of, solve_slots) ||
      !expri::build_solve_schedule(s->sym, bs, false, U, s->slot_pos, s->slot_col, s->row_of, solve_slots)) {
    s->slot_pos.clear();
    s->slot_col.clear();
    s->row_of.clear();
    return EXPRI_EINVAL;
  }
  auto flat = [](const std::vector<expri::SolveLevel> &v, std::vector<int32_t> &o) {
    o.clear();
    for (const auto &l : v) o.insert(o.end(), {l.G, l.P, l.passes, l.rows, l.slot_base, l.row_base});
  };
  flat(L, s->lsched);
  flat(U, s->usched);
  s->pass_code = expri::pass_codes(L, bs);
  const std::vector<int32_t> up = expri::pass_codes(U, bs);
  s->pass_code.insert(s->pass_code.end(), up.begin(), up.end());
  const int32_t k = expri::build_c_ell(s->sym, s->c_ell_col);
  s->c_ell_col.push_back(k);  // last element: the ELL width
  return EXPRI_OK;
}

expri_status expri_symbolic_array(const expri_symbolic *s, const char *name, int32_t *out, int64_t cap,
                                  int64_t *len) {
  if (!s || !name || !len) return EXPRI_EINVAL;
  const expri::Symbolic &S = s->sym;
  const std::vector<int32_t> *v = nullptr;
  const std::string nm(name);
#define A(X) if (nm == #X) v = &S.X;
  A(perm) A(lu_rowptr) A(lu_col) A(lu_diag) A(lev_ptr) A(lev_rows) A(ulev_ptr) A(ulev_rows)
  A(row_grp) A(grp_pos) A(grp_diag) A(grp_ptr) A(pair_src) A(pair_dst) A(lu_gidx) A(jac_ptr)
  A(jac_code) A(node_ptr) A(node_code) A(g_rowptr) A(g_col) A(g_src) A(c_rowptr) A(c_col)
  A(c_src) A(b_rowptr) A(b_col) A(b_src) A(dev_node) A(block_of)
#undef A
#define B(X) if (nm == #X) v = &s->X;
  B(lsched) B(usched) B(slot_pos) B(slot_col) B(row_of) B(pass_code) B(c_ell_col)
#undef B
  if (!v) return EXPRI_EINVAL;
  *len = (int64_t)v->size();
  if (out && cap > 0) std::memcpy(out, v->data(), sizeof(int32_t) * (size_t)std::min<int64_t>(cap, *len));
  return EXPRI_OK;
}

void expri_symbolic_destroy(expri_symbolic *s) { delete s; }

expri_status expri_frontal_create(expri_frontal **out, const expri_circuit *k, int32_t leaf) {
  if (!out || !k) return EXPRI_EINVAL;
  *out = nullptr;
  if (k->G.n_rows != k->n || k->C.n_rows != k->n || k->B.n_rows != k->n || k->B.n_cols != k->n_src)
    return EXPRI_EINVAL;
  expri::PatternInput pin;
  pin.n = k->n;
  pin.g_rowptr = k->G.rowptr; pin.g_col = k->G.colidx;
  pin.c_rowptr = k->C.rowptr; pin.c_col = k->C.colidx;
  pin.b_rowptr = k->B.rowptr; pin.b_col = k->B.colidx;
  pin.n_src = k->n_src;
  pin.n_dev = k->dev.n;
  pin.dev_d = k->dev.d; pin.dev_g = k->dev.g; pin.dev_s = k->dev.s;
  expri_frontal *f = new (std::nothrow) expri_frontal();
  if (!f) return EXPRI_ENOMEM;
  if (!expri::analyse_frontal(pin, f->fs, leaf)) {
    delete f;
    return EXPRI_EINVAL;
  }
  *out = f;
  return EXPRI_OK;
}

expri_status expri_frontal_array(const expri_frontal *f, const char *name, int64_t *out, int64_t cap,
                                 int64_t *len) {
  if (!f || !name || !len) return EXPRI_EINVAL;
  const expri::FrontalSym &S = f->fs;
  const std::string nm(name);
  const std::vector<int32_t> *v = nullptr;
  const std::vector<int64_t> *w = nullptr;
#define A(X) if (nm == #X) v = &S.X;
  A(perm) A(c0) A(nc) A(fsz) A(parent) A(height) A(r_ptr) A(r_idx) A(rel) A(u_off) A(owner) A(lev_ptr)
  A(lev_front) A(ch_ptr) A(ch) A(ent_row) A(ent_g) A(ent_jptr) A(ent_jcode) A(g_rowptr) A(g_col) A(g_src) A(c_rowptr)
  A(c_col) A(c_src) A(b_rowptr) A(b_col) A(b_src) A(dev_node) A(node_ptr) A(node_code)
#undef A
  if (nm == "f_off") w = &S.f_off;
  if (nm == "ent_pos") w = &S.ent_pos;
  if (!v && !w) return EXPRI_EINVAL;
  *len = v ? (int64_t)v->size() : (int64_t)w->size();
  if (out && cap > 0) {
    const int64_t m = std::min<int64_t>(cap, *len);
    for (int64_t i = 0; i < m; ++i) out[i] = v ? (*v)[i] : (*w)[i];
  }
  return EXPRI_OK;
}

expri_status expri_frontal_stats(const expri_frontal *f, double *out) {
  if (!f || !out) return EXPRI_EINVAL;
  const expri::FrontalSym &S = f->fs;
  out[0] = S.n_front;
  out[1] = (double)S.front_doubles;
  out[2] = (double)S.lu_entries;
  out[3] = S.flops;
  out[4] = S.max_front;
  out[5] = S.max_nc;
  out[6] = (double)S.lev_ptr.size() - 1;
  out[7] = (double)S.upd_doubles;
  return EXPRI_OK;
}

void expri_frontal_destroy(expri_frontal *f) { delete f; }

}  // extern "C"
