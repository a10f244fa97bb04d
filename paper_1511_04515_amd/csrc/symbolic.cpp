// Host symbolic analysis: ordering, elimination tree, L\U pattern, level
// schedules, refactor update lists and scatter maps (see symbolic.hpp).
#include "symbolic.hpp"

#include <algorithm>
#include <cstring>
#include <numeric>

namespace expri {

namespace {

constexpr int32_t kGND = -1;
constexpr int32_t kVDD = -2;
constexpr int32_t kLeaf = 3;
constexpr int64_t kMaxPairs = int64_t(1) << 31;

bool check_csr(int32_t rows, int32_t cols, const int32_t *rp, const int32_t *ci, const char *name,
               std::string &err) {
  if (rows < 0 || cols < 0) { err = std::string(name) + ": negative size"; return false; }
  if (rows > 0 && (rp == nullptr)) { err = std::string(name) + ": null rowptr"; return false; }
  if (rows == 0) return true;
  if (rp[0] != 0) { err = std::string(name) + ": rowptr[0] != 0"; return false; }
  for (int32_t i = 0; i < rows; ++i) {
    if (rp[i + 1] < rp[i]) { err = std::string(name) + ": rowptr not monotone"; return false; }
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
      if (ci[e] < 0 || ci[e] >= cols) { err = std::string(name) + ": column out of range"; return false; }
      if (e > rp[i] && ci[e] <= ci[e - 1]) {
        err = std::string(name) + ": columns not sorted / duplicated";
        return false;
      }
    }
  }
  return true;
}

// BFS restricted to nodes with mark[v] == tag; returns nodes in BFS order and
// fills lev[] for them.
void bfs(int32_t root, int32_t tag, const std::vector<int32_t> &mark, const std::vector<int32_t> &ap,
         const std::vector<int32_t> &adj, std::vector<int32_t> &lev, std::vector<int32_t> &out,
         std::vector<int32_t> &seen, int32_t seen_tag) {
  out.clear();
  out.push_back(root);
  seen[root] = seen_tag;
  lev[root] = 0;
  for (size_t h = 0; h < out.size(); ++h) {
    int32_t u = out[h];
    for (int32_t e = ap[u]; e < ap[u + 1]; ++e) {
      int32_t v = adj[e];
      if (mark[v] == tag && seen[v] != seen_tag) {
        seen[v] = seen_tag;
        lev[v] = lev[u] + 1;
        out.push_back(v);
      }
    }
  }
}

struct NDState {
  const std::vector<int32_t> &ap, &adj;
  std::vector<int32_t> mark, lev, seen, bufA, bufB;
  int32_t next_tag = 1, next_seen = 1;
  std::vector<int32_t> order;
  NDState(int32_t n, const std::vector<int32_t> &ap_, const std::vector<int32_t> &adj_)
      : ap(ap_), adj(adj_), mark(n, 0), lev(n, 0), seen(n, 0) {}

  // order one connected set (all members carry mark == tag)
  void dissect(std::vector<int32_t> nodes, int depth) {
    if ((int32_t)nodes.size() <= kLeaf || depth > 64) {
      std::sort(nodes.begin(), nodes.end());
      order.insert(order.end(), nodes.begin(), nodes.end());
      return;
    }
    const int32_t tag = mark[nodes[0]];
    // pseudo-peripheral root
    int32_t root = *std::min_element(nodes.begin(), nodes.end());
    int32_t ecc = -1;
    std::vector<int32_t> seq;
    for (int it = 0; it < 6; ++it) {
      bfs(root, tag, mark, ap, adj, lev, seq, seen, next_seen++);
      int32_t far = seq.back();
      int32_t e = lev[far];
      // among the last level pick the smallest id (deterministic)
      for (int32_t v : seq)
        if (lev[v] == e && v < far) far = v;
      if (e <= ecc) break;
      ecc = e;
      root = far;
    }
    bfs(root, tag, mark, ap, adj, lev, seq, seen, next_seen++);
    int32_t depthmax = lev[seq.back()];
    if (depthmax < 2) {  // no useful separator (clique-like): keep BFS order
      std::sort(seq.begin(), seq.end());
      order.insert(order.end(), seq.begin(), seq.end());
      return;
    }
    // separator level: first level at which half of the nodes lie strictly below
    std::vector<int32_t> cnt(depthmax + 1, 0);
    for (int32_t v : seq) cnt[lev[v]]++;
    int32_t half = (int32_t)seq.size() / 2, acc = 0, L = 1;
    for (int32_t l = 0; l <= depthmax; ++l) {
      if (acc + cnt[l] > half) { L = l; break; }
      acc += cnt[l];
    }
    if (L == 0) L = 1;
    if (L >= depthmax) L = depthmax - 1;
    std::vector<int32_t> A, B, S;
    for (int32_t v : seq) {
      if (lev[v] < L) A.push_back(v);
      else if (lev[v] > L) B.push_back(v);
      else S.push_back(v);
    }
    components(A, depth + 1);
    components(B, depth + 1);
    std::sort(S.begin(), S.end());
    order.insert(order.end(), S.begin(), S.end());
  }

  // split a node set into connected components and dissect each
  void components(std::vector<int32_t> &set, int depth) {
    if (set.empty()) return;
    const int32_t tag = next_tag++;
    for (int32_t v : set) mark[v] = tag;
    std::sort(set.begin(), set.end());
    std::vector<std::vector<int32_t>> comps;
    std::vector<int32_t> seq;
    const int32_t st = next_seen++;
    for (int32_t v : set) {
      if (seen[v] == st) continue;
      bfs(v, tag, mark, ap, adj, lev, seq, seen, st);
      comps.push_back(seq);
    }
    for (auto &c : comps) {
      const int32_t t2 = next_tag++;
      for (int32_t v : c) mark[v] = t2;
    }
    for (auto &c : comps) dissect(c, depth);
  }
};

// Tarjan's strongly connected components, iterative.  Returns the component
// id of every node; ids are in reverse topological order of the condensation
// (a component is numbered after every component reachable from it).
int32_t tarjan_scc(int32_t n, const std::vector<int32_t> &ap, const std::vector<int32_t> &adj,
                   std::vector<int32_t> &comp) {
  std::vector<int32_t> index(n, -1), low(n, 0), stack, callv, calle;
  std::vector<char> on(n, 0);
  comp.assign(n, -1);
  int32_t idx = 0, nc = 0;
  for (int32_t s = 0; s < n; ++s) {
    if (index[s] >= 0) continue;
    callv.push_back(s);
    calle.push_back(ap[s]);
    index[s] = low[s] = idx++;
    stack.push_back(s);
    on[s] = 1;
    while (!callv.empty()) {
      int32_t v = callv.back();
      int32_t &e = calle.back();
      if (e < ap[v + 1]) {
        int32_t w = adj[e++];
        if (index[w] < 0) {
          index[w] = low[w] = idx++;
          stack.push_back(w);
          on[w] = 1;
          callv.push_back(w);
          calle.push_back(ap[w]);
        } else if (on[w]) {
          low[v] = std::min(low[v], index[w]);
        }
      } else {
        if (low[v] == index[v]) {
          int32_t w;
          do {
            w = stack.back();
            stack.pop_back();
            on[w] = 0;
            comp[w] = nc;
          } while (w != v);
          ++nc;
        }
        callv.pop_back();
        calle.pop_back();
        if (!callv.empty()) {
          int32_t u = callv.back();
          low[u] = std::min(low[u], low[v]);
        }
      }
    }
  }
  return nc;
}

void fnv(uint64_t &h, const void *p, size_t bytes) {
  const unsigned char *c = static_cast<const unsigned char *>(p);
  for (size_t i = 0; i < bytes; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
}

}  // namespace

bool check_csr_pattern(int32_t rows, int32_t cols, const int32_t *rp, const int32_t *ci, const char *name,
                       std::string &err) {
  return check_csr(rows, cols, rp, ci, name, err);
}

std::vector<int32_t> nested_dissection(int32_t n, const std::vector<int32_t> &ap,
                                       const std::vector<int32_t> &adj) {
  NDState st(n, ap, adj);
  std::vector<int32_t> all(n);
  std::iota(all.begin(), all.end(), 0);
  st.components(all, 0);
  return st.order;
}

uint64_t pattern_hash(const PatternInput &in) {
  uint64_t h = 1469598103934665603ull;
  fnv(h, &in.n, sizeof(in.n));
  fnv(h, &in.n_src, sizeof(in.n_src));
  fnv(h, &in.n_dev, sizeof(in.n_dev));
  if (in.n > 0) {
    fnv(h, in.g_rowptr, sizeof(int32_t) * (in.n + 1));
    fnv(h, in.g_col, sizeof(int32_t) * in.g_rowptr[in.n]);
    fnv(h, in.c_rowptr, sizeof(int32_t) * (in.n + 1));
    fnv(h, in.c_col, sizeof(int32_t) * in.c_rowptr[in.n]);
    fnv(h, in.b_rowptr, sizeof(int32_t) * (in.n + 1));
    fnv(h, in.b_col, sizeof(int32_t) * in.b_rowptr[in.n]);
  }
  if (in.n_dev > 0) {
    fnv(h, in.dev_d, sizeof(int32_t) * in.n_dev);
    fnv(h, in.dev_g, sizeof(int32_t) * in.n_dev);
    fnv(h, in.dev_s, sizeof(int32_t) * in.n_dev);
  }
  return h;
}

bool analyse(const PatternInput &in, Symbolic &sym) {
  const int32_t n = in.n;
  sym = Symbolic();
  sym.n = n;
  sym.n_src = in.n_src;
  sym.n_dev = in.n_dev;
  std::string &err = sym.error;
  if (n <= 0) { err = "n must be positive"; return false; }
  if (!check_csr(n, n, in.g_rowptr, in.g_col, "G", err)) return false;
  if (!check_csr(n, n, in.c_rowptr, in.c_col, "C", err)) return false;
  if (!check_csr(n, in.n_src, in.b_rowptr, in.b_col, "B", err)) return false;
  if (in.n_dev < 0) { err = "negative device count"; return false; }
  auto node_ok = [&](int32_t v) { return v == kGND || v == kVDD || (v >= 0 && v < n); };
  for (int32_t k = 0; k < in.n_dev; ++k)
    if (!node_ok(in.dev_d[k]) || !node_ok(in.dev_g[k]) || !node_ok(in.dev_s[k])) {
      err = "device terminal out of range";
      return false;
    }

  // -- structural pattern P = G_lin + device stamps + diagonal, symmetrised --
  std::vector<std::vector<int32_t>> nb(n);
  auto add_edge = [&](int32_t a, int32_t b) {
    if (a == b) return;
    nb[a].push_back(b);
    nb[b].push_back(a);
  };
  for (int32_t i = 0; i < n; ++i)
    for (int32_t e = in.g_rowptr[i]; e < in.g_rowptr[i + 1]; ++e) add_edge(i, in.g_col[e]);
  for (int32_t k = 0; k < in.n_dev; ++k) {
    const int32_t t[3] = {in.dev_d[k], in.dev_g[k], in.dev_s[k]};
    for (int eq : {0, 2})
      for (int var = 0; var < 3; ++var)
        if (t[eq] >= 0 && t[var] >= 0) add_edge(t[eq], t[var]);
  }
  std::vector<int32_t> ap(n + 1, 0), adj;
  for (int32_t i = 0; i < n; ++i) {
    auto &v = nb[i];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    ap[i + 1] = ap[i] + (int32_t)v.size();
  }
  adj.reserve(ap[n]);
  for (int32_t i = 0; i < n; ++i) adj.insert(adj.end(), nb[i].begin(), nb[i].end());

  // -- fill-reducing order --
  sym.perm = nested_dissection(n, ap, adj);
  if ((int32_t)sym.perm.size() != n) { err = "ordering lost nodes"; return false; }
  sym.iperm.assign(n, -1);
  for (int32_t i = 0; i < n; ++i) sym.iperm[sym.perm[i]] = i;
  for (int32_t i = 0; i < n; ++i)
    if (sym.iperm[i] < 0) { err = "ordering is not a permutation"; return false; }
  const auto &P = sym.perm;
  const auto &IP = sym.iperm;

  // permuted symmetric adjacency, lower part per row
  std::vector<std::vector<int32_t>> low(n);
  for (int32_t iold = 0; iold < n; ++iold)
    for (int32_t e = ap[iold]; e < ap[iold + 1]; ++e) {
      int32_t i = IP[iold], j = IP[adj[e]];
      if (j < i) low[i].push_back(j);
    }

  // -- elimination tree (Liu, path compression) --
  std::vector<int32_t> parent(n, -1), anc(n, -1);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t j : low[i]) {
      int32_t r = j;
      while (anc[r] != -1 && anc[r] != i) {
        int32_t nx = anc[r];
        anc[r] = i;
        r = nx;
      }
      if (anc[r] == -1) {
        anc[r] = i;
        parent[r] = i;
      }
    }

  // -- row structures of L (row subtrees) and of U (transposed) --
  std::vector<std::vector<int32_t>> Lrow(n), Urow(n);
  std::vector<int32_t> mark(n, -1);
  for (int32_t i = 0; i < n; ++i) {
    mark[i] = i;
    for (int32_t j : low[i]) {
      int32_t r = j;
      while (r != -1 && mark[r] != i) {
        Lrow[i].push_back(r);
        mark[r] = i;
        r = parent[r];
      }
    }
    std::sort(Lrow[i].begin(), Lrow[i].end());
    for (int32_t k : Lrow[i]) Urow[k].push_back(i);
  }

  // -- combined L\U CSR --
  sym.lu_rowptr.assign(n + 1, 0);
  sym.lu_diag.assign(n, 0);
  for (int32_t i = 0; i < n; ++i)
    sym.lu_rowptr[i + 1] = sym.lu_rowptr[i] + (int32_t)(Lrow[i].size() + 1 + Urow[i].size());
  const int64_t nnz = sym.lu_rowptr[n];
  sym.lu_col.resize(nnz);
  for (int32_t i = 0; i < n; ++i) {
    int32_t p = sym.lu_rowptr[i];
    for (int32_t k : Lrow[i]) sym.lu_col[p++] = k;
    sym.lu_diag[i] = p;
    sym.lu_col[p++] = i;
    for (int32_t j : Urow[i]) sym.lu_col[p++] = j;
    sym.max_row = std::max(sym.max_row, sym.lu_rowptr[i + 1] - sym.lu_rowptr[i]);
  }

  // -- level schedules --
  std::vector<int32_t> lev(n, 0), ulev(n, 0);
  int32_t nl = 0, nu = 0;
  for (int32_t i = 0; i < n; ++i) {
    int32_t l = 0;
    for (int32_t k : Lrow[i]) l = std::max(l, lev[k] + 1);
    lev[i] = l;
    nl = std::max(nl, l + 1);
  }
  for (int32_t i = n - 1; i >= 0; --i) {
    int32_t l = 0;
    for (int32_t j : Urow[i]) l = std::max(l, ulev[j] + 1);
    ulev[i] = l;
    nu = std::max(nu, l + 1);
  }
  auto bucket = [&](const std::vector<int32_t> &L, int32_t nlev, std::vector<int32_t> &ptr,
                    std::vector<int32_t> &rows) {
    ptr.assign(nlev + 1, 0);
    for (int32_t i = 0; i < n; ++i) ptr[L[i] + 1]++;
    for (int32_t l = 0; l < nlev; ++l) ptr[l + 1] += ptr[l];
    rows.assign(n, 0);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int32_t i = 0; i < n; ++i) rows[fill[L[i]]++] = i;
  };
  bucket(lev, nl, sym.lev_ptr, sym.lev_rows);
  bucket(ulev, nu, sym.ulev_ptr, sym.ulev_rows);

  // -- refactor update lists (row-wise Doolittle) --
  std::vector<int32_t> pos(n, -1);
  sym.row_grp.assign(n + 1, 0);
  sym.grp_ptr.push_back(0);
  int64_t pairs = 0;
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t p = sym.lu_rowptr[i]; p < sym.lu_rowptr[i + 1]; ++p) pos[sym.lu_col[p]] = p;
    for (int32_t k : Lrow[i]) {
      sym.grp_pos.push_back(pos[k]);
      sym.grp_diag.push_back(sym.lu_diag[k]);
      for (int32_t q = sym.lu_diag[k] + 1; q < sym.lu_rowptr[k + 1]; ++q) {
        int32_t j = sym.lu_col[q];
        int32_t d = pos[j];
        if (d < 0) { err = "symbolic fill is not closed"; return false; }
        sym.pair_src.push_back(q);
        sym.pair_dst.push_back(d);
        ++pairs;
        if (pairs >= kMaxPairs) { err = "refactor update list too large"; return false; }
      }
      sym.grp_ptr.push_back((int32_t)sym.pair_src.size());
    }
    sym.row_grp[i + 1] = (int32_t)sym.grp_pos.size();
    for (int32_t p = sym.lu_rowptr[i]; p < sym.lu_rowptr[i + 1]; ++p) pos[sym.lu_col[p]] = -1;
  }
  sym.flops = pairs;

  // -- permuted G, C, B --
  auto permute_csr = [&](const int32_t *rp, const int32_t *ci, int32_t rows, bool perm_cols,
                         std::vector<int32_t> &orp, std::vector<int32_t> &oci,
                         std::vector<int32_t> &osrc) {
    orp.assign(rows + 1, 0);
    for (int32_t inew = 0; inew < rows; ++inew) {
      int32_t iold = P[inew];
      orp[inew + 1] = orp[inew] + (rp[iold + 1] - rp[iold]);
    }
    oci.resize(orp[rows]);
    osrc.resize(orp[rows]);
    std::vector<std::pair<int32_t, int32_t>> tmp;
    for (int32_t inew = 0; inew < rows; ++inew) {
      int32_t iold = P[inew];
      tmp.clear();
      for (int32_t e = rp[iold]; e < rp[iold + 1]; ++e)
        tmp.emplace_back(perm_cols ? IP[ci[e]] : ci[e], e);
      std::sort(tmp.begin(), tmp.end());
      int32_t o = orp[inew];
      for (auto &pr : tmp) {
        oci[o] = pr.first;
        osrc[o] = pr.second;
        ++o;
      }
    }
  };
  permute_csr(in.g_rowptr, in.g_col, n, true, sym.g_rowptr, sym.g_col, sym.g_src);
  permute_csr(in.c_rowptr, in.c_col, n, true, sym.c_rowptr, sym.c_col, sym.c_src);
  permute_csr(in.b_rowptr, in.b_col, n, false, sym.b_rowptr, sym.b_col, sym.b_src);

  // position of (i, j) (internal ids) in the LU storage
  auto lu_pos = [&](int32_t i, int32_t j) -> int32_t {
    auto b = sym.lu_col.begin() + sym.lu_rowptr[i], e = sym.lu_col.begin() + sym.lu_rowptr[i + 1];
    auto it = std::lower_bound(b, e, j);
    if (it == e || *it != j) return -1;
    return (int32_t)(it - sym.lu_col.begin());
  };

  // -- G_lin value index per LU position --
  sym.lu_gidx.assign(nnz, -1);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t e = sym.g_rowptr[i]; e < sym.g_rowptr[i + 1]; ++e) {
      int32_t p = lu_pos(i, sym.g_col[e]);
      if (p < 0) { err = "G entry missing from LU pattern"; return false; }
      sym.lu_gidx[p] = e;
    }

  // -- DC blocks (SCC of the dependency graph, internal ids) --
  {
    std::vector<std::vector<int32_t>> dep(n);
    for (int32_t i = 0; i < n; ++i)
      for (int32_t e = sym.g_rowptr[i]; e < sym.g_rowptr[i + 1]; ++e)
        if (sym.g_col[e] != i) dep[i].push_back(sym.g_col[e]);
    for (int32_t k = 0; k < in.n_dev; ++k) {
      const int32_t t[3] = {in.dev_d[k], in.dev_g[k], in.dev_s[k]};
      for (int eq : {0, 2})
        for (int var = 0; var < 3; ++var)
          if (t[eq] >= 0 && t[var] >= 0 && t[eq] != t[var]) dep[IP[t[eq]]].push_back(IP[t[var]]);
    }
    std::vector<int32_t> dp(n + 1, 0), da;
    for (int32_t i = 0; i < n; ++i) {
      std::sort(dep[i].begin(), dep[i].end());
      dep[i].erase(std::unique(dep[i].begin(), dep[i].end()), dep[i].end());
      dp[i + 1] = dp[i] + (int32_t)dep[i].size();
      da.insert(da.end(), dep[i].begin(), dep[i].end());
    }
    sym.n_blocks = tarjan_scc(n, dp, da, sym.block_of);
  }

  // -- device stamp gather per LU position, node current gather --
  std::vector<std::vector<int32_t>> contrib(nnz);
  std::vector<std::vector<int32_t>> ncontrib(n);
  sym.dev_node.assign(3 * (size_t)in.n_dev, kGND);
  for (int32_t k = 0; k < in.n_dev; ++k) {
    const int32_t t[3] = {in.dev_d[k], in.dev_g[k], in.dev_s[k]};
    for (int v = 0; v < 3; ++v) sym.dev_node[3 * k + v] = t[v] >= 0 ? IP[t[v]] : t[v];
    for (int eqi = 0; eqi < 2; ++eqi) {
      const int32_t eqn = t[eqi == 0 ? 0 : 2];
      if (eqn < 0) continue;
      ncontrib[IP[eqn]].push_back((k << 1) | eqi);
      for (int var = 0; var < 3; ++var) {
        if (t[var] < 0) continue;
        int32_t p = lu_pos(IP[eqn], IP[t[var]]);
        if (p < 0) { err = "device entry missing from LU pattern"; return false; }
        int32_t cross = sym.block_of[IP[eqn]] != sym.block_of[IP[t[var]]] ? 1 : 0;
        contrib[p].push_back((k << 4) | (cross << 3) | (eqi << 2) | var);
      }
    }
  }
  if (in.n_dev >= (1 << 26)) { err = "too many devices"; return false; }
  sym.jac_ptr.assign(nnz + 1, 0);
  for (int64_t p = 0; p < nnz; ++p) sym.jac_ptr[p + 1] = sym.jac_ptr[p] + (int32_t)contrib[p].size();
  for (int64_t p = 0; p < nnz; ++p) sym.jac_code.insert(sym.jac_code.end(), contrib[p].begin(), contrib[p].end());
  sym.node_ptr.assign(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) sym.node_ptr[i + 1] = sym.node_ptr[i] + (int32_t)ncontrib[i].size();
  for (int32_t i = 0; i < n; ++i) sym.node_code.insert(sym.node_code.end(), ncontrib[i].begin(), ncontrib[i].end());

  sym.hash = pattern_hash(in);
  return true;
}

constexpr int kSlotMax = 8;  // entries per lane and pass (the kernel's register budget)

// Flattened schedule of one triangular solve.  Every pass of one direction
// gives each lane the same number P of slots (P in {1, 2, 4, 8}), so that the
// kernel's loads per pass are a fixed set it can issue one pass ahead.  A
// level's rows are handled by groups of G lanes (the smallest power of two
// with ceil(K / G) <= P for the level's longest row K); lane t of pass q of
// the direction reads slots (q * P + j) * bs + t, j < P (coalesced), and group
// t / G owns row row_of[q * bs + t / G].  P is chosen per direction to
// minimise passes * (1 + P / 8): a pass costs a dependent load round trip and
// a barrier, its padding only bandwidth.  Returns false (and builds nothing)
// when a row is longer than 64 lanes x kSlotMax slots.
bool build_solve_schedule(const Symbolic &S, int bs, bool lower, std::vector<SolveLevel> &sched,
                          std::vector<int32_t> &slot_pos, std::vector<int32_t> &slot_col,
                          std::vector<int32_t> &row_of, int force_p) {
  const auto &ptr = lower ? S.lev_ptr : S.ulev_ptr;
  const auto &rows = lower ? S.lev_rows : S.ulev_rows;
  const int nlev = (int)ptr.size() - 1;
  auto row_len = [&](int i) {
    return lower ? S.lu_diag[i] - S.lu_rowptr[i] : S.lu_rowptr[i + 1] - S.lu_diag[i] - 1;
  };
  std::vector<int> Kl(nlev, 0);
  for (int l = 0; l < nlev; ++l)
    for (int q = ptr[l]; q < ptr[l + 1]; ++q) Kl[l] = std::max(Kl[l], row_len(rows[q]));
  auto group = [](int K, int P) {
    int G = 1;
    while (G < 64 && (K + G - 1) / G > P) G *= 2;
    return G;
  };
  int bestP = 1;
  double best = 1e300;
  bool forced_fits = false;
  for (int P = 1; P <= kSlotMax; P *= 2) {
    bool fits = true;
    long passes = 0;
    for (int l = 0; l < nlev; ++l) {
      if (lower && Kl[l] == 0) continue;
      const int G = group(Kl[l], P);
      if ((Kl[l] + G - 1) / G > P) fits = false;
      const int nr = ptr[l + 1] - ptr[l];
      passes += (nr + bs / G - 1) / (bs / G);
    }
    const double cost = fits ? passes * (1.0 + P / 8.0) : 1e300;
    if (cost < best) { best = cost; bestP = P; }
    if (P == force_p) forced_fits = fits;
  }
  if (!(best < 1e300)) return false;
  // a requested P is taken only where every level's longest row fits it
  const int P = forced_fits ? force_p : bestP;
  sched.clear();
  for (int l = 0; l < nlev; ++l) {
    const int r0 = ptr[l], r1 = ptr[l + 1], nr = r1 - r0;
    if (lower && Kl[l] == 0) continue;  // unit diagonal: nothing to do on this level
    const int G = group(Kl[l], P);
    const int per_pass = bs / G;
    const int passes = (nr + per_pass - 1) / per_pass;
    SolveLevel L{};
    L.G = G;
    L.P = P;
    L.passes = passes;
    L.rows = nr;
    L.slot_base = (int32_t)slot_pos.size();
    L.row_base = (int32_t)row_of.size();
    slot_pos.resize(slot_pos.size() + (size_t)passes * P * bs, -1);
    slot_col.resize(slot_col.size() + (size_t)passes * P * bs, 0);
    row_of.resize(row_of.size() + (size_t)passes * bs, -1);
    for (int idx = 0; idx < nr; ++idx) {
      const int i = rows[r0 + idx];
      const int q = idx / per_pass, g = idx % per_pass;
      row_of[L.row_base + q * bs + g] = i;
      const int b = lower ? S.lu_rowptr[i] : S.lu_diag[i] + 1;
      const int e = lower ? S.lu_diag[i] : S.lu_rowptr[i + 1];
      for (int k = 0; k < e - b; ++k) {
        const int li = k % G, j = k / G;
        const int t = g * G + li;
        const size_t o = (size_t)L.slot_base + ((size_t)q * P + j) * bs + t;
        slot_pos[o] = b + k;
        slot_col[o] = S.lu_col[b + k];
      }
    }
    sched.push_back(L);
  }
  return true;
}

std::vector<int32_t> pass_codes(const std::vector<SolveLevel> &sched, int bs) {
  std::vector<int32_t> out;
  for (const auto &L : sched)
    for (int q = 0; q < L.passes; ++q) {
      int lg = 0;
      while ((1 << lg) < L.G) ++lg;
      const int per_pass = bs / L.G;
      const int active = std::min(per_pass, L.rows - q * per_pass) * L.G;
      out.push_back((active << 16) | (lg << 8) | (q == L.passes - 1 ? kPassSync : 0));
    }
  return out;
}

// ELL layout of C's pattern: entry k of row i at k * ld + i (ld >= n, or n
// when ld is 0; -1 on padding); returns K.
int32_t build_c_ell(const Symbolic &S, std::vector<int32_t> &col, int ld) {
  const int n = S.n;
  if (ld < n) ld = n;
  int K = 0;
  for (int i = 0; i < n; ++i) K = std::max(K, S.c_rowptr[i + 1] - S.c_rowptr[i]);
  col.assign((size_t)std::max(K, 1) * ld, -1);
  for (int i = 0; i < n; ++i)
    for (int e = S.c_rowptr[i]; e < S.c_rowptr[i + 1]; ++e) col[(size_t)(e - S.c_rowptr[i]) * ld + i] = S.c_col[e];
  return K;
}


}  // namespace expri
