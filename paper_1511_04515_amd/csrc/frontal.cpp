// Host symbolic analysis for the multifrontal engine (see frontal.hpp).
#include "frontal.hpp"

#include <algorithm>
#include <numeric>

namespace expri {

namespace {

constexpr int32_t kRailG = -1;
constexpr int32_t kRailV = -2;

// Nested dissection that keeps its separator tree.  A set larger than `leaf`
// is split by a middle BFS level from a pseudo-peripheral node (the level at
// which half of the set lies strictly closer to the root); the level becomes a
// tree node and every connected component on either side is dissected below
// it.
struct TreeND {
  const std::vector<int32_t> &ap, &adj;
  int32_t leaf;
  std::vector<int32_t> mark, lev, seen;
  int32_t next_tag = 1, next_seen = 1;
  std::vector<std::vector<int32_t>> members;  // tree nodes in creation (pre-)order
  std::vector<int32_t> parent;

  TreeND(int32_t n, const std::vector<int32_t> &ap_, const std::vector<int32_t> &adj_, int32_t leaf_)
      : ap(ap_), adj(adj_), leaf(leaf_), mark(n, 0), lev(n, 0), seen(n, 0) {}

  void bfs(int32_t root, int32_t tag, std::vector<int32_t> &out, int32_t st) {
    out.clear();
    out.push_back(root);
    seen[root] = st;
    lev[root] = 0;
    for (size_t h = 0; h < out.size(); ++h) {
      const int32_t u = out[h];
      for (int32_t e = ap[u]; e < ap[u + 1]; ++e) {
        const int32_t v = adj[e];
        if (mark[v] == tag && seen[v] != st) {
          seen[v] = st;
          lev[v] = lev[u] + 1;
          out.push_back(v);
        }
      }
    }
  }

  int32_t add_node(std::vector<int32_t> &&nodes, int32_t par) {
    std::sort(nodes.begin(), nodes.end());
    members.push_back(std::move(nodes));
    parent.push_back(par);
    return (int32_t)members.size() - 1;
  }

  // split `set` (members carry no common tag yet) into connected components,
  // each dissected below `par`
  void components(std::vector<int32_t> &set, int32_t par) {
    if (set.empty()) return;
    const int32_t tag = next_tag++;
    for (int32_t v : set) mark[v] = tag;
    std::sort(set.begin(), set.end());
    std::vector<std::vector<int32_t>> comps;
    std::vector<int32_t> seq;
    const int32_t st = next_seen++;
    for (int32_t v : set) {
      if (seen[v] == st) continue;
      bfs(v, tag, seq, st);
      comps.push_back(seq);
    }
    for (auto &c : comps) {
      const int32_t t2 = next_tag++;
      for (int32_t v : c) mark[v] = t2;
    }
    for (auto &c : comps) dissect(c, par);
  }

  // one connected set whose members share one tag
  void dissect(std::vector<int32_t> &nodes, int32_t par) {
    if ((int32_t)nodes.size() <= leaf) {
      add_node(std::move(nodes), par);
      return;
    }
    const int32_t tag = mark[nodes[0]];
    int32_t root = *std::min_element(nodes.begin(), nodes.end());
    int32_t ecc = -1;
    std::vector<int32_t> seq;
    for (int it = 0; it < 6; ++it) {
      bfs(root, tag, seq, next_seen++);
      int32_t far = seq.back();
      const int32_t e = lev[far];
      for (int32_t v : seq)
        if (lev[v] == e && v < far) far = v;
      if (e <= ecc) break;
      ecc = e;
      root = far;
    }
    bfs(root, tag, seq, next_seen++);
    const int32_t dmax = lev[seq.back()];
    if (dmax < 2) {  // clique-like: no separator helps
      add_node(std::move(nodes), par);
      return;
    }
    std::vector<int32_t> cnt(dmax + 1, 0);
    for (int32_t v : seq) cnt[lev[v]]++;
    const int32_t half = (int32_t)seq.size() / 2;
    int32_t acc = 0, L = 1;
    for (int32_t l = 0; l <= dmax; ++l) {
      if (acc + cnt[l] > half) { L = l; break; }
      acc += cnt[l];
    }
    L = std::min(std::max(L, 1), dmax - 1);
    std::vector<int32_t> A, B, S;
    for (int32_t v : seq) {
      if (lev[v] < L) A.push_back(v);
      else if (lev[v] > L) B.push_back(v);
      else S.push_back(v);
    }
    std::vector<int32_t>().swap(nodes);
    const int32_t x = add_node(std::move(S), par);
    components(A, x);
    components(B, x);
  }
};

}  // namespace

bool analyse_frontal(const PatternInput &in, FrontalSym &fs, int32_t leaf) {
  const int32_t n = in.n;
  fs = FrontalSym();
  fs.n = n;
  fs.n_src = in.n_src;
  fs.n_dev = in.n_dev;
  std::string &err = fs.error;
  if (n <= 0) { err = "n must be positive"; return false; }
  if (!check_csr_pattern(n, n, in.g_rowptr, in.g_col, "G", err)) return false;
  if (!check_csr_pattern(n, n, in.c_rowptr, in.c_col, "C", err)) return false;
  if (!check_csr_pattern(n, in.n_src, in.b_rowptr, in.b_col, "B", err)) return false;
  if (in.n_dev < 0) { err = "negative device count"; return false; }
  auto node_ok = [&](int32_t v) { return v == kRailG || v == kRailV || (v >= 0 && v < n); };
  for (int32_t k = 0; k < in.n_dev; ++k)
    if (!node_ok(in.dev_d[k]) || !node_ok(in.dev_g[k]) || !node_ok(in.dev_s[k])) {
      err = "device terminal out of range";
      return false;
    }
  if (leaf < 1) leaf = 1;

  // -- symmetrised pattern of G_k (G_lin and the device stamp positions) --
  std::vector<int32_t> deg(n, 0);
  auto each_edge = [&](auto &&f) {
    for (int32_t i = 0; i < n; ++i)
      for (int32_t e = in.g_rowptr[i]; e < in.g_rowptr[i + 1]; ++e)
        if (in.g_col[e] != i) f(i, in.g_col[e]);
    for (int32_t k = 0; k < in.n_dev; ++k) {
      const int32_t t[3] = {in.dev_d[k], in.dev_g[k], in.dev_s[k]};
      for (int eq : {0, 2})
        for (int var = 0; var < 3; ++var)
          if (t[eq] >= 0 && t[var] >= 0 && t[eq] != t[var]) f(t[eq], t[var]);
    }
  };
  each_edge([&](int32_t a, int32_t b) { deg[a]++; deg[b]++; });
  std::vector<int32_t> ap(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) ap[i + 1] = ap[i] + deg[i];
  std::vector<int32_t> adj(ap[n]);
  {
    std::vector<int32_t> fill(ap.begin(), ap.end() - 1);
    each_edge([&](int32_t a, int32_t b) {
      adj[fill[a]++] = b;
      adj[fill[b]++] = a;
    });
    // sort and deduplicate every row in place, then compact
    int32_t w = 0;
    std::vector<int32_t> ap2(n + 1, 0);
    for (int32_t i = 0; i < n; ++i) {
      auto b = adj.begin() + ap[i], e = adj.begin() + ap[i + 1];
      std::sort(b, e);
      const int32_t start = w;
      for (auto it = b; it != e; ++it)
        if (w == start || adj[w - 1] != *it) adj[w++] = *it;
      ap2[i + 1] = w;
    }
    adj.resize(w);
    ap.swap(ap2);
  }

  // -- separator tree by nested dissection --
  TreeND nd(n, ap, adj, leaf);
  {
    std::vector<int32_t> all(n);
    std::iota(all.begin(), all.end(), 0);
    nd.components(all, -1);
  }
  const int32_t T = (int32_t)nd.members.size();
  // postorder of the tree (children before parents; roots in creation order)
  std::vector<int32_t> kid_ptr(T + 1, 0), kids;
  for (int32_t t = 0; t < T; ++t)
    if (nd.parent[t] >= 0) kid_ptr[nd.parent[t] + 1]++;
  for (int32_t t = 0; t < T; ++t) kid_ptr[t + 1] += kid_ptr[t];
  kids.resize(kid_ptr[T]);
  {
    std::vector<int32_t> fill(kid_ptr.begin(), kid_ptr.end() - 1);
    for (int32_t t = 0; t < T; ++t)
      if (nd.parent[t] >= 0) kids[fill[nd.parent[t]]++] = t;
  }
  std::vector<int32_t> post;
  post.reserve(T);
  {
    std::vector<std::pair<int32_t, int32_t>> stack;
    for (int32_t r = 0; r < T; ++r) {
      if (nd.parent[r] >= 0) continue;
      stack.push_back({r, kid_ptr[r]});
      while (!stack.empty()) {
        auto &top = stack.back();
        if (top.second < kid_ptr[top.first + 1]) {
          const int32_t c = kids[top.second++];
          stack.push_back({c, kid_ptr[c]});
        } else {
          post.push_back(top.first);
          stack.pop_back();
        }
      }
    }
  }
  if ((int32_t)post.size() != T) { err = "separator tree is not a forest"; return false; }
  std::vector<int32_t> front_of(T);
  for (int32_t s = 0; s < T; ++s) front_of[post[s]] = s;

  // -- the new order: each front's members, fronts in postorder --
  fs.n_front = T;
  fs.perm.reserve(n);
  fs.c0.resize(T);
  fs.nc.resize(T);
  fs.parent.resize(T);
  for (int32_t s = 0; s < T; ++s) {
    const auto &mem = nd.members[post[s]];
    fs.c0[s] = (int32_t)fs.perm.size();
    fs.nc[s] = (int32_t)mem.size();
    fs.perm.insert(fs.perm.end(), mem.begin(), mem.end());
    fs.parent[s] = nd.parent[post[s]] >= 0 ? front_of[nd.parent[post[s]]] : -1;
  }
  if ((int32_t)fs.perm.size() != n) { err = "ordering lost nodes"; return false; }
  fs.iperm.assign(n, -1);
  for (int32_t i = 0; i < n; ++i) fs.iperm[fs.perm[i]] = i;
  for (int32_t i = 0; i < n; ++i)
    if (fs.iperm[i] < 0) { err = "ordering is not a permutation"; return false; }
  fs.owner.resize(n);
  for (int32_t s = 0; s < T; ++s)
    for (int32_t i = fs.c0[s]; i < fs.c0[s] + fs.nc[s]; ++i) fs.owner[i] = s;

  // -- children lists and heights --
  fs.ch_ptr.assign(T + 1, 0);
  for (int32_t s = 0; s < T; ++s)
    if (fs.parent[s] >= 0) fs.ch_ptr[fs.parent[s] + 1]++;
  for (int32_t s = 0; s < T; ++s) fs.ch_ptr[s + 1] += fs.ch_ptr[s];
  fs.ch.resize(fs.ch_ptr[T]);
  {
    std::vector<int32_t> fill(fs.ch_ptr.begin(), fs.ch_ptr.end() - 1);
    for (int32_t s = 0; s < T; ++s)
      if (fs.parent[s] >= 0) fs.ch[fill[fs.parent[s]]++] = s;
  }
  fs.height.assign(T, 0);
  for (int32_t s = 0; s < T; ++s)
    if (fs.parent[s] >= 0) fs.height[fs.parent[s]] = std::max(fs.height[fs.parent[s]], fs.height[s] + 1);

  // -- row structures R_s: the later nodes that the pivot columns of s or the
  // update matrices of its children reach --
  std::vector<int32_t> stamp(n, -1);
  fs.r_ptr.assign(T + 1, 0);
  for (int32_t s = 0; s < T; ++s) {
    const int32_t c1 = fs.c0[s] + fs.nc[s];
    std::vector<int32_t> R;
    for (int32_t i = fs.c0[s]; i < c1; ++i) {
      const int32_t iold = fs.perm[i];
      for (int32_t e = ap[iold]; e < ap[iold + 1]; ++e) {
        const int32_t j = fs.iperm[adj[e]];
        if (j >= c1 && stamp[j] != s) { stamp[j] = s; R.push_back(j); }
      }
    }
    for (int32_t q = fs.ch_ptr[s]; q < fs.ch_ptr[s + 1]; ++q) {
      const int32_t c = fs.ch[q];
      for (int32_t a = fs.r_ptr[c]; a < fs.r_ptr[c + 1]; ++a) {
        const int32_t j = fs.r_idx[a];
        if (j >= c1 && stamp[j] != s) { stamp[j] = s; R.push_back(j); }
      }
    }
    std::sort(R.begin(), R.end());
    fs.r_idx.insert(fs.r_idx.end(), R.begin(), R.end());
    fs.r_ptr[s + 1] = (int32_t)fs.r_idx.size();
  }
  fs.fsz.resize(T);
  for (int32_t s = 0; s < T; ++s) fs.fsz[s] = fs.nc[s] + fs.r_ptr[s + 1] - fs.r_ptr[s];

  // local index of global new index j in front s (-1 if absent)
  auto local = [&](int32_t s, int32_t j) -> int32_t {
    if (j >= fs.c0[s] && j < fs.c0[s] + fs.nc[s]) return j - fs.c0[s];
    const auto b = fs.r_idx.begin() + fs.r_ptr[s], e = fs.r_idx.begin() + fs.r_ptr[s + 1];
    const auto it = std::lower_bound(b, e, j);
    if (it == e || *it != j) return -1;
    return fs.nc[s] + (int32_t)(it - b);
  };
  fs.rel.resize(fs.r_idx.size());
  for (int32_t s = 0; s < T; ++s) {
    const int32_t p = fs.parent[s];
    for (int32_t a = fs.r_ptr[s]; a < fs.r_ptr[s + 1]; ++a) {
      const int32_t l = p >= 0 ? local(p, fs.r_idx[a]) : -1;
      if (l < 0) { err = "a child's update row is not in its parent's front"; return false; }
      fs.rel[a] = l;
    }
  }

  // -- levels by height --
  int32_t hmax = 0;
  for (int32_t s = 0; s < T; ++s) hmax = std::max(hmax, fs.height[s]);
  fs.lev_ptr.assign(hmax + 2, 0);
  for (int32_t s = 0; s < T; ++s) fs.lev_ptr[fs.height[s] + 1]++;
  for (int32_t h = 0; h <= hmax; ++h) fs.lev_ptr[h + 1] += fs.lev_ptr[h];
  fs.lev_front.resize(T);
  {
    std::vector<int32_t> fill(fs.lev_ptr.begin(), fs.lev_ptr.end() - 1);
    for (int32_t s = 0; s < T; ++s) fs.lev_front[fill[fs.height[s]]++] = s;
  }

  // -- storage offsets (256-byte aligned) and statistics --
  fs.f_off.resize(T);
  fs.u_off.resize(T);
  int64_t off = 0, uoff = 0;
  for (int32_t s = 0; s < T; ++s) {
    fs.f_off[s] = off;
    off += ((int64_t)fs.fsz[s] * fs.fsz[s] + 31) / 32 * 32;
    fs.u_off[s] = (int32_t)uoff;
    uoff += ((int64_t)(fs.fsz[s] - fs.nc[s]) + 31) / 32 * 32;
    const double f = fs.fsz[s], p = fs.nc[s], r = f - p;
    fs.lu_entries += (int64_t)fs.nc[s] * (2 * (int64_t)fs.fsz[s] - fs.nc[s]);
    fs.flops += 2.0 / 3.0 * p * p * p + 2.0 * r * p * p + 2.0 * r * r * p;
    fs.max_front = std::max(fs.max_front, fs.fsz[s]);
    fs.max_nc = std::max(fs.max_nc, fs.nc[s]);
  }
  if (uoff > INT32_MAX) { err = "update vectors too large"; return false; }
  fs.front_doubles = off;
  fs.upd_doubles = uoff;

  // -- permuted G_lin, C, B --
  auto permute = [&](const int32_t *rp, const int32_t *ci, int32_t cols, bool permute_cols, std::vector<int32_t> &orp,
                     std::vector<int32_t> &oci, std::vector<int32_t> &osrc) {
    orp.assign(n + 1, 0);
    oci.clear();
    osrc.clear();
    std::vector<std::pair<int32_t, int32_t>> row;
    for (int32_t i = 0; i < n; ++i) {
      const int32_t io = fs.perm[i];
      row.clear();
      for (int32_t e = rp[io]; e < rp[io + 1]; ++e) row.push_back({permute_cols ? fs.iperm[ci[e]] : ci[e], e});
      std::sort(row.begin(), row.end());
      for (auto &pr : row) {
        oci.push_back(pr.first);
        osrc.push_back(pr.second);
      }
      orp[i + 1] = (int32_t)oci.size();
    }
    (void)cols;
  };
  permute(in.g_rowptr, in.g_col, n, true, fs.g_rowptr, fs.g_col, fs.g_src);
  permute(in.c_rowptr, in.c_col, n, true, fs.c_rowptr, fs.c_col, fs.c_src);
  permute(in.b_rowptr, in.b_col, in.n_src, false, fs.b_rowptr, fs.b_col, fs.b_src);

  // -- devices in the new order --
  fs.dev_node.resize(3 * (size_t)in.n_dev);
  auto newid = [&](int32_t v) { return v >= 0 ? fs.iperm[v] : v; };
  for (int32_t k = 0; k < in.n_dev; ++k) {
    fs.dev_node[3 * k] = newid(in.dev_d[k]);
    fs.dev_node[3 * k + 1] = newid(in.dev_g[k]);
    fs.dev_node[3 * k + 2] = newid(in.dev_s[k]);
  }
  fs.node_ptr.assign(n + 1, 0);
  for (int32_t k = 0; k < in.n_dev; ++k)
    for (int eq = 0; eq < 2; ++eq) {
      const int32_t v = fs.dev_node[3 * k + (eq ? 2 : 0)];
      if (v >= 0) fs.node_ptr[v + 1]++;
    }
  for (int32_t i = 0; i < n; ++i) fs.node_ptr[i + 1] += fs.node_ptr[i];
  fs.node_code.resize(fs.node_ptr[n]);
  {
    std::vector<int32_t> fill(fs.node_ptr.begin(), fs.node_ptr.end() - 1);
    for (int32_t k = 0; k < in.n_dev; ++k)
      for (int eq = 0; eq < 2; ++eq) {
        const int32_t v = fs.dev_node[3 * k + (eq ? 2 : 0)];
        if (v >= 0) fs.node_code[fill[v]++] = (k << 1) | eq;
      }
  }

  // -- assembly entries: every G_lin nonzero and device derivative, at its
  // front position (the front that owns the earlier of row and column) --
  struct Src {
    int64_t pos;
    int32_t g;     // permuted G_lin index or -1
    int32_t code;  // device code or -1
    int32_t row;   // row of G_k (new order)
  };
  std::vector<Src> src;
  src.reserve(fs.g_col.size() + 6 * (size_t)in.n_dev);
  auto pos_of = [&](int32_t i, int32_t j, int64_t &pos) -> bool {
    const int32_t s = fs.owner[std::min(i, j)];
    const int32_t li = local(s, i), lj = local(s, j);
    if (li < 0 || lj < 0) return false;
    pos = fs.f_off[s] + (int64_t)li + (int64_t)lj * fs.fsz[s];
    return true;
  };
  for (int32_t i = 0; i < n; ++i)
    for (int32_t e = fs.g_rowptr[i]; e < fs.g_rowptr[i + 1]; ++e) {
      int64_t pos;
      if (!pos_of(i, fs.g_col[e], pos)) { err = "G entry outside its front"; return false; }
      src.push_back({pos, e, -1, i});
    }
  for (int32_t k = 0; k < in.n_dev; ++k)
    for (int eq = 0; eq < 2; ++eq) {
      const int32_t row = fs.dev_node[3 * k + (eq ? 2 : 0)];
      if (row < 0) continue;
      for (int var = 0; var < 3; ++var) {
        const int32_t col = fs.dev_node[3 * k + var];
        if (col < 0) continue;
        int64_t pos;
        if (!pos_of(row, col, pos)) { err = "device entry outside its front"; return false; }
        src.push_back({pos, -1, (k << 3) | (eq << 2) | var, row});
      }
    }
  std::sort(src.begin(), src.end(), [](const Src &a, const Src &b) {
    if (a.pos != b.pos) return a.pos < b.pos;
    if (a.g != b.g) return a.g > b.g;  // the G_lin source first
    return a.code < b.code;
  });
  fs.ent_jptr.push_back(0);
  for (size_t q = 0; q < src.size();) {
    size_t e = q;
    int32_t g = -1;
    while (e < src.size() && src[e].pos == src[q].pos) {
      if (src[e].g >= 0) {
        if (g >= 0) { err = "duplicate G entry"; return false; }
        g = src[e].g;
      } else {
        fs.ent_jcode.push_back(src[e].code);
      }
      ++e;
    }
    fs.ent_pos.push_back(src[q].pos);
    fs.ent_row.push_back(src[q].row);
    fs.ent_g.push_back(g);
    fs.ent_jptr.push_back((int32_t)fs.ent_jcode.size());
    q = e;
  }
  return true;
}

}  // namespace expri
