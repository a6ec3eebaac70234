// Host plan for the MRPT2 energy: STP-DAS categories and strings (Sec. 2.4),
// external space by excitation class, excitation lists with fermionic signs,
// and the device memory layout.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>

namespace mrpt2 {
namespace {

int popc(uint64_t x) { return __builtin_popcountll(x); }

int64_t binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

struct Layout {
  size_t cur = 0;
  size_t take(size_t bytes) {
    size_t o = cur;
    cur = align_up(cur + bytes);
    return o;
  }
};

// All electron counts m with sum m = ne and 0 <= m_k <= s_k, in lexicographic
// order of (m_0, m_1, ...).
void categories(const std::vector<int>& s, int ne, std::vector<std::vector<int>>* out) {
  std::vector<int> m(s.size(), 0);
  std::vector<int> suffix(s.size() + 1, 0);
  for (int k = (int)s.size() - 1; k >= 0; --k) suffix[k] = suffix[k + 1] + s[k];
  std::function<void(int, int)> rec = [&](int k, int left) {
    if (k == (int)s.size()) {
      if (left == 0) out->push_back(m);
      return;
    }
    for (int x = 0; x <= std::min(s[k], left); ++x) {
      if (left - x > suffix[k + 1]) continue;
      m[k] = x;
      rec(k + 1, left - x);
    }
  };
  rec(0, ne);
}

// Strings of one category: product over subspaces of the combinations of m_k
// spinors among s_k (lexicographic), the last subspace varying fastest.
void category_strings(const std::vector<int>& s, const std::vector<int>& off,
                      const std::vector<int>& m, std::vector<uint64_t>* out) {
  std::vector<std::vector<uint64_t>> per(s.size());
  for (size_t k = 0; k < s.size(); ++k) {
    std::vector<int> c(m[k]);
    for (int i = 0; i < m[k]; ++i) c[i] = i;
    while (true) {
      uint64_t b = 0;
      for (int i = 0; i < m[k]; ++i) b |= 1ull << (off[k] + c[i]);
      per[k].push_back(b);
      int i = m[k] - 1;
      while (i >= 0 && c[i] == s[k] - m[k] + i) --i;
      if (i < 0) break;
      ++c[i];
      for (int j = i + 1; j < m[k]; ++j) c[j] = c[j - 1] + 1;
    }
  }
  std::vector<size_t> idx(s.size(), 0);
  while (true) {
    uint64_t b = 0;
    for (size_t k = 0; k < s.size(); ++k) b |= per[k][idx[k]];
    out->push_back(b);
    int k = (int)s.size() - 1;
    while (k >= 0) {
      if (++idx[k] < per[k].size()) break;
      idx[k] = 0;
      --k;
    }
    if (k < 0) break;
  }
}

// Sign of applying the active operators to string beta (active bits only):
// annihilations in `ann` order, then creations in `cre` order.  Each operator
// on spinor p takes (-1)^(occupied active spinors below p).  Returns 0 when
// the product vanishes; *res receives the resulting string.
int op_sign(uint64_t beta, const int* ann, int na, const int* cre, int nc, uint64_t* res) {
  int sgn = 1;
  uint64_t d = beta;
  for (int i = 0; i < na; ++i) {
    uint64_t bit = 1ull << ann[i];
    if (!(d & bit)) return 0;
    if (popc(d & (bit - 1)) & 1) sgn = -sgn;
    d &= ~bit;
  }
  for (int i = 0; i < nc; ++i) {
    uint64_t bit = 1ull << cre[i];
    if (d & bit) return 0;
    if (popc(d & (bit - 1)) & 1) sgn = -sgn;
    d |= bit;
  }
  *res = d;
  return sgn;
}

std::vector<int> bits_of(uint64_t x) {
  std::vector<int> b;
  while (x) {
    int p = __builtin_ctzll(x);
    b.push_back(p);
    x &= x - 1;
  }
  return b;
}

struct PatKey {
  int32_t kind, a0, a1, r0, r1, w;
  bool operator==(const PatKey& o) const {
    return kind == o.kind && a0 == o.a0 && a1 == o.a1 && r0 == o.r0 && r1 == o.r1 && w == o.w;
  }
};
struct PatHash {
  size_t operator()(const PatKey& k) const {
    return ((((size_t)k.kind * 131 + k.a0 + 1) * 131 + k.a1 + 1) * 131 + k.r0 + 1) * 131 * 131 +
           (k.r1 + 1) * 131 + k.w + 1;
  }
};

// Excitation lists of one class.  For external active string alpha and a
// reference string beta = (alpha - R) + A:
//   rank-2 patterns: |R| = 2 - v active creations, |A| = 2 - h annihilations;
//   rank-1 patterns (h <= 1, v <= 1): |R| = 1 - v, |A| = 1 - h, as a one-body
//   pattern and one spectator pattern per w in alpha - R.
// Operator order (fixes the sign and the integral slots): core annihilations
// ascending, active annihilations ascending (then w for a spectator), active
// creations (w first for a spectator) ascending, virtual creations descending.
void build_class(InstancePlan& ip, ClassPlan& cp) {
  const int h = cp.h, v = cp.v;
  std::unordered_map<PatKey, int, PatHash> pid;
  auto get_pid = [&](const PatKey& k) {
    auto it = pid.find(k);
    if (it != pid.end()) return it->second;
    int id = (int)cp.patterns.size();
    pid.emplace(k, id);
    cp.patterns.push_back(Pattern{k.kind, k.a0, k.a1, k.r0, k.r1, k.w, 0, 0});
    return id;
  };
  // fixed pattern order for the dense classes: patterns indexed by their
  // orbitals so that the integral layouts are regular
  cp.conn_ptr.assign(cp.strings.size() + 1, 0);
  const int n_a = ip.n_a;
  const uint64_t amask = (n_a == 64) ? ~0ull : ((1ull << n_a) - 1);
  for (size_t s = 0; s < cp.strings.size(); ++s) {
    const uint64_t al = cp.strings[s];
    const std::vector<int> occ = bits_of(al);
    const std::vector<int> fre = bits_of(amask & ~al);
    for (int rank = 1; rank <= 2; ++rank) {
      const int nr = rank - v, na = rank - h;
      if (nr < 0 || na < 0) continue;
      // subsets R of occ of size nr, A of fre of size na
      std::vector<int> R(nr), A(na);
      std::function<void(int, int)> recA;
      std::function<void(int, int)> recR = [&](int i0, int k) {
        if (k == nr) {
          recA(0, 0);
          return;
        }
        for (int i = i0; i < (int)occ.size(); ++i) {
          R[k] = occ[i];
          recR(i + 1, k + 1);
        }
      };
      recA = [&](int i0, int k) {
        if (k < na) {
          for (int i = i0; i < (int)fre.size(); ++i) {
            A[k] = fre[i];
            recA(i + 1, k + 1);
          }
          return;
        }
        uint64_t beta = al;
        for (int x : R) beta &= ~(1ull << x);
        for (int x : A) beta |= 1ull << x;
        auto it = ip.pindex.find(beta);
        if (it == ip.pindex.end()) return;
        const int32_t bidx = it->second;
        auto emit = [&](int kind, int w) {
          int ann[3], cre[3], nan = 0, ncr = 0;
          for (int x : A) ann[nan++] = x;
          if (kind == PAT_SPECT) {
            ann[nan++] = w;
            cre[ncr++] = w;
          }
          for (int x : R) cre[ncr++] = x;
          uint64_t res = 0;
          int sg = op_sign(beta, ann, nan, cre, ncr, &res);
          if (sg == 0 || res != al) return;
          PatKey key{kind, na > 0 ? A[0] : -1, na > 1 ? A[1] : -1, nr > 0 ? R[0] : -1,
                     nr > 1 ? R[1] : -1, kind == PAT_SPECT ? w : -1};
          int id = get_pid(key);
          cp.conn.push_back(bidx | (sg < 0 ? (int32_t)0x80000000 : 0));
          cp.conn.push_back(id);
        };
        if (rank == 2) {
          emit(PAT_DOUBLE, -1);
        } else {
          emit(PAT_SINGLE, -1);
          for (int w : occ) {
            bool inR = false;
            for (int x : R) inR |= (x == w);
            if (!inR) emit(PAT_SPECT, w);
          }
        }
      };
      recR(0, 0);
    }
    cp.conn_ptr[s + 1] = (int32_t)(cp.conn.size() / 2);
  }
  cp.n_conn = (int64_t)(cp.conn.size() / 2);
}

// Reorder the strings of a class so that strings coupling to the same set of
// active orbitals (same annihilated-orbital pattern set) are adjacent; the
// register-resident coupling kernels then walk runs of identical masks.
void sort_by_pattern_mask(InstancePlan& ip, ClassPlan& cp) {
  const size_t S = cp.strings.size();
  std::vector<uint64_t> key(S, 0);
  for (size_t s = 0; s < S; ++s)
    for (int e = cp.conn_ptr[s]; e < cp.conn_ptr[s + 1]; ++e) {
      const Pattern& p = cp.patterns[cp.conn[2 * e + 1]];
      // the orbital a pattern is indexed by: the annihilated active spinor
      // (class (1,2)) or the created one (class (2,1))
      const int o = p.a0 >= 0 ? p.a0 : p.r0;
      if (o >= 0) key[s] |= 1ull << o;
    }
  std::vector<size_t> ord(S);
  for (size_t s = 0; s < S; ++s) ord[s] = s;
  std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return key[x] < key[y]; });
  std::vector<uint64_t> sorted(S);
  for (size_t s = 0; s < S; ++s) sorted[s] = cp.strings[ord[s]];
  cp.strings.swap(sorted);
  cp.patterns.clear();
  cp.conn.clear();
  cp.conn_ptr.clear();
  build_class(ip, cp);
}

}  // namespace

int64_t sigma_blocks(const InstancePlan& ip, int k) {
  const ClassPlan& cp = ip.cls[k];
  if (cp.strings.empty() || cp.n_rows == 0) return 0;
  const int64_t rb = (cp.n_rows + 255) / 256;
  const int64_t target = cp.sigma_target > 0 ? cp.sigma_target : 8192;
  int64_t nsc = std::max<int64_t>(1, std::min<int64_t>((int64_t)cp.strings.size(), (target + rb - 1) / rb));
  return rb * nsc;
}

namespace {

int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Append one launch over the given per-instance jobs (skipping empty grids).
void add_launch(Plan* P, std::vector<Launch>* seq, int kid, int stage, const std::vector<JobH>& js,
                size_t dyn = 0, int arg = 0) {
  Launch L;
  L.kid = kid;
  L.stage = stage;
  L.job0 = (int64_t)P->jobs.size();
  L.dyn_lds = dyn;
  L.arg = arg;
  int64_t blk = 0;
  for (JobH j : js) {
    if (j.gx <= 0 || j.gy <= 0) continue;
    j.blk0 = blk;
    blk += (int64_t)j.gx * j.gy;
    P->jobs.push_back(j);
  }
  L.njobs = (int)((int64_t)P->jobs.size() - L.job0);
  L.nblocks = blk;
  if (L.njobs > 0) seq->push_back(L);
}

JobH job(int inst, int64_t gx, int64_t gy, int arg = 0) {
  JobH j;
  j.inst = inst;
  j.gx = (int32_t)gx;
  j.gy = (int32_t)gy;
  j.arg = arg;
  j.blk0 = 0;
  return j;
}

// Factor tables and the occupied-block integrals for the instances in `which`.
void table_launches(Plan* P, std::vector<Launch>* seq, const std::vector<int>& which) {
  std::vector<JobH> js;
  for (int i : which) {
    const InstancePlan& ip = P->inst[i];
    for (int t = 0; t < ip.d.n_sets; ++t)
      if (ip.d.rank[t] > 0) js.push_back(job(i, cdiv64(ip.d.rank[t], 64), ip.n_corr, t));
  }
  add_launch(P, seq, K_PACK, ST_TABLES, js);
  js.clear();
  for (int i : which) {
    const InstancePlan& ip = P->inst[i];
    for (int t = 0; t < ip.d.n_sets; ++t)
      if (ip.d.rank[t] > 0) js.push_back(job(i, cdiv64(ip.n, 256), ip.d.rank[t], t));
  }
  add_launch(P, seq, K_DIAG, ST_TABLES, js);
  js.clear();
  for (int i : which) js.push_back(job(i, cdiv64(P->inst[i].n, 256), P->inst[i].n));
  add_launch(P, seq, K_WPASS, ST_TABLES, js);
  js.clear();
  for (int i : which) js.push_back(job(i, cdiv64(P->inst[i].n_corr, 256), 1));
  add_launch(P, seq, K_EPS, ST_TABLES, js);
  js.clear();
  for (int i : which) js.push_back(job(i, cdiv64(P->inst[i].n_l, 256), 1));
  add_launch(P, seq, K_DSUM, ST_TABLES, js);
  js.clear();
  for (int i : which) {
    const InstancePlan& ip = P->inst[i];
    if (ip.n_fc + ip.n_c > 0)
      js.push_back(job(i, cdiv64(ip.n_a + ip.n_v, 64) * cdiv64(ip.n_o, 64), ip.n_fc + ip.n_c));
  }
  add_launch(P, seq, K_FOCKX, ST_TABLES, js);
  js.clear();
  for (int i : which) js.push_back(job(i, P->inst[i].n_o, P->inst[i].n_a + P->inst[i].n_v));
  add_launch(P, seq, K_FOCK, ST_TABLES, js);
  js.clear();
  for (int i : which) {
    const InstancePlan& ip = P->inst[i];
    if (ip.n_a == 0) continue;
    const int64_t M = (int64_t)ip.n_o * (ip.n_a + ip.n_v), N = (int64_t)ip.n_o * ip.n_a;
    js.push_back(job(i, cdiv64(N, 64), cdiv64(M, 64)));
  }
  add_launch(P, seq, K_GBUILD, ST_GBUILD, js);
}

// Class (0,2): order the strings of each occupation category by the set of
// active pairs they couple through, then cut them into tiles of at most
// kStrTile consecutive strings of one category.  A tile's support is the
// union of its strings' pairs; its coefficients form a dense [tile][support]
// block whose product with the pair integrals is one small complex GEMM.
// Returns false (generic kernel) if some string has no coupling.
bool tile_by_support(InstancePlan& ip, ClassPlan& cp, const std::vector<int>& ss, const std::vector<int>& off) {
  const size_t S = cp.strings.size();
  auto category = [&](uint64_t al) {
    std::vector<int> m(ss.size());
    for (size_t q = 0; q < ss.size(); ++q)
      m[q] = popc((al >> off[q]) & (ss[q] >= 64 ? ~0ull : (1ull << ss[q]) - 1));
    return m;
  };
  std::vector<std::pair<std::vector<int>, std::vector<int>>> key(S);
  for (size_t s = 0; s < S; ++s) {
    key[s].first = category(cp.strings[s]);
    for (int e = cp.conn_ptr[s]; e < cp.conn_ptr[s + 1]; ++e) {
      const Pattern& p = cp.patterns[cp.conn[2 * e + 1]];
      key[s].second.push_back(p.a0 * 64 + p.a1);
    }
    if (key[s].second.empty()) return false;
    std::sort(key[s].second.begin(), key[s].second.end());
  }
  std::vector<size_t> ord(S);
  for (size_t s = 0; s < S; ++s) ord[s] = s;
  std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return key[x] < key[y]; });
  std::vector<uint64_t> sorted(S);
  std::vector<std::vector<int>> cat(S);
  for (size_t s = 0; s < S; ++s) {
    sorted[s] = cp.strings[ord[s]];
    cat[s] = key[ord[s]].first;
  }
  cp.strings.swap(sorted);
  cp.patterns.clear();
  cp.conn.clear();
  cp.conn_ptr.clear();
  build_class(ip, cp);
  cp.tile_s0.assign(1, 0);
  cp.tile_k0.assign(1, 0);
  cp.tile_sup.clear();
  cp.ccol.assign(cp.n_conn, -1);
  std::vector<int32_t> col(cp.patterns.size(), -1);
  size_t s = 0;
  while (s < S) {
    size_t e = s;
    while (e < S && e - s < (size_t)kStrTile && cat[e] == cat[s]) ++e;
    std::vector<int> used;
    for (size_t t = s; t < e; ++t)
      for (int c = cp.conn_ptr[t]; c < cp.conn_ptr[t + 1]; ++c) {
        const int j = cp.conn[2 * c + 1];
        if (col[j] < 0) {
          col[j] = (int32_t)used.size();
          used.push_back(j);
        }
        cp.ccol[c] = col[j];
      }
    for (int j : used) {
      const Pattern& p = cp.patterns[j];
      const int x = ip.n_c + p.a0, y = ip.n_c + p.a1;
      cp.tile_sup.push_back((int32_t)((int64_t)x * ip.n_o - (int64_t)x * (x + 1) / 2 + (y - x - 1)));
      col[j] = -1;
    }
    if (used.size() & 1) cp.tile_sup.push_back(-1);
    cp.tile_s0.push_back((int32_t)e);
    cp.tile_k0.push_back((int32_t)cp.tile_sup.size());
    s = e;
  }
  cp.n_tiles = (int64_t)cp.tile_s0.size() - 1;
  return true;
}

}  // namespace

void build_launches(Plan* P) {
  P->jobs.clear();
  P->energy.clear();
  P->backward.clear();
  P->stats.clear();
  P->reference.clear();
  const int ni = (int)P->inst.size();
  std::vector<int> all(ni);
  for (int i = 0; i < ni; ++i) all[i] = i;
  std::vector<Launch>* seq = &P->energy;
  add_launch(P, seq, K_CLEAR, ST_NONE, {job(0, 1, 1)});
  table_launches(P, seq, all);
  std::vector<JobH> js;
  for (int i : all) {
    const int np = (int)P->inst[i].pstrings.size();
    js.push_back(job(i, cdiv64(np, 16), cdiv64(np, 16)));
  }
  add_launch(P, seq, K_HPP, ST_REF, js, 0, 0);
  js.clear();
  for (int i : all) js.push_back(job(i, (int64_t)P->inst[i].pstrings.size(), 1));
  add_launch(P, seq, K_SIGP, ST_REF, js);
  js.clear();
  for (int i : all) js.push_back(job(i, 1, 1));
  add_launch(P, seq, K_E0, ST_REF, js);
  {
    // FP64: 128 x 128 blocks of virtual pairs where at least 90 % of their
    // waves have a tile to compute (n_tp tiles over 4 n2 (n2 + 1) / 2 wave
    // pairs), else one 64 x 64 tile per block, unless the tuning fixes the
    // block edge; mixed form: its own kernel
    std::vector<JobH> j128, j64, j32;
    for (int i : all) {
      const InstancePlan& ip = P->inst[i];
      if (ip.n_v < 2 || ip.n_pairs == 0) continue;
      const int64_t n2 = (ip.n_vt + 1) / 2, nstp = n2 * (n2 + 1) / 2;
      if (ip.d.precision == MRPT2_MIXED) j32.push_back(job(i, ip.n_tp, ip.n_pairs));
      else if (ip.pair_tile == 128 || (ip.pair_tile == 0 && 10 * ip.n_tp >= 9 * 4 * nstp))
        j128.push_back(job(i, nstp, ip.n_pairs));
      else j64.push_back(job(i, ip.n_tp, ip.n_pairs));
    }
    add_launch(P, seq, K_ABUILD, ST_ABUILD, j128);
    add_launch(P, seq, K_ABUILD64, ST_ABUILD, j64);
    add_launch(P, seq, K_ABUILD32, ST_ABUILD, j32);
  }
  for (int k = 0; k < MRPT2_N_CLASS; ++k) {
    js.clear();
    for (int i : all) {
      const InstancePlan& ip = P->inst[i];
      const ClassPlan& cp = ip.cls[k];
      if (cp.strings.empty() || cp.n_rows == 0) continue;
      js.push_back(job(i, (int64_t)cp.strings.size(), cdiv64(std::max(std::max(ip.n_c, ip.n_v), 1), 256), k));
    }
    add_launch(P, seq, K_CTAB, ST_PREP0 + k, js);
    js.clear();
    for (int i : all) {
      const ClassPlan& cp = P->inst[i].cls[k];
      if (cp.strings.empty() || cp.n_rows == 0 || cp.v == 2 || cp.patterns.empty()) continue;
      js.push_back(job(i, cdiv64(cp.n_rows, 256), (int64_t)cp.patterns.size(), k));
    }
    add_launch(P, seq, K_XBUILD, ST_PREP0 + k, js);
    js.clear();
    for (int i : all) {
      const ClassPlan& cp = P->inst[i].cls[k];
      if ((cp.kernel == KERN_E12 || cp.kernel == KERN_E21) && !cp.strings.empty() && cp.n_rows > 0)
        js.push_back(job(i, cdiv64((int64_t)cp.strings.size(), 256), 1, k));
    }
    add_launch(P, seq, K_DCOEF, ST_PREP0 + k, js);
    js.clear();
    for (int i : all) {
      const ClassPlan& cp = P->inst[i].cls[k];
      if (cp.kernel == KERN_E02 && !cp.strings.empty() && cp.n_rows > 0) js.push_back(job(i, cp.n_tiles, 1, k));
    }
    add_launch(P, seq, K_E02COEF, ST_PREP0 + k, js);
    // sigma: dedicated kernels, then the generic kernel for the rest
    // (index 1 of each pair: the level-shifted variant)
    std::vector<JobH> e22[2], e12[2][5], e12f[5], e21[2][5], e02[2], e02f[2], gen;
    for (int i : all) {
      const InstancePlan& ip = P->inst[i];
      const ClassPlan& cp = ip.cls[k];
      if (cp.strings.empty() || cp.n_rows == 0) continue;
      const int ls = ip.d.level_shift_b != 0.0 ? 1 : 0;
      if (cp.kernel == KERN_E22) {
        e22[ls].push_back(job(i, cp.n_holes, ip.n_tp, k));
      } else if (cp.kernel == KERN_E12) {
        const size_t J = cp.patterns.size();
        const int v = J <= 8 ? 0 : J <= 16 ? 1 : J <= 20 ? 4 : J <= 24 ? 2 : 3;
        (ip.d.precision == MRPT2_MIXED && !ls ? e12f[v] : e12[ls][v]).push_back(job(i, cp.n_holes, ip.n_tp * 8, k));
      } else if (cp.kernel == KERN_E21) {
        const size_t J = cp.patterns.size();
        const int v = J <= 8 ? 0 : J <= 16 ? 1 : J <= 20 ? 2 : J <= 24 ? 3 : 4;
        e21[ls][v].push_back(job(i, cp.n_holes, cdiv64(ip.n_v, 256), k));
      } else if (cp.kernel == KERN_E02) {
        (ip.d.precision == MRPT2_MIXED ? e02f[ls] : e02[ls]).push_back(job(i, cp.n_tiles, ip.n_tp * 64, k));
      } else {
        gen.push_back(job(i, sigma_blocks(ip, k), 1, k));
      }
    }
    add_launch(P, seq, K_E22, ST_SIGMA0 + k, e22[0]);
    add_launch(P, seq, K_E12_8, ST_SIGMA0 + k, e12[0][0]);
    add_launch(P, seq, K_E12_16, ST_SIGMA0 + k, e12[0][1]);
    add_launch(P, seq, K_E12_24, ST_SIGMA0 + k, e12[0][2]);
    add_launch(P, seq, K_E12_32, ST_SIGMA0 + k, e12[0][3]);
    add_launch(P, seq, K_E12_20, ST_SIGMA0 + k, e12[0][4]);
    for (int v = 0; v < 5; ++v) add_launch(P, seq, K_E12F_8 + v, ST_SIGMA0 + k, e12f[v]);
    add_launch(P, seq, K_E02, ST_SIGMA0 + k, e02[0]);
    add_launch(P, seq, K_E02F, ST_SIGMA0 + k, e02f[0]);
    add_launch(P, seq, K_E22S, ST_SIGMA0 + k, e22[1]);
    add_launch(P, seq, K_E12S_8, ST_SIGMA0 + k, e12[1][0]);
    add_launch(P, seq, K_E12S_16, ST_SIGMA0 + k, e12[1][1]);
    add_launch(P, seq, K_E12S_24, ST_SIGMA0 + k, e12[1][2]);
    add_launch(P, seq, K_E12S_32, ST_SIGMA0 + k, e12[1][3]);
    add_launch(P, seq, K_E12S_20, ST_SIGMA0 + k, e12[1][4]);
    add_launch(P, seq, K_E02S, ST_SIGMA0 + k, e02[1]);
    add_launch(P, seq, K_E02FS, ST_SIGMA0 + k, e02f[1]);
    for (int v = 0; v < 5; ++v) {
      add_launch(P, seq, K_E21_8 + v, ST_SIGMA0 + k, e21[0][v]);
      add_launch(P, seq, K_E21S_8 + v, ST_SIGMA0 + k, e21[1][v]);
    }
    add_launch(P, seq, K_SIG22 + k, ST_SIGMA0 + k, gen);
  }
  js.clear();
  for (int i : all) js.push_back(job(i, 1, 1));
  add_launch(P, seq, K_FINISH, ST_FINISH, js);
  // denominator statistics: the forward tables up to the per-string
  // denominator tables (no pair integrals, no sigma), one pass per class,
  // then the fold per instance
  seq = &P->stats;
  for (const Launch& L : P->energy)
    if (L.stage == ST_NONE || L.stage == ST_TABLES || L.stage == ST_GBUILD || L.stage == ST_REF ||
        L.kid == K_CTAB)
      seq->push_back(L);
  for (int k = 0; k < MRPT2_N_CLASS; ++k) {
    js.clear();
    for (int i : all) {
      const ClassPlan& cp = P->inst[i].cls[k];
      if (cp.n_dstat > 0) js.push_back(job(i, cdiv64(cp.n_rows, 256), cp.dstat_chunks, k));
    }
    add_launch(P, seq, K_DSTAT22 + k, ST_NONE, js);
  }
  js.clear();
  for (int i : all) js.push_back(job(i, 1, 1));
  add_launch(P, seq, K_DSTATFIN, ST_NONE, js);
  // adjoint: clear the gradient workspace, recompute the forward pass, then
  // the per-class passes and the chain back through the tables
  seq = &P->backward;
  js.clear();
  for (int i : all) {
    const int64_t n32 = (int64_t)(P->inst[i].grad_bytes / 32);
    js.push_back(job(i, std::max<int64_t>(1, std::min<int64_t>(cdiv64(n32, 256), 65536)), 1));
  }
  add_launch(P, seq, K_BZERO, ST_BZERO, js);
  // the forward pass without its sigma and E2 kernels: the row passes below
  // recompute every determinant's term and write E2 per block
  for (const Launch& L : P->energy)
    if (!(L.stage >= ST_SIGMA0 && L.stage < ST_SIGMA0 + MRPT2_N_CLASS) && L.kid != K_FINISH) seq->push_back(L);
  js.clear();
  for (int k = 0; k < MRPT2_N_CLASS; ++k)
    for (int i : all) {
      const ClassPlan& cp = P->inst[i].cls[k];
      if (cp.strings.empty() || cp.n_rows == 0 || cp.n_conn == 0) continue;
      js.push_back(job(i, cdiv64(cp.n_conn, 256), 1, k));
    }
  add_launch(P, seq, K_BECOEF, ST_BZERO, js);
  for (int k = 0; k < MRPT2_N_CLASS; ++k) {
    std::vector<JobH> jr, jsr, j22a, j22b, j22w, jt, j12r[6], j12s[5], j02r, j02s, j02w;
    size_t lds = 0, lds12 = 0, lds12w = 0, lds02 = 0;
    for (int i : all) {
      const InstancePlan& ip = P->inst[i];
      const ClassPlan& cp = ip.cls[k];
      if (cp.strings.empty() || cp.n_rows == 0) continue;
      // string tables transposed for the generic string-owned pass of the
      // one-virtual classes (arg 2 k: Uv, 2 k + 1: Uc)
      if (cp.kernel_bwd == KERN_GENERIC && cp.v <= 1) {
        const int64_t sb = cdiv64((int64_t)cp.strings.size(), 32);
        if (cp.v >= 1) jt.push_back(job(i, sb, cdiv64(ip.n_v, 32), 2 * k));
        if (cp.h >= 1) jt.push_back(job(i, sb, cdiv64(ip.n_c, 32), 2 * k + 1));
      }
      if (cp.kernel_bwd == KERN_E22) {
        j22a.push_back(job(i, cp.n_holes, ip.n_tp, k));
        j22b.push_back(job(i, cdiv64((int64_t)cp.strings.size(), kB22Threads), cp.parts, k));

        j22w.push_back(job(i, cdiv64((int64_t)ip.n_v * ip.n_a, 256), 1, k));
        continue;
      }
      if (cp.kernel_bwd == KERN_E02) {
        j02r.push_back(job(i, 64 * ip.n_tp, 1, k));
        int64_t nkb = 1;   // the widest tile's support in blocks of 64 columns
        for (int64_t t = 0; t < cp.n_tiles; ++t) nkb = std::max<int64_t>(nkb, cdiv64(cp.tile_k0[t + 1] - cp.tile_k0[t], 64));
        j02s.push_back(job(i, nkb * cp.n_tiles, cp.parts, k));
        const int64_t vb = cdiv64(ip.n_v, 256);
        j02w.push_back(job(i, vb, std::min<int64_t>((int64_t)cp.strings.size(), cdiv64(1024, vb)), k));
        lds02 = std::max(lds02, (size_t)ip.n_a * 256 * 8);
        continue;
      }
      if (cp.kernel_bwd == KERN_E12) {
        const size_t J = cp.patterns.size();
        const int v = J <= 8 ? 0 : J <= 16 ? 1 : J <= 24 ? 2 : 3;
        const int vs = (J > 16 && J <= 20) ? 4 : v;
        // + a row for padding adds; the 20-pattern row pass takes 64-string
        // chunks (about 40 KB of static LDS) where its spinor sums leave room
        const size_t ly = (size_t)(ip.n_a + 1) * 256 * 8;
        const bool wide_chunk = vs == 4 && ly + 40960 <= 160 * 1024;
        j12r[wide_chunk ? 5 : vs].push_back(job(i, cp.n_holes, ip.n_tp * 16, k));
        (wide_chunk ? lds12w : lds12) = std::max(wide_chunk ? lds12w : lds12, ly);
        j12s[vs].push_back(job(i, cdiv64((int64_t)cp.strings.size(), 256), cp.parts, k));
        continue;
      }
      jr.push_back(job(i, cdiv64(cp.n_rows, 256), cp.row_split, k));
      jsr.push_back(job(i, cdiv64((int64_t)cp.strings.size(), 256), cp.parts, k));
      lds = std::max(lds, (size_t)ip.n_a * 256 * 8);
    }
    add_launch(P, seq, K_BTRANS, ST_BSTR0 + k, jt);
    add_launch(P, seq, K_B22A, ST_BROW0 + k, j22a);
    add_launch(P, seq, K_B22B, ST_BSTR0 + k, j22b);
    add_launch(P, seq, K_B22WR, ST_BSTR0 + k, j22w);
    for (int v = 0; v < 4; ++v) {
      add_launch(P, seq, K_B12R_8 + v, ST_BROW0 + k, j12r[v], lds12);
      add_launch(P, seq, K_B12S_8 + v, ST_BSTR0 + k, j12s[v]);
    }
    add_launch(P, seq, K_B12R_20, ST_BROW0 + k, j12r[4], lds12);
    add_launch(P, seq, K_B12R_20W, ST_BROW0 + k, j12r[5], lds12w);
    add_launch(P, seq, K_B12S_20, ST_BSTR0 + k, j12s[4]);
    add_launch(P, seq, K_B02R, ST_BROW0 + k, j02r);
    add_launch(P, seq, K_B02S, ST_BSTR0 + k, j02s);
    add_launch(P, seq, K_B02W, ST_BSTR0 + k, j02w, lds02);
    add_launch(P, seq, K_BROW22 + k, ST_BROW0 + k, jr, lds);
    {
      std::vector<JobH> jx;
      for (int i : all) {
        const ClassPlan& cp = P->inst[i].cls[k];
        if (cp.xb_private && !cp.strings.empty() && cp.n_rows > 0)
          jx.push_back(job(i, cdiv64((int64_t)cp.patterns.size() * cp.n_rows, 256), 1, k));
      }
      add_launch(P, seq, K_BXBRED, ST_BROW0 + k, jx);
    }
    add_launch(P, seq, K_BSTR22 + k, ST_BSTR0 + k, jsr);
  }
  for (int k = 0; k < MRPT2_N_CLASS; ++k) {
    js.clear();
    std::vector<JobH> j22;
    for (int i : all) {
      const ClassPlan& cp = P->inst[i].cls[k];
      if (cp.strings.empty() || cp.n_rows == 0) continue;
      if (cp.kernel_bwd == KERN_E22) j22.push_back(job(i, cdiv64((int64_t)cp.strings.size(), 256), 1, k));
      else js.push_back(job(i, cdiv64(std::max<int64_t>((int64_t)cp.strings.size(), cp.n_conn), 256), 1, k));
    }
    add_launch(P, seq, K_B22FIN, ST_BFIN, j22);
    add_launch(P, seq, K_BSFIN, ST_BFIN, js);
  }
  js.clear();
  for (int i : all) js.push_back(job(i, 1, 1));
  add_launch(P, seq, K_FINISH, ST_BFIN, js);   // E2 of the row passes' block sums
  js.clear();
  for (int i : all) {
    const int np = (int)P->inst[i].pstrings.size();
    js.push_back(job(i, cdiv64(np, 16), cdiv64(np, 16)));
  }
  add_launch(P, seq, K_BHPP, ST_BHPP, js);
  js.clear();
  for (int k = 0; k < MRPT2_N_CLASS; ++k)
    for (int i : all) {
      const ClassPlan& cp = P->inst[i].cls[k];
      if (cp.strings.empty() || cp.n_rows == 0 || cp.v == 2 || cp.patterns.empty()) continue;
      js.push_back(job(i, cdiv64(cp.n_rows, 256), (int64_t)cp.patterns.size(), k));
    }
  add_launch(P, seq, K_BXB, ST_BXB, js);
  // pair-integral adjoint GEMM: FP64 (128 x 128 blocks for large n_v and
  // N_L, else 64 x 64), or FP32 (Gauss) in the mixed form
  {
    std::vector<JobH> j64, j128, j32;
    for (int i : all) {
      const InstancePlan& ip = P->inst[i];
      if (ip.n_v < 2 || ip.n_o < 2) continue;
      if (ip.d.precision == MRPT2_MIXED) j32.push_back(job(i, cdiv64(ip.n_l, 64), cdiv64(ip.n_v, 64) * ip.n_o));
      else if (ip.n_v >= 512 && ip.n_l >= 512)
        j128.push_back(job(i, cdiv64(ip.n_l, 128), cdiv64(ip.n_vt, 2) * ip.n_o));
      else j64.push_back(job(i, cdiv64(ip.n_l, 64), cdiv64(ip.n_v, 64) * ip.n_o));
    }
    add_launch(P, seq, K_BAG128, ST_BPAIR, j128);
    add_launch(P, seq, K_BAG, ST_BPAIR, j64);
    add_launch(P, seq, K_BAGF, ST_BPAIR, j32);
  }
  for (int which = 0; which < 2; ++which) {
    js.clear();
    for (int i : all) {
      const InstancePlan& ip = P->inst[i];
      if (ip.n_a == 0) continue;
      const int64_t M = (int64_t)ip.n_o * (ip.n_a + ip.n_v), N = (int64_t)ip.n_o * ip.n_a;
      js.push_back(job(i, cdiv64(ip.n_l, 64), cdiv64(which ? N : M, 64), which));
    }
    add_launch(P, seq, K_BGG, ST_BOCC, js);
  }
  js.clear();
  for (int i : all) js.push_back(job(i, P->inst[i].n_occ, P->inst[i].n_corr));
  add_launch(P, seq, K_BFOCK, ST_BTAB, js);
  js.clear();
  for (int i : all) js.push_back(job(i, cdiv64(P->inst[i].n_l, 256), 1));
  add_launch(P, seq, K_BDSUM, ST_BTAB, js);
  js.clear();
  for (int i : all) {
    const InstancePlan& ip = P->inst[i];
    js.push_back(job(i, cdiv64(std::max(ip.n_corr, ip.n_a + ip.n_v), 256), 1 + ip.n_o));
  }
  add_launch(P, seq, K_BHFE, ST_BTAB, js);
  js.clear();
  for (int i : all) js.push_back(job(i, cdiv64(P->inst[i].n, 256), P->inst[i].n));
  add_launch(P, seq, K_BWSYM, ST_BTAB, js);
  js.clear();
  for (int i : all) js.push_back(job(i, cdiv64(P->inst[i].n, 256), P->inst[i].n_l));
  add_launch(P, seq, K_BDG, ST_BTAB, js);
  js.clear();
  for (int i : all) {
    const InstancePlan& ip = P->inst[i];
    const int64_t nt = cdiv64(ip.n, 32);
    for (int t = 0; t < ip.d.n_sets; ++t)
      if (ip.d.rank[t] > 0) js.push_back(job(i, nt, nt * ip.d.rank[t], t));
  }
  add_launch(P, seq, K_BDB, ST_BOUT, js);
  js.clear();
  for (int i : all) js.push_back(job(i, cdiv64(P->inst[i].n, 256), P->inst[i].n));
  add_launch(P, seq, K_BDH, ST_BOUT, js);
  js.clear();
  for (int i : all) js.push_back(job(i, cdiv64((int64_t)P->inst[i].pstrings.size(), 256), 1));
  add_launch(P, seq, K_BDC, ST_BOUT, js);
  // reference Hamiltonian of one instance: its tables and H_PP
  P->reference.resize(ni);
  for (int i = 0; i < ni; ++i) {
    std::vector<Launch>* r = &P->reference[i];
    add_launch(P, r, K_CLEAR, ST_NONE, {job(0, 1, 1)});
    table_launches(P, r, {i});
    const int np = (int)P->inst[i].pstrings.size();
    add_launch(P, r, K_HPP, ST_REF, {job(i, cdiv64(np, 16), cdiv64(np, 16))}, 0, 1);
  }
  // the same tables without H_PP (the direct sigma-build in P)
  P->reference_tables.resize(ni);
  for (int i = 0; i < ni; ++i) {
    std::vector<Launch>* r = &P->reference_tables[i];
    add_launch(P, r, K_CLEAR, ST_NONE, {job(0, 1, 1)});
    table_launches(P, r, {i});
  }
}

void class_block(const InstancePlan& ip, int k, int64_t b, mrpt2_block* o) {
  const ClassPlan& cp = ip.cls[k];
  std::memset(o, 0, sizeof(*o));
  const int64_t S = (int64_t)cp.strings.size();
  o->s_lo = 0;
  o->s_hi = S;
  auto set_holes = [&](int64_t hidx) {
    o->n_holes = cp.h;
    if (cp.h == 1) o->hole[0] = (int)hidx;
    if (cp.h == 2) {
      o->hole[0] = ip.hole_pairs[2 * hidx];
      o->hole[1] = ip.hole_pairs[2 * hidx + 1];
    }
  };
  auto clampv = [&](int x) { return std::min(std::max(x, 0), ip.n_v); };
  o->kind = 0;
  if (cp.kernel == KERN_E22) {
    const int64_t hp = b / ip.n_tp, tp = b % ip.n_tp;
    set_holes(hp);
    const int I = ip.tile_pairs[2 * tp], J = ip.tile_pairs[2 * tp + 1];
    o->a_lo = clampv(I * 64); o->a_hi = clampv(I * 64 + 64);
    o->b_lo = clampv(J * 64); o->b_hi = clampv(J * 64 + 64);
    return;
  }
  if (cp.kernel == KERN_E12) {
    const int64_t c = b / (ip.n_tp * 16), r = b % (ip.n_tp * 16);
    const int64_t tp = r / 16;
    const int sub = (int)(r % 16), sa = sub >> 2, sb = sub & 3;
    set_holes(c);
    const int I = ip.tile_pairs[2 * tp], J = ip.tile_pairs[2 * tp + 1];
    o->a_lo = clampv(I * 64 + sa * 16); o->a_hi = clampv(I * 64 + sa * 16 + 16);
    o->b_lo = clampv(J * 64 + sb * 16); o->b_hi = clampv(J * 64 + sb * 16 + 16);
    return;
  }
  if (cp.kernel == KERN_E21) {
    const int64_t hp = b % cp.n_holes, at = b / cp.n_holes;
    set_holes(hp);
    o->a_lo = clampv((int)(at * 256));
    o->a_hi = clampv((int)(at * 256 + 256));
    return;
  }
  if (cp.kernel == KERN_E02) {
    const int64_t t = b % cp.n_tiles, rc = b / cp.n_tiles;
    const int64_t tp = rc >> 6;
    const int la = (int)(rc & 63);
    set_holes(0);
    const int I = ip.tile_pairs[2 * tp], J = ip.tile_pairs[2 * tp + 1];
    o->a_lo = clampv(I * 64 + la); o->a_hi = clampv(I * 64 + la + 1);
    o->b_lo = clampv(J * 64); o->b_hi = clampv(J * 64 + 64);
    o->s_lo = cp.tile_s0[t];
    o->s_hi = cp.tile_s0[t + 1];
    return;
  }
  // generic kernel: rows x string chunk
  const int64_t rb = (cp.n_rows + 255) / 256;
  const int64_t nsc = rb > 0 ? sigma_blocks(ip, k) / rb : 1;
  const int64_t rbi = b / nsc, sc = b % nsc;
  const int64_t chunk = (S + nsc - 1) / nsc;
  o->s_lo = std::min(S, sc * chunk);
  o->s_hi = std::min(S, o->s_lo + chunk);
  const int64_t r0 = rbi * 256, r1 = std::min(cp.n_rows, r0 + 256);
  if (cp.v == 2) {
    const int64_t per = ip.n_tp * 4096;
    const int64_t hole = r0 / per, rab = r0 % per, tp = rab >> 12;
    const int la = (int)((rab >> 6) & 63);
    set_holes(hole);
    const int I = ip.tile_pairs[2 * tp], J = ip.tile_pairs[2 * tp + 1];
    o->a_lo = clampv(I * 64 + la); o->a_hi = clampv(I * 64 + la + 4);
    o->b_lo = clampv(J * 64); o->b_hi = clampv(J * 64 + 64);
    return;
  }
  o->kind = 1;
  o->row_lo = r0;
  o->row_hi = r1;
}

mrpt2_status build_plan(const mrpt2_desc* dd, int n_inst, const mrpt2_tuning* tuning, Plan* out,
                        std::string* err) {
  if (!dd || n_inst < 1 || !out) {
    *err = "null argument or n_inst < 1";
    return MRPT2_ERR_ARG;
  }
  out->inst.clear();
  out->inst.resize(n_inst);
  size_t pers = 0, work = 0, grad = 0;
  for (int ii = 0; ii < n_inst; ++ii) {
    const mrpt2_desc& d = dd[ii];
    InstancePlan& ip = out->inst[ii];
    ip.d = d;
    if (d.n_sub < 0 || d.n_sub > MRPT2_MAX_SUB || d.n_sets < 1 || d.n_sets > MRPT2_MAX_SETS ||
        d.n_frozen_core < 0 || d.n_core < 0 || d.n_virt < 0 || d.n_act_elec < 0 || d.max_hops < 0 ||
        (d.q_mode != 0 && d.q_mode != 1)) {
      *err = "descriptor field out of range";
      return MRPT2_ERR_ARG;
    }
    if (d.precision != MRPT2_FP64 && d.precision != MRPT2_MIXED) {
      *err = "unknown precision";
      return MRPT2_ERR_UNSUPPORTED;
    }
    if (d.layout != MRPT2_LAYOUT_FULL && d.layout != MRPT2_LAYOUT_PACKED) {
      *err = "unknown factor layout";
      return MRPT2_ERR_UNSUPPORTED;
    }
    if (!std::isfinite(d.level_shift_b)) {
      *err = "level shift b must be finite";
      return MRPT2_ERR_ARG;
    }
    ip.n_fc = d.n_frozen_core;
    ip.n_c = d.n_core;
    ip.n_v = d.n_virt;
    ip.n_e = d.n_act_elec;
    ip.n_a = 0;
    std::vector<int> ss, off;
    int basesum = 0;
    for (int k = 0; k < d.n_sub; ++k) {
      if (d.sub_size[k] < 1 || d.sub_base[k] < 0 || d.sub_base[k] > d.sub_size[k]) {
        *err = "bad subspace size or base occupation";
        return MRPT2_ERR_SHAPE;
      }
      off.push_back(ip.n_a);
      ss.push_back(d.sub_size[k]);
      ip.n_a += d.sub_size[k];
      basesum += d.sub_base[k];
    }
    if (ip.n_a > kMaxAct || ip.n_e > ip.n_a || basesum != ip.n_e) {
      *err = "active space inconsistent (electrons, base occupations or > 64 spinors)";
      return MRPT2_ERR_SHAPE;
    }
    ip.n_l = 0;
    for (int t = 0; t < d.n_sets; ++t) {
      if (d.rank[t] < 0 || !std::isfinite(d.weight[t])) {
        *err = "bad factor set";
        return MRPT2_ERR_ARG;
      }
      for (int l = 0; l < d.rank[t]; ++l) {
        ip.set_sign.push_back(d.weight[t] < 0 ? -1.0 : 1.0);
        ip.set_scale.push_back(std::sqrt(std::fabs(d.weight[t])));
      }
      ip.n_l += d.rank[t];
    }
    if (ip.n_l < 1) {
      *err = "no Cholesky vectors";
      return MRPT2_ERR_SHAPE;
    }
    ip.n_o = ip.n_c + ip.n_a;
    ip.n_occ = ip.n_fc + ip.n_o;
    ip.n_corr = ip.n_o + ip.n_v;
    ip.n = ip.n_fc + ip.n_corr;
    // primary space (Sec. 2.4)
    std::vector<std::vector<int>> cats;
    categories(ss, ip.n_e, &cats);
    for (auto& m : cats) {
      int hops = 0;
      for (int k = 0; k < d.n_sub; ++k) hops += std::max(0, m[k] - d.sub_base[k]);
      if (hops <= d.max_hops) ip.pcats.push_back(m);
    }
    for (auto& m : ip.pcats) category_strings(ss, off, m, &ip.pstrings);
    if (ip.pstrings.empty() || ip.pstrings.size() >= (1u << 24)) {
      *err = "reference space empty or too large";
      return MRPT2_ERR_SHAPE;
    }
    for (size_t i = 0; i < ip.pstrings.size(); ++i) ip.pindex[ip.pstrings[i]] = (int32_t)i;
    // excitation lists of the reference space: for every reference string,
    // the reference strings reached from it by one or two replacements of
    // active spinors, in ascending order (the off-diagonal couplings of H_PP,
    // which the sigma-build in P applies without storing H_PP)
    {
      const uint64_t act = ip.n_a >= 64 ? ~0ull : ((1ull << ip.n_a) - 1);
      ip.plist_ptr.assign(1, 0);
      std::vector<int> occ, emp;
      std::vector<int32_t> row;
      for (size_t i = 0; i < ip.pstrings.size(); ++i) {
        const uint64_t b = ip.pstrings[i];
        occ.clear();
        emp.clear();
        for (int t = 0; t < ip.n_a; ++t) (b >> t & 1 ? occ : emp).push_back(t);
        row.clear();
        auto add = [&](uint64_t bj) {
          auto it = ip.pindex.find(bj & act);
          if (it != ip.pindex.end()) row.push_back(it->second);
        };
        for (int q : occ)
          for (int p : emp) add(b ^ (1ull << q) ^ (1ull << p));
        for (size_t x = 0; x < occ.size(); ++x)
          for (size_t y = x + 1; y < occ.size(); ++y)
            for (size_t u = 0; u < emp.size(); ++u)
              for (size_t w = u + 1; w < emp.size(); ++w)
                add(b ^ (1ull << occ[x]) ^ (1ull << occ[y]) ^ (1ull << emp[u]) ^ (1ull << emp[w]));
        std::sort(row.begin(), row.end());
        ip.plist_col.insert(ip.plist_col.end(), row.begin(), row.end());
        ip.plist_ptr.push_back((int64_t)ip.plist_col.size());
      }
    }
    // external space by class: level = v + min over P categories of the
    // surplus sum_k max(0, m_k - m'_k) must not exceed 2
    int64_t n_ext = 0;
    if (tuning) {
      const int pt = tuning[ii].pair_tile;
      if (pt != 0 && pt != 64 && pt != 128) {
        *err = "pair_tile must be 0, 64 or 128";
        return MRPT2_ERR_ARG;
      }
      ip.pair_tile = pt;
    }
    for (int k = 0; k < MRPT2_N_CLASS; ++k) {
      ClassPlan& cp = ip.cls[k];
      cp.h = kClassH[k];
      cp.v = kClassV[k];
      if (tuning) {
        const mrpt2_tuning& tu = tuning[ii];
        if (tu.sigma_blocks[k] < 0 || tu.bwd_blocks[k] < 0 || tu.bwd_row_blocks[k] < 0) {
          *err = "negative launch-shape target";
          return MRPT2_ERR_ARG;
        }
        cp.sigma_target = tu.sigma_blocks[k];
        cp.bwd_target = tu.bwd_blocks[k];
        cp.bwd_row_target = tu.bwd_row_blocks[k];
      }
      const int ne = ip.n_e + cp.h - cp.v;
      if (ne < 0 || ne > ip.n_a || cp.h > ip.n_c || cp.v > ip.n_v) continue;
      if (cp.h == 0 && cp.v == 0 && d.q_mode == 1) continue;
      std::vector<std::vector<int>> cc;
      categories(ss, ne, &cc);
      for (auto& m : cc) {
        int best = 1 << 30;
        bool inP = false;
        for (auto& mp : ip.pcats) {
          int sur = 0;
          for (int q = 0; q < d.n_sub; ++q) sur += std::max(0, m[q] - mp[q]);
          best = std::min(best, sur);
          if (m == mp) inP = true;
        }
        if (cp.v + best > 2) continue;
        if (cp.h == 0 && cp.v == 0 && inP) continue;
        category_strings(ss, off, m, &cp.strings);
      }
      cp.n_holes = binom(ip.n_c, cp.h);
      cp.n_ext = cp.n_holes * binom(ip.n_v, cp.v) * (int64_t)cp.strings.size();
      n_ext += cp.n_ext;
      if (!cp.strings.empty()) build_class(ip, cp);
      if ((k == 1 || k == 3) && !cp.strings.empty() && cp.patterns.size() <= (size_t)kMaxDenseJ)
        sort_by_pattern_mask(ip, cp);
      if (k == 2 && !cp.strings.empty() && !tile_by_support(ip, cp, ss, off)) {
        cp.n_tiles = 0;
        cp.tile_s0.clear();
        cp.tile_k0.clear();
        cp.tile_sup.clear();
        cp.ccol.clear();
      }
    }
    // the (2,2) class walks the reference strings themselves
    if (!ip.cls[0].strings.empty() && ip.cls[0].strings != ip.pstrings) {
      *err = "internal: (2,2) strings differ from the reference strings";
      return MRPT2_ERR_SHAPE;
    }
    // tiles of virtual pairs
    ip.n_vt = (ip.n_v + kTile - 1) / kTile;
    for (int I = 0; I < ip.n_vt; ++I)
      for (int J = I; J < ip.n_vt; ++J) {
        ip.tile_pairs.push_back(I);
        ip.tile_pairs.push_back(J);
      }
    ip.n_tp = (int64_t)ip.tile_pairs.size() / 2;
    for (int c = 0; c < ip.n_c; ++c)
      for (int c2 = c + 1; c2 < ip.n_c; ++c2) {
        ip.hole_pairs.push_back(c);
        ip.hole_pairs.push_back(c2);
      }
    ip.n_pairs = (int64_t)ip.n_o * (ip.n_o - 1) / 2;
    for (int k = 0; k < MRPT2_N_CLASS; ++k) {
      ClassPlan& cp = ip.cls[k];
      if (cp.v == 2) cp.n_rows = cp.n_holes * ip.n_tp * kTile * kTile;
      else if (cp.v == 1) cp.n_rows = cp.n_holes * ip.n_v;
      else cp.n_rows = cp.n_holes;
      if (cp.strings.empty()) cp.n_rows = 0;
    }
    // ---- persistent layout (plan tables) ----
    Layout P;
    ip.off_pstrings = P.take(ip.pstrings.size() * 8);
    ip.off_plist_ptr = P.take(ip.plist_ptr.size() * 8);
    ip.off_plist_col = P.take(std::max<size_t>(ip.plist_col.size(), 1) * 4);
    ip.off_hole_pairs = P.take(std::max<size_t>(ip.hole_pairs.size(), 2) * 4);
    ip.off_tile_pairs = P.take(std::max<size_t>(ip.tile_pairs.size(), 2) * 4);
    ip.off_sign = P.take(ip.n_l * 8);
    ip.off_scale = P.take(ip.n_l * 8);
    for (int k = 0; k < MRPT2_N_CLASS; ++k) {
      ClassPlan& cp = ip.cls[k];
      cp.off_strings = P.take(cp.strings.size() * 8);
      cp.off_conn_ptr = P.take(cp.conn_ptr.size() * 4);
      cp.off_conn = P.take(cp.conn.size() * 4);
      cp.off_pat = P.take(cp.patterns.size() * sizeof(Pattern));
      // coupling keys: the pattern index (v < 2), or the part of the pair
      // integral's occupied pair that the pattern fixes (v = 2: none with two
      // core holes, the active spinor with one, the active pair with none)
      cp.ekey.resize(cp.n_conn);
      for (int64_t e = 0; e < cp.n_conn; ++e) {
        const int j = cp.conn[2 * e + 1];
        const Pattern& pt = cp.patterns[j];
        int32_t key = j;
        if (cp.v == 2) {
          if (cp.h == 2) key = 0;
          else if (cp.h == 1) key = pt.a0;
          else {
            const int x = ip.n_c + pt.a0, y = ip.n_c + pt.a1;
            key = (int32_t)((int64_t)x * ip.n_o - (int64_t)x * (x + 1) / 2 + (y - x - 1));
          }
        }
        cp.ekey[e] = key | (cp.conn[2 * e] < 0 ? (int32_t)0x80000000 : 0);
      }
      cp.off_ekey = P.take(cp.ekey.size() * 4);
      cp.off_tile_s0 = P.take(cp.tile_s0.size() * 4);
      cp.off_tile_k0 = P.take(cp.tile_k0.size() * 4);
      cp.off_tile_sup = P.take(cp.tile_sup.size() * 4);
      cp.off_ccol = P.take(cp.ccol.size() * 4);
    }
    ip.persistent_bytes = P.cur;
    ip.host_blob.assign(ip.persistent_bytes, 0);
    auto put = [&](size_t o, const void* src, size_t bytes) {
      if (bytes) std::memcpy(ip.host_blob.data() + o, src, bytes);
    };
    put(ip.off_pstrings, ip.pstrings.data(), ip.pstrings.size() * 8);
    put(ip.off_plist_ptr, ip.plist_ptr.data(), ip.plist_ptr.size() * 8);
    put(ip.off_plist_col, ip.plist_col.data(), ip.plist_col.size() * 4);
    put(ip.off_hole_pairs, ip.hole_pairs.data(), ip.hole_pairs.size() * 4);
    put(ip.off_tile_pairs, ip.tile_pairs.data(), ip.tile_pairs.size() * 4);
    put(ip.off_sign, ip.set_sign.data(), ip.n_l * 8);
    put(ip.off_scale, ip.set_scale.data(), ip.n_l * 8);
    for (int k = 0; k < MRPT2_N_CLASS; ++k) {
      ClassPlan& cp = ip.cls[k];
      put(cp.off_strings, cp.strings.data(), cp.strings.size() * 8);
      put(cp.off_conn_ptr, cp.conn_ptr.data(), cp.conn_ptr.size() * 4);
      put(cp.off_conn, cp.conn.data(), cp.conn.size() * 4);
      put(cp.off_pat, cp.patterns.data(), cp.patterns.size() * sizeof(Pattern));
      put(cp.off_ekey, cp.ekey.data(), cp.ekey.size() * 4);
      put(cp.off_tile_s0, cp.tile_s0.data(), cp.tile_s0.size() * 4);
      put(cp.off_tile_k0, cp.tile_k0.data(), cp.tile_k0.size() * 4);
      put(cp.off_tile_sup, cp.tile_sup.data(), cp.tile_sup.size() * 4);
      put(cp.off_ccol, cp.ccol.data(), cp.ccol.size() * 4);
    }
    // ---- workspace layout ----
    Layout W;
    const size_t NP = ip.pstrings.size();
    ip.off_dg = W.take((size_t)ip.n_l * ip.n * 8);
    ip.off_slab = W.take((size_t)ip.n_occ * ip.n_corr * ip.n_l * 16);
    ip.off_slab32 = W.take((ip.d.precision == MRPT2_MIXED && ip.n_v >= 2)
                               ? (size_t)ip.n_o * ip.n_v * (ip.n_l + (ip.n_l & 1)) * 8 : 0);
    ip.off_W = W.take((size_t)ip.n * ip.n * 8);
    ip.off_eps = W.take((size_t)ip.n * 8);
    ip.off_f = W.take((size_t)(ip.n_a + ip.n_v) * ip.n_o * 16);
    ip.off_fx = W.take((size_t)(ip.n_fc + ip.n_c) * (ip.n_a + ip.n_v) * ip.n_o * 16);
    ip.off_G = W.take((size_t)ip.n_o * (ip.n_a + ip.n_v) * ip.n_o * std::max(ip.n_a, 1) * 16);
    ip.off_A = W.take(ip.n_v >= 2 ? (size_t)ip.n_pairs * ip.n_tp * kTile * kTile * 16 : 0);
    ip.off_hpp = W.take(NP * NP * 16);
    ip.off_sigp = W.take(NP * 16);
    ip.off_scal = W.take(16 * 8);
    ip.off_dsum = W.take((size_t)ip.n_l * 8);
    ip.off_dstat_out = W.take(MRPT2_N_CLASS * 16);
    ip.n_part = 0;
    for (int k = 0; k < MRPT2_N_CLASS; ++k) {
      ClassPlan& cp = ip.cls[k];
      const size_t S = cp.strings.size();
      cp.off_T = W.take(S * 8);
      cp.off_Uc = W.take(cp.h > 0 ? S * ip.n_c * 8 : 0);
      cp.off_Uv = W.take(cp.v > 0 ? S * ip.n_v * 8 : 0);
      cp.off_X = W.take((cp.v < 2 && S) ? (size_t)cp.patterns.size() * cp.n_rows * 16 : 0);
      // denominator statistics: row blocks of 256, strings split into enough
      // chunks for about 4096 blocks
      cp.dstat_chunks = 1;
      cp.n_dstat = 0;
      if (S && cp.n_rows > 0) {
        const int64_t rb = cdiv64(cp.n_rows, 256);
        cp.dstat_chunks = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)S, cdiv64(4096, rb)));
        cp.n_dstat = rb * cp.dstat_chunks;
      }
      cp.off_dstat = W.take((size_t)cp.n_dstat * 16);
      // a level shift changes every denominator: the dedicated forward
      // kernels have shifted variants, the adjoint then runs on the generic
      // passes (the only ones that carry the shifted weight's derivative)
      const bool shifted = ip.d.level_shift_b != 0.0;
      cp.dense_coef = (k == 1 || k == 3) && S && cp.patterns.size() <= (size_t)kMaxDenseJ;
      cp.off_D = W.take(cp.dense_coef ? S * cp.patterns.size() * 16 : 0);
      cp.off_mask = W.take(cp.dense_coef ? S * 4 : 0);
      // kernel choice and partial-sum blocks: the dedicated kernels' grids
      // ((2,2): tile pair x core pair; (1,2): 16 sub-tiles per tile pair x
      // core; (0,2): string tile x 64 rows of a tile pair) or the generic kernel's
      cp.kernel = KERN_GENERIC;
      if (S && cp.n_rows > 0) {
        if (k == 0) cp.kernel = KERN_E22;
        else if (k == 1 && cp.dense_coef) cp.kernel = KERN_E12;
        else if (k == 2 && cp.n_tiles > 0) cp.kernel = KERN_E02;
        else if (k == 3 && cp.dense_coef) cp.kernel = KERN_E21;
      }
      // class (2,1) has no dedicated adjoint: its generic passes serve
      cp.kernel_bwd = (shifted || cp.kernel == KERN_E21) ? KERN_GENERIC : cp.kernel;
      cp.off_Md = W.take(cp.kernel == KERN_E02 ? (size_t)kStrTile * cp.tile_k0.back() * 16 : 0);
      cp.n_blocks = (cp.kernel == KERN_E22)   ? ip.n_tp * cp.n_holes
                    : (cp.kernel == KERN_E12) ? ip.n_tp * 16 * cp.n_holes
                    : (cp.kernel == KERN_E02) ? ip.n_tp * 64 * cp.n_tiles
                    : (cp.kernel == KERN_E21) ? cp.n_holes * cdiv64(ip.n_v, 256)
                                              : sigma_blocks(ip, k);
      ip.n_part_class[k] = cp.n_blocks;
      ip.off_part_class[k] = W.take(std::max<int64_t>(ip.n_part_class[k], 1) * 8);
    }
    ip.workspace_bytes = W.cur;
  }
  // Work of each class's generic adjoint row pass over the whole plan (row
  // blocks x strings): one launch covers every instance, so a batch shares
  // the pass's block target among its instances in proportion to their work
  // instead of giving each instance the whole target.
  int64_t row_blocks[MRPT2_N_CLASS] = {0}, row_work[MRPT2_N_CLASS] = {0};
  for (const InstancePlan& ip : out->inst)
    for (int k = 0; k < MRPT2_N_CLASS; ++k) {
      const ClassPlan& cp = ip.cls[k];
      const int64_t S = (int64_t)cp.strings.size();
      if (S > 0 && cp.n_rows > 0 && cp.kernel_bwd != KERN_E22 && cp.kernel_bwd != KERN_E12 &&
          cp.kernel_bwd != KERN_E02) {
        row_blocks[k] += (cp.n_rows + 255) / 256;
        row_work[k] += (cp.n_rows + 255) / 256 * S;
      }
    }
  for (int ii = 0; ii < n_inst; ++ii) {
    InstancePlan& ip = out->inst[ii];
    const size_t NP = ip.pstrings.size();
    int64_t n_ext = 0;
    for (int k = 0; k < MRPT2_N_CLASS; ++k) n_ext += ip.cls[k].n_ext;
    // ---- gradient workspace layout (adjoint) ----
    Layout Gw;
    ip.off_gs = Gw.take(16 * 8);
    ip.off_Wb = Gw.take((size_t)ip.n * ip.n * 8);
    ip.off_Wsym = Gw.take((size_t)ip.n * ip.n * 8);
    ip.off_epsb = Gw.take((size_t)ip.n_corr * 8);
    ip.off_fb = Gw.take((size_t)(ip.n_a + ip.n_v) * ip.n_o * 16);
    ip.off_Gb = Gw.take((size_t)ip.n_o * (ip.n_a + ip.n_v) * ip.n_o * std::max(ip.n_a, 1) * 16);
    ip.off_Ab = Gw.take(ip.n_v >= 2 ? (size_t)ip.n_pairs * ip.n_tp * kTile * kTile * 16 : 0);
    ip.off_slabb = Gw.take((size_t)ip.n_occ * ip.n_corr * ip.n_l * 16);
    ip.off_dgb = Gw.take((size_t)ip.n_l * ip.n * 8);
    ip.off_dsumb = Gw.take((size_t)ip.n_l * 8);
    ip.off_hb = Gw.take((size_t)ip.n * ip.n * 16);
    ip.off_cb = Gw.take(NP * 16);
    for (int k = 0; k < MRPT2_N_CLASS; ++k) {
      ClassPlan& cp = ip.cls[k];
      const int64_t S = (int64_t)cp.strings.size();
      cp.parts = 1;
      cp.rows_per_part = std::max<int64_t>(cp.n_rows, 1);
      cp.row_split = 1;
      const int64_t bt = cp.bwd_target > 0 ? cp.bwd_target : 2048;
      if (S > 0 && cp.n_rows > 0 && cp.kernel_bwd == KERN_E22) {
        // (2,2) string-owned adjoint kernel (kB22Threads strings per block): parts = groups of core pairs
        const int64_t sblk = (S + kB22Threads - 1) / kB22Threads;
        int64_t parts = std::min<int64_t>(cp.n_holes, std::max<int64_t>(1, (bt + sblk - 1) / sblk));
        parts = std::max<int64_t>(parts, (cp.n_holes + kB22PairsPerPart - 1) / kB22PairsPerPart);
        const int64_t grp = (cp.n_holes + parts - 1) / parts;
        cp.rows_per_part = grp;
        cp.parts = (int)((cp.n_holes + grp - 1) / grp);
      } else if (S > 0 && cp.n_rows > 0 && cp.kernel_bwd == KERN_E12) {
        // (1,2) string pass: parts = core x group of tile pairs
        const int64_t sblk = (S + 255) / 256;
        int64_t ngr = std::min<int64_t>(ip.n_tp, std::max<int64_t>(1, (bt + sblk * cp.n_holes - 1) / (sblk * cp.n_holes)));
        const int64_t tpg = (ip.n_tp + ngr - 1) / ngr;
        ngr = (ip.n_tp + tpg - 1) / tpg;
        cp.rows_per_part = tpg;
        cp.parts = (int)(cp.n_holes * ngr);
      } else if (S > 0 && cp.n_rows > 0 && cp.kernel_bwd == KERN_E02) {
        // (0,2) string pass: parts = groups of (tile pair, a) rows, enough
        // (string tile, part) blocks to fill the device
        const int64_t nrow = 64 * ip.n_tp;
        const int64_t parts = std::min<int64_t>(nrow, std::max<int64_t>(1, (bt + cp.n_tiles - 1) / std::max<int64_t>(cp.n_tiles, 1)));
        cp.rows_per_part = (nrow + parts - 1) / parts;
        cp.parts = (int)((nrow + cp.rows_per_part - 1) / cp.rows_per_part);
      } else if (S > 0 && cp.n_rows > 0) {
        // string-owned pass: enough (string block, row part) blocks to fill the
        // device, partial coupling adjoints bounded to 256 MB
        const int64_t sblk = (S + 255) / 256;
        int64_t parts = std::min<int64_t>(cp.n_rows, std::max<int64_t>(1, (bt + sblk - 1) / sblk));
        parts = std::min<int64_t>(parts, std::max<int64_t>(1, (int64_t)((256ull << 20) / (16 * std::max<int64_t>(cp.n_conn, 1)))));
        cp.rows_per_part = (cp.n_rows + parts - 1) / parts;
        cp.parts = (int)((cp.n_rows + cp.rows_per_part - 1) / cp.rows_per_part);
        // row pass: few rows -> split the strings over blocks as well; the
        // instance takes its share S rb / row_work of the target, so every
        // block of the launch gets about the same number of (row, string)
        // items (a single instance: ceil(target / rb) string chunks)
        const int64_t rt = cp.bwd_row_target > 0 ? cp.bwd_row_target : 2048;
        if (row_blocks[k] < 512)
          cp.row_split = (int)std::min<int64_t>(S, std::max<int64_t>(1, (rt * S + row_work[k] - 1) / row_work[k]));
      }
      cp.off_Xb = Gw.take((cp.v < 2 && S) ? (size_t)cp.patterns.size() * cp.n_rows * 16 : 0);
      // with several string chunks per row block the generic row pass writes
      // each chunk's coupling adjoints into its own slice (plain adds, summed
      // in order afterwards) where that stays within 4 GiB, else it adds them
      // atomically into one array
      const size_t xbp = (size_t)cp.row_split * cp.patterns.size() * (size_t)std::max<int64_t>(cp.n_rows, 0) * 16;
      cp.xb_private = cp.kernel_bwd == KERN_GENERIC && cp.v < 2 && S > 0 && cp.row_split > 1 && xbp <= (4ull << 30);
      cp.off_Xbp = Gw.take(cp.xb_private ? xbp : 0);
      cp.off_Tb = Gw.take((size_t)cp.parts * S * 8);
      const bool b22 = cp.kernel_bwd == KERN_E22, b12 = cp.kernel_bwd == KERN_E12;
      cp.off_cbe = Gw.take((b22 || b12) ? 0 : (size_t)cp.parts * cp.n_conn * 16);
      cp.off_r1 = Gw.take(b22 ? (size_t)cp.parts * S * 8 : 0);
      cp.off_dbp = Gw.take(b12 ? (size_t)cp.parts * S * cp.patterns.size() * 16 : 0);
      cp.off_ecoef = Gw.take((size_t)cp.n_conn * 16);
      cp.off_wpart = Gw.take(b22 ? (size_t)cp.parts * ((S + kB22Threads - 1) / kB22Threads) * ip.n_v * ip.n_a * 8 : 0);
      cp.off_u2 = Gw.take((cp.kernel_bwd == KERN_E02 && S > 0 && cp.n_rows > 0) ? (size_t)cp.parts * S * ip.n_v * 8 : 0);
      // E2 share of every block of the class's row pass
      cp.n_e2part = 0;
      if (S > 0 && cp.n_rows > 0) {
        if (cp.kernel_bwd == KERN_E22) cp.n_e2part = cp.n_holes * ip.n_tp;
        else if (cp.kernel_bwd == KERN_E12) cp.n_e2part = cp.n_holes * 16 * ip.n_tp;
        else if (cp.kernel_bwd == KERN_E02) cp.n_e2part = 64 * ip.n_tp;
        else cp.n_e2part = cdiv64(cp.n_rows, 256) * cp.row_split;
      }
      cp.off_e2part = Gw.take((size_t)cp.n_e2part * 8);
      // string tables transposed for the generic string-owned pass of the
      // one-virtual classes (lanes = strings)
      const bool pass = S > 0 && cp.n_rows > 0 && cp.kernel_bwd == KERN_GENERIC && cp.v <= 1;
      cp.off_UvT = Gw.take((pass && cp.v >= 1) ? (size_t)S * ip.n_v * 8 : 0);
      cp.off_UcT = Gw.take((pass && cp.h >= 1) ? (size_t)S * ip.n_c * 8 : 0);
    }
    ip.grad_bytes = Gw.cur;
    // info
    mrpt2_info& inf = ip.info;
    std::memset(&inf, 0, sizeof(inf));
    inf.n_orb = ip.n;
    inf.n_corr = ip.n_corr;
    inf.n_chol = ip.n_l;
    inf.n_ref = (int64_t)NP;
    inf.n_ext = n_ext;
    inf.n_ref_couplings = (int64_t)ip.plist_col.size();
    double fs = 0;
    for (int k = 0; k < MRPT2_N_CLASS; ++k) {
      const ClassPlan& cp = ip.cls[k];
      inf.n_ext_class[k] = cp.n_ext;
      inf.n_strings_class[k] = (int64_t)cp.strings.size();
      inf.n_conn_class[k] = cp.n_conn;
      inf.n_patterns_class[k] = (int32_t)cp.patterns.size();
      inf.kernel_class[k] = cp.kernel;
      // complex multiply-adds of the sigma contraction: one per coupling and
      // external determinant (nonzero couplings only); the double core ->
      // virtual class has no contraction (sigma = integral x coefficient)
      if (k != 0) fs += 8.0 * (double)cp.n_conn * (double)cp.n_holes * (double)binom(ip.n_v, cp.v);
    }
    inf.flop_sigma = fs;
    const double nv = ip.n_v, nl = ip.n_l;
    inf.flop_integral = 8.0 * (double)ip.n_pairs * nv * (nv - 1) * nl +
                        8.0 * (double)ip.n_o * (ip.n_a + ip.n_v) * ip.n_o * ip.n_a * nl;
    inf.bytes_factors = 16.0 * nl * ip.n * ip.n;
    ip.persistent_base = pers;
    ip.workspace_base = work;
    ip.grad_base = grad;
    pers = align_up(pers + ip.persistent_bytes);
    work = align_up(work + ip.workspace_bytes);
    grad = align_up(grad + ip.grad_bytes);
  }
  out->grad_bytes = grad;
  out->off_flag = work;
  work = align_up(work + 256);
  out->off_insts = work;
  work = align_up(work + kInstBytes * n_inst);
  build_launches(out);
  out->off_jobs = pers;
  pers = align_up(pers + out->jobs.size() * sizeof(JobH));
  out->persistent_bytes = pers;
  out->workspace_bytes = work;
  out->host_blob.assign(pers, 0);
  out->static_stage.assign(kInstBytes * (size_t)n_inst, 0);
  for (auto& ip : out->inst)
    std::memcpy(out->host_blob.data() + ip.persistent_base, ip.host_blob.data(), ip.persistent_bytes);
  if (!out->jobs.empty())
    std::memcpy(out->host_blob.data() + out->off_jobs, out->jobs.data(), out->jobs.size() * sizeof(JobH));
  return MRPT2_OK;
}

}  // namespace mrpt2
