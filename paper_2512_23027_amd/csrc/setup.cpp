// Host-side problem setup (see setup.h).
#include "setup.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>
#include <tuple>

namespace sgw {

// ---------------------------------------------------------------------------
// Hermite chaos (Eq. PCEOrtho with the normalised basis; Eq.
// galerproject_chap2).  Triple products come from the linearisation
// He_a He_b = sum_r C(a,r) C(b,r) r! He_{a+b-2r} and <He_m He_c> = c! d_mc.
// ---------------------------------------------------------------------------
static void gen_level(int L, int pos, int rem, std::vector<int>& a,
                      std::vector<std::vector<int>>& out) {
  if (pos == L - 1) {
    a[pos] = rem;
    out.push_back(a);
    return;
  }
  for (int v = rem; v >= 0; --v) {
    a[pos] = v;
    gen_level(L, pos + 1, rem - v, a, out);
  }
}

static std::vector<std::vector<int>> graded(int L, int p) {
  std::vector<std::vector<int>> out;
  if (L == 0) {
    out.push_back({});
    return out;
  }
  std::vector<int> a(L, 0);
  for (int deg = 0; deg <= p; ++deg) gen_level(L, 0, deg, a, out);
  return out;
}

static double fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

static double binom(int n, int r) {
  double b = 1.0;
  for (int i = 1; i <= r; ++i) b = b * (n - r + i) / i;
  return b;
}

// <psi_a psi_b psi_c> for normalised 1-D Hermite polynomials.
static double triple1(int a, int b, int c) {
  int twice = a + b - c;
  if (twice < 0 || (twice & 1)) return 0.0;
  int r = twice / 2;
  if (r > std::min(a, b)) return 0.0;
  double e = binom(a, r) * binom(b, r) * fact(r) * fact(c);
  return e / std::sqrt(fact(a) * fact(b) * fact(c));
}

Galerkin build_galerkin(int L, int p_in, int p_out) {
  Galerkin g;
  g.L = L;
  g.p_in = p_in;
  g.p_out = p_out;
  g.in_idx = graded(L, p_in);
  g.out_idx = graded(L, p_out);
  g.nk = (int)g.in_idx.size();
  g.P = (int)g.out_idx.size();
  for (int k = 0; k < g.nk; ++k)
    for (int i = 0; i < g.P; ++i)
      for (int j = 0; j < g.P; ++j) {
        double v = 1.0;
        for (int d = 0; d < L && v != 0.0; ++d)
          v *= triple1(g.in_idx[k][d], g.out_idx[i][d], g.out_idx[j][d]);
        if (v != 0.0) {
          g.k.push_back(k);
          g.i.push_back(i);
          g.j.push_back(j);
          g.v.push_back(v);
        }
      }
  return g;
}

// ---------------------------------------------------------------------------
// KLE of the separable exponential kernel (Eq. CovarKer2D_chapt2,
// KLEchapt2): closed-form 1-D eigenpairs on [-a, a], a = 1/2, roots of the
// even / odd transcendental equations found by bisection.
// ---------------------------------------------------------------------------
struct Mode1 {
  double w, lam;
  int odd;
};

static double bisect(double lo, double hi, double c, double a, int odd) {
  auto f = [&](double w) {
    return odd ? w * std::cos(w * a) + c * std::sin(w * a)
               : c * std::cos(w * a) - w * std::sin(w * a);
  };
  double flo = f(lo);
  for (int it = 0; it < 400; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    double fm = f(mid);
    if (fm == 0.0) return mid;
    if ((fm > 0) == (flo > 0)) {
      lo = mid;
      flo = fm;
    } else {
      hi = mid;
    }
  }
  return 0.5 * (lo + hi);
}

static std::vector<Mode1> modes1(double b, int nm) {
  const double a = 0.5, c = 1.0 / b, pi = M_PI;
  std::vector<Mode1> m;
  for (int n = 0; (int)m.size() < nm; ++n) {
    double lo = n * pi / a, mid = lo + pi / (2 * a), hi = (n + 1) * pi / a;
    double w = bisect(lo, mid, c, a, 0);
    m.push_back({w, 2 * c / (w * w + c * c), 0});
    if ((int)m.size() == nm) break;
    w = bisect(mid, hi, c, a, 1);
    m.push_back({w, 2 * c / (w * w + c * c), 1});
  }
  return m;
}

static double phi1(const Mode1& m, double x) {
  const double a = 0.5;
  double t = x - a;
  if (!m.odd) return std::cos(m.w * t) / std::sqrt(a + std::sin(2 * m.w * a) / (2 * m.w));
  return std::sin(m.w * t) / std::sqrt(a - std::sin(2 * m.w * a) / (2 * m.w));
}

// ---------------------------------------------------------------------------
// P1 element matrices (Sec. 2 weak form): stiffness for unit coefficient and
// consistent mass of a triangle.
// ---------------------------------------------------------------------------
static void p1_element(const double* px, const double* py, double ke[3][3],
                       double me[3][3]) {
  double area = 0.5 * ((px[1] - px[0]) * (py[2] - py[0]) -
                       (px[2] - px[0]) * (py[1] - py[0]));
  double gx[3] = {py[1] - py[2], py[2] - py[0], py[0] - py[1]};
  double gy[3] = {px[2] - px[1], px[0] - px[2], px[1] - px[0]};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      ke[a][b] = (gx[a] * gx[b] + gy[a] * gy[b]) / (4 * area);
      me[a][b] = area / 12.0 * (a == b ? 2.0 : 1.0);
    }
}

// slot of neighbour offset (di, dj) in the 7-point pattern of this mesh
static int slot_of(int di, int dj) {
  if (di == 0 && dj == 0) return 0;
  if (di == 1 && dj == 0) return 1;
  if (di == -1 && dj == 0) return 2;
  if (di == 0 && dj == 1) return 3;
  if (di == 0 && dj == -1) return 4;
  if (di == 1 && dj == 1) return 5;
  if (di == -1 && dj == -1) return 6;
  return -1;
}
static const int kDi[7] = {0, 1, -1, 0, 0, 1, -1};
static const int kDj[7] = {0, 0, 0, 1, -1, 1, -1};

// ---------------------------------------------------------------------------
// Nested dissection of a set of grid points: recursive bisection of the
// bounding box by one grid line (a separator for the 7-point pattern, whose
// neighbours differ by at most one in each coordinate).  Points are appended
// in post-order: left part, right part, separator.  Every leaf box and every
// separator becomes one supernode; level = depth below the top call.
// ---------------------------------------------------------------------------
struct Pt {
  int i, j, id;
};
struct SN {
  int beg, w, level;
};

static void nested_dissection(std::vector<Pt> pts, int level,
                              std::vector<int>& order, std::vector<SN>& sns,
                              int leaf) {
  if (pts.empty()) return;
  int imin = 1 << 30, imax = -1, jmin = 1 << 30, jmax = -1;
  for (auto& p : pts) {
    imin = std::min(imin, p.i);
    imax = std::max(imax, p.i);
    jmin = std::min(jmin, p.j);
    jmax = std::max(jmax, p.j);
  }
  auto lex = [](const Pt& a, const Pt& b) {
    return a.j != b.j ? a.j < b.j : a.i < b.i;
  };
  bool splitx = (imax - imin) >= (jmax - jmin);
  int ext = splitx ? imax - imin : jmax - jmin;
  if ((int)pts.size() <= leaf || ext < 2) {
    std::sort(pts.begin(), pts.end(), lex);
    SN s{(int)order.size(), (int)pts.size(), level};
    for (auto& p : pts) order.push_back(p.id);
    sns.push_back(s);
    return;
  }
  int m = splitx ? (imin + imax) / 2 : (jmin + jmax) / 2;
  std::vector<Pt> lo, hi, sep;
  for (auto& p : pts) {
    int c = splitx ? p.i : p.j;
    (c < m ? lo : c > m ? hi : sep).push_back(p);
  }
  nested_dissection(lo, level + 1, order, sns, leaf);
  nested_dissection(hi, level + 1, order, sns, leaf);
  if (!sep.empty()) {
    std::sort(sep.begin(), sep.end(), lex);
    SN s{(int)order.size(), (int)sep.size(), level};
    for (auto& p : sep) order.push_back(p.id);
    sns.push_back(s);
  }
}

// ---------------------------------------------------------------------------
// Sparse Cholesky (up-looking, row by row along the elimination tree) of one
// symmetric block given as adjacency lists (local indices, both triangles).
// Returns false on a non-positive pivot.  L is produced in CSC form with the
// diagonal first in every column.
// ---------------------------------------------------------------------------
struct CSC {
  int n = 0;
  std::vector<int> p, i;
  std::vector<double> x;
};

static bool cholesky(int n, const std::vector<std::vector<std::pair<int, double>>>& A,
                     CSC& L) {
  std::vector<int> parent(n, -1), anc(n, -1);
  for (int k = 0; k < n; ++k)
    for (auto& e : A[k]) {
      int i = e.first;
      while (i != -1 && i < k) {
        int nx = anc[i];
        anc[i] = k;
        if (nx == -1) parent[i] = k;
        i = nx;
      }
    }
  // row patterns (reach of A[0:k, k] in the etree) and column counts
  std::vector<int> mark(n, -1), cnt(n, 1);
  std::vector<std::vector<int>> rowpat(n);
  for (int k = 0; k < n; ++k) {
    mark[k] = k;
    for (auto& e : A[k]) {
      int i = e.first;
      while (i < k && mark[i] != k) {
        mark[i] = k;
        rowpat[k].push_back(i);
        cnt[i]++;
        i = parent[i];
      }
    }
    std::sort(rowpat[k].begin(), rowpat[k].end());
  }
  L.n = n;
  L.p.assign(n + 1, 0);
  for (int j = 0; j < n; ++j) L.p[j + 1] = L.p[j] + cnt[j];
  L.i.assign(L.p[n], 0);
  L.x.assign(L.p[n], 0.0);
  std::vector<int> fill(n);
  for (int j = 0; j < n; ++j) fill[j] = L.p[j] + 1;  // slot 0 = diagonal
  std::vector<double> x(n, 0.0);
  for (int k = 0; k < n; ++k) {
    double d = 0.0;
    for (auto& e : A[k]) {
      if (e.first < k) x[e.first] += e.second;
      else if (e.first == k) d += e.second;
    }
    for (int j : rowpat[k]) {
      double lkj = x[j] / L.x[L.p[j]];
      x[j] = 0.0;
      for (int q = L.p[j] + 1; q < fill[j]; ++q) x[L.i[q]] -= L.x[q] * lkj;
      d -= lkj * lkj;
      L.i[fill[j]] = k;
      L.x[fill[j]] = lkj;
      fill[j]++;
    }
    if (!(d > 0.0)) return false;
    L.i[L.p[k]] = k;
    L.x[L.p[k]] = std::sqrt(d);
  }
  return true;
}

// Append one block's factor to the batched pull-form structure.
static void append_factor(Factor& f, const CSC& L, const std::vector<SN>& sns) {
  int n = L.n;
  int row0 = f.row_off.back();
  f.row_off.push_back(row0 + n);
  f.max_rows = std::max(f.max_rows, n);
  f.nnz_l += L.p[n];
  std::vector<int> sn_of(n);
  int nlev = 0;
  for (size_t s = 0; s < sns.size(); ++s) {
    for (int r = sns[s].beg; r < sns[s].beg + sns[s].w; ++r) sn_of[r] = (int)s;
    nlev = std::max(nlev, sns[s].level + 1);
  }
  f.max_levels = std::max(f.max_levels, nlev);
  // supernodes sorted by level (root level 0 first)
  std::vector<int> ordsn(sns.size());
  std::iota(ordsn.begin(), ordsn.end(), 0);
  std::stable_sort(ordsn.begin(), ordsn.end(),
                   [&](int a, int b) { return sns[a].level < sns[b].level; });
  int sn0 = (int)f.sn_beg.size();
  f.lvl_off.push_back((int)f.lvl_ptr.size() + nlev + 1);
  std::vector<int> lvcount(nlev, 0), lvrows(nlev, 0), lvd(nlev, 0);
  for (auto& s : sns) {
    lvcount[s.level]++;
    lvrows[s.level] += s.w;
    lvd[s.level] += s.w * s.w;
  }
  for (int l = 0; l < nlev; ++l) f.max_lvl_d = std::max(f.max_lvl_d, lvd[l]);
  int acc = sn0;
  for (int l = 0; l < nlev; ++l) {
    f.lvl_ptr.push_back(acc);
    acc += lvcount[l];
    f.max_level_rows = std::max(f.max_level_rows, lvrows[l]);
  }
  f.lvl_ptr.push_back(acc);
  {
    int racc = (int)f.lrow_list.size();
    for (int l = 0; l < nlev; ++l) {
      f.lrow_ptr.push_back(racc);
      racc += lvrows[l];
    }
    f.lrow_ptr.push_back(racc);
    int gsn = sn0;
    for (int s : ordsn) {
      for (int r = sns[s].beg; r < sns[s].beg + sns[s].w; ++r) {
        f.lrow_list.push_back(r);
        f.lrow_sn.push_back(gsn);
      }
      ++gsn;
    }
  }
  for (int s : ordsn) {
    const SN& q = sns[s];
    f.sn_beg.push_back(q.beg);
    f.sn_w.push_back(q.w);
    f.sn_dinv.push_back((int)f.dinv.size());
    f.max_w = std::max(f.max_w, q.w);
    // dense diagonal block and its inverse (lower triangular)
    int w = q.w;
    std::vector<double> D(w * w, 0.0), Inv(w * w, 0.0);
    for (int c = 0; c < w; ++c) {
      int col = q.beg + c;
      for (int t = L.p[col]; t < L.p[col + 1]; ++t) {
        int r = L.i[t];
        if (r < q.beg + w) D[(r - q.beg) * w + c] = L.x[t];
      }
    }
    for (int c = 0; c < w; ++c) {  // solve D Inv[:, c] = e_c
      for (int r = 0; r < w; ++r) {
        double s = (r == c) ? 1.0 : 0.0;
        for (int t = 0; t < r; ++t) s -= D[r * w + t] * Inv[t * w + c];
        Inv[r * w + c] = s / D[r * w + r];
      }
    }
    f.dinv.insert(f.dinv.end(), Inv.begin(), Inv.end());
    for (int c = 0; c < w; ++c)
      for (int r = 0; r < w; ++r) f.dinvT.push_back(Inv[r * w + c]);
  }
  // off-diagonal entries (rows outside the column's supernode), stored in
  // the order of the level lists: position li of the block owns
  // [lr_ptr[li], lr_ptr[li+1]) (its row of L) and [lc_ptr[li], lc_ptr[li+1])
  // (its column of L); indices are block-local rows.
  std::vector<std::vector<std::pair<int, double>>> byrow(n), bycol(n);
  for (int c = 0; c < n; ++c) {
    const SN& q = sns[sn_of[c]];
    for (int t = L.p[c] + 1; t < L.p[c + 1]; ++t) {
      int r = L.i[t];
      if (r >= q.beg + q.w) {
        bycol[c].push_back({r, L.x[t]});
        byrow[r].push_back({c, L.x[t]});
      }
    }
  }
  for (int s : ordsn)
    for (int r = sns[s].beg; r < sns[s].beg + sns[s].w; ++r) {
      for (auto& e : byrow[r]) {
        f.lr_col.push_back(e.first);
        f.lr_val.push_back(e.second);
      }
      f.lr_ptr.push_back((int)f.lr_col.size());
      for (auto& e : bycol[r]) {
        f.lc_row.push_back(e.first);
        f.lc_val.push_back(e.second);
      }
      f.lc_ptr.push_back((int)f.lc_row.size());
    }
  f.max_sn = std::max(f.max_sn, (int)sns.size());
  // lanes per row for the pull phases of each level: a power of two that
  // leaves about four entries per lane for the longest row (0: no entries)
  {
    std::vector<int> mr(nlev, 0), mc(nlev, 0);
    for (size_t s = 0; s < sns.size(); ++s)
      for (int r = sns[s].beg; r < sns[s].beg + sns[s].w; ++r) {
        mr[sns[s].level] = std::max(mr[sns[s].level], (int)byrow[r].size());
        mc[sns[s].level] = std::max(mc[sns[s].level], (int)bycol[r].size());
      }
    // lanes per row: the power of two G that minimises the dependent load
    // rounds ceil(rows G / 1024) * ceil(longest row / (8 G)) of a 1024-thread
    // workgroup issuing eight entry loads per lane at a time
    auto lanes_for = [](int rows, int m) {
      if (m == 0) return 0;
      int best = 1;
      long long bestr = -1;
      for (int g = 1; g <= 64; g *= 2) {
        long long r = ((long long)rows * g + 1023) / 1024 * ((m + 8 * g - 1) / (8 * g));
        if (bestr < 0 || r < bestr) {
          bestr = r;
          best = g;
        }
      }
      return best;
    };
    for (int l = 0; l < nlev; ++l) {
      f.lvl_gf.push_back(lanes_for(lvrows[l], mr[l]));
      f.lvl_gb.push_back(lanes_for(lvrows[l], mc[l]));
    }
    f.lvl_gf.push_back(0);  // keeps the same indexing as lvl_ptr
    f.lvl_gb.push_back(0);
  }
  f.nb++;
}

// ---------------------------------------------------------------------------
// Problem build.
// ---------------------------------------------------------------------------
// Spectral interval [lo, hi] of the Jacobi-scaled mean matrix
// D^{-1/2} K~_0 D^{-1/2} of every block [off[b], off[b+1]) of E (k = 0
// values, slot 0 = diagonal).  hi: the smaller of the Gershgorin bound and
// 1.05 x the largest Ritz value; lo: the smallest Ritz value of a 60-step
// Lanczos run (the Chebyshev preconditioner built from them is SPD for any
// spectrum inside (0, lo + hi), which these bounds always contain).
// Returns false if a block has a non-positive diagonal or couples to a row
// outside itself.
static bool cheb_bounds(const Ell& E, const std::vector<int>& off, std::vector<double>& out) {
  const int nb = (int)off.size() - 1, W = E.W, NR = E.nrows;
  out.assign(2 * (size_t)nb, 0.0);
  for (int b = 0; b < nb; ++b) {
    const int r0 = off[b], n = off[b + 1] - r0;
    if (n <= 0) continue;
    std::vector<double> isd(n);
    for (int r = 0; r < n; ++r) {
      const size_t o = (size_t)r0 + r;
      if (E.col[o] != r0 + r || !(E.val[o] > 0.0)) return false;
      isd[r] = 1.0 / std::sqrt(E.val[o]);
    }
    double gersh = 0.0;
    for (int r = 0; r < n; ++r) {
      double s = 0.0;
      for (int sl = 0; sl < W; ++sl) {
        const size_t o = (size_t)sl * NR + r0 + r;
        const int c = E.col[o] - r0;
        if (c < 0 || c >= n) return false;
        s += std::fabs(E.val[o]) * isd[r] * isd[c];
      }
      gersh = std::max(gersh, s);
    }
    auto matvec = [&](const std::vector<double>& x, std::vector<double>& y) {
      for (int r = 0; r < n; ++r) {
        double s = 0.0;
        for (int sl = 0; sl < W; ++sl) {
          const size_t o = (size_t)sl * NR + r0 + r;
          const int c = E.col[o] - r0;
          s += E.val[o] * isd[r] * isd[c] * x[c];
        }
        y[r] = s;
      }
    };
    // Lanczos with full reorthogonalisation (n ~ 1e3, m = 60)
    const int m = std::min(n, 60);
    std::vector<std::vector<double>> V;
    std::vector<double> al, be;
    std::vector<double> v(n), w(n);
    double nv = 0.0;
    for (int r = 0; r < n; ++r) {
      v[r] = 1.0 + 0.25 * std::sin(0.7 * r + 0.3 * b);
      nv += v[r] * v[r];
    }
    for (auto& x : v) x /= std::sqrt(nv);
    for (int it = 0; it < m; ++it) {
      V.push_back(v);
      matvec(v, w);
      double a = 0.0;
      for (int r = 0; r < n; ++r) a += w[r] * v[r];
      al.push_back(a);
      for (const auto& u : V) {
        double d = 0.0;
        for (int r = 0; r < n; ++r) d += w[r] * u[r];
        for (int r = 0; r < n; ++r) w[r] -= d * u[r];
      }
      double bnorm = 0.0;
      for (double x : w) bnorm += x * x;
      bnorm = std::sqrt(bnorm);
      if (it + 1 == m || bnorm < 1e-12) break;
      be.push_back(bnorm);
      for (int r = 0; r < n; ++r) v[r] = w[r] / bnorm;
    }
    // extreme eigenvalues of the tridiagonal matrix by Sturm bisection
    const int k = (int)al.size();
    auto count_below = [&](double x) {
      int cnt = 0;
      double q = al[0] - x;
      if (q < 0) ++cnt;
      for (int i = 1; i < k; ++i) {
        if (q == 0.0) q = 1e-300;
        q = al[i] - x - be[i - 1] * be[i - 1] / q;
        if (q < 0) ++cnt;
      }
      return cnt;
    };
    auto kth = [&](int idx) {  // idx-th smallest (0-based)
      double lo = -1.0, hi = gersh + 1.0;
      for (int t = 0; t < 200; ++t) {
        double mid = 0.5 * (lo + hi);
        if (count_below(mid) > idx) hi = mid;
        else lo = mid;
      }
      return 0.5 * (lo + hi);
    };
    double tmin = kth(0), tmax = kth(k - 1);
    if (!(tmin > 0.0)) return false;
    out[2 * (size_t)b] = tmin;
    out[2 * (size_t)b + 1] = std::min(gersh, 1.05 * tmax);
  }
  return true;
}

int build_host(const sgw_problem_desc& d, Host& h, std::string& err) {
  h.d = d;
  const int n = d.n;
  if (n < 2 || d.nsx < 1 || d.nsy < 1 || !d.xsplits || !d.ysplits || d.L < 0 ||
      d.p_in < 0 || d.p_out < 0 || !(d.dt > 0) || !(d.zeta > 0) ||
      (d.L > 0 && (!(d.bx > 0) || !(d.by > 0) || d.sigma < 0)) ||
      (d.precond != SGW_PRECOND_NN2 && d.precond != SGW_PRECOND_NN1 &&
       d.precond != SGW_PRECOND_LUMPED)) {
    err = "invalid problem description";
    return SGW_EINVAL;
  }
  h.xs.assign(d.xsplits, d.xsplits + d.nsx + 1);
  h.ys.assign(d.ysplits, d.ysplits + d.nsy + 1);
  for (auto* v : {&h.xs, &h.ys}) {
    if (v->front() != 0 || v->back() != n) {
      err = "splits must start at 0 and end at n";
      return SGW_EINVAL;
    }
    for (size_t q = 1; q < v->size(); ++q)
      if ((*v)[q] < (*v)[q - 1] + 2) {
        err = "every subdomain strip must be at least 2 cells wide";
        return SGW_EINVAL;
      }
  }
  if (d.nsx * d.nsy < 2) {
    err = "at least two subdomains are needed (no interface otherwise)";
    return SGW_EINVAL;
  }
  h.n = n;
  h.nn = (n + 1) * (n + 1);
  const int nsx = d.nsx, nsy = d.nsy;
  h.nsub = nsx * nsy;
  h.g = build_galerkin(d.L, d.p_in, d.p_out);
  const int nk = h.g.nk;
  const double z = d.zeta, gm = d.gamma, dt = d.dt;
  h.a_m = 1.0 / (z * dt * dt) + gm * d.alpha0 / (z * dt);
  h.s_k = 1.0 + gm * d.alpha1 / (z * dt);

  // ----- random field: KLE and log-normal PCE at element centroids -----
  const int ne = 2 * n * n;
  std::vector<double> cx(ne), cy(ne);
  for (int cj = 0; cj < n; ++cj)
    for (int ci = 0; ci < n; ++ci) {
      int e = 2 * (ci + n * cj);
      cx[e] = (ci + 2.0 / 3.0) / n;  // (0,0),(1,0),(1,1)
      cy[e] = (cj + 1.0 / 3.0) / n;
      cx[e + 1] = (ci + 1.0 / 3.0) / n;  // (0,0),(1,1),(0,1)
      cy[e + 1] = (cj + 2.0 / 3.0) / n;
    }
  std::vector<std::vector<double>> gl(d.L, std::vector<double>(ne));
  if (d.L > 0) {
    int nm = d.L + 2;
    auto mx = modes1(d.bx, nm), my = modes1(d.by, nm);
    std::vector<std::tuple<double, int, int>> cand;
    for (int a = 0; a < nm; ++a)
      for (int b = 0; b < nm; ++b)
        cand.emplace_back(-(d.sigma * d.sigma * (mx[a].lam * my[b].lam)), a, b);
    std::sort(cand.begin(), cand.end());
    for (int l = 0; l < d.L; ++l) {
      double lam = -std::get<0>(cand[l]);
      int a = std::get<1>(cand[l]), b = std::get<2>(cand[l]);
      h.kle_lambda.push_back(lam);
      double sl = std::sqrt(lam);
      for (int e = 0; e < ne; ++e) gl[l][e] = sl * phi1(mx[a], cx[e]) * phi1(my[b], cy[e]);
    }
  }
  h.kappa.assign((size_t)nk * ne, 0.0);
  for (int e = 0; e < ne; ++e) {
    double s2 = 0.0;
    for (int l = 0; l < d.L; ++l) s2 += gl[l][e] * gl[l][e];
    double c0 = std::exp(0.5 * s2);  // Eq. LNL0 with g_0 = 0
    for (int k = 0; k < nk; ++k) {
      double v = c0;
      for (int l = 0; l < d.L; ++l) {
        int a = h.g.in_idx[k][l];
        for (int t = 0; t < a; ++t) v *= gl[l][e];
        v /= std::sqrt(fact(a));
      }
      h.kappa[(size_t)k * ne + e] = v;
    }
  }

  // ----- partition: strips containing each grid line -----
  auto strips = [&](const std::vector<int>& cuts, int c, int& s0, int& s1) {
    s0 = -1;
    s1 = -1;
    for (int a = 0; a + 1 < (int)cuts.size(); ++a)
      if (cuts[a] <= c && c <= cuts[a + 1]) {
        if (s0 < 0) s0 = a;
        else s1 = a;
      }
  };
  std::vector<int> mult(h.nn, 0);
  for (int j = 0; j <= n; ++j)
    for (int i = 0; i <= n; ++i) {
      int a0, a1, b0, b1;
      strips(h.xs, i, a0, a1);
      strips(h.ys, j, b0, b1);
      mult[i + (n + 1) * j] = (a1 >= 0 ? 2 : 1) * (b1 >= 0 ? 2 : 1);
    }
  auto is_free = [&](int i, int j) { return i > 0 && i < n && j > 0 && j < n; };
  // corners (cross points of the cut lines) carry the coarse grid of the
  // two-level preconditioner; the one-level variants have none
  const bool two_level = d.precond == SGW_PRECOND_NN2;
  auto is_corner = [&](int v) { return two_level && mult[v] >= 3; };
  // nodes of a subdomain's local (torn) problem of the preconditioner:
  // two-level NN every node but the corners, one-level NN all of them,
  // lumped only the interface nodes (the local interface block K~^s_GG)
  auto in_torn = [&](int v) {
    if (d.precond == SGW_PRECOND_LUMPED) return mult[v] >= 2;
    return !is_corner(v);
  };
  auto cell_sub = [&](int ci, int cj) {
    int a = int(std::upper_bound(h.xs.begin(), h.xs.end(), ci) - h.xs.begin()) - 1;
    int b = int(std::upper_bound(h.ys.begin(), h.ys.end(), cj) - h.ys.begin()) - 1;
    return a + nsx * b;
  };

  // ----- DD numbering: interior blocks (ND order), then interface -----
  const int LEAF = 20;
  h.mesh2dd.assign(h.nn, -1);
  h.Ioff.assign(1, 0);
  std::vector<std::vector<SN>> dsn(h.nsub);
  for (int b = 0; b < nsy; ++b)
    for (int a = 0; a < nsx; ++a) {
      int s = a + nsx * b;
      std::vector<Pt> pts;
      for (int j = h.ys[b] + 1; j < h.ys[b + 1]; ++j)
        for (int i = h.xs[a] + 1; i < h.xs[a + 1]; ++i)
          if (is_free(i, j)) pts.push_back({i, j, i + (n + 1) * j});
      std::vector<int> order;
      nested_dissection(pts, 0, order, dsn[s], LEAF);
      for (int v : order) {
        h.mesh2dd[v] = (int)h.dd2mesh.size();
        h.dd2mesh.push_back(v);
      }
      h.Ioff.push_back((int)h.dd2mesh.size());
    }
  h.nI = (int)h.dd2mesh.size();
  for (int v = 0; v < h.nn; ++v) {
    int i = v % (n + 1), j = v / (n + 1);
    if (is_free(i, j) && mult[v] >= 2) {
      int gi = (int)h.dd2mesh.size() - h.nI;
      h.mesh2dd[v] = (int)h.dd2mesh.size();
      h.dd2mesh.push_back(v);
      if (is_corner(v)) {
        h.g2c.push_back((int)h.c2g.size());
        h.c2g.push_back(gi);
      } else {
        h.g2c.push_back(-1);
      }
    }
  }
  h.NF = (int)h.dd2mesh.size();
  h.nG = h.NF - h.nI;
  h.nC = (int)h.c2g.size();

  // ----- torn (Neumann) numbering: interior + remaining nodes per subdomain
  h.Toff.assign(1, 0);
  std::vector<std::vector<SN>> nsn(h.nsub);
  std::vector<std::vector<int>> tloc(h.nsub);  // local box index -> torn row
  for (int b = 0; b < nsy; ++b)
    for (int a = 0; a < nsx; ++a) {
      int s = a + nsx * b;
      int wx = h.xs[a + 1] - h.xs[a] + 1, wy = h.ys[b + 1] - h.ys[b] + 1;
      tloc[s].assign(wx * wy, -1);
      std::vector<Pt> pts;
      for (int j = h.ys[b]; j <= h.ys[b + 1]; ++j)
        for (int i = h.xs[a]; i <= h.xs[a + 1]; ++i) {
          int v = i + (n + 1) * j;
          if (is_free(i, j) && in_torn(v)) pts.push_back({i, j, v});
        }
      std::vector<int> order;
      nested_dissection(pts, 0, order, nsn[s], LEAF);
      for (int v : order) {
        int i = v % (n + 1), j = v / (n + 1);
        tloc[s][(i - h.xs[a]) + wx * (j - h.ys[b])] = (int)h.torn2dd.size();
        h.torn2dd.push_back(h.mesh2dd[v]);
      }
      h.Toff.push_back((int)h.torn2dd.size());
    }
  h.NT = (int)h.torn2dd.size();
  auto torn_of = [&](int s, int i, int j) {
    int a = s % nsx, b = s / nsx;
    if (i < h.xs[a] || i > h.xs[a + 1] || j < h.ys[b] || j > h.ys[b + 1]) return -1;
    int wx = h.xs[a + 1] - h.xs[a] + 1;
    return tloc[s][(i - h.xs[a]) + wx * (j - h.ys[b])];
  };

  // ----- assembly into ELL -----
  const int W = 7;
  auto init_ell = [&](Ell& E, int nrows) {
    E.nrows = nrows;
    E.W = W;
    E.nk = nk;
    E.col.assign((size_t)W * nrows, 0);
    for (int s = 0; s < W; ++s)
      for (int r = 0; r < nrows; ++r) E.col[(size_t)s * nrows + r] = r;
    E.val.assign((size_t)nk * W * nrows, 0.0);
    E.mval.assign((size_t)W * nrows, 0.0);
  };
  init_ell(h.glob, h.NF);
  init_ell(h.dir, h.nI);
  init_ell(h.neu, h.NT);
  h.cc_ptr.assign(1, 0);
  h.sc_ptr.assign(1, 0);
  // per subdomain corner lists
  std::vector<std::vector<int>> corners(h.nsub);
  for (int v = 0; v < h.nn; ++v) {
    int i = v % (n + 1), j = v / (n + 1);
    if (!is_free(i, j) || !is_corner(v)) continue;
    for (int s = 0; s < h.nsub; ++s) {
      int a = s % nsx, b = s / nsx;
      if (h.xs[a] <= i && i <= h.xs[a + 1] && h.ys[b] <= j && j <= h.ys[b + 1])
        corners[s].push_back(v);
    }
  }
  // corner row accumulators: per (subdomain, corner) map slot -> values
  std::vector<std::vector<double>> crow(h.nsub);  // [corner][slot][k]
  for (int s = 0; s < h.nsub; ++s) crow[s].assign(corners[s].size() * W * nk, 0.0);

  const double hh = 1.0 / n;
  for (int cj = 0; cj < n; ++cj)
    for (int ci = 0; ci < n; ++ci) {
      int s = cell_sub(ci, cj);
      int v00 = ci + (n + 1) * cj, v10 = v00 + 1, v01 = v00 + n + 1, v11 = v01 + 1;
      int tri[2][3] = {{v00, v10, v11}, {v00, v11, v01}};
      for (int t = 0; t < 2; ++t) {
        int e = 2 * (ci + n * cj) + t;
        double px[3], py[3];
        for (int q = 0; q < 3; ++q) {
          px[q] = (tri[t][q] % (n + 1)) * hh;
          py[q] = (tri[t][q] / (n + 1)) * hh;
        }
        double ke[3][3], me[3][3];
        p1_element(px, py, ke, me);
        for (int qa = 0; qa < 3; ++qa) {
          int va = tri[t][qa];
          int ia = va % (n + 1), ja = va / (n + 1);
          if (!is_free(ia, ja)) continue;
          for (int qb = 0; qb < 3; ++qb) {
            int vb = tri[t][qb];
            int ib = vb % (n + 1), jb = vb / (n + 1);
            if (!is_free(ib, jb)) continue;
            int sl = slot_of(ib - ia, jb - ja);
            double mv = me[qa][qb];
            // K~_0 = a_m M + s_k K_0 ; K~_k = s_k K_k  (Eq. K_T_Sto)
            auto add = [&](Ell& E, int row, int colr) {
              size_t o = (size_t)sl * E.nrows + row;
              E.col[o] = colr;
              E.mval[o] += mv;
              for (int k = 0; k < nk; ++k)
                E.val[((size_t)k * W + sl) * E.nrows + row] +=
                    h.s_k * h.kappa[(size_t)k * ne + e] * ke[qa][qb] + (k == 0 ? h.a_m * mv : 0.0);
            };
            int ra = h.mesh2dd[va], rb = h.mesh2dd[vb];
            add(h.glob, ra, rb);
            if (ra < h.nI && rb < h.nI) add(h.dir, ra, rb);
            int ta = torn_of(s, ia, ja), tb = torn_of(s, ib, jb);
            if (ta >= 0 && tb >= 0) add(h.neu, ta, tb);
            if (is_corner(va) && (tb >= 0 || vb == va)) {
              int lc = int(std::find(corners[s].begin(), corners[s].end(), va) - corners[s].begin());
              for (int k = 0; k < nk; ++k)
                crow[s][((size_t)lc * W + sl) * nk + k] +=
                    h.s_k * h.kappa[(size_t)k * ne + e] * ke[qa][qb] + (k == 0 ? h.a_m * mv : 0.0);
            }
          }
        }
      }
    }
  // corner coupling lists
  for (int s = 0; s < h.nsub; ++s) {
    for (size_t lc = 0; lc < corners[s].size(); ++lc) {
      int v = corners[s][lc];
      int i = v % (n + 1), j = v / (n + 1);
      int gi = h.mesh2dd[v] - h.nI;
      h.sc_coarse.push_back(h.g2c[gi]);
      h.sc_gidx.push_back(gi);
      h.sc_w.push_back(1.0 / mult[v]);
      for (int sl = 0; sl < W; ++sl) {
        const double* cv = &crow[s][((size_t)lc * W + sl) * nk];
        if (sl == 0) {
          for (int k = 0; k < nk; ++k) h.cself.push_back(cv[k]);
          continue;
        }
        int t = torn_of(s, i + kDi[sl], j + kDj[sl]);
        if (t < 0) continue;
        h.cc_torn.push_back(t);
        for (int k = 0; k < nk; ++k) h.cc_val.push_back(cv[k]);
      }
      h.cc_ptr.push_back((int)h.cc_torn.size());
    }
    h.sc_ptr.push_back((int)h.sc_coarse.size());
  }
  // D_s R_s (interface -> torn) and sum_s R_s^T D_s (torn -> interface)
  h.torn_gidx.assign(h.NT, -1);
  h.torn_w.assign(h.NT, 0.0);
  std::vector<std::vector<std::pair<int, double>>> gcopies(h.nG);
  for (int t = 0; t < h.NT; ++t) {
    int dd = h.torn2dd[t];
    if (dd >= h.nI) {
      int v = h.dd2mesh[dd];
      h.torn_gidx[t] = dd - h.nI;
      h.torn_w[t] = 1.0 / mult[v];
      gcopies[dd - h.nI].push_back({t, 1.0 / mult[v]});
    }
  }
  h.gam_ptr.assign(1, 0);
  for (int gi = 0; gi < h.nG; ++gi) {
    for (auto& c : gcopies[gi]) {
      h.gam_torn.push_back(c.first);
      h.gam_w.push_back(c.second);
    }
    h.gam_ptr.push_back((int)h.gam_torn.size());
  }

  // ----- spectral interval of every block for the Chebyshev preconditioner
  if (!cheb_bounds(h.dir, h.Ioff, h.chebD) || !cheb_bounds(h.neu, h.Toff, h.chebN)) {
    err = "a subdomain block couples outside itself or has a non-positive diagonal";
    return SGW_ENOTSPD;
  }

  // ----- mean-matrix factors (Dirichlet: interior; Neumann: torn) -----
  auto factor_blocks = [&](const Ell& E, const std::vector<int>& off,
                           std::vector<std::vector<SN>>& sns, Factor& F) -> bool {
    F = Factor();
    F.row_off.assign(1, 0);
    F.lvl_off.assign(1, 0);
    F.lr_ptr.assign(1, 0);
    F.lc_ptr.assign(1, 0);
    std::vector<int> lr0, lc0;
    for (int s = 0; s < h.nsub; ++s) {
      int r0 = off[s], nb = off[s + 1] - off[s];
      std::vector<std::vector<std::pair<int, double>>> A(nb);
      for (int r = 0; r < nb; ++r)
        for (int sl = 0; sl < E.W; ++sl) {
          size_t o = (size_t)sl * E.nrows + r0 + r;
          double v = E.val[o];  // k = 0 block
          int c = E.col[o] - r0;
          if (v != 0.0) A[r].push_back({c, v});
        }
      CSC L;
      if (!cholesky(nb, A, L)) return false;
      append_factor(F, L, sns[s]);
    }
    return true;
  };
  if (!factor_blocks(h.dir, h.Ioff, dsn, h.fD) ||
      !factor_blocks(h.neu, h.Toff, nsn, h.fN)) {
    err = "non-positive pivot in a mean-matrix factor";
    return SGW_ENOTSPD;
  }
  return 0;
}

}  // namespace sgw
