// Basis-function reordering by overlap-signature clustering (Sec. III-B.2, "Locality-Preserving
// Reordering"; appendix on reordering details, eqs. overlap_signature, cosine_similarity and
// cosine_distance), run on the host once per geometry.
//
// Row i of the overlap matrix S is the signature of basis function i; functions are compared by the
// cosine distance d(i, j) = 1 - s_i . s_j / (|s_i| |s_j|).  Average-linkage agglomerative clustering
// merges, from singletons, the two clusters of smallest mean inter-cluster distance until one cluster
// remains.  The merges are found with the nearest-neighbour chain (average linkage is reducible, so the
// chain finds the same merges as the greedy procedure) over a condensed matrix updated by the
// Lance-Williams rule d(k, a+b) = (n_a d(k, a) + n_b d(k, b)) / (n_a + n_b); they are then put in
// order of distance and numbered as the greedy procedure forms them.  Each merge joins the leaf
// sequences of its two sub-trees, the earlier-formed one first, each taken forward or reversed so
// that the junction pair has the smallest distance (ties in the order forward/forward,
// reversed/forward, forward/reversed, reversed/reversed).  The leaf order is the basis permutation;
// the library applies it per shell (a shell's components stay together), shells sorted stably by the
// first leaf position of any of their components.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "kldi_impl.h"

namespace {

struct OrderError {
  kldi_status code;
  std::string msg;
};

int ncart_l(int l) { return (l + 1) * (l + 2) / 2; }

// condensed index of (i, j), i < j, in the row-major upper triangle of an n x n matrix
inline size_t cidx(size_t n, size_t i, size_t j) { return i * n - i * (i + 1) / 2 + (j - i - 1); }

// Gram matrix of the normalised rows, as cosine distances in condensed form.  Host threads take blocks
// of 4 rows (dealt cyclically: block i has n - 4 i entries to its right, so the work evens out); each
// 4 x 4 block of the upper triangle keeps 16 sums in registers, each summed over k in order (the same
// sum as one dot product at a time, 8x fewer loads).
void cosine_distances(const std::vector<double> &U, size_t n, std::vector<double> &d) {
  d.assign(n * (n - 1) / 2, 0.0);
  const size_t nb = (n + 3) / 4;
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) {
    th.emplace_back([&, t] {
      for (size_t ib = t; ib < nb; ib += nt) {
        const size_t i0 = 4 * ib, ni = std::min<size_t>(4, n - i0);
        const double *u[4];
        for (size_t a = 0; a < 4; ++a) u[a] = U.data() + std::min(i0 + a, n - 1) * n;
        for (size_t jb = ib; jb < nb; ++jb) {
          const size_t j0 = 4 * jb, nj = std::min<size_t>(4, n - j0);
          const double *v[4];
          for (size_t b = 0; b < 4; ++b) v[b] = U.data() + std::min(j0 + b, n - 1) * n;
          double s[4][4] = {};
          for (size_t k = 0; k < n; ++k) {
            const double x0 = u[0][k], x1 = u[1][k], x2 = u[2][k], x3 = u[3][k];
            const double y0 = v[0][k], y1 = v[1][k], y2 = v[2][k], y3 = v[3][k];
            s[0][0] += x0 * y0; s[0][1] += x0 * y1; s[0][2] += x0 * y2; s[0][3] += x0 * y3;
            s[1][0] += x1 * y0; s[1][1] += x1 * y1; s[1][2] += x1 * y2; s[1][3] += x1 * y3;
            s[2][0] += x2 * y0; s[2][1] += x2 * y1; s[2][2] += x2 * y2; s[2][3] += x2 * y3;
            s[3][0] += x3 * y0; s[3][1] += x3 * y1; s[3][2] += x3 * y2; s[3][3] += x3 * y3;
          }
          for (size_t a = 0; a < ni; ++a)
            for (size_t b = 0; b < nj; ++b)
              if (j0 + b > i0 + a) d[cidx(n, i0 + a, j0 + b)] = 1.0 - s[a][b];
        }
      }
    });
  }
  for (auto &x : th) x.join();
}

struct Merge {
  int a, b;      // slots (cluster representatives) merged
  double dist;
};

// nearest-neighbour chain over the condensed matrix d (overwritten by the Lance-Williams updates)
std::vector<Merge> nn_chain(std::vector<double> &d, size_t n) {
  std::vector<int> size(n, 1);
  std::vector<char> alive(n, 1);
  std::vector<int> chain;
  std::vector<Merge> out;
  out.reserve(n - 1);
  auto D = [&](size_t i, size_t j) -> double & { return i < j ? d[cidx(n, i, j)] : d[cidx(n, j, i)]; };
  size_t remaining = n;
  size_t first = 0;
  while (remaining > 1) {
    if (chain.empty()) {
      while (!alive[first]) ++first;
      chain.push_back(int(first));
    }
    const int a = chain.back();
    const int prev = chain.size() >= 2 ? chain[chain.size() - 2] : -1;
    int b = -1;
    double best = 0.0;
    if (prev >= 0) {
      b = prev;
      best = D(a, prev);
    }
    for (size_t c = 0; c < n; ++c) {
      if (!alive[c] || int(c) == a) continue;
      const double v = D(a, c);
      if (b < 0 || v < best) {
        best = v;
        b = int(c);
      }
    }
    if (b == prev) {
      chain.pop_back();
      chain.pop_back();
      const int lo = std::min(a, b), hi = std::max(a, b);
      out.push_back(Merge{lo, hi, best});
      // the merged cluster lives in slot lo
      const double na = size[lo], nb = size[hi];
      for (size_t k = 0; k < n; ++k) {
        if (!alive[k] || int(k) == lo || int(k) == hi) continue;
        D(lo, k) = (na * D(lo, k) + nb * D(hi, k)) / (na + nb);
      }
      size[lo] += size[hi];
      alive[hi] = 0;
      --remaining;
    } else {
      chain.push_back(b);
    }
  }
  return out;
}

}  // namespace

extern "C" kldi_status kldi_overlap_order(const kldi_basis *b, const double *S, int32_t *ao_order, int32_t *shell_order) {
  try {
    if (!b || !S || !shell_order || b->n_shells <= 0 || !b->shell_l) throw OrderError{KLDI_E_ARG, "bad arguments to kldi_overlap_order"};
    const int ns = b->n_shells;
    std::vector<int> ao_shell;
    for (int s = 0; s < ns; ++s) {
      if (b->shell_l[s] < 0 || b->shell_l[s] > 2) throw OrderError{KLDI_E_ARG, "shell_l must be 0, 1 or 2"};
      for (int c = 0; c < ncart_l(b->shell_l[s]); ++c) ao_shell.push_back(s);
    }
    const size_t n = ao_shell.size();
    // normalised signatures
    std::vector<double> U(n * n);
    for (size_t i = 0; i < n; ++i) {
      double nr = 0.0;
      for (size_t k = 0; k < n; ++k) {
        const double v = S[i * n + k];
        if (!std::isfinite(v)) throw OrderError{KLDI_E_ARG, "overlap matrix not finite"};
        nr += v * v;
      }
      nr = std::sqrt(nr);
      if (!(nr > 0.0)) throw OrderError{KLDI_E_ARG, "overlap matrix has a zero row"};
      for (size_t k = 0; k < n; ++k) U[i * n + k] = S[i * n + k] / nr;
    }
    std::vector<int> leaves;
    if (n == 1) {
      leaves.push_back(0);
    } else {
      std::vector<double> d;
      cosine_distances(U, n, d);
      std::vector<Merge> m = nn_chain(d, n);
      std::stable_sort(m.begin(), m.end(), [](const Merge &x, const Merge &y) { return x.dist < y.dist; });
      // number the clusters as they form: slot -> current cluster's leaf sequence
      std::vector<std::vector<int>> seq(n);
      std::vector<size_t> formed(n);   // formation index of the cluster a slot holds (leaf i: i)
      for (size_t i = 0; i < n; ++i) {
        seq[i] = {int(i)};
        formed[i] = i;
      }
      // the slots of a merge in sorted order are its clusters' representatives: union by slot
      std::vector<int> rep(n);
      std::iota(rep.begin(), rep.end(), 0);
      auto find = [&](int x) {
        while (rep[x] != x) x = rep[x] = rep[rep[x]];
        return x;
      };
      auto dist = [&](int i, int j) {
        const double *ui = U.data() + size_t(i) * n, *uj = U.data() + size_t(j) * n;
        double s = 0.0;
        for (size_t k = 0; k < n; ++k) s += ui[k] * uj[k];
        return 1.0 - s;
      };
      size_t next = n;
      for (const Merge &mg : m) {
        int ra = find(mg.a), rb = find(mg.b);
        if (formed[ra] > formed[rb]) std::swap(ra, rb);   // the earlier-formed cluster goes first
        std::vector<int> &A = seq[ra], &B = seq[rb];
        const double c0 = dist(A.back(), B.front()), c1 = dist(A.front(), B.front());
        const double c2 = dist(A.back(), B.back()), c3 = dist(A.front(), B.back());
        int pick = 0;
        double best = c0;
        if (c1 < best) { best = c1; pick = 1; }
        if (c2 < best) { best = c2; pick = 2; }
        if (c3 < best) { best = c3; pick = 3; }
        if (pick & 1) std::reverse(A.begin(), A.end());
        if (pick & 2) std::reverse(B.begin(), B.end());
        A.insert(A.end(), B.begin(), B.end());
        std::vector<int>().swap(B);
        rep[rb] = ra;
        formed[ra] = next++;
      }
      leaves = seq[find(0)];
    }
    if (ao_order)
      for (size_t i = 0; i < n; ++i) ao_order[i] = leaves[i];
    std::vector<size_t> first(ns, n);
    for (size_t pos = 0; pos < n; ++pos) first[ao_shell[leaves[pos]]] = std::min(first[ao_shell[leaves[pos]]], pos);
    std::vector<int> so(ns);
    std::iota(so.begin(), so.end(), 0);
    std::stable_sort(so.begin(), so.end(), [&](int x, int y) { return first[x] < first[y]; });
    for (int s = 0; s < ns; ++s) shell_order[s] = so[s];
    return KLDI_OK;
  } catch (const OrderError &e) {
    kldi::set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    kldi::set_error("host allocation failed");
    return KLDI_E_OOM;
  }
}
