// Operator algebra of the two-site DMRG superblock (host side).
//
// Every operator of an enlarged block is written as a short list of groups
// sum_g (sum_k c_k O_k) (x) M_g, where O_k are renormalized block operators
// (or the identity) and M_g is an exact matrix on the explicitly treated sites.
// The rules follow from splitting the ab initio Hamiltonian (Eq. 1) over two
// parts X | Y (X to the left):
//   H = H_X + H_Y + sum_{x in X}(a+_x S^Y_x + h.c.) + sum_{y in Y}(S^X_y a_y + h.c.)
//       + sum_{p<q in X}(a+_p a+_q P^Y_pq + h.c.) + sum_{p,q in X} a+_p a_q Q^Y_pq
//   S^Y_x  = sum_{y in Y} t_xy a_y + 1/2 sum_{qrs in Y}(g_xqrs - g_qxrs) a+_q a_r a_s
//   S^X_y  = 1/2 sum_{pqu in X}(g_pquy - g_pqyu) a+_p a+_q a_u
//   P^Y_pq = 1/2 sum_{rs in Y}(g_pqrs - g_qprs) a_r a_s
//   Q^Y_pq = sum_{y,y' in Y}(g_{p y y' q} - g_{p y q y'}) a+_y a_y'
// with H = sum t a+ a + 1/2 sum g a+ a+ a a in spin-orbitals (t_pq = h_ij for equal
// spins, g_pqrs = (i_p i_s | i_q i_r) for sigma_p = sigma_s, sigma_q = sigma_r).
// Fermionic products of consecutive parts are graded: an odd operator on a
// right part picks up (-1)^{n} of the parts to its left.
#include "internal.h"

namespace bsd {

const Q kSiteQ[4] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};

Mat mat_mul(const Mat& x, const Mat& y) {
  Mat r(x.n);
  for (int i = 0; i < x.n; ++i)
    for (int k = 0; k < x.n; ++k) {
      double v = x(i, k);
      if (v == 0.0) continue;
      for (int j = 0; j < x.n; ++j) r(i, j) += v * y(k, j);
    }
  return r;
}
Mat mat_T(const Mat& x) {
  Mat r(x.n);
  for (int i = 0; i < x.n; ++i)
    for (int j = 0; j < x.n; ++j) r(j, i) = x(i, j);
  return r;
}
Mat mat_scale(const Mat& x, double c) {
  Mat r = x;
  for (double& v : r.a) v *= c;
  return r;
}
void mat_axpy(Mat& y, double c, const Mat& x) {
  for (size_t i = 0; i < y.a.size(); ++i) y.a[i] += c * x.a[i];
}
Mat mat_eye(int n) {
  Mat r(n);
  for (int i = 0; i < n; ++i) r(i, i) = 1.0;
  return r;
}

SiteSet make_siteset(int first, int nsites) {
  SiteSet S;
  S.first = first;
  S.nsites = nsites;
  S.dim = 1;
  for (int k = 0; k < nsites; ++k) S.dim *= 4;
  S.q.resize(S.dim);
  for (int c = 0; c < S.dim; ++c) {
    Q qq;
    int x = c;
    for (int k = nsites - 1; k >= 0; --k) {
      qq = qq + kSiteQ[x % 4];
      x /= 4;
    }
    S.q[c] = qq;
  }
  // one-site matrices in the basis |0>, a+_a|0>, a+_b|0>, a+_a a+_b|0>
  Mat cda(4), cdb(4);
  cda(1, 0) = 1.0;
  cda(3, 2) = 1.0;
  cdb(2, 0) = 1.0;
  cdb(3, 1) = -1.0;
  for (int k = 0; k < nsites; ++k)
    for (int sg = 0; sg < 2; ++sg) {
      const Mat& loc = sg == 0 ? cda : cdb;
      Mat M(S.dim);
      for (int c = 0; c < S.dim; ++c) {
        // digits of c, site 0 most significant
        int dig[4] = {0, 0, 0, 0};
        int x = c;
        for (int j = nsites - 1; j >= 0; --j) {
          dig[j] = x % 4;
          x /= 4;
        }
        int s = dig[k];
        for (int s2 = 0; s2 < 4; ++s2) {
          double v = loc(s2, s);
          if (v == 0.0) continue;
          int sign = 1;
          for (int j = 0; j < k; ++j) sign *= kSiteQ[dig[j]].parity() ? -1 : 1;
          int c2 = 0;
          for (int j = 0; j < nsites; ++j) c2 = c2 * 4 + (j == k ? s2 : dig[j]);
          M(c2, c) += sign * v;
        }
      }
      S.cd.push_back(M);
    }
  return S;
}

int local_parity(const Mat& M, const SiteSet& C) {
  for (int i = 0; i < M.n; ++i)
    for (int j = 0; j < M.n; ++j)
      if (M(i, j) != 0.0) return (C.q[i] - C.q[j]).parity();
  return -1;
}

Q key_dq(const OpKey& k, bool left_block) {
  switch (k.kind) {
    case 'I':
    case 'H':
      return {0, 0};
    case 'c':
      return mode_q(k.p);
    case 'A':
      return mode_q(k.p) + mode_q(k.q);
    case 'B':
      return mode_q(k.p) - mode_q(k.q);
    case 'S':
      return left_block ? mode_q(k.p) : -mode_q(k.p);
    case 'P':
      return -(mode_q(k.p) + mode_q(k.q));
    case 'Q':
      return mode_q(k.q) - mode_q(k.p);
  }
  throw Error(1, "bad op key");
}

// ---------------------------------------------------------------- local operators
namespace {

OpKey K(char kind, int p = -1, int q = -1) {
  OpKey k;
  k.kind = kind;
  k.p = p;
  k.q = q;
  return k;
}
const OpKey kIdent = {'I', -1, -1};

Mat H_local(const SiteSet& C, const Integrals& I) {
  Mat M(C.dim);
  int m0 = C.mode0(), m1 = m0 + C.nmodes();
  for (int a = m0; a < m1; ++a)
    for (int b = m0; b < m1; ++b) {
      double t = I.t(a, b);
      if (t != 0.0) mat_axpy(M, t, mat_mul(C.CD(a), C.C(b)));
    }
  for (int p = m0; p < m1; ++p)
    for (int q = m0; q < m1; ++q)
      for (int r = m0; r < m1; ++r)
        for (int s = m0; s < m1; ++s) {
          double g = I.g(p, q, r, s);
          if (g != 0.0)
            mat_axpy(M, 0.5 * g, mat_mul(mat_mul(C.CD(p), C.CD(q)), mat_mul(C.C(r), C.C(s))));
        }
  return M;
}

// S^C_x with x to the left of C (C on the complementary side)
Mat S_right_role(const SiteSet& C, int x, const Integrals& I) {
  Mat M(C.dim);
  int m0 = C.mode0(), m1 = m0 + C.nmodes();
  for (int a = m0; a < m1; ++a) {
    double t = I.t(x, a);
    if (t != 0.0) mat_axpy(M, t, C.C(a));
  }
  for (int q = m0; q < m1; ++q)
    for (int r = m0; r < m1; ++r)
      for (int s = m0; s < m1; ++s) {
        double w = 0.5 * (I.g(x, q, r, s) - I.g(q, x, r, s));
        if (w != 0.0) mat_axpy(M, w, mat_mul(C.CD(q), mat_mul(C.C(r), C.C(s))));
      }
  return M;
}

// S^C_y with y to the right of C (C on the normal side)
Mat S_left_role(const SiteSet& C, int y, const Integrals& I) {
  Mat M(C.dim);
  int m0 = C.mode0(), m1 = m0 + C.nmodes();
  for (int p = m0; p < m1; ++p)
    for (int q = m0; q < m1; ++q)
      for (int u = m0; u < m1; ++u) {
        double w = 0.5 * (I.g(p, q, u, y) - I.g(p, q, y, u));
        if (w != 0.0) mat_axpy(M, w, mat_mul(mat_mul(C.CD(p), C.CD(q)), C.C(u)));
      }
  return M;
}

Mat P_right_role(const SiteSet& C, int p, int q, const Integrals& I) {
  Mat M(C.dim);
  int m0 = C.mode0(), m1 = m0 + C.nmodes();
  for (int r = m0; r < m1; ++r)
    for (int s = m0; s < m1; ++s) {
      double w = 0.5 * (I.g(p, q, r, s) - I.g(q, p, r, s));
      if (w != 0.0) mat_axpy(M, w, mat_mul(C.C(r), C.C(s)));
    }
  return M;
}

Mat Q_right_role(const SiteSet& C, int p, int q, const Integrals& I) {
  Mat M(C.dim);
  int m0 = C.mode0(), m1 = m0 + C.nmodes();
  for (int y = m0; y < m1; ++y)
    for (int y2 = m0; y2 < m1; ++y2) {
      double w = I.g(p, y, y2, q) - I.g(p, y, q, y2);
      if (w != 0.0) mat_axpy(M, w, mat_mul(C.CD(y), C.C(y2)));
    }
  return M;
}

void push(std::vector<Group>& out, const Mat& M, std::vector<Term> terms) {
  if (M.zero() || terms.empty()) return;
  std::vector<Term> kept;
  for (auto& t : terms)
    if (t.coef != 0.0) kept.push_back(t);
  if (kept.empty()) return;
  Group g;
  g.M = M;
  g.terms = std::move(kept);
  out.push_back(std::move(g));
}

}  // namespace

// ---------------------------------------------------------------- left (normal) role
std::vector<Group> expand_left(const OpKey& key, int nL, const SiteSet& C, const Integrals& I) {
  std::vector<Group> out;
  const int c0 = C.mode0(), c1 = c0 + C.nmodes();
  const Mat Id = mat_eye(C.dim);
  auto inL = [&](int p) { return p < nL; };
  switch (key.kind) {
    case 'c': {
      if (inL(key.p))
        push(out, Id, {{1.0, K('c', key.p), false}});
      else
        push(out, C.CD(key.p), {{1.0, kIdent, false}});
      break;
    }
    case 'A': {
      int p = key.p, q = key.q;
      if (inL(q))
        push(out, Id, {{1.0, K('A', p, q), false}});
      else if (inL(p))
        push(out, C.CD(q), {{1.0, K('c', p), false}});
      else
        push(out, mat_mul(C.CD(p), C.CD(q)), {{1.0, kIdent, false}});
      break;
    }
    case 'B': {
      int p = key.p, q = key.q;
      if (inL(p) && inL(q))
        push(out, Id, {{1.0, K('B', p, q), false}});
      else if (inL(p))
        push(out, C.C(q), {{1.0, K('c', p), false}});
      else if (inL(q))
        push(out, mat_scale(C.CD(p), -1.0), {{1.0, K('c', q), true}});
      else
        push(out, mat_mul(C.CD(p), C.C(q)), {{1.0, kIdent, false}});
      break;
    }
    case 'S': {
      const int y = key.p;
      auto Kc = [&](int p, int q, int u) { return 0.5 * (I.g(p, q, u, y) - I.g(p, q, y, u)); };
      if (nL > 0) push(out, Id, {{1.0, K('S', y), false}});
      push(out, S_left_role(C, y, I), {{1.0, kIdent, false}});
      for (int u = c0; u < c1; ++u) {  // two in L, one in C
        std::vector<Term> t;
        for (int p = 0; p < nL; ++p)
          for (int q = p + 1; q < nL; ++q) {
            double w = Kc(p, q, u) - Kc(q, p, u);
            if (w != 0.0) t.push_back({w, K('A', p, q), false});
          }
        push(out, C.C(u), t);
      }
      for (int a = c0; a < c1; ++a) {
        std::vector<Term> t;
        for (int p = 0; p < nL; ++p)
          for (int u = 0; u < nL; ++u) {
            double w = Kc(a, p, u) - Kc(p, a, u);
            if (w != 0.0) t.push_back({w, K('B', p, u), false});
          }
        push(out, C.CD(a), t);
      }
      for (int x = 0; x < nL; ++x) {  // one creator in L, two in C
        Mat M(C.dim);
        for (int b = c0; b < c1; ++b)
          for (int c = c0; c < c1; ++c) {
            double w = Kc(x, b, c) - Kc(b, x, c);
            if (w != 0.0) mat_axpy(M, w, mat_mul(C.CD(b), C.C(c)));
          }
        push(out, M, {{1.0, K('c', x), false}});
      }
      for (int u = 0; u < nL; ++u) {  // one annihilator in L
        Mat M(C.dim);
        for (int p = c0; p < c1; ++p)
          for (int q = c0; q < c1; ++q) {
            double w = Kc(p, q, u);
            if (w != 0.0) mat_axpy(M, w, mat_mul(C.CD(p), C.CD(q)));
          }
        push(out, M, {{1.0, K('c', u), true}});
      }
      break;
    }
    case 'H': {
      if (nL > 0) push(out, Id, {{1.0, K('H'), false}});
      push(out, H_local(C, I), {{1.0, kIdent, false}});
      for (int x = 0; x < nL; ++x) {
        Mat M = S_right_role(C, x, I);
        push(out, M, {{1.0, K('c', x), false}});
        push(out, mat_scale(mat_T(M), -1.0), {{1.0, K('c', x), true}});
      }
      if (nL > 0)
        for (int a = c0; a < c1; ++a) {
          push(out, C.C(a), {{1.0, K('S', a), false}});
          push(out, mat_scale(C.CD(a), -1.0), {{1.0, K('S', a), true}});
        }
      // sum_{p<q in L} A_pq (x) P^C_pq + h.c., grouped by local monomial a_r a_s (r<s)
      for (int r = c0; r < c1; ++r)
        for (int s = r + 1; s < c1; ++s) {
          std::vector<Term> t, tT;
          for (int p = 0; p < nL; ++p)
            for (int q = p + 1; q < nL; ++q) {
              double w = 0.5 * ((I.g(p, q, r, s) - I.g(q, p, r, s)) - (I.g(p, q, s, r) - I.g(q, p, s, r)));
              if (w != 0.0) {
                t.push_back({w, K('A', p, q), false});
                tT.push_back({w, K('A', p, q), true});
              }
            }
          Mat M = mat_mul(C.C(r), C.C(s));
          push(out, M, t);
          push(out, mat_T(M), tT);
        }
      // sum_{pq in L} B_pq (x) Q^C_pq, grouped by local monomial a+_y a_y'
      for (int y = c0; y < c1; ++y)
        for (int y2 = c0; y2 < c1; ++y2) {
          std::vector<Term> t;
          for (int p = 0; p < nL; ++p)
            for (int q = 0; q < nL; ++q) {
              double w = I.g(p, y, y2, q) - I.g(p, y, q, y2);
              if (w != 0.0) t.push_back({w, K('B', p, q), false});
            }
          push(out, mat_mul(C.CD(y), C.C(y2)), t);
        }
      break;
    }
    default:
      throw Error(1, "expand_left: bad key");
  }
  return out;
}

// ---------------------------------------------------------------- right (complementary) role
std::vector<Group> expand_right(const OpKey& key, const SiteSet& s, int r0, int nmodes,
                                const Integrals& I, bool R_normal) {
  std::vector<Group> out;
  const int s0 = s.mode0(), s1 = s0 + s.nmodes();
  const Mat Id = mat_eye(s.dim);
  const bool haveR = r0 < nmodes;
  switch (key.kind) {
    case 'A': {   // a+_p a+_q, p < q, both in s . R (normal right block)
      BSD_CHECK(R_normal, 1, "expand_right: normal key on a complementary block");
      const int p = key.p, q = key.q;
      if (p >= r0)
        push(out, Id, {{1.0, K('A', p, q), false}});
      else if (q >= r0)
        push(out, s.CD(p), {{1.0, K('c', q), false}});
      else
        push(out, mat_mul(s.CD(p), s.CD(q)), {{1.0, kIdent, false}});
      break;
    }
    case 'B': {   // a+_p a_q, both in s . R (normal right block)
      BSD_CHECK(R_normal, 1, "expand_right: normal key on a complementary block");
      const int p = key.p, q = key.q;
      if (p >= r0 && q >= r0)
        push(out, Id, {{1.0, K('B', p, q), false}});
      else if (q >= r0)
        push(out, s.CD(p), {{1.0, K('c', q), true}});
      else if (p >= r0)   // a+_p a_q = -a_q a+_p with a_q on s
        push(out, mat_scale(s.C(q), -1.0), {{1.0, K('c', p), false}});
      else
        push(out, mat_mul(s.CD(p), s.C(q)), {{1.0, kIdent, false}});
      break;
    }
    case 'c': {
      if (s.has(key.p))
        push(out, s.CD(key.p), {{1.0, kIdent, false}});
      else
        push(out, Id, {{1.0, K('c', key.p), false}});
      break;
    }
    case 'H': {
      if (haveR) push(out, Id, {{1.0, K('H'), false}});
      push(out, H_local(s, I), {{1.0, kIdent, false}});
      if (!haveR) break;
      for (int a = s0; a < s1; ++a) {
        push(out, s.CD(a), {{1.0, K('S', a), false}});
        push(out, mat_scale(s.C(a), -1.0), {{1.0, K('S', a), true}});
      }
      for (int r = r0; r < nmodes; ++r) {
        Mat M = S_left_role(s, r, I);
        push(out, M, {{1.0, K('c', r), true}});
        push(out, mat_scale(mat_T(M), -1.0), {{1.0, K('c', r), false}});
      }
      for (int p = s0; p < s1; ++p)
        for (int q = p + 1; q < s1; ++q) {
          Mat M = mat_mul(s.CD(p), s.CD(q));
          push(out, M, {{1.0, K('P', p, q), false}});
          push(out, mat_T(M), {{1.0, K('P', p, q), true}});
        }
      for (int p = s0; p < s1; ++p)
        for (int q = s0; q < s1; ++q) push(out, mat_mul(s.CD(p), s.C(q)), {{1.0, K('Q', p, q), false}});
      break;
    }
    case 'S': {
      const int x = key.p;
      if (haveR) push(out, Id, {{1.0, K('S', x), false}});
      push(out, S_right_role(s, x, I), {{1.0, kIdent, false}});
      if (!haveR) break;
      for (int q = s0; q < s1; ++q) push(out, s.CD(q), {{1.0, K('P', x, q), false}});
      for (int a = s0; a < s1; ++a) push(out, s.C(a), {{1.0, K('Q', x, a), false}});
      // two modes in s, one in R: aggregated over the R mode
      for (int a = s0; a < s1; ++a)
        for (int b = s0; b < s1; ++b) {
          std::vector<Term> t1, t3;
          for (int u = r0; u < nmodes; ++u) {
            double w1 = 0.5 * (I.g(x, a, b, u) - I.g(a, x, b, u)) - 0.5 * (I.g(x, a, u, b) - I.g(a, x, u, b));
            if (w1 != 0.0) t1.push_back({w1, K('c', u), true});
            double w3 = 0.5 * (I.g(x, u, a, b) - I.g(u, x, a, b));
            if (w3 != 0.0) t3.push_back({w3, K('c', u), false});
          }
          push(out, mat_mul(s.CD(a), s.C(b)), t1);
          push(out, mat_mul(s.C(a), s.C(b)), t3);
        }
      break;
    }
    case 'P': {
      const int p = key.p, q = key.q;
      if (haveR) push(out, Id, {{1.0, K('P', p, q), false}});
      push(out, P_right_role(s, p, q, I), {{1.0, kIdent, false}});
      for (int a = s0; a < s1; ++a) {
        std::vector<Term> t;
        for (int y = r0; y < nmodes; ++y) {
          double w = I.g(p, q, a, y) - I.g(p, q, y, a);
          if (w != 0.0) t.push_back({w, K('c', y), true});
        }
        push(out, s.C(a), t);
      }
      break;
    }
    case 'Q': {
      const int p = key.p, q = key.q;
      if (haveR) push(out, Id, {{1.0, K('Q', p, q), false}});
      push(out, Q_right_role(s, p, q, I), {{1.0, kIdent, false}});
      for (int a = s0; a < s1; ++a) {
        std::vector<Term> t1, t2;
        for (int y = r0; y < nmodes; ++y) {
          double w1 = I.g(p, a, y, q) - I.g(p, a, q, y);
          if (w1 != 0.0) t1.push_back({w1, K('c', y), true});
          double w2 = -(I.g(p, y, a, q) - I.g(p, y, q, a));
          if (w2 != 0.0) t2.push_back({w2, K('c', y), false});
        }
        push(out, s.CD(a), t1);
        push(out, s.C(a), t2);
      }
      break;
    }
    default:
      throw Error(1, "expand_right: bad key");
  }
  if (!R_normal || !haveR) return out;
  // R holds normal operators: P^R_pq and Q^R_pq become sums over them.
  //   P^R_pq = 1/2 sum_{r,s in R} (g_pqrs - g_qprs) a_r a_s, and with
  //   A_rs = a+_r a+_s (r < s): a_r a_s = -A_rs^T, a_s a_r = A_rs^T, so
  //   P^R_pq = sum_{r<s} 1/2 [(g_pqsr - g_qpsr) - (g_pqrs - g_qprs)] A_rs^T;
  //   Q^R_pq = sum_{y,y' in R} (g_{p y y' q} - g_{p y q y'}) B_yy'.
  // A transposed P or Q term transposes every term of its sum.
  std::vector<Group> res;
  for (auto& g : out) {
    Group h;
    h.M = g.M;
    for (const auto& t : g.terms) {
      if (t.key.kind == 'P') {
        const int p = t.key.p, q = t.key.q;
        for (int r = r0; r < nmodes; ++r)
          for (int u = r + 1; u < nmodes; ++u) {
            const double w = 0.5 * ((I.g(p, q, u, r) - I.g(q, p, u, r)) - (I.g(p, q, r, u) - I.g(q, p, r, u)));
            if (w != 0.0) h.terms.push_back({t.coef * w, K('A', r, u), !t.trans});
          }
      } else if (t.key.kind == 'Q') {
        const int p = t.key.p, q = t.key.q;
        for (int y = r0; y < nmodes; ++y)
          for (int y2 = r0; y2 < nmodes; ++y2) {
            const double w = I.g(p, y, y2, q) - I.g(p, y, q, y2);
            if (w != 0.0) h.terms.push_back({t.coef * w, K('B', y, y2), t.trans});
          }
      } else {
        h.terms.push_back(t);
      }
    }
    push(res, h.M, h.terms);
  }
  return res;
}

std::vector<Group> transpose_groups(const std::vector<Group>& gs, const SiteSet& C, int total_par) {
  std::vector<Group> out;
  for (const auto& g : gs) {
    int mp = local_parity(g.M, C);
    if (mp < 0) continue;
    int op_par = total_par ^ mp;
    double sign = (mp && op_par) ? -1.0 : 1.0;
    Group h;
    h.M = mat_T(g.M);
    for (auto t : g.terms) {
      t.trans = !t.trans;
      t.coef *= sign;
      h.terms.push_back(t);
    }
    out.push_back(std::move(h));
  }
  return out;
}

}  // namespace bsd
