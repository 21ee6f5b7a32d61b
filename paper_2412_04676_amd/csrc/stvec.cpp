// Start vector of the next two-site position ("StVec" in the profile of one
// sweep, Fig. 9; Sec. II.B: the wave function of one step is carried into the
// next).  After the split of psi at sites (i, i+1):
//   left to right, new left-canonical A_i:
//     T[(q_m, s2, r)]        = sum_{s1} A_i[(q_l, s1)]^T psi[(q_l, s1, s2, r)]
//     guess[(q_m, s2, s3, r')] = T[(q_m, s2, r)] B_{i+2}[(q_b, s3)]
//   right to left, new right-canonical B_{i+1}:
//     T[(q_l, s1, q_m)]      = sum_{s2} psi[(q_l, s1, s2, r)] B_{i+1}[(q_m, s2)]^T
//     guess[(q_ll, s0, s1, q_m)] = A_{i-1}[(q_ll, s0)] T[(q_l, s1, q_m)]
// so the guess is S V^T B (or A U S) expressed in the bases of the next
// position's environment blocks.  Both contractions run as float64 grouped
// GEMMs (K concatenated over the summed local state).
#include "stvec.h"

namespace bsd {

namespace {

struct TKey {
  Q qa;        // left label (q_m for left to right, q_l for right to left)
  int s;       // the local state that is carried (s2, or s1)
  Q qb;        // right label: bond label of the right index (left to right), q_m (right to left)
  bool operator<(const TKey& o) const {
    if (!(qa == o.qa)) return qa < o.qa;
    if (s != o.s) return s < o.s;
    return qb < o.qb;
  }
};

int find_block(const SiteTensor& T, const Q& ql, int s) {
  int l = T.left.find(ql);
  if (l < 0) return -1;
  auto it = T.by_ls.find({l, s});
  return it == T.by_ls.end() ? -1 : it->second;
}

}  // namespace

void next_guess(Ctx& ctx, int site, bool left_to_right, const double* psi, double* guess, DevBuf& work,
                hipStream_t s) {
  const int L = ctx.L;
  Block* Lb = get_block(ctx, true, site);
  Block* Rb = get_block(ctx, false, site + 2);
  BSD_CHECK(Lb && Rb, 2, "environment blocks of the split position are not built");
  const int nsite = left_to_right ? site + 1 : site - 1;
  BSD_CHECK(nsite >= 0 && nsite + 1 < L, 1, "no next two-site position in this direction");
  Block* nLb = get_block(ctx, true, nsite);
  Block* nRb = get_block(ctx, false, nsite + 2);
  BSD_CHECK(nLb && nRb, 2, "environment blocks of the next position are not built");
  const SiteTensor& Tnew = ctx.sites[left_to_right ? site : site + 1];
  const SiteTensor& Tfar = ctx.sites[left_to_right ? site + 2 : site - 1];
  BSD_CHECK(Tnew.set && Tfar.set, 2, "site tensors of the transformation are not set");
  const SiteSet C = make_siteset(site, 2);
  const SiteSet nC = make_siteset(nsite, 2);
  PsiLayout lay, nlay;
  build_psi_layout(*Lb, *Rb, C, ctx.target, lay);
  build_psi_layout(*nLb, *nRb, nC, ctx.target, nlay);
  const Q tgt = ctx.target;

  // intermediate blocks T and their shapes
  std::map<TKey, int> tidx;
  struct TBlk {
    int rows, cols;
    int64_t off;
  };
  std::vector<TBlk> tb;
  int64_t tsize = 0;
  auto tblock = [&](const TKey& k, int rows, int cols) -> int {
    auto it = tidx.find(k);
    if (it != tidx.end()) {
      BSD_CHECK(tb[it->second].rows == rows && tb[it->second].cols == cols, 3, "inconsistent intermediate shape");
      return it->second;
    }
    tidx[k] = (int)tb.size();
    tb.push_back({rows, cols, tsize});
    tsize += (int64_t)rows * cols;
    return (int)tb.size() - 1;
  };
  // first pass: shapes of T from the psi blocks
  struct Seg1 {
    int t, psi_blk, tensor_blk;
  };
  std::vector<Seg1> seg1;
  for (int b = 0; b < (int)lay.blocks.size(); ++b) {
    const PsiBlk& pb = lay.blocks[b];
    const int s1 = pb.c / 4, s2 = pb.c % 4;
    const Q ql = Lb->basis.q[pb.l];
    const Q qr_bond = tgt - Rb->basis.q[pb.r];   // bond label of bond site+2
    if (left_to_right) {
      const int ab = find_block(Tnew, ql, s1);
      if (ab < 0) continue;                    // this (q_l, s1) was truncated away
      const Q qm = ql + kSiteQ[s1];
      const int t = tblock({qm, s2, qr_bond}, Tnew.blocks[ab].cols, pb.cols);
      seg1.push_back({t, b, ab});
    } else {
      const Q qm = ql + kSiteQ[s1];             // bond label of bond site+1
      const int bb = find_block(Tnew, qm, s2);
      if (bb < 0) continue;
      const int t = tblock({ql, s1, qm}, pb.rows, Tnew.blocks[bb].rows);
      seg1.push_back({t, b, bb});
    }
  }
  work.reserve((size_t)std::max<int64_t>(1, tsize) * sizeof(double));
  double* Tm = static_cast<double*>(work.p);
  zero_fill(guess, nlay.n_elems, s);
  std::vector<GemmProblem> p1(tb.size());
  for (size_t t = 0; t < tb.size(); ++t) {
    p1[t].C = tag_ptr(0, (uint64_t)(Tm + tb[t].off));
    p1[t].ldc = tb[t].cols;
    p1[t].M = tb[t].rows;
    p1[t].N = tb[t].cols;
    p1[t].beta = 0.0;
  }
  for (const auto& sg : seg1) {
    const PsiBlk& pb = lay.blocks[sg.psi_blk];
    const auto& tk = Tnew.blocks[sg.tensor_blk];
    GSeg g;
    g.alpha = 1.0;
    if (left_to_right) {
      // A^T (k x d_l) psi (d_l x d_r): A row-major d_l x k, read transposed
      g.A = tag_ptr(0, (uint64_t)Tnew.ptr(sg.tensor_blk));
      g.lda = tk.cols;
      g.B = tag_ptr(0, (uint64_t)(psi + pb.off));
      g.ldb = pb.cols;
      g.K = pb.rows;
      g.flags = kTransA;
    } else {
      // psi (d_l x d_r) B^T (d_r x k): B row-major k x d_r, read transposed
      g.A = tag_ptr(0, (uint64_t)(psi + pb.off));
      g.lda = pb.cols;
      g.B = tag_ptr(0, (uint64_t)Tnew.ptr(sg.tensor_blk));
      g.ldb = tk.cols;
      g.K = pb.cols;
      g.flags = kTransB;
    }
    p1[sg.t].segs.push_back(g);
  }
  std::vector<GemmProblem> p2;
  for (int b = 0; b < (int)nlay.blocks.size(); ++b) {
    const PsiBlk& nb = nlay.blocks[b];
    const int s1 = nb.c / 4, s2 = nb.c % 4;
    const Q ql = nLb->basis.q[nb.l];             // bond label of bond nsite
    const Q qr_bond = tgt - nRb->basis.q[nb.r];   // bond label of bond nsite+2
    int t = -1, fb = -1;
    bool tensor_left = false;
    if (left_to_right) {
      // guess[(q_m, s2', s3, r')] = T[(q_m, s2', q_b)] B_{i+2}[(q_b, s3)], q_b = q_r' - q_s3
      const Q qb = qr_bond - kSiteQ[s2];
      fb = find_block(Tfar, qb, s2);
      auto it = tidx.find({ql, s1, qb});
      if (fb < 0 || it == tidx.end()) continue;
      t = it->second;
    } else {
      // guess[(q_ll, s0, s1', q_m)] = A_{i-1}[(q_ll, s0)] T[(q_ll + s0, s1', q_m)]
      fb = find_block(Tfar, ql, s1);
      auto it = tidx.find({ql + kSiteQ[s1], s2, qr_bond});
      if (fb < 0 || it == tidx.end()) continue;
      t = it->second;
      tensor_left = true;
    }
    const auto& fk = Tfar.blocks[fb];
    GemmProblem gp;
    gp.C = tag_ptr(0, (uint64_t)(guess + nb.off));
    gp.ldc = nb.cols;
    gp.M = nb.rows;
    gp.N = nb.cols;
    gp.beta = 0.0;
    GSeg g;
    g.alpha = 1.0;
    g.flags = 0;
    if (!tensor_left) {
      BSD_CHECK(tb[t].rows == nb.rows && fk.cols == nb.cols && fk.rows == tb[t].cols, 3,
                "guess block shape mismatch");
      g.A = tag_ptr(0, (uint64_t)(Tm + tb[t].off));
      g.lda = tb[t].cols;
      g.B = tag_ptr(0, (uint64_t)Tfar.ptr(fb));
      g.ldb = fk.cols;
      g.K = fk.rows;
    } else {
      BSD_CHECK(fk.rows == nb.rows && tb[t].cols == nb.cols && fk.cols == tb[t].rows, 3,
                "guess block shape mismatch");
      g.A = tag_ptr(0, (uint64_t)Tfar.ptr(fb));
      g.lda = fk.cols;
      g.B = tag_ptr(0, (uint64_t)(Tm + tb[t].off));
      g.ldb = tb[t].cols;
      g.K = fk.cols;
    }
    gp.segs.push_back(g);
    p2.push_back(std::move(gp));
  }
  // problems of T with no segment (no kept state) stay zero: drop them, and
  // clear T so that guess blocks reading them see zeros
  std::vector<GemmProblem> p1k;
  for (auto& p : p1)
    if (!p.segs.empty()) p1k.push_back(std::move(p));
  zero_fill(Tm, tsize, s);
  GBases bases{{0, 0, 0, 0}};
  GemmPlan g1, g2;
  g1.build(p1k);
  g2.build(p2);
  g1.launch(bases, s);
  g2.launch(bases, s);
  BSD_HIP(hipStreamSynchronize(s));
}

}  // namespace bsd
