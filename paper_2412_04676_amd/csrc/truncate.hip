// Truncation of the two-site wave function (Sec. II.B step 3, where the
// enlarged block's new basis comes from a singular value decomposition),
// float64 on the device.
//
// psi is split across the middle bond: rows (s1, q_l), columns (s2, q_r) for
// each middle sector q_m = q_l + q_s1.  The left (right) singular vectors are
// the eigenvectors of the Gram matrix G = M M^T (M^T M), formed by the
// grouped-GEMM engine with the K dimension concatenated over the other local
// state, and diagonalized by a parallel round-robin Jacobi method spread over
// several workgroups per sector (a launch per round).  Singular values are
// sqrt of the eigenvalues.  The
// kept states follow one global rule: the D largest, extended to every value
// >= sigma_D (1 - 1e-10), values <= 1e-6 sigma_max dropped.  A sector has at
// most min(rows, cols) nonzero singular values; the Gram matrix of its larger
// side carries the others as rounding-level eigenvalues, which never count.
// The floor sits well above what the Gram route resolves (sigma down to about
// sqrt(eps) sigma_max) and above the eigensolver's noise in psi.
#include "truncate.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>

namespace bsd {

// Cyclic parallel Jacobi on the Gram matrix of every sector (m x m, ld m,
// m even).  A sweep is m - 1 rounds of the round-robin pairing; a round
// rotates m / 2 disjoint index pairs (p, q) at once.  With the rotations R_k
// of a round fixed, the update R^T A R splits into independent 2 x 2 blocks,
// one per pair of pairs (k1, k2).
//
// A sector is spread over several workgroups, each owning a range of row
// pairs k1 (rows p1, q1 of A and of the eigenvector rows Z).  One launch is
// one round for every sector: a workgroup first derives the rotations of the
// whole round from the current A (every workgroup of the sector derives the
// same ones), then writes its rows of the next A into the other of two
// buffers, so no workgroup reads what another writes in the same launch.
// Eigenvector rows rotate in place (each pair's rows belong to one workgroup).
// No divisions beyond the rotation angles.
constexpr int kJacobiMaxDim = 4096;       // 2048 rotations per round: 48 KiB of LDS
constexpr double kSigmaFloor = 1e-6;      // relative to sigma_max: numerically zero below
constexpr int kJacobiPairsPerGroup = 8;   // row pairs per workgroup (two per wave)

struct JTask {
  int sec;    // sector
  int k1a;    // first row pair
  int k1b;    // one past the last
  int par;    // buffer of the sector's current A at round 0 of this sweep
};

__global__ void __launch_bounds__(256)
jacobi_identity_kernel(const int64_t* __restrict__ goff, const int* __restrict__ dims, double* __restrict__ Z) {
  const int m = dims[blockIdx.x];
  double* z = Z + goff[blockIdx.x];
  for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += blockDim.x) z[e] = (e / m == e % m) ? 1.0 : 0.0;
}

// off-diagonal and diagonal squared norms of the current A of each listed sector
__global__ void __launch_bounds__(1024)
jacobi_norms_kernel(const int* __restrict__ list, const int* __restrict__ par, const int64_t* __restrict__ goff,
                    const int* __restrict__ dims, const double* __restrict__ A0, const double* __restrict__ A1,
                    double* __restrict__ out) {
  const int sec = list[blockIdx.x];
  const int m = dims[sec];
  const double* A = (par[blockIdx.x] ? A1 : A0) + goff[sec];
  __shared__ double red[2][16];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63, nw = blockDim.x >> 6;
  double o = 0.0, d = 0.0;
  for (int i = wave; i < m; i += nw)
    for (int j = lane; j < m; j += 64) {
      const double v = A[(int64_t)i * m + j];
      if (i == j) d += v * v;
      else o += v * v;
    }
  for (int w = 32; w > 0; w >>= 1) {
    o += __shfl_xor(o, w);
    d += __shfl_xor(d, w);
  }
  if (lane == 0) {
    red[0][wave] = o;
    red[1][wave] = d;
  }
  __syncthreads();
  if (t == 0) {
    double so = 0.0, sd = 0.0;
    for (int w = 0; w < nw; ++w) {
      so += red[0][w];
      sd += red[1][w];
    }
    out[2 * blockIdx.x] = so;
    out[2 * blockIdx.x + 1] = sd;
  }
}

__global__ void __launch_bounds__(256)
jacobi_round_kernel(const JTask* __restrict__ tasks, const int64_t* __restrict__ goff, const int* __restrict__ dims,
                    double* __restrict__ A0, double* __restrict__ A1, double* __restrict__ Z, int r) {
  const JTask tk = tasks[blockIdx.x];
  const int m = dims[tk.sec];
  if (r >= m - 1) return;   // this sector's sweep has fewer rounds
  const int half = m / 2;
  const int64_t off = goff[tk.sec];
  const bool odd = (tk.par + r) & 1;
  const double* Ac = (odd ? A1 : A0) + off;
  double* An = (odd ? A0 : A1) + off;
  double* Zs = Z + off;
  extern __shared__ double lds_rot[];
  const int hmax = kJacobiMaxDim / 2;
  double* cs = lds_rot;
  double* sn = lds_rot + hmax;
  int* pp = reinterpret_cast<int*>(lds_rot + 2 * hmax);
  int* qq = pp + hmax;
  const int t = threadIdx.x, nt = blockDim.x;
  const int wave = t >> 6, lane = t & 63, nw = nt >> 6;
  // the rotations of round r (pairing of m - 1 rotating indices and a fixed one)
  for (int k = t; k < half; k += nt) {
    int p, q;
    if (k == 0) {
      p = r;
      q = m - 1;
    } else {
      p = r + k;
      if (p >= m - 1) p -= m - 1;
      q = r - k;
      if (q < 0) q += m - 1;
    }
    if (p > q) {
      const int x = p;
      p = q;
      q = x;
    }
    const double apq = Ac[(int64_t)p * m + q];
    double c = 1.0, sv = 0.0;
    if (fabs(apq) > 1e-300) {
      const double tau = (Ac[(int64_t)q * m + q] - Ac[(int64_t)p * m + p]) / (2.0 * apq);
      const double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
      c = 1.0 / sqrt(1.0 + tt * tt);
      sv = tt * c;
    }
    cs[k] = c;
    sn[k] = sv;
    pp[k] = p;
    qq[k] = q;
  }
  __syncthreads();
  // blocks (k1, k2): B' = R1^T B R2 with R = [[c, s], [-s, c]] on (p, q)
  const int k1e = min(tk.k1b, half);
  for (int k1 = tk.k1a + wave; k1 < k1e; k1 += nw) {
    const double c1 = cs[k1], s1 = sn[k1];
    const int p1 = pp[k1], q1 = qq[k1];
    const double* rp = Ac + (int64_t)p1 * m;
    const double* rq = Ac + (int64_t)q1 * m;
    double* wp = An + (int64_t)p1 * m;
    double* wq = An + (int64_t)q1 * m;
    for (int k2 = lane; k2 < half; k2 += 64) {
      const double c2 = cs[k2], s2 = sn[k2];
      const int p2 = pp[k2], q2 = qq[k2];
      const double b00 = rp[p2], b01 = rp[q2], b10 = rq[p2], b11 = rq[q2];
      const double t00 = c1 * b00 - s1 * b10, t01 = c1 * b01 - s1 * b11;
      const double t10 = s1 * b00 + c1 * b10, t11 = s1 * b01 + c1 * b11;
      const bool diag = k1 == k2;   // the rotated pair itself is diagonalized
      wp[p2] = c2 * t00 - s2 * t01;
      wp[q2] = diag ? 0.0 : s2 * t00 + c2 * t01;
      wq[p2] = diag ? 0.0 : c2 * t10 - s2 * t11;
      wq[q2] = s2 * t10 + c2 * t11;
    }
  }
  // eigenvector rows p, q of this workgroup's pairs
  for (int k = tk.k1a + wave; k < k1e; k += nw) {
    const double c = cs[k], sv = sn[k];
    if (sv == 0.0) continue;
    double* zp = Zs + (int64_t)pp[k] * m;
    double* zq = Zs + (int64_t)qq[k] * m;
    for (int i = lane; i < m; i += 64) {
      const double a = zp[i], b = zq[i];
      zp[i] = c * a - sv * b;
      zq[i] = sv * a + c * b;
    }
  }
}

TruncResult truncate_psi(Ctx& ctx, const HpsiPlan& plan, const double* psi, int D, bool left_to_right,
                         DevBuf& work, hipStream_t s) {
  Block* Lb = get_block(ctx, true, plan.site);
  Block* Rb = get_block(ctx, false, plan.site + 2);
  BSD_CHECK(Lb && Rb, 2, "environment blocks missing");
  // BSDMRG_VERBOSE: host wall time of the stages
  const bool verbose = std::getenv("BSDMRG_VERBOSE") != nullptr;
  auto t_last = std::chrono::steady_clock::now();
  auto note = [&](const char* what) {
    if (!verbose) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "truncate: %s %.3f s\n", what, std::chrono::duration<double>(now - t_last).count());
    t_last = now;
  };
  const SiteSet C = make_siteset(plan.site, 2);
  const PsiLayout& lay = plan.lay;
  // middle sectors and their row (s1, l) / column (s2, r) index spaces
  struct Sec {
    Q qm;
    std::vector<std::pair<int, int>> rows, cols;   // (s, basis idx)
    std::vector<int> roff, coff;
    int nr = 0, nc = 0, m = 0;
    int64_t goff = 0;
  };
  std::map<Q, int> sidx;
  std::vector<Sec> secs;
  for (const auto& b : lay.blocks) {
    const int s1 = b.c / 4;
    Q qm = Lb->basis.q[b.l] + kSiteQ[s1];
    if (sidx.find(qm) == sidx.end()) {
      sidx[qm] = (int)secs.size();
      Sec x;
      x.qm = qm;
      secs.push_back(x);
    }
  }
  for (auto& x : secs) {
    for (int s1 = 0; s1 < 4; ++s1) {
      int l = Lb->basis.find(x.qm - kSiteQ[s1]);
      if (l >= 0) {
        x.rows.push_back({s1, l});
        x.roff.push_back(x.nr);
        x.nr += Lb->basis.dim[l];
      }
    }
    for (int s2 = 0; s2 < 4; ++s2) {
      // right block label counts electrons to the right: target - (q_m + q_s2)
      int r = Rb->basis.find(ctx.target - (x.qm + kSiteQ[s2]));
      if (r >= 0) {
        x.cols.push_back({s2, r});
        x.coff.push_back(x.nc);
        x.nc += Rb->basis.dim[r];
      }
    }
    const int n = left_to_right ? x.nr : x.nc;
    x.m = n + (n & 1);
    BSD_CHECK(x.m <= kJacobiMaxDim, 3, "middle sector larger than 4096 states");
  }
  int64_t gtot = 0;
  for (auto& x : secs) {
    x.goff = gtot;
    gtot += (int64_t)x.m * x.m;
  }
  work.reserve((size_t)std::max<int64_t>(1, 3 * gtot + 2 * (int64_t)secs.size()) * sizeof(double));
  double* G = static_cast<double*>(work.p);
  double* V = G + gtot;
  double* A1 = V + gtot;   // the other buffer of the Jacobi rounds
  zero_fill(G, gtot, s);
  // Gram matrices by the grouped GEMM (psi blocks: rows d_l, cols d_r)
  std::vector<GemmProblem> probs;
  for (auto& x : secs) {
    const auto& outer = left_to_right ? x.rows : x.cols;
    const auto& offs = left_to_right ? x.roff : x.coff;
    for (size_t a = 0; a < outer.size(); ++a)
      for (size_t b = 0; b < outer.size(); ++b) {
        GemmProblem gp;
        const int da = left_to_right ? Lb->basis.dim[outer[a].second] : Rb->basis.dim[outer[a].second];
        const int db = left_to_right ? Lb->basis.dim[outer[b].second] : Rb->basis.dim[outer[b].second];
        gp.C = tag_ptr(0, (uint64_t)(G + x.goff + (int64_t)offs[a] * x.m + offs[b]));
        gp.ldc = x.m;
        gp.M = da;
        gp.N = db;
        gp.beta = 0.0;
        const auto& inner = left_to_right ? x.cols : x.rows;
        for (const auto& in : inner) {
          int la, lb, ra, rb, ca, cb;
          if (left_to_right) {
            la = outer[a].second, lb = outer[b].second;
            ca = outer[a].first * 4 + in.first;
            cb = outer[b].first * 4 + in.first;
            ra = rb = in.second;
          } else {
            la = lb = in.second;
            ca = in.first * 4 + outer[a].first;
            cb = in.first * 4 + outer[b].first;
            ra = outer[a].second, rb = outer[b].second;
          }
          auto ia = lay.index.find({la, ca, ra});
          auto ib = lay.index.find({lb, cb, rb});
          if (ia == lay.index.end() || ib == lay.index.end()) continue;
          const PsiBlk& A = lay.blocks[ia->second];
          const PsiBlk& B = lay.blocks[ib->second];
          GSeg sg;
          sg.alpha = 1.0;
          sg.A = tag_ptr(1, (uint64_t)(A.off * sizeof(double)));
          sg.B = tag_ptr(1, (uint64_t)(B.off * sizeof(double)));
          sg.lda = A.cols;
          sg.ldb = B.cols;
          if (left_to_right) {
            sg.K = A.cols;           // sum over the right index
            sg.flags = kTransB;      // A (d_la x d_r) * B^T (d_r x d_lb)
          } else {
            sg.K = A.rows;           // sum over the left index
            sg.flags = kTransA;      // A^T (d_ra x d_l) * B (d_l x d_rb)
          }
          gp.segs.push_back(sg);
        }
        if (!gp.segs.empty()) probs.push_back(std::move(gp));
      }
  }
  {
    GemmPlan gplan;
    gplan.build(probs);
    GBases b{{0, (uint64_t)psi, 0, 0}};
    gplan.launch(b, s);
    BSD_HIP(hipStreamSynchronize(s));
  }
  note("sectors and Gram matrices");
  // Jacobi per sector
  std::vector<int64_t> goffs;
  std::vector<int> dims;
  for (auto& x : secs) {
    goffs.push_back(x.goff);
    dims.push_back(x.m);
  }
  if (!secs.empty()) {
    const int nsec = (int)secs.size();
    DevBuf dg, dd, dlist, dpar, dnorm, dtasks;
    dg.reserve(goffs.size() * sizeof(int64_t));
    dd.reserve(dims.size() * sizeof(int));
    dlist.reserve(nsec * sizeof(int));
    dpar.reserve(nsec * sizeof(int));
    dnorm.reserve(2 * nsec * sizeof(double));
    BSD_HIP(hipMemcpy(dg.p, goffs.data(), goffs.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    BSD_HIP(hipMemcpy(dd.p, dims.data(), dims.size() * sizeof(int), hipMemcpyHostToDevice));
    const int64_t* pg = static_cast<const int64_t*>(dg.p);
    const int* pd = static_cast<const int*>(dd.p);
    hipLaunchKernelGGL(jacobi_identity_kernel, dim3(nsec), dim3(256), 0, s, pg, pd, V);
    BSD_HIP(hipGetLastError());
    // rounds done per sector (its current A is in buffer rounds % 2) and the
    // sectors still rotating; at most 40 sweeps
    std::vector<int64_t> rounds(nsec, 0);
    std::vector<int> active;
    for (int k = 0; k < nsec; ++k)
      if (secs[k].m >= 2) active.push_back(k);
    const size_t lds = (size_t)(kJacobiMaxDim / 2) * (2 * sizeof(double) + 2 * sizeof(int));
    std::vector<JTask> tasks;   // host copy kept until the next synchronization
    for (int sweep = 0; sweep < 40 && !active.empty(); ++sweep) {
      // convergence: off-diagonal norm against the diagonal norm, per sector
      std::vector<int> par(active.size());
      for (size_t i = 0; i < active.size(); ++i) par[i] = (int)(rounds[active[i]] & 1);
      BSD_HIP(hipMemcpyAsync(dlist.p, active.data(), active.size() * sizeof(int), hipMemcpyHostToDevice, s));
      BSD_HIP(hipMemcpyAsync(dpar.p, par.data(), par.size() * sizeof(int), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(jacobi_norms_kernel, dim3((unsigned)active.size()), dim3(1024), 0, s,
                         static_cast<const int*>(dlist.p), static_cast<const int*>(dpar.p), pg, pd,
                         (const double*)G, (const double*)A1, static_cast<double*>(dnorm.p));
      BSD_HIP(hipGetLastError());
      std::vector<double> nrm(2 * active.size());
      BSD_HIP(hipMemcpyAsync(nrm.data(), dnorm.p, nrm.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      BSD_HIP(hipStreamSynchronize(s));
      std::vector<int> still;
      for (size_t i = 0; i < active.size(); ++i)
        if (!(nrm[2 * i] <= 1e-32 * nrm[2 * i + 1] || nrm[2 * i] == 0.0)) still.push_back(active[i]);
      active.swap(still);
      if (active.empty()) break;
      // one sweep: rounds in lockstep across the sectors, a launch per round
      tasks.clear();
      int rmax = 0;
      for (int k : active) {
        const int half = secs[k].m / 2;
        for (int a = 0; a < half; a += kJacobiPairsPerGroup)
          tasks.push_back({k, a, std::min(half, a + kJacobiPairsPerGroup), (int)(rounds[k] & 1)});
        rmax = std::max(rmax, secs[k].m - 1);
      }
      dtasks.reserve(tasks.size() * sizeof(JTask));
      BSD_HIP(hipMemcpyAsync(dtasks.p, tasks.data(), tasks.size() * sizeof(JTask), hipMemcpyHostToDevice, s));
      for (int r = 0; r < rmax; ++r)
        hipLaunchKernelGGL(jacobi_round_kernel, dim3((unsigned)tasks.size()), dim3(256), lds, s,
                           static_cast<const JTask*>(dtasks.p), pg, pd, G, A1, V, r);
      BSD_HIP(hipGetLastError());
      for (int k : active) rounds[k] += secs[k].m - 1;
      if (verbose) std::fprintf(stderr, "truncate: sweep %d, %zu sectors, %d rounds\n", sweep, active.size(), rmax);
    }
    // every sector's final A back into G
    for (int k = 0; k < nsec; ++k)
      if (rounds[k] & 1)
        BSD_HIP(hipMemcpyAsync(G + secs[k].goff, A1 + secs[k].goff, (size_t)secs[k].m * secs[k].m * sizeof(double),
                               hipMemcpyDeviceToDevice, s));
    BSD_HIP(hipStreamSynchronize(s));
  }
  note("Jacobi");
  // eigenvalues and vectors to the host (small: at most (4D)^2 per sector)
  std::vector<double> Gh(gtot), Vh(gtot);
  BSD_HIP(hipMemcpy(Gh.data(), G, gtot * sizeof(double), hipMemcpyDeviceToHost));
  BSD_HIP(hipMemcpy(Vh.data(), V, gtot * sizeof(double), hipMemcpyDeviceToHost));
  note("copies to the host");
  struct SV {
    double lam;
    int sec, col;
  };
  std::vector<SV> all;
  std::vector<SV> beyond_rank;
  for (int k = 0; k < (int)secs.size(); ++k) {
    const auto& x = secs[k];
    const int n = left_to_right ? x.nr : x.nc;
    std::vector<SV> sec;
    for (int j = 0; j < n; ++j) sec.push_back({std::max(0.0, Gh[x.goff + (int64_t)j * x.m + j]), k, j});
    // the rank bound: only the min(rows, cols) largest can be nonzero
    std::sort(sec.begin(), sec.end(), [](const SV& a, const SV& b) { return a.lam > b.lam; });
    const size_t rank = (size_t)std::min(x.nr, x.nc);
    for (size_t j = 0; j < sec.size(); ++j) (j < rank ? all : beyond_rank).push_back(sec[j]);
  }
  std::sort(all.begin(), all.end(), [](const SV& a, const SV& b) { return a.lam > b.lam; });
  TruncResult res;
  double total = 0.0;
  for (auto& a : all) total += a.lam;
  double disc = 0.0;
  for (auto& a : beyond_rank) {
    total += a.lam;
    disc += a.lam;
  }
  const double smax = all.empty() ? 0.0 : std::sqrt(all[0].lam);
  double cut = -1.0;
  if ((int)all.size() > D && D > 0) cut = std::sqrt(all[D - 1].lam) * (1.0 - 1e-10);
  std::vector<std::vector<int>> kept(secs.size());
  for (auto& a : all) {
    const double sg = std::sqrt(a.lam);
    if (sg >= cut && sg > kSigmaFloor * smax) {
      kept[a.sec].push_back(a.col);
      res.sv.push_back(sg);
    } else {
      disc += a.lam;
    }
  }
  res.trunc_err = disc;
  res.norm2 = total;
  // new site tensor: for left_to_right the blocks (q_l, s1) -> q_m are rows of
  // the kept eigenvectors; for right_to_left the blocks (q_m, s2) are the kept
  // eigenvectors transposed
  for (int k = 0; k < (int)secs.size(); ++k) {
    const auto& x = secs[k];
    const auto& kc = kept[k];
    if (kc.empty()) continue;
    res.D_kept += (int)kc.size();
    const auto& outer = left_to_right ? x.rows : x.cols;
    const auto& offs = left_to_right ? x.roff : x.coff;
    for (size_t a = 0; a < outer.size(); ++a) {
      const int d = left_to_right ? Lb->basis.dim[outer[a].second] : Rb->basis.dim[outer[a].second];
      TruncBlock tb;
      tb.s = outer[a].first;
      if (left_to_right) {
        tb.ql = Lb->basis.q[outer[a].second];
        tb.rows = d;
        tb.cols = (int)kc.size();
        tb.data.resize((size_t)d * kc.size());
        for (int i = 0; i < d; ++i)
          for (size_t j = 0; j < kc.size(); ++j)
            tb.data[i * kc.size() + j] = Vh[x.goff + (int64_t)kc[j] * x.m + offs[a] + i];
      } else {
        tb.ql = x.qm;   // left bond label of site+1 is the middle sector
        tb.rows = (int)kc.size();
        tb.cols = d;
        tb.data.resize((size_t)d * kc.size());
        for (size_t j = 0; j < kc.size(); ++j)
          for (int i = 0; i < d; ++i) tb.data[j * d + i] = Vh[x.goff + (int64_t)kc[j] * x.m + offs[a] + i];
      }
      res.blocks.push_back(std::move(tb));
    }
  }
  note("selection and new site tensor");
  return res;
}

}  // namespace bsd
