// Davidson eigensolver for the lowest eigenpair of the two-site effective
// Hamiltonian (Sec. II.B step 2), float64 on the device.
//
// Subspace vectors V and their products W = H V live in HBM in the psi
// layout; the projected matrix, its eigensolve (cyclic Jacobi in one
// workgroup), the Ritz vector, the residual and the diagonal preconditioner
// (diag H_eff - theta)^-1 are all device kernels.  New directions are
// orthogonalized twice (classical Gram-Schmidt, repeated).  The only host
// traffic per iteration is one 16-byte read of (theta, |r|).
#include "davidson.h"

#include <algorithm>
#include <cmath>

namespace bsd {

constexpr int kRedBlocks = 512;

// partial[b * k + j] = sum over this block's slice of V_j . w
__global__ void __launch_bounds__(256)
multi_dot_kernel(const double* __restrict__ V, int64_t ldv, int k, const double* __restrict__ w, int64_t n,
                 double* __restrict__ partial) {
  __shared__ double red[256];
  for (int j = 0; j < k; ++j) {
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
      s += V[(int64_t)j * ldv + i] * w[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * k + j] = red[0];
    __syncthreads();
  }
}

// out[j] = scale * sum_b partial[b * k + j]
__global__ void finish_dot_kernel(const double* __restrict__ partial, int nb, int k, double* __restrict__ out) {
  const int j = threadIdx.x;
  if (j < k) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[(int64_t)b * k + j];
    out[j] = s;
  }
}

// y = beta y + sum_j c[j] V_j   (c on the device)
__global__ void __launch_bounds__(256)
combine_kernel(const double* __restrict__ V, int64_t ldv, int k, const double* __restrict__ c, double beta,
               double cscale, double* __restrict__ y, int64_t n) {
  __shared__ double cs[64];
  if (threadIdx.x < k) cs[threadIdx.x] = c[threadIdx.x] * cscale;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = beta == 0.0 ? 0.0 : beta * y[i];
    for (int j = 0; j < k; ++j) s += cs[j] * V[(int64_t)j * ldv + i];
    y[i] = s;
  }
}

// y = x * (1 / s[0]) (normalization by a device scalar norm)
__global__ void scale_by_inv_kernel(const double* __restrict__ x, const double* __restrict__ s, double* __restrict__ y,
                                    int64_t n) {
  const double inv = 1.0 / sqrt(s[0]);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i] * inv;
}

// r = Hx - theta x ; t = r / (diag - theta) with |denominator| >= floor, or t = r
__global__ void residual_kernel(const double* __restrict__ x, const double* __restrict__ hx,
                                const double* __restrict__ diag, const double* __restrict__ theta, double floor_,
                                int precond, double* __restrict__ r, double* __restrict__ t, int64_t n) {
  const double th = theta[0];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double ri = hx[i] - th * x[i];
    r[i] = ri;
    if (precond == 0) {
      double d = diag[i] - th;
      if (fabs(d) < floor_) d = d < 0 ? -floor_ : floor_;
      t[i] = ri / d;
    } else {
      t[i] = ri;
    }
  }
}

// Lowest eigenpairs of the symmetric k x k matrix S (row-major, lds = 32) by
// cyclic Jacobi rotations in one workgroup; writes eigenvalues ascending to
// evals and the matching eigenvectors as columns of Y (ld 32).
__global__ void __launch_bounds__(64)
small_eig_kernel(const double* __restrict__ S, int k, double* __restrict__ evals, double* __restrict__ Y,
                 double* __restrict__ theta_out) {
  __shared__ double A[32][33];
  __shared__ double Z[32][33];
  __shared__ double cs[2];
  const int t = threadIdx.x;
  for (int e = t; e < k * k; e += 64) {
    const int i = e / k, j = e % k;
    A[i][j] = 0.5 * (S[i * 32 + j] + S[j * 32 + i]);
    Z[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    __shared__ double off;
    if (t == 0) {
      double o = 0.0, d = 0.0;
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
          if (i != j) o += A[i][j] * A[i][j];
          else d += A[i][j] * A[i][j];
        }
      off = (o <= 1e-30 * (d + 1e-300)) ? -1.0 : o;
    }
    __syncthreads();
    if (off < 0.0) break;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        if (t == 0) {
          const double apq = A[p][q];
          double c = 1.0, s = 0.0;
          if (fabs(apq) > 1e-300) {
            const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
            const double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
          cs[0] = c;
          cs[1] = s;
        }
        __syncthreads();
        const double c = cs[0], s = cs[1];
        if (s != 0.0) {
          if (t < k) {  // rows p, q
            const double ap = A[p][t], aq = A[q][t];
            A[p][t] = c * ap - s * aq;
            A[q][t] = s * ap + c * aq;
          }
          __syncthreads();
          if (t < k) {  // columns p, q and eigenvectors
            const double ap = A[t][p], aq = A[t][q];
            A[t][p] = c * ap - s * aq;
            A[t][q] = s * ap + c * aq;
            const double zp = Z[t][p], zq = Z[t][q];
            Z[t][p] = c * zp - s * zq;
            Z[t][q] = s * zp + c * zq;
          }
        }
        __syncthreads();
      }
  }
  if (t == 0) {
    // selection sort of eigenvalues with their vectors
    int idx[32];
    for (int i = 0; i < k; ++i) idx[i] = i;
    for (int i = 0; i < k; ++i)
      for (int j = i + 1; j < k; ++j)
        if (A[idx[j]][idx[j]] < A[idx[i]][idx[i]]) {
          int tmp = idx[i];
          idx[i] = idx[j];
          idx[j] = tmp;
        }
    for (int i = 0; i < k; ++i) {
      evals[i] = A[idx[i]][idx[i]];
      for (int r = 0; r < k; ++r) Y[r * 32 + i] = Z[r][idx[i]];
    }
    theta_out[0] = evals[0];
  }
}

// copy the first column of Y (ld 32) into a dense coefficient vector
__global__ void column_kernel(const double* __restrict__ Y, int k, int col, double* __restrict__ c) {
  const int t = threadIdx.x;
  if (t < k) c[t] = Y[t * 32 + col];
}

// S[i][j] = S[j][i] = d[i] for i < k (new column j)
__global__ void set_col_kernel(double* __restrict__ S, int j, int k, const double* __restrict__ d) {
  const int i = threadIdx.x;
  if (i < k) {
    S[i * 32 + j] = d[i];
    S[j * 32 + i] = d[i];
  }
}

// rotate the subspace: out_j = sum_i V_i Y[i][j] for j < m
__global__ void __launch_bounds__(256)
rotate_kernel(const double* __restrict__ V, int64_t ldv, int k, const double* __restrict__ Y, int m,
              double* __restrict__ out, int64_t n) {
  __shared__ double ys[32 * 32];
  for (int e = threadIdx.x; e < k * 32; e += blockDim.x) ys[e] = Y[e];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v[32];
    for (int a = 0; a < k; ++a) v[a] = V[(int64_t)a * ldv + i];
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int a = 0; a < k; ++a) s += v[a] * ys[a * 32 + j];
      out[(int64_t)j * ldv + i] = s;
    }
  }
}

namespace {

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + 255) / 256)); }

struct Work {
  int64_t n;
  double* V;
  double* W;
  double* x;
  double* hx;
  double* r;
  double* t;
  double* tmp;      // rotation scratch, max_sub vectors
  double* partial;  // kRedBlocks * 32
  double* d;        // 32 dots
  double* S;        // 32 x 32
  double* Y;        // 32 x 32
  double* ev;       // 32
  double* sc;       // scalars: [0] theta, [1] |r|^2, [2] norm^2
};

void dots(const Work& w, const double* Vb, int k, const double* v, double* out, hipStream_t s) {
  int nb = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (w.n + 255) / 256));
  hipLaunchKernelGGL(multi_dot_kernel, dim3(nb), dim3(256), 0, s, Vb, w.n, k, v, w.n, w.partial);
  hipLaunchKernelGGL(finish_dot_kernel, dim3(1), dim3(64), 0, s, w.partial, nb, k, out);
}

}  // namespace

DavidsonResult davidson(HpsiPlan& plan, const double* diag, double* psi, const DavidsonOpts& o,
                        DevBuf& work, hipStream_t s) {
  DavidsonResult res;
  const int64_t n = plan.lay.n_elems;
  const int M = std::min(std::max(o.max_sub, 4), 30);
  const int R = std::min(std::max(o.restart, 1), M - 2);
  const int64_t nvec = 2 * (int64_t)M + 4 + M;
  const int64_t small = kRedBlocks * 32 + 32 + 32 * 32 * 2 + 32 + 8;
  work.reserve((size_t)(nvec * n + small) * sizeof(double));
  Work w;
  w.n = n;
  double* base = static_cast<double*>(work.p);
  w.V = base;
  w.W = w.V + M * n;
  w.x = w.W + M * n;
  w.hx = w.x + n;
  w.r = w.hx + n;
  w.t = w.r + n;
  w.tmp = w.t + n;
  w.partial = w.tmp + M * n;
  w.d = w.partial + kRedBlocks * 32;
  w.S = w.d + 32;
  w.Y = w.S + 32 * 32;
  w.ev = w.Y + 32 * 32;
  w.sc = w.ev + 32;
  const int G = grid_for(n);
  // every product replays one captured graph on fixed staging buffers
  plan.stage_in.reserve(std::max<int64_t>(1, n) * sizeof(double));
  plan.stage_out.reserve(std::max<int64_t>(1, n) * sizeof(double));
  double* sin = static_cast<double*>(plan.stage_in.p);
  double* sout = static_cast<double*>(plan.stage_out.p);
  int prec = o.precision;
  auto H = [&](const double* in, double* out) {
    BSD_HIP(hipMemcpyAsync(sin, in, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    run_hpsi_graph(plan, sin, sout, s, prec);
    BSD_HIP(hipMemcpyAsync(out, sout, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    ++res.products;
  };
  auto normalize_into = [&](const double* in, double* out) {
    dots(w, in, 1, in, w.sc + 2, s);
    hipLaunchKernelGGL(scale_by_inv_kernel, dim3(G), dim3(256), 0, s, in, w.sc + 2, out, n);
  };
  double theta = 0.0, rn = 0.0;
  int total = 0;
  bool reached = false;   // the last solve stopped at its residual bound
  // one Davidson run from psi with products at `prec`; stops when the residual
  // is below tol (rel_floor * |theta| counts too: the noise level of a split
  // product) or after max_it iterations; leaves the Ritz vector in psi
  auto solve = [&](double tol, double rel_floor, int max_it) {
    reached = false;
    normalize_into(psi, w.V);
    H(w.V, w.W);
    int k = 1;
    dots(w, w.V, 1, w.W, w.d, s);
    hipLaunchKernelGGL(set_col_kernel, dim3(1), dim3(32), 0, s, w.S, 0, 1, w.d);
    int it = 0;
    for (; it < max_it; ++it) {
      hipLaunchKernelGGL(small_eig_kernel, dim3(1), dim3(64), 0, s, w.S, k, w.ev, w.Y, w.sc);
      hipLaunchKernelGGL(column_kernel, dim3(1), dim3(32), 0, s, w.Y, k, 0, w.d);
      hipLaunchKernelGGL(combine_kernel, dim3(G), dim3(256), 0, s, w.V, n, k, w.d, 0.0, 1.0, w.x, n);
      hipLaunchKernelGGL(combine_kernel, dim3(G), dim3(256), 0, s, w.W, n, k, w.d, 0.0, 1.0, w.hx, n);
      hipLaunchKernelGGL(residual_kernel, dim3(G), dim3(256), 0, s, w.x, w.hx, diag, w.sc, o.precond_floor,
                         o.precond, w.r, w.t, n);
      dots(w, w.r, 1, w.r, w.sc + 1, s);
      double hs[2];
      BSD_HIP(hipMemcpyAsync(hs, w.sc, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      BSD_HIP(hipStreamSynchronize(s));
      theta = hs[0];
      rn = std::sqrt(std::max(0.0, hs[1]));
      res.ritz.push_back(theta);
      if (rn <= std::max(tol, rel_floor * std::fabs(theta))) {
        reached = true;
        break;
      }
      if (k == M) {
        // thick restart: keep the R lowest Ritz vectors (and their products)
        hipLaunchKernelGGL(rotate_kernel, dim3(G), dim3(256), 0, s, w.V, n, k, w.Y, R, w.tmp, n);
        BSD_HIP(hipMemcpyAsync(w.V, w.tmp, R * n * sizeof(double), hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(rotate_kernel, dim3(G), dim3(256), 0, s, w.W, n, k, w.Y, R, w.tmp, n);
        BSD_HIP(hipMemcpyAsync(w.W, w.tmp, R * n * sizeof(double), hipMemcpyDeviceToDevice, s));
        k = R;
        // projected matrix becomes diagonal in the Ritz basis
        std::vector<double> Sh(32 * 32, 0.0), evh(32);
        BSD_HIP(hipMemcpyAsync(evh.data(), w.ev, 32 * sizeof(double), hipMemcpyDeviceToHost, s));
        BSD_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < k; ++i) Sh[i * 32 + i] = evh[i];
        BSD_HIP(hipMemcpyAsync(w.S, Sh.data(), Sh.size() * sizeof(double), hipMemcpyHostToDevice, s));
      }
      // two passes of Gram-Schmidt against V
      for (int pass = 0; pass < 2; ++pass) {
        dots(w, w.V, k, w.t, w.d, s);
        hipLaunchKernelGGL(combine_kernel, dim3(G), dim3(256), 0, s, w.V, n, k, w.d, 1.0, -1.0, w.t, n);
      }
      double* vk = w.V + (int64_t)k * n;
      normalize_into(w.t, vk);
      H(vk, w.W + (int64_t)k * n);
      ++k;
      dots(w, w.V, k, w.W + (int64_t)(k - 1) * n, w.d, s);
      hipLaunchKernelGGL(set_col_kernel, dim3(1), dim3(32), 0, s, w.S, k - 1, k, w.d);
    }
    // eigenvector into psi (x is normalized up to rounding: renormalize)
    normalize_into(w.x, psi);
    total += std::min(it + 1, max_it);
  };
  // energy and residual of the normalized psi from one float64 product (no
  // new direction): the Rayleigh quotient that finishes a split run
  auto rayleigh = [&]() {
    normalize_into(psi, w.V);
    H(w.V, w.W);
    dots(w, w.V, 1, w.W, w.sc, s);
    hipLaunchKernelGGL(residual_kernel, dim3(G), dim3(256), 0, s, w.V, w.W, diag, w.sc, o.precond_floor, 1, w.r,
                       w.t, n);
    dots(w, w.r, 1, w.r, w.sc + 1, s);
    double hs[2];
    BSD_HIP(hipMemcpyAsync(hs, w.sc, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    BSD_HIP(hipMemcpyAsync(psi, w.V, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    BSD_HIP(hipStreamSynchronize(s));
    theta = hs[0];
    rn = std::sqrt(std::max(0.0, hs[1]));
    res.ritz.push_back(theta);
  };
  if (o.precision == 0) {
    solve(o.tol, 0.0, o.max_iter);
  } else {
    // split-bf16 products down to their noise level (relative product error
    // about 5e-8 for six products, 5e-6 for three), then float64 products from
    // the Ritz vector for the iterations left; with none left, one float64
    // product gives the Rayleigh quotient of the split run's vector.  Either
    // way the energy and the residual returned are float64 quantities.
    const double eps = o.precision == 2 ? 5e-8 : 5e-6;
    solve(o.tol, 4.0 * eps, o.max_iter);
    prec = 0;
    if (reached && total < o.max_iter) solve(o.tol, 0.0, o.max_iter - total);
    else rayleigh();
  }
  BSD_HIP(hipStreamSynchronize(s));
  res.energy = theta;
  res.resid = rn;
  res.iters = total;
  return res;
}

}  // namespace bsd
