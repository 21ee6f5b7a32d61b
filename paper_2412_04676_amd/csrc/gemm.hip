// Grouped block GEMM on CDNA4 FP64 matrix cores.
//
// One workgroup computes one output tile of one output matrix:
//   C_tile = beta C_tile + sum_seg alpha_seg op(A_seg)[tile rows, 0:K_seg] op(B_seg)[0:K_seg, tile cols]
// so a block of the effective-Hamiltonian product, a renormalized operator
// block, or a projected block is one "tile list + K-segment list" entry and
// every uneven sector GEMM of one phase runs in a single launch.  Operands are
// staged through LDS in K-slices of 16; each wave owns a 32x32 sub-tile made of
// 2x2 v_mfma_f64_16x16x4 accumulators.
#include "internal.h"

#include <algorithm>

namespace bsd {

typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ const double* resolve(uint64_t t, const GBases& b) {
  return reinterpret_cast<const double*>(b.b[t >> kTagShift] + (t & ((1ull << kTagShift) - 1)));
}

constexpr int KB = 16;

template <int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN)
grouped_gemm_kernel(const GTile* __restrict__ tiles, const GSeg* __restrict__ segs, GBases bases) {
  constexpr int TM = 32 * WM, TN = 32 * WN, NT = 64 * WM * WN;
  __shared__ double As[TM][KB + 1];
  __shared__ double Bs[KB][TN + 1];

  const GTile tile = tiles[blockIdx.x];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave / WN) * 32;
  const int wc = (wave % WN) * 32;
  const int mt = min(TM, tile.M - tile.m0);
  const int nt = min(TN, tile.N - tile.n0);

  double4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};

  for (int sidx = 0; sidx < tile.nseg; ++sidx) {
    const GSeg sg = segs[tile.seg0 + sidx];
    const double* A = resolve(sg.A, bases);
    const double* B = resolve(sg.B, bases);
    const bool ta = sg.flags & kTransA, tb = sg.flags & kTransB, ia = sg.flags & kIdentA;
    const double alpha = sg.alpha;
    for (int k0 = 0; k0 < sg.K; k0 += KB) {
      // stage op(A)[m0 + i][k0 + k] * alpha
      for (int e = tid; e < TM * KB; e += NT) {
        int i, k;
        if (ta) { k = e / TM; i = e % TM; } else { i = e / KB; k = e % KB; }
        const int gi = tile.m0 + i, gk = k0 + k;
        double v = 0.0;
        if (i < mt && gk < sg.K) {
          if (ia) v = (gi == gk) ? alpha : 0.0;
          else v = alpha * (ta ? A[(int64_t)gk * sg.lda + gi] : A[(int64_t)gi * sg.lda + gk]);
        }
        As[i][k] = v;
      }
      // stage op(B)[k0 + k][n0 + j]
      for (int e = tid; e < KB * TN; e += NT) {
        int j, k;
        if (tb) { j = e / KB; k = e % KB; } else { k = e / TN; j = e % TN; }
        const int gj = tile.n0 + j, gk = k0 + k;
        double v = 0.0;
        if (j < nt && gk < sg.K) v = tb ? B[(int64_t)gj * sg.ldb + gk] : B[(int64_t)gk * sg.ldb + gj];
        Bs[k][j] = v;
      }
      __syncthreads();
      const int kend = min(KB, sg.K - k0);
#pragma unroll
      for (int kk = 0; kk < KB; kk += 4) {
        if (kk >= kend) break;
        double a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = As[wr + i * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = Bs[kk + (lane >> 4)][wc + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      __syncthreads();
    }
  }
  double* C = const_cast<double*>(resolve(tile.C, bases));
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // f64 16x16x4 output: accumulator register v of lane l holds row 4 v + l / 16
        const int r = wr + i * 16 + 4 * v + (lane >> 4);
        const int c = wc + j * 16 + (lane & 15);
        if (r < mt && c < nt) {
          double* p = C + (int64_t)(tile.m0 + r) * tile.ldc + (tile.n0 + c);
          double x = acc[i][j][v];
          if (tile.beta != 0.0) x += tile.beta * (*p);
          *p = x;
        }
      }
}

// ---------------------------------------------------------------- split-bf16 variant
// Each float64 operand x is split while it is staged into LDS:
//   2 parts: x ~ h + m,          3 parts: x ~ h + m + l,
// with h = bf16(x), m = bf16(x - h), l = bf16(x - h - m) (round to nearest
// even).  The products kept are h h + h m + m h (3 MFMA products) or
// h h + h m + m h + h l + m m + l h (6 products); v_mfma_f32_16x16x32_bf16
// accumulates them in float32, and the float32 accumulators are added into
// float64 accumulators after every 256 values of K.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ double bf16_to_double(unsigned short h) {
  return (double)__uint_as_float(((unsigned int)h) << 16);
}

constexpr int KB16 = 32;     // K per MFMA step
constexpr int KPAD = 40;     // LDS row stride in bf16 (80 bytes)
constexpr int kFlushSteps = 8;

template <int WM, int WN, int NPARTS>
__global__ void __launch_bounds__(64 * WM * WN)
grouped_gemm_bf16_kernel(const GTile* __restrict__ tiles, const GSeg* __restrict__ segs, GBases bases) {
  constexpr int TM = 32 * WM, TN = 32 * WN, NT = 64 * WM * WN;
  __shared__ __attribute__((aligned(16))) unsigned short As[NPARTS][TM][KPAD];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[NPARTS][TN][KPAD];

  const GTile tile = tiles[blockIdx.x];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave / WN) * 32;
  const int wc = (wave % WN) * 32;
  const int mt = min(TM, tile.M - tile.m0);
  const int nt = min(TN, tile.N - tile.n0);

  float4_t acc[2][2];
  double4_t acc64[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
      acc64[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
    }
  int steps = 0;

  for (int sidx = 0; sidx < tile.nseg; ++sidx) {
    const GSeg sg = segs[tile.seg0 + sidx];
    const double* A = resolve(sg.A, bases);
    const double* B = resolve(sg.B, bases);
    const bool ta = sg.flags & kTransA, tb = sg.flags & kTransB, ia = sg.flags & kIdentA;
    const double alpha = sg.alpha;
    for (int k0 = 0; k0 < sg.K; k0 += KB16) {
      for (int e = tid; e < TM * KB16; e += NT) {
        int i, k;
        if (ta) { k = e / TM; i = e % TM; } else { i = e / KB16; k = e % KB16; }
        const int gi = tile.m0 + i, gk = k0 + k;
        double v = 0.0;
        if (i < mt && gk < sg.K) {
          if (ia) v = (gi == gk) ? alpha : 0.0;
          else v = alpha * (ta ? A[(int64_t)gk * sg.lda + gi] : A[(int64_t)gi * sg.lda + gk]);
        }
        const unsigned short h = bf16_rne((float)v);
        As[0][i][k] = h;
        const double r1 = v - bf16_to_double(h);
        const unsigned short m = bf16_rne((float)r1);
        As[1][i][k] = m;
        if (NPARTS == 3) As[NPARTS - 1][i][k] = bf16_rne((float)(r1 - bf16_to_double(m)));
      }
      for (int e = tid; e < KB16 * TN; e += NT) {
        int j, k;
        if (tb) { j = e / KB16; k = e % KB16; } else { k = e / TN; j = e % TN; }
        const int gj = tile.n0 + j, gk = k0 + k;
        double v = 0.0;
        if (j < nt && gk < sg.K) v = tb ? B[(int64_t)gj * sg.ldb + gk] : B[(int64_t)gk * sg.ldb + gj];
        const unsigned short h = bf16_rne((float)v);
        Bs[0][j][k] = h;
        const double r1 = v - bf16_to_double(h);
        const unsigned short m = bf16_rne((float)r1);
        Bs[1][j][k] = m;
        if (NPARTS == 3) Bs[NPARTS - 1][j][k] = bf16_rne((float)(r1 - bf16_to_double(m)));
      }
      __syncthreads();
      const int kq = (lane >> 4) * 8;
      bf16x8_t a[NPARTS][2], b[NPARTS][2];
#pragma unroll
      for (int p = 0; p < NPARTS; ++p) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
          a[p][i] = *reinterpret_cast<const bf16x8_t*>(&As[p][wr + i * 16 + (lane & 15)][kq]);
#pragma unroll
        for (int j = 0; j < 2; ++j)
          b[p][j] = *reinterpret_cast<const bf16x8_t*>(&Bs[p][wc + j * 16 + (lane & 15)][kq]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          float4_t c = acc[i][j];
          if (NPARTS == 3) {
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2][i], b[0][j], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[1][j], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[2][j], c, 0, 0, 0);
          }
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[0][j], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[1][j], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[0][j], c, 0, 0, 0);
          acc[i][j] = c;
        }
      __syncthreads();
      if (++steps == kFlushSteps) {
        steps = 0;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[i][j][v] += (double)acc[i][j][v];
            acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
          }
      }
    }
  }
  double* C = const_cast<double*>(resolve(tile.C, bases));
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wr + i * 16 + 4 * (lane >> 4) + v;
        const int c = wc + j * 16 + (lane & 15);
        if (r < mt && c < nt) {
          double* p = C + (int64_t)(tile.m0 + r) * tile.ldc + (tile.n0 + c);
          double x = acc64[i][j][v] + (double)acc[i][j][v];
          if (tile.beta != 0.0) x += tile.beta * (*p);
          *p = x;
        }
      }
}

// ---------------------------------------------------------------- wave tiles
// For small sector blocks (at most 64 x 64) the K dimension arrives in many
// short segments, so LDS staging and workgroup barriers per segment would
// dominate.  Here every wave owns one TW x TW output tile (TW = 16 or 32),
// loads its MFMA operands straight from global memory / L2 (lane l holds
// A[l % 16][k + l / 16] and B[k + l / 16][l % 16]) and never synchronizes; a
// workgroup is four independent waves.
template <int TW>
__global__ void __launch_bounds__(256)
wave_gemm_kernel(const GTile* __restrict__ tiles, int ntiles, const GSeg* __restrict__ segs, GBases bases) {
  constexpr int NI = TW / 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ti = blockIdx.x * 4 + wave;
  if (ti >= ntiles) return;
  const GTile tile = tiles[ti];
  const int mt = min(TW, tile.M - tile.m0);
  const int nt = min(TW, tile.N - tile.n0);
  const int r16 = lane & 15, kq = lane >> 4;
  double4_t acc[NI][NI];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
  for (int sidx = 0; sidx < tile.nseg; ++sidx) {
    const GSeg sg = segs[tile.seg0 + sidx];
    const double* A = resolve(sg.A, bases);
    const double* B = resolve(sg.B, bases);
    const bool ta = sg.flags & kTransA, tb = sg.flags & kTransB, ia = sg.flags & kIdentA;
    const double alpha = sg.alpha;
    bool rowok[NI], colok[NI];
    int gi[NI], gj[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      rowok[i] = i * 16 + r16 < mt;
      gi[i] = tile.m0 + i * 16 + r16;
      colok[i] = i * 16 + r16 < nt;
      gj[i] = tile.n0 + i * 16 + r16;
    }
    // 16 values of K per pass: every operand load of the pass is issued before its MFMAs
    for (int k0 = 0; k0 < sg.K; k0 += 16) {
      double a[4][NI], b[4][NI];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int k = k0 + 4 * st + kq;
        const bool kok = k < sg.K;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          double v = 0.0;
          if (rowok[i] && kok) {
            if (ia) v = (gi[i] == k) ? alpha : 0.0;
            else v = alpha * (ta ? A[(int64_t)k * sg.lda + gi[i]] : A[(int64_t)gi[i] * sg.lda + k]);
          }
          a[st][i] = v;
        }
#pragma unroll
        for (int j = 0; j < NI; ++j) {
          double v = 0.0;
          if (colok[j] && kok) v = tb ? B[(int64_t)gj[j] * sg.ldb + k] : B[(int64_t)k * sg.ldb + gj[j]];
          b[st][j] = v;
        }
      }
      const int nst = min(4, (sg.K - k0 + 3) / 4);
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        if (st >= nst) break;
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int j = 0; j < NI; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st][i], b[st][j], acc[i][j], 0, 0, 0);
      }
    }
  }
  double* C = const_cast<double*>(resolve(tile.C, bases));
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = i * 16 + 4 * v + kq;
        const int c = j * 16 + r16;
        if (r < mt && c < nt) {
          double* p = C + (int64_t)(tile.m0 + r) * tile.ldc + (tile.n0 + c);
          double x = acc[i][j][v];
          if (tile.beta != 0.0) x += tile.beta * (*p);
          *p = x;
        }
      }
}

// tile shape classes: 0 64x64, 1 32x32, 2 32x64, 3 64x32 (workgroup tiles),
// 4 16x16 and 5 32x32 wave tiles (float64 only; split-bf16 uses 1 and 0)
template <int WM, int WN>
static void launch_shape(const GTile* tiles, int ntiles, const GSeg* segs, const GBases& b, hipStream_t s,
                         int precision) {
  const dim3 grid(ntiles), block(64 * WM * WN);
  if (precision == 0)
    hipLaunchKernelGGL((grouped_gemm_kernel<WM, WN>), grid, block, 0, s, tiles, segs, b);
  else if (precision == 1)
    hipLaunchKernelGGL((grouped_gemm_bf16_kernel<WM, WN, 2>), grid, block, 0, s, tiles, segs, b);
  else
    hipLaunchKernelGGL((grouped_gemm_bf16_kernel<WM, WN, 3>), grid, block, 0, s, tiles, segs, b);
}

void launch_grouped_gemm(const GTile* tiles, int ntiles, int shape, const GSeg* segs,
                         const GBases& b, hipStream_t s, int precision) {
  if (ntiles <= 0) return;
  if (shape >= 4 && precision == 0) {
    const dim3 grid((ntiles + 3) / 4), block(256);
    if (shape == 4)
      hipLaunchKernelGGL((wave_gemm_kernel<16>), grid, block, 0, s, tiles, ntiles, segs, b);
    else
      hipLaunchKernelGGL((wave_gemm_kernel<32>), grid, block, 0, s, tiles, ntiles, segs, b);
    BSD_HIP(hipGetLastError());
    return;
  }
  switch (shape) {
    case 0: launch_shape<2, 2>(tiles, ntiles, segs, b, s, precision); break;
    case 1: launch_shape<1, 1>(tiles, ntiles, segs, b, s, precision); break;
    case 2: launch_shape<1, 2>(tiles, ntiles, segs, b, s, precision); break;
    case 3: launch_shape<2, 1>(tiles, ntiles, segs, b, s, precision); break;
    default: throw Error(1, "wave-tile lists are float64 only");
  }
  BSD_HIP(hipGetLastError());
}

// out = sum_t coef_t op(in_t); one workgroup per output block
__global__ void __launch_bounds__(256)
aggregate_kernel(const AggTask* __restrict__ tasks, const AggTerm* __restrict__ terms) {
  const AggTask t = tasks[blockIdx.x];
  const int n = t.rows * t.cols;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int r = e / t.cols, c = e % t.cols;
    double acc = 0.0;
    for (int k = 0; k < t.nt; ++k) {
      const AggTerm a = terms[t.t0 + k];
      double v;
      if (a.flags & kIdentA) v = (r == c) ? 1.0 : 0.0;
      else if (a.flags & kTransA) v = a.in[(int64_t)c * a.ldi + r];
      else v = a.in[(int64_t)r * a.ldi + c];
      acc += a.coef * v;
    }
    t.out[(int64_t)r * t.ldo + c] = acc;
  }
}

void launch_aggregate(const AggTask* tasks, const AggTerm* terms, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(aggregate_kernel, dim3(ntasks), dim3(256), 0, s, tasks, terms);
  BSD_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- plan building (host)
void GemmPlan::build(const std::vector<GemmProblem>& probs, bool wave_tiles) {
  std::vector<GTile> t[kShapes];
  std::vector<double> work[kShapes];
  std::vector<GSeg> sg;
  flops = 0.0;
  for (int c = 0; c < kShapes; ++c) shape_flops[c] = 0.0;
  for (const auto& p : probs) {
    if (p.M <= 0 || p.N <= 0) continue;
    int seg0 = (int)sg.size();
    // wave tiles for blocks up to 64 x 64 (float64 lists); otherwise the
    // workgroup tile with the smallest padded area, then fewer tiles
    const int TMs[kShapes] = {64, 32, 32, 64, 16, 32}, TNs[kShapes] = {64, 32, 64, 32, 16, 32};
    int cls = 0;
    int64_t best = -1;
    if (wave_tiles && p.M <= 64 && p.N <= 64) {
      cls = (p.M <= 16 && p.N <= 16) ? 4 : 5;
      best = 0;
    }
    for (int c = 0; c < 4 && best != 0; ++c) {
      const int64_t tm = (p.M + TMs[c] - 1) / TMs[c], tn = (p.N + TNs[c] - 1) / TNs[c];
      const int64_t area = tm * tn * TMs[c] * TNs[c];
      const int64_t score = area * 4 + tm * tn;  // area first, tile count as tie-break
      if (best < 0 || score < best) {
        best = score;
        cls = c;
      }
    }
    int64_t ktot = 0;
    for (const auto& s : p.segs) {
      if (s.K <= 0) continue;
      sg.push_back(s);
      ktot += s.K;
      if (!(s.flags & kIdentA)) {
        double f = 2.0 * p.M * (double)p.N * s.K;
        flops += f;
        shape_flops[cls] += f;
      }
    }
    int nseg = (int)sg.size() - seg0;
    for (int m0 = 0; m0 < p.M; m0 += TMs[cls])
      for (int n0 = 0; n0 < p.N; n0 += TNs[cls]) {
        GTile x;
        x.C = p.C;
        x.ldc = p.ldc;
        x.M = p.M;
        x.N = p.N;
        x.m0 = m0;
        x.n0 = n0;
        x.seg0 = seg0;
        x.nseg = nseg;
        x.beta = p.beta;
        t[cls].push_back(x);
        work[cls].push_back((double)ktot + 16.0 * nseg);
      }
  }
  wave = wave_tiles;
  // longest tiles first inside every launch (LPT order)
  std::vector<GTile> all;
  for (int c = 0; c < kShapes; ++c) {
    std::vector<int> idx(t[c].size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return work[c][a] > work[c][b]; });
    first[c] = (int)all.size();
    count[c] = (int)idx.size();
    for (int i : idx) all.push_back(t[c][i]);
  }
  tiles.reserve(std::max<size_t>(1, all.size()) * sizeof(GTile));
  segs.reserve(std::max<size_t>(1, sg.size()) * sizeof(GSeg));
  if (!all.empty()) BSD_HIP(hipMemcpy(tiles.p, all.data(), all.size() * sizeof(GTile), hipMemcpyHostToDevice));
  if (!sg.empty()) BSD_HIP(hipMemcpy(segs.p, sg.data(), sg.size() * sizeof(GSeg), hipMemcpyHostToDevice));
}

void GemmPlan::launch_shape_class(int c, const GBases& bases, hipStream_t s, int precision) const {
  BSD_CHECK(!(wave && count[4] + count[5] > 0 && precision != 0), 1, "float64 tile list launched at split precision");
  launch_grouped_gemm(static_cast<const GTile*>(tiles.p) + first[c], count[c], c,
                      static_cast<const GSeg*>(segs.p), bases, s, precision);
}

void GemmPlan::launch(const GBases& bases, hipStream_t s, int precision) const {
  for (int c = 0; c < kShapes; ++c) launch_shape_class(c, bases, s, precision);
}

}  // namespace bsd
