// Grouped block GEMM on CDNA4 FP64 matrix cores.
//
// One workgroup computes one output tile of one output matrix:
//   C_tile = beta C_tile + sum_seg alpha_seg op(A_seg)[tile rows, 0:K_seg] op(B_seg)[0:K_seg, tile cols]
// so a block of the effective-Hamiltonian product, a renormalized operator
// block, or a projected block is one "tile list + K-segment list" entry and
// every uneven sector GEMM of one phase runs in a single launch.  Operands are
// staged through LDS in K-slices of 16; each wave owns a 32x32 sub-tile made of
// 2x2 v_mfma_f64_16x16x4 accumulators.
#include <atomic>
#include <exception>
#include <system_error>
#include <thread>
#include "devutil.h"

#include <algorithm>
#include <map>
#include <set>

namespace bsd {


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
          double* p = C + (int64_t)r * tile.ldc + c;
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
          double* p = C + (int64_t)r * tile.ldc + c;
          double x = acc64[i][j][v] + (double)acc[i][j][v];
          if (tile.beta != 0.0) x += tile.beta * (*p);
          *p = x;
        }
      }
}

// ---------------------------------------------------------------- wave tiles
// For small sector blocks (at most 64 x 64) the K dimension arrives in many
// short segments, so LDS staging and workgroup barriers per segment would
// dominate.  Here every wave owns one TW x TW output tile (TW = 16 or 32) and
// never synchronizes; a workgroup is four independent waves.  The host cuts
// the segments into steps of 16 values of K.  Per step a lane (r, q) (r =
// lane % 16, q = lane / 16) feeds MFMA step s with A[r][4 s + q] (times alpha)
// and B[4 s + q][r]; operands come through buffer loads (lanes outside the
// tile or past K get an offset beyond the buffer and read zeros), descriptors
// through scalar loads two steps ahead, and two operand sets alternate.
typedef __attribute__((address_space(4))) const GSeg* cseg64_ptr;
typedef __attribute__((address_space(4))) const GTile* ctile64_ptr;
constexpr unsigned kOut64 = 0x80000000u;   // byte offset past every operand buffer
constexpr int kRawFlags = 0x00020000;      // raw buffer, 32-bit data

__device__ __forceinline__ GSeg ld_seg64(cseg64_ptr p, int i) {
  GSeg g;
  g.A = p[i].A;
  g.B = p[i].B;
  g.lda = p[i].lda;
  g.ldb = p[i].ldb;
  g.K = p[i].K;
  g.flags = p[i].flags;
  g.alpha = p[i].alpha;
  return g;
}
__device__ __forceinline__ GTile ld_tile64(ctile64_ptr p, int i) {
  GTile t;
  t.C = p[i].C;
  t.ldc = p[i].ldc;
  t.M = p[i].M;
  t.N = p[i].N;
  t.m0 = p[i].m0;
  t.n0 = p[i].n0;
  t.seg0 = p[i].seg0;
  t.nseg = p[i].nseg;
  t.beta = p[i].beta;
  return t;
}

struct WStep {
  __amdgpu_buffer_rsrc_t ra, rb;
  int ai, ak, bk, bj;   // element strides of A along (row, k) and of B along (k, column)
  int K;                // values of K left from this step (<= 0: empty step)
  int kbase;            // first K index of the step (identity operand)
  bool ident;
  double alpha;
};

__device__ __forceinline__ WStep decode64(const GSeg& g, bool valid, const GBases& bases) {
  WStep w;
  w.ra = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(resolve(g.A, bases)), (short)0, 0x7FFFFFFF, kRawFlags);
  w.rb = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(resolve(g.B, bases)), (short)0, 0x7FFFFFFF, kRawFlags);
  const bool ta = g.flags & kTransA, tb = g.flags & kTransB;
  w.ai = ta ? 1 : (int)g.lda;
  w.ak = ta ? (int)g.lda : 1;
  w.bk = tb ? 1 : (int)g.ldb;
  w.bj = tb ? (int)g.ldb : 1;
  w.K = valid ? g.K : 0;
  w.kbase = (g.flags >> kStepPassShift) * 16;
  w.ident = g.flags & kIdentA;
  w.alpha = g.alpha;
  return w;
}

template <int NI>
__device__ __forceinline__ void load_step64(const WStep& d, const bool* rowok, const int* gi, const bool* colok,
                                            const int* gj, int q, double (&a)[4][NI], double (&b)[4][NI]) {
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int k = 4 * st + q;
    const bool kok = k < d.K;
    // loads on every path (the identity operand's read zeros and its diagonal
    // is added), so the loads in flight do not depend on the operand kind and
    // the waits before the MFMAs stay exact
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const unsigned o = (rowok[i] && kok && !d.ident) ? (unsigned)(gi[i] * d.ai + k * d.ak) * 8u : kOut64;
      const double v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(d.ra, o, 0, 0));
      const double id = (d.ident && rowok[i] && kok && gi[i] == d.kbase + k) ? d.alpha : 0.0;
      a[st][i] = d.alpha * v + id;
    }
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const unsigned o = (colok[j] && kok) ? (unsigned)(k * d.bk + gj[j] * d.bj) * 8u : kOut64;
      b[st][j] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(d.rb, o, 0, 0));
    }
  }
}

template <int TW>
__global__ void __launch_bounds__(256)
wave_gemm_kernel(const GTile* __restrict__ tiles_g, int ntiles, const GSeg* __restrict__ segs_g, GBases bases) {
  constexpr int NI = TW / 16;
  const cseg64_ptr segs = (cseg64_ptr)segs_g;
  const ctile64_ptr tiles = (ctile64_ptr)tiles_g;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ti = uni(blockIdx.x * 4 + wave);
  if (ti >= ntiles) return;
  const GTile tile = ld_tile64(tiles, ti);
  const int M = tile.M, N = tile.N, m0 = tile.m0, n0 = tile.n0;
  const int seg0 = tile.seg0, nseg = tile.nseg;
  const int mt = min(TW, M - m0);
  const int nt = min(TW, N - n0);
  const int ni = (mt + 15) >> 4, nj = (nt + 15) >> 4;   // 16 x 16 sub-tiles inside the block
  const int r16 = lane & 15, q = lane >> 4;
  bool rowok[NI], colok[NI];
  int gi[NI], gj[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    rowok[i] = i * 16 + r16 < mt;
    gi[i] = m0 + i * 16 + r16;
    colok[i] = i * 16 + r16 < nt;
    gj[i] = n0 + i * 16 + r16;
  }
  double4_t acc[NI][NI];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
  auto mfma = [&](const double (&a)[4][NI], const double (&b)[4][NI], int nst) {
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      if (st >= nst) break;
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
          if (NI == 1 || (i < ni && j < nj))   // sub-tiles outside the block are skipped
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st][i], b[st][j], acc[i][j], 0, 0, 0);
    }
  };

  if (nseg > 0) {
    double a0[4][NI], b0[4][NI], a1[4][NI], b1[4][NI];
    WStep d0 = decode64(ld_seg64(segs, seg0), true, bases);
    GSeg gn = ld_seg64(segs, seg0 + min(1, nseg - 1));
    load_step64<NI>(d0, rowok, gi, colok, gj, q, a0, b0);
    for (int s = 0;; s += 2) {
      const WStep d1 = decode64(gn, s + 1 < nseg, bases);
      gn = ld_seg64(segs, seg0 + min(s + 2, nseg - 1));
      load_step64<NI>(d1, rowok, gi, colok, gj, q, a1, b1);
      mfma(a0, b0, min(4, (d0.K + 3) >> 2));
      if (s + 1 >= nseg) break;
      d0 = decode64(gn, s + 2 < nseg, bases);
      gn = ld_seg64(segs, seg0 + min(s + 3, nseg - 1));
      load_step64<NI>(d0, rowok, gi, colok, gj, q, a0, b0);
      mfma(a1, b1, min(4, (d1.K + 3) >> 2));
      if (s + 2 >= nseg) break;
    }
  }
  double* C = const_cast<double*>(resolve(tile.C, bases));
  const double beta = tile.beta;
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // f64 16x16x4 output: accumulator register v of lane l holds row 4 v + l / 16
        const int r = i * 16 + 4 * v + q;
        const int c = j * 16 + r16;
        if (r < mt && c < nt) {
          double* p = C + (int64_t)r * tile.ldc + c;
          double x = acc[i][j][v];
          if (beta != 0.0) x += beta * (*p);
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
  // one term's value at (r, c); the term is wave-uniform
  auto val = [&](const AggTerm& a, int r, int c) -> double {
    if (a.flags & kIdentA) return (r == c) ? 1.0 : 0.0;
    if (a.flags & kTransA) return a.in[(int64_t)c * a.ldi + r];
    return a.in[(int64_t)r * a.ldi + c];
  };
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    // neighbouring lanes read neighbouring addresses of most terms: row by row
    // for terms read as stored, column by column for terms read transposed
    const int r = t.col_major ? e % t.rows : e / t.cols;
    const int c = t.col_major ? e / t.rows : e % t.cols;
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    int k = 0;
    // four independent loads in flight per lane
    for (; k + 4 <= t.nt; k += 4) {
      const AggTerm a0 = terms[t.t0 + k], a1 = terms[t.t0 + k + 1];
      const AggTerm a2 = terms[t.t0 + k + 2], a3 = terms[t.t0 + k + 3];
      const double v0 = val(a0, r, c), v1 = val(a1, r, c), v2 = val(a2, r, c), v3 = val(a3, r, c);
      acc0 += a0.coef * v0;
      acc1 += a1.coef * v1;
      acc2 += a2.coef * v2;
      acc3 += a3.coef * v3;
    }
    for (; k < t.nt; ++k) {
      const AggTerm a = terms[t.t0 + k];
      acc0 += a.coef * val(a, r, c);
    }
    t.out[(int64_t)r * t.ldo + c] = (acc0 + acc1) + (acc2 + acc3);
  }
}

void launch_aggregate(const AggTask* tasks, const AggTerm* terms, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(aggregate_kernel, dim3(ntasks), dim3(256), 0, s, tasks, terms);
  BSD_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- plan building (host)
__global__ void __launch_bounds__(256)
split_reduce_kernel(const GReduce* __restrict__ red, GBases bases) {
  const GReduce t = red[blockIdx.x];
  double* C = const_cast<double*>(resolve(t.C, bases));
  const int n = t.rows * t.cols;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int r = e / t.cols, c = e % t.cols;
    const double* q = t.parts + (int64_t)r * t.ldp + c;
    double x = 0.0;
    for (int p = 0; p < t.nparts; ++p) x += q[p * t.part_stride];
    double* o = C + (int64_t)r * t.ldc + c;
    if (t.beta != 0.0) x += t.beta * (*o);
    *o = x;
  }
}

void launch_split_reduce(const GReduce* red, int n, const GBases& b, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(split_reduce_kernel, dim3(n), dim3(256), 0, s, red, b);
  BSD_HIP(hipGetLastError());
}

void GemmPlan::build(const std::vector<GemmProblem>& probs, const GemmBuildOpts& opts) {
  auto upload = [&](void* dst, const void* src, size_t bytes) {
    if (opts.upload) {
      BSD_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, opts.upload));
      BSD_HIP(hipStreamSynchronize(opts.upload));
    } else {
      BSD_HIP(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    }
  };
  const bool wave_tiles = opts.wave_tiles, plane_operands = opts.plane_operands || opts.plane_output;
  const bool split_k = opts.split_k && !opts.plane_output;
  // tile shape classes and the waves one tile of each class occupies
  const int TMs[kShapes] = {64, 32, 32, 64, 16, 32}, TNs[kShapes] = {64, 32, 64, 32, 16, 32};
  const int waves_per_tile[kShapes] = {4, 1, 2, 2, 1, 1};
  // split-K targets: about this many waves per launch, and parts of at least
  // this much work (work = sum of K + 16 per segment)
  const double kTargetWaves = opts.target_waves, kMinPartWork = opts.min_part_work;
  struct Pending {
    GTile t;
    double work;
    int group;
    double f;   // where the unit starts in its tile's segment list (fraction of the work)
  };
  std::vector<Pending> t[kShapes];
  std::vector<GSeg> sg;
  std::vector<double> segwork;
  flops = 0.0;
  for (int c = 0; c < kShapes; ++c) shape_flops[c] = shape_in_elems[c] = shape_out_bytes[c] = 0.0;
  // operands read by each shape class: (address, elements); each distinct
  // address counts once in shape_in_elems
  std::vector<std::pair<uint64_t, double>> operands[kShapes];
  for (const auto& p : probs) {
    if (p.M <= 0 || p.N <= 0) continue;
    int seg0 = (int)sg.size();
    // wave tiles for blocks up to 64 x 64 (float64 lists); otherwise the
    // workgroup tile with the smallest padded area, then fewer tiles
    int cls = 0;
    int64_t best = -1;
    if (plane_operands && p.M > opts.wave_max && p.N > opts.wave_max) {
      cls = 0;   // 64 x 64 workgroup tile on planes (operands shared through LDS)
      best = 0;
    } else if (plane_operands || (wave_tiles && p.M <= opts.wave_max && p.N <= opts.wave_max)) {
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
    double ktot = 0;
    for (const auto& s : p.segs) {
      if (s.K <= 0) continue;
      sg.push_back(s);
      segwork.push_back(s.K + 16.0);
      ktot += s.K + 16.0;
      const double kk = plane_operands ? (s.K + 7) / 8 * 8.0 : (double)s.K;
      if (!(s.flags & kIdentA)) {
        double f = 2.0 * p.M * (double)p.N * s.K;
        flops += f;
        shape_flops[cls] += f;
        operands[cls].push_back({s.A, p.M * kk});
      }
      operands[cls].push_back({s.B, p.N * kk});
    }
    shape_out_bytes[cls] += opts.plane_output ? (double)p.M * p.N * 2.0 * kPlaneParts
                                              : (double)p.M * p.N * sizeof(double) * (p.beta != 0.0 ? 2 : 1);
    int nseg = (int)sg.size() - seg0;
    for (int m0 = 0; m0 < p.M; m0 += TMs[cls])
      for (int n0 = 0; n0 < p.N; n0 += TNs[cls]) {
        GTile x;
        // tile origin: element (m0, n0) of C, or of the planes of C^T (row n0, chunk m0 / 8;
        // n0 is a multiple of 8, so the tile's rows start a row group)
        x.C = opts.plane_output
                  ? p.C + (uint64_t)(plane_off(n0, m0 / 8, 0, p.ldc) * (int64_t)sizeof(uint16_t))
                  : p.C + (uint64_t)(((int64_t)m0 * p.ldc + n0) * (int64_t)sizeof(double));
        x.ldc = p.ldc;
        x.M = p.M;
        x.N = p.N;
        x.m0 = m0;
        x.n0 = n0;
        x.seg0 = seg0;
        x.nseg = nseg;
        x.beta = p.beta;
        t[cls].push_back({x, ktot, p.group, 0.0});
      }
  }
  for (int c = 0; c < kShapes; ++c) {
    auto& v = operands[c];
    std::sort(v.begin(), v.end());
    for (size_t i = 0; i < v.size(); ++i)
      if (i == 0 || v[i].first != v[i - 1].first) shape_in_elems[c] += v[i].second;
    std::vector<std::pair<uint64_t, double>>().swap(v);
  }
  wave = wave_tiles || plane_operands;
  planes = plane_operands;
  planes_out = opts.plane_output;
  // split long tiles into parts of about equal work: each part accumulates its
  // own contiguous run of segments into a workspace slot, and one reduction per
  // split tile adds the parts in a fixed order (deterministic results)
  std::vector<GTile> all;
  std::vector<int64_t> slot;      // per entry of `all`: workspace offset (doubles), -1 = direct
  std::vector<GReduce> red;
  std::vector<int64_t> red_off;   // per reduction: workspace offset of part 0
  int64_t ws_elems = 0;
  for (int c = 0; c < kShapes; ++c) {
    double total = 0.0;
    for (const auto& x : t[c]) total += x.work;
    const double target = std::max(kMinPartWork, total * waves_per_tile[c] / kTargetWaves);
    std::vector<std::pair<Pending, int64_t>> units;
    for (const auto& x : t[c]) {
      const int nparts = split_k ? (int)std::min<double>(x.t.nseg, std::ceil(x.work / target)) : 1;
      if (nparts <= 1) {
        units.push_back({x, -1});
        continue;
      }
      const int64_t stride = (int64_t)TMs[c] * TNs[c];
      const double per = x.work / nparts;
      const int send = x.t.seg0 + x.t.nseg;
      int s0 = x.t.seg0, made = 0;
      double acc = 0.0;
      for (int si = x.t.seg0; si < send; ++si) {
        acc += segwork[si];
        if (si == send - 1 || acc >= per * (made + 1)) {
          Pending u = x;
          u.t.seg0 = s0;
          u.t.nseg = si + 1 - s0;
          u.t.ldc = TNs[c];
          u.t.beta = 0.0;
          u.work = 0.0;
          for (int k = s0; k <= si; ++k) u.work += segwork[k];
          u.f = (acc - u.work) / x.work;
          units.push_back({u, ws_elems + (int64_t)made * stride});
          ++made;
          s0 = si + 1;
        }
      }
      GReduce r;
      r.C = x.t.C;
      r.ldc = x.t.ldc;
      r.parts = nullptr;
      r.rows = std::min(TMs[c], x.t.M - x.t.m0);
      r.cols = std::min(TNs[c], x.t.N - x.t.n0);
      r.nparts = made;
      r.ldp = TNs[c];
      r.part_stride = stride;
      r.beta = x.t.beta;
      red.push_back(r);
      red_off.push_back(ws_elems);
      ws_elems += (int64_t)made * stride;
    }
    bool grouped = opts.xcd_order && !units.empty();
    for (const auto& u : units) grouped = grouped && u.first.group >= 0;
    if (grouped) {
      // workgroup b runs on XCD b % 8 (round-robin dispatch).  Groups go whole
      // to the least loaded XCD; inside an XCD, units run in the order of
      // where they start in their segment lists, so the waves resident at one
      // time on an XCD read the same operands through its L2.
      constexpr int kXcd = 8;
      const int per_wg = c >= 4 ? 4 : 1;
      std::map<int, double> gwork;
      for (const auto& u : units) gwork[u.first.group] += u.first.work;
      std::vector<std::pair<double, int>> gl;
      for (const auto& kv : gwork) gl.push_back({kv.second, kv.first});
      std::sort(gl.begin(), gl.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
        return a.first > b.first || (a.first == b.first && a.second < b.second);
      });
      std::map<int, int> xcd_of;
      double load[kXcd] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (const auto& g : gl) {
        const int x = (int)(std::min_element(load, load + kXcd) - load);
        xcd_of[g.second] = x;
        load[x] += g.first;
      }
      std::vector<std::pair<Pending, int64_t>> lists[kXcd];
      for (const auto& u : units) lists[xcd_of[u.first.group]].push_back(u);
      for (auto& l : lists)
        std::stable_sort(l.begin(), l.end(),
                         [](const std::pair<Pending, int64_t>& a, const std::pair<Pending, int64_t>& b) {
                           return a.first.f < b.first.f || (a.first.f == b.first.f && a.first.work > b.first.work);
                         });
      size_t pos[kXcd] = {0, 0, 0, 0, 0, 0, 0, 0};
      std::vector<std::pair<Pending, int64_t>> order;
      order.reserve(units.size());
      for (int wg = 0; order.size() < units.size(); ++wg) {
        int x = wg % kXcd;
        for (int k = 0; k < per_wg && order.size() < units.size(); ++k) {
          if (pos[x] >= lists[x].size()) {   // this XCD's list is done: lend from the longest
            size_t best = 0;
            for (int y = 0; y < kXcd; ++y)
              if (lists[y].size() - pos[y] > best) {
                best = lists[y].size() - pos[y];
                x = y;
              }
          }
          order.push_back(lists[x][pos[x]++]);
        }
      }
      units.swap(order);
    } else {
      // longest units first inside every launch (LPT order), ties in list order
      std::vector<std::pair<double, uint32_t>> key(units.size());
      for (size_t i = 0; i < key.size(); ++i) key[i] = {-units[i].first.work, (uint32_t)i};
      std::sort(key.begin(), key.end());
      std::vector<std::pair<Pending, int64_t>> order;
      order.reserve(units.size());
      for (const auto& k : key) order.push_back(units[k.second]);
      units.swap(order);
    }
    first[c] = (int)all.size();
    count[c] = (int)units.size();
    for (const auto& u : units) {
      all.push_back(u.first.t);
      slot.push_back(u.second);
    }
  }
  if (plane_operands) {
    // one step per pass of 32 K values; split-K cuts above fall on segment
    // boundaries, so every unit starts fresh and ends with a flush
    BSD_CHECK(slot.size() == all.size(), 1, "tile bookkeeping");
    std::vector<GSeg> steps;
    std::vector<int> first_step(sg.size() + 1);
    for (size_t si = 0; si < sg.size(); ++si) {
      first_step[si] = (int)steps.size();
      const GSeg& g = sg[si];
      BSD_CHECK((g.A >> kTagShift) == 0 && (g.B >> kTagShift) == 0, 1, "plane operands must be absolute addresses");
      const int npass = (g.K + 31) / 32;
      for (int p = 0; p < npass; ++p) {
        GSeg x = g;
        x.K = g.K - 32 * p;
        x.flags = (g.flags & kIdentA) | (p == 0 ? kStepFresh : 0) | (p == npass - 1 ? kStepEnd : 0) |
                  (p << kStepPassShift);
        const uint64_t adv = (uint64_t)p * 4 * kPlaneParts * 64 * sizeof(uint16_t);
        if (!(g.flags & kIdentA)) x.A += adv;
        x.B += adv;
        steps.push_back(x);
      }
    }
    first_step[sg.size()] = (int)steps.size();
    for (auto& x : all) {
      const int a = first_step[x.seg0], b = first_step[x.seg0 + x.nseg];
      x.seg0 = a;
      x.nseg = b - a;
    }
    sg.swap(steps);
  }
  if (!plane_operands && count[4] + count[5] > 0) {
    // float64 wave tiles: steps of 16 values of K; a step's K counts the values
    // left from its start, the pass index rides in the flags (identity operand)
    std::vector<GSeg> st;
    std::vector<int> first_step(sg.size() + 1);
    for (size_t si = 0; si < sg.size(); ++si) {
      first_step[si] = (int)st.size();
      const GSeg& g = sg[si];
      const int npass = (g.K + 15) / 16;
      for (int p = 0; p < npass; ++p) {
        GSeg x = g;
        x.K = g.K - 16 * p;
        x.flags = (g.flags & (kTransA | kTransB | kIdentA)) | (p << kStepPassShift);
        const uint64_t da = (uint64_t)(16 * p) * ((g.flags & kTransA) ? (uint64_t)g.lda : 1u) * sizeof(double);
        const uint64_t db = (uint64_t)(16 * p) * ((g.flags & kTransB) ? 1u : (uint64_t)g.ldb) * sizeof(double);
        if (!(g.flags & kIdentA)) x.A += da;
        x.B += db;
        st.push_back(x);
      }
    }
    first_step[sg.size()] = (int)st.size();
    for (int c = 4; c <= 5; ++c)
      for (int i = first[c]; i < first[c] + count[c]; ++i) {
        GTile& x = all[i];
        const int a = first_step[x.seg0], b = first_step[x.seg0 + x.nseg];
        x.seg0 = a;
        x.nseg = b - a;
      }
    steps.reserve(std::max<size_t>(1, st.size()) * sizeof(GSeg));
    if (!st.empty()) upload(steps.p, st.data(), st.size() * sizeof(GSeg));
  }
  if (ws_elems > 0) parts.reserve(ws_elems * sizeof(double));
  double* ws = static_cast<double*>(parts.p);
  for (size_t i = 0; i < all.size(); ++i)
    if (slot[i] >= 0) all[i].C = tag_ptr(0, (uint64_t)(uintptr_t)(ws + slot[i]));
  for (size_t i = 0; i < red.size(); ++i) red[i].parts = ws + red_off[i];
  nreduce = (int)red.size();
  tiles.reserve(std::max<size_t>(1, all.size()) * sizeof(GTile));
  segs.reserve(std::max<size_t>(1, sg.size()) * sizeof(GSeg));
  if (!all.empty()) upload(tiles.p, all.data(), all.size() * sizeof(GTile));
  if (!sg.empty()) upload(segs.p, sg.data(), sg.size() * sizeof(GSeg));
  if (nreduce > 0) {
    reduces.reserve(red.size() * sizeof(GReduce));
    upload(reduces.p, red.data(), red.size() * sizeof(GReduce));
  }
}

void parallel_jobs(int n, const std::function<void(int, hipStream_t)>& fn) {
  if (n <= 0) return;
  const int nt = std::min<int>(n, (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
  int dev = 0;
  BSD_HIP(hipGetDevice(&dev));
  std::atomic<int> next{0};
  std::vector<std::exception_ptr> errs(n);
  std::vector<std::thread> pool;
  auto worker = [&] {
    hipStream_t up = nullptr;
    try {
      BSD_HIP(hipSetDevice(dev));
      BSD_HIP(hipStreamCreateWithFlags(&up, hipStreamNonBlocking));
    } catch (...) {
      up = nullptr;
    }
    for (int i; (i = next.fetch_add(1)) < n;) {
      try {
        BSD_CHECK(up != nullptr, 1, "no copy stream for a planning thread");
        fn(i, up);
      } catch (...) {
        errs[i] = std::current_exception();
      }
    }
    if (up) (void)hipStreamDestroy(up);
  };
  for (int t = 0; t < nt; ++t) {
    try {
      pool.emplace_back(worker);
    } catch (const std::system_error&) {
      break;   // fewer threads: the running ones (or this one) take every job
    }
  }
  if (pool.empty()) worker();
  for (auto& th : pool) th.join();
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
}

void GemmPlan::launch_shape_class(int c, const GBases& bases, hipStream_t s, int precision) const {
  if (planes) {
    BSD_CHECK(precision != 0, 1, "plane-operand tile list launched at float64 precision");
    launch_planes_gemm(static_cast<const GTile*>(tiles.p) + first[c], count[c], c,
                       static_cast<const GSeg*>(segs.p), bases, s, precision, planes_out);
    return;
  }
  BSD_CHECK(!(wave && count[4] + count[5] > 0 && precision != 0), 1, "float64 tile list launched at split precision");
  // wave classes read the 16-K steps, workgroup classes the segments
  const void* sp = (c == 4 || c == 5) ? steps.p : segs.p;
  launch_grouped_gemm(static_cast<const GTile*>(tiles.p) + first[c], count[c], c, static_cast<const GSeg*>(sp),
                      bases, s, precision);
}

void GemmPlan::launch_reduce(const GBases& bases, hipStream_t s) const {
  launch_split_reduce(static_cast<const GReduce*>(reduces.p), nreduce, bases, s);
}

void GemmPlan::launch(const GBases& bases, hipStream_t s, int precision) const {
  for (int c = 0; c < kShapes; ++c) launch_shape_class(c, bases, s, precision);
  launch_reduce(bases, s);
}

}  // namespace bsd
