/*
 * bsdmrg: block-sparse U(1)xU(1) two-site DMRG hot path on AMD MI355X (gfx950).
 *
 * C ABI of the shared library libbsdmrg.so.  The calls follow the problem
 * statement of the ab initio DMRG sweep (Menczer & Legeza, arXiv:2412.04676):
 * load one- and two-electron integrals (Hamiltonian, Eq. 1), set MPS site
 * tensors (Eq. 2), build and renormalize block operators (Sec. II.B, steps 1
 * and 3), apply the effective Hamiltonian to a two-site wave function
 * (Sec. II.B, step 2), and serialize / deserialize / offload block operators
 * (Sec. III.A strategy 2 and Sec. III.B.2).
 *
 * Conventions
 *  - Spatial orbital i is site i.  Spin-orbital p = 2 i + sigma (sigma 0 alpha,
 *    1 beta); Jordan-Wigner order 0a, 0b, 1a, 1b, ...  Local site basis:
 *    0 |0>, 1 a+_a|0>, 2 a+_b|0>, 3 a+_a a+_b|0>.
 *  - Hamiltonian: H = sum h_pq a+_ps a_qs
 *        + 1/2 sum (pq|rs) a+_ps a+_rt a_st a_qs  (chemists' order, no core term).
 *  - A quantum number is (n_alpha, n_beta).  Bond n lies between sites n-1 and
 *    n; its sector label counts the electrons on sites 0..n-1.
 *  - All floating-point data are float64, row-major.
 *  - Buffers are owned by the caller.  "dev" pointers are device memory on the
 *    current HIP device, "host" pointers are host memory; pinned host memory is
 *    required where stated.  The library owns only its context and the block
 *    operators it builds.
 *  - Stream-ordered calls enqueue work on the given stream and return; calls
 *    documented as synchronizing wait for their stream before returning.
 *  - Every call returns a status code (BSDMRG_OK = 0).  On error nothing is
 *    launched, and bsdmrg_last_error() (thread-local) describes the failure.
 *    No C++ exception crosses this interface.
 */
#ifndef BSDMRG_H
#define BSDMRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* bsdmrg_stream_t; /* a hipStream_t (NULL = default stream) */
typedef struct bsdmrg_ctx bsdmrg_ctx;

enum {
  BSDMRG_OK = 0,
  BSDMRG_EINVAL = 1,   /* invalid argument */
  BSDMRG_ESTATE = 2,   /* call out of order (missing integrals, tensors or blocks) */
  BSDMRG_ESHAPE = 3,   /* sizes or sectors inconsistent */
  BSDMRG_ENOMEM = 4,   /* buffer too small or allocation failure */
  BSDMRG_EHIP = 5,     /* HIP runtime error */
  BSDMRG_EBUSY = 6,    /* block is not resident on the device */
  BSDMRG_ECORRUPT = 7  /* serialized stream does not match the target */
};

enum { BSDMRG_LEFT = 0, BSDMRG_RIGHT = 1 };
/* Precision of the sector GEMMs.  FP64: float64 matrix cores.  BF16X3 /
 * BF16X6: every float64 operand is split into 2 / 3 bfloat16 parts (round to
 * nearest even) and the 3 / 6 leading cross products run on bf16 matrix cores
 * with float32 accumulation over one K-segment (one sector product), whose sum
 * times its coefficient is added into float64; the channels with the largest
 * operators stay float64 (bsdmrg_set_split_policy).  Inputs, outputs and all
 * vector arithmetic stay float64. */
enum { BSDMRG_FP64 = 0, BSDMRG_BF16X3 = 1, BSDMRG_BF16X6 = 2 };

/* Last error message of the calling thread (never NULL). */
const char* bsdmrg_last_error(void);

/* Configuration of a context.  The problem is Eq. 1 restricted to the
 * (n_alpha, n_beta) sector (U(1) x U(1)); the sizes below are device budgets of
 * the steps of one DMRG iteration (Sec. II.B).  Zero selects the default. */
typedef struct {
  int32_t L;                  /* spatial orbitals (2 .. 512) */
  int32_t n_alpha, n_beta;    /* electrons of each spin */
  int32_t D_max;              /* largest bond dimension the caller will keep (advisory, >= 0) */
  size_t hpsi_ws_bytes;       /* per-chunk intermediate workspace of H.psi (default 16 GiB) */
  size_t renorm_ws_bytes;     /* workspace of one renormalization batch (default 8 GiB) */
  size_t hbm_budget_bytes;    /* device bytes the two environment blocks of a product may
                                 occupy; a product prepared above it streams its right-block
                                 operators from pinned host memory (bsdmrg_set_hbm_budget).
                                 0: no limit */
  int32_t right_normal_from;  /* as bsdmrg_set_right_normal; 0: no normal right blocks */
  int32_t flags;              /* reserved, must be 0 */
} bsdmrg_config;

/* Create a context for cfg->L spatial orbitals holding n_alpha + n_beta
 * electrons.  EINVAL if L is out of range, the electron counts do not fit, or
 * flags != 0.  Uses the current device. */
int bsdmrg_create(bsdmrg_ctx** out, const bsdmrg_config* cfg);
int bsdmrg_destroy(bsdmrg_ctx* ctx);

/* Integrals of Eq. 1: h (host, L*L) and eri (host, L^4, (pq|rs) at
 * ((p*L+q)*L+r)*L+s).  Copied into the context.  EINVAL if h is not symmetric
 * or eri violates the 8-fold permutational symmetry by more than
 * 1e-12 * max|eri|, or e_core != 0 (electronic energies only). */
int bsdmrg_load_integrals(bsdmrg_ctx* ctx, const double* h, const double* eri, double e_core);

/* MPS site tensor (Eq. 2) of `site`, given as n_blocks dense blocks.
 * meta (host, n_blocks x 5 int32): q_left_alpha, q_left_beta, s, rows, cols, where
 * q_left is the left-bond sector, s the local state, rows = d_left(q_left) and
 * cols = d_right(q_left + q_s).  data (host): the blocks one after another,
 * each row-major and compact.  The tensor must be left-canonical for sites left
 * of the two-site position and right-canonical to its right; the library does
 * not check orthogonality.  Copied to the device (synchronizing).  ESHAPE if two
 * blocks give a bond sector different dimensions. */
int bsdmrg_set_site_tensor(bsdmrg_ctx* ctx, int site, int n_blocks, const int32_t* meta,
                           const double* data);

/* Read an MPS site tensor (Eq. 2) back in the format of
 * bsdmrg_set_site_tensor (blocks in ascending (q_left, s) order).  With
 * meta == NULL only *n_blocks and *n_elems are returned; otherwise meta (host,
 * n_blocks x 5 int32) and data (host, n_elems float64) are filled.  Tensors
 * written by bsdmrg_truncate are read the same way.  ESTATE if the site has no
 * tensor.  Synchronizing. */
int bsdmrg_get_site_tensor(bsdmrg_ctx* ctx, int site, int* n_blocks, int64_t* n_elems, int32_t* meta,
                           double* data);

/* Build renormalized block operators (Sec. II.B: preprocessing and
 * renormalization).  side = BSDMRG_LEFT: blocks for bonds 0..bond from the left
 * site tensors 0..bond-1 (left blocks keep H, a+_p, a+_p a+_q, a+_p a_q and the
 * three-operator complementary operators).  side = BSDMRG_RIGHT: blocks for bonds
 * L..bond from the right site tensors bond..L-1 (right blocks keep H, a+_r and
 * the complementary operators S_x, P_pq, Q_pq of every spin-orbital to their
 * left).  Growth starts from the nearest existing block on the way to `bond`;
 * built blocks are kept.  Synchronizes `stream`. */
int bsdmrg_build_env(bsdmrg_ctx* ctx, int side, int bond, bsdmrg_stream_t stream);

/* One renormalization step (Sec. II.B step 4): the block of `bond` is
 * enlarged by one site and projected on the site tensor next to it, giving
 * the block of bond + 1 (side LEFT, site tensor `bond`, left-canonical) or of
 * bond - 1 (side RIGHT, site tensor bond - 1, right-canonical).  The source
 * block must exist and be resident (ESTATE / EBUSY otherwise).  A block that
 * already exists at the target bond is replaced.  Synchronizes `stream`. */
int bsdmrg_renormalize(bsdmrg_ctx* ctx, int side, int bond, bsdmrg_stream_t stream);

/* Free a renormalized block (0 < bond < L; the vacuum blocks stay) and every
 * prepared product plan; a later bsdmrg_build_env rebuilds the block when it
 * is needed.  Lets a caller keep only the blocks at the front of a growing
 * environment on the device.  EBUSY while an offload of the block is in
 * flight.  Synchronizes the device. */
int bsdmrg_drop_block(bsdmrg_ctx* ctx, int side, int bond);

/* Device workspace budget of one renormalization step (bytes, default 8 GiB):
 * the new block's operators are produced in batches whose aggregated operators
 * and intermediates fit it (a batch holds at least one operator).  Applies to
 * later bsdmrg_build_env calls.  EINVAL for 0. */
int bsdmrg_set_renorm_workspace(bsdmrg_ctx* ctx, size_t bytes);

/* Operator sets of right blocks built from now on: blocks at bonds >= `bond`
 * keep the normal operators of their own spin-orbitals (H, a+_r, a+_r a+_s,
 * a+_r a_s) plus S_x, the smaller set near the chain's right end; blocks at
 * lower bonds keep the complementary set (H, a+_r, S_x, P_pq, Q_pq over every
 * spin-orbital to their left; Sec. II.B step 4).  The block that switches
 * builds its complementary two-index operators as sums over the normal ones of
 * its source.  Products need the complementary set at bond site+2.  Default:
 * no normal blocks.  A normal block can only be grown from a normal block or
 * the vacuum (ESTATE from bsdmrg_build_env otherwise); a product at a site
 * whose right block is normal fails with ESTATE.  EINVAL for bond < 1. */
int bsdmrg_set_right_normal(bsdmrg_ctx* ctx, int bond);

/* Running totals of the renormalization steps done so far (Sec. II.B step 4):
 * useful flops of the grouped-GEMM phases (2mnk per product), wall seconds,
 * device seconds (per batch of new operators, from the start of its first
 * kernel to the end of its last, by events on `stream`; host planning of later
 * batches overlaps them) and the step count.  Any pointer may be NULL. */
int bsdmrg_renorm_stats(bsdmrg_ctx* ctx, double* flops, double* wall_s, double* device_s, int64_t* steps);

/* Layout of the two-site wave function at sites (site, site+1), between the
 * left block of bond `site` and the right block of bond site+2.  With meta ==
 * NULL only *n_blocks and *n_elems are returned.  Otherwise meta (host, cap >=
 * n_blocks x 8 int32) receives q_left_a, q_left_b, s1, s2, q_right_a, q_right_b
 * (bond labels), rows, cols per block, and offsets (host, n_blocks int64) each
 * block's element offset.  Blocks are compact row-major and grouped by right
 * sector. */
int bsdmrg_psi_layout(bsdmrg_ctx* ctx, int site, int* n_blocks, int64_t* n_elems, int32_t* meta,
                      int64_t* offsets);

/* Prepare the effective-Hamiltonian product at `site` (the "Tables" step:
 * term list, aggregated operators, grouped-GEMM tile lists, and the split-bf16
 * planes of the left operators).  ws_bytes bounds the per-chunk intermediate
 * workspace, the float64 products of the right operators with psi plus their
 * bf16 planes (0 = 16 GiB); larger problems are split into chunks of channels.
 * Synchronizes `stream`.  Optional: bsdmrg_hpsi prepares on first use. */
int bsdmrg_hpsi_prepare(bsdmrg_ctx* ctx, int site, int precision, size_t ws_bytes,
                        bsdmrg_stream_t stream);

/* Choose the schedule of the prepared product at `site` for `precision` (the
 * Tables step's tile and sector schedule): candidate split-K wave targets, XCD
 * placement of locality groups and, for float64, the largest block given wave
 * tiles are timed by graph replays on a scratch vector and the fastest is kept
 * for this site.  best_ms and default_ms (optional) receive the product time of
 * the chosen and of the default schedule, n_candidates (optional) the number
 * tried.  Results are identical up to the order of float64 additions.
 * Synchronizes `stream`. */
int bsdmrg_hpsi_autotune(bsdmrg_ctx* ctx, int site, int precision, bsdmrg_stream_t stream, double* best_ms,
                         double* default_ms, int* n_candidates);

/* Set the schedule of the prepared product at `site` for `precision` directly
 * (one candidate of bsdmrg_hpsi_autotune): the split-K target of waves per
 * launch (256 .. 2^20), XCD placement of locality groups (0/1) and the
 * largest block dimension given wave tiles (>= 16): for float64 larger blocks
 * use workgroup tiles; for the split precisions blocks larger in both
 * dimensions use 64 x 64 workgroup tiles whose operands go through LDS (the
 * default is 32; 2^30 keeps wave tiles everywhere).  Rebuilds the phase-2 tile lists; results are
 * identical up to the order of float64 additions.  ESTATE if not prepared. */
int bsdmrg_hpsi_schedule(bsdmrg_ctx* ctx, int site, int precision, double target_waves, int xcd_order,
                         int wave_max);

/* Device budget of the environment (Sec. III.A strategy 2; the
 * CAS(113,76) runs of Sec. IV hold more operator data than the accelerators'
 * memory).  Products prepared from now on whose left and right blocks together
 * exceed `bytes` are built in streamed form: the right block's operator blocks
 * are gathered once, chunk by chunk in the order the product reads them, into
 * pinned host memory owned by the plan; every product then copies chunk k into
 * device slot k % 2 on a side stream while chunk k - 1 computes (event
 * ordered, the compute stream waits only for a copy that is not done), and
 * reads them there.  Results are bit-identical to the resident product.  After
 * preparing, the caller may release the right block (bsdmrg_offload with
 * release); the streamed product does not read it.  0 disables streaming.
 * chunk_bytes > 0 bounds the right operators of one chunk of every product
 * prepared from now on, streamed or resident (0: no bound for resident
 * products, 1 GiB for streamed ones); two slots of the largest chunk hold
 * them on the device.  A resident and a streamed product with the same chunk
 * bound give bit-identical results. */
int bsdmrg_set_hbm_budget(bsdmrg_ctx* ctx, size_t bytes, size_t chunk_bytes);
/* Whether the prepared product at `site` streams its right operators, the
 * pinned host bytes it copies per product, and its chunk count (optional). */
int bsdmrg_hpsi_streamed(bsdmrg_ctx* ctx, int site, int* streamed, size_t* host_bytes, int* n_chunks);

/* out = H_eff psi (Sec. II.B step 2) at two-site position `site`; psi and out
 * are device buffers in the layout of bsdmrg_psi_layout and must not overlap.
 * The product (output zero-fill and every grouped launch) is captured once
 * per (psi, out, precision) into a hipGraph and replayed by later calls.
 * Stream-ordered; psi and out must stay valid until the stream reaches it. */
int bsdmrg_hpsi(bsdmrg_ctx* ctx, int site, const double* psi_dev, double* out_dev, int precision,
                bsdmrg_stream_t stream);

/* Davidson options (Sec. II.B step 2; the paper names the method but fixes
 * no parameters).  Defaults: max_iter 50, max_subspace 24, restart 4,
 * float64 products, diagonal preconditioner, tol 1e-8 on the residual 2-norm,
 * preconditioner floor 1e-4.  precond 0: t = (diag H_eff - theta)^-1 r;
 * precond 1: t = r (no preconditioner; converges faster when the block bases
 * are far from converged, e.g. random isometries). */
typedef struct {
  int32_t max_iter, max_subspace, restart, precision;  /* precision of the H.psi products */
  double tol, precond_floor;
  int32_t precond, pad;
} bsdmrg_dav_opts;

/* Lowest eigenpair of H_eff at `site` by Davidson in float64 on the device:
 * diagonal preconditioner (diag H_eff - theta)^-1 with |denominator| >= floor,
 * two Gram-Schmidt passes per new direction, thick restart.  psi_dev holds the
 * guess on entry (any nonzero vector) and the normalized eigenvector on return.
 * energy, iters, resid (host) receive the Ritz value, the iteration count and
 * the final residual norm; ritz (host, optional, cap entries) the lowest Ritz
 * value after every iteration.  opts == NULL uses the defaults.  With a split
 * precision the products run split until the residual reaches the product's
 * noise level (2e-7 |theta| for BF16X6, 2e-5 |theta| for BF16X3), then the run
 * restarts from that Ritz vector with float64 products down to tol for the
 * iterations left; if the split stage used every iteration, one float64
 * product on its Ritz vector gives the energy (the Rayleigh quotient) and the
 * residual.  Either way the energy and the residual returned are float64
 * quantities; iters counts the iterations of both stages (max_iter at most)
 * and the final float64 evaluation counts as none.  Synchronizes `stream` once per
 * iteration (a 16-byte read of theta and |r|). */
int bsdmrg_davidson(bsdmrg_ctx* ctx, int site, double* psi_dev, const bsdmrg_dav_opts* opts, double* energy,
                    int* iters, double* resid, double* ritz, int cap, bsdmrg_stream_t stream);

/* Truncation (Sec. II.B step 3) of the two-site wave function psi_dev at
 * `site` across its middle bond: the Gram matrix of each middle sector is
 * formed by the grouped GEMM and diagonalized by a parallel Jacobi method
 * (float64, one workgroup per sector, sectors up to 4096 states; ESHAPE
 * beyond).  Kept states:
 * the D largest singular values, extended to every value >= sigma_D (1 - 1e-10),
 * values <= 1e-14 sigma_max dropped.  direction 0 (left to right) replaces the
 * site tensor of `site` by the kept left singular vectors (left-canonical);
 * direction 1 replaces the tensor of site+1 by the kept right singular vectors
 * (right-canonical).  Blocks depending on the replaced tensor are dropped.
 * trunc_err receives the discarded weight, D_kept the kept count, sv (optional,
 * cap entries) the kept singular values in descending order.  Synchronizing. */
int bsdmrg_truncate(bsdmrg_ctx* ctx, int site, const double* psi_dev, int D, int direction, double* trunc_err,
                    int* D_kept, double* sv, int cap, bsdmrg_stream_t stream);

/* Start vector of the next two-site position (Fig. 9 "StVec"; Sec. II.B:
 * the wave function of one iteration step is carried into the next).  Call
 * after bsdmrg_truncate(site, psi_dev, ..., direction) and after building the
 * environment of the next position: direction 0 moves to site + 1 (left block
 * of bond site+1, right block of bond site+3 must exist) and forms
 * S V^T B_{site+2} = A_site^T psi B_{site+2}; direction 1 moves to site - 1
 * (left block of bond site-1, right block of bond site+1) and forms
 * A_{site-1} U S = A_{site-1} psi B_{site+1}^T.  psi_dev is the wave function
 * that was truncated, in the layout of `site` (its environment blocks must
 * still exist); guess_dev receives the start vector in the layout of the next
 * position (bsdmrg_psi_layout), float64 grouped GEMMs on the device.  Its
 * norm is sqrt(1 - discarded weight) for a normalized psi.  Synchronizes
 * `stream`. */
int bsdmrg_next_guess(bsdmrg_ctx* ctx, int site, int direction, const double* psi_dev, double* guess_dev,
                      bsdmrg_stream_t stream);

/* Diagonal of H_eff at `site` into diag_dev (psi layout), stream-ordered. */
int bsdmrg_hpsi_diagonal(bsdmrg_ctx* ctx, int site, double* diag_dev, bsdmrg_stream_t stream);

/* Statistics of the last prepared product at `site` (the work of Sec. II.B
 * step 2): useful flops per product (2 m n k summed over all non-identity
 * sector GEMMs), number of channels, K-segments and aggregated operators,
 * workspace bytes, and the elements of the distinct operator blocks one
 * product reads (stored and aggregated; each counted once).  Any output
 * pointer may be NULL.  ESTATE if not prepared. */
int bsdmrg_hpsi_info(bsdmrg_ctx* ctx, int site, int precision, double* flops, int64_t* n_channels,
                     int64_t* n_segments, int64_t* n_aggregates, int64_t* ws_bytes, int64_t* op_elems);

/* One product as bsdmrg_hpsi with a HIP event between consecutive kernel
 * launches (synchronizing).  For launch i (i < cap) it returns the elapsed
 * milliseconds ms[i], the algorithmic flops flops[i] of that launch, its
 * algorithmic HBM bytes bytes[i] (every distinct operand block read once plus
 * the output; bytes may be NULL) and its kind
 * kind[i] (0 output zero-fill; 10 + c phase-1 and 20 + c phase-2 grouped GEMM
 * with tile shape class c: 0 64x64, 1 32x32, 2 32x64, 3 64x32 workgroup tiles,
 * 4 16x16 and 5 32x32 wave tiles; 16 and 26 the reduction that sums the
 * split-K parts of phase 1 and phase 2).  Launches with no tiles are skipped.
 * *n_launches receives the number of launches. */
int bsdmrg_hpsi_profile(bsdmrg_ctx* ctx, int site, const double* psi_dev, double* out_dev, int precision,
                        bsdmrg_stream_t stream, int cap, double* ms, double* flops, double* bytes,
                        int* kind, int* n_launches);

/* Copy one renormalized block operator to the host (synchronizing).  kind is
 * one of 'H','c','A','B','S','P','Q' with spin-orbital indices p, q (-1 if
 * unused).  With data == NULL, *n_blocks and *n_elems are returned.  Otherwise
 * meta (n_blocks x 6 int32: q_in_a, q_in_b, q_out_a, q_out_b, rows, cols; labels
 * count the electrons inside the block) and data (compact row-major) are filled.
 * ESTATE if the operator does not exist. */
int bsdmrg_get_block_op(bsdmrg_ctx* ctx, int side, int bond, char kind, int p, int q,
                        int* n_blocks, int64_t* n_elems, int32_t* meta, double* data);

/* Batched dense block GEMMs on the matrix cores, the primitive behind every
 * sector product: C_i = alpha_i op(A_i) op(B_i) + beta_i C_i for each problem
 * (device pointers, row-major, op = transpose if trans != 0).  Problems must
 * not write overlapping C regions.  Synchronizes `stream` (problem lists are
 * uploaded per call). */
typedef struct {
  const double* A;
  const double* B;
  double* C;
  int32_t M, N, K;
  int32_t transA, transB;
  int32_t pad;
  int64_t lda, ldb, ldc;
  double alpha, beta;
} bsdmrg_gemm_desc;
int bsdmrg_block_gemm(int n, const bsdmrg_gemm_desc* problems, int precision, bsdmrg_stream_t stream);

/* ---------------------------------------------------------------- serializer
 * Stream format: header (64 B), family table (64 B per family), block tables
 * (32 B per block), zero padding to 256 B, then every family's payload
 * (n_layers layers of its blocks, compact row-major, layer after layer) padded
 * to 256 B.  The size is exact and known before packing (Sec. III.B.2). */
typedef struct {
  uint64_t tag;                 /* caller-defined id stored in the stream */
  int32_t dq[2];                /* quantum-number change of every layer */
  int32_t n_layers, n_blocks;
  const int32_t* block_q;       /* host, n_blocks x 2: input sector of each block */
  const int32_t* rows;          /* host, n_blocks */
  const int32_t* cols;          /* host, n_blocks */
  const int32_t* ld;            /* host, n_blocks: leading dimension in memory (>= cols) */
  const int64_t* elem_offset;   /* host, n_blocks: element offset of each block inside a layer */
  int64_t layer_stride;         /* elements between consecutive layers */
  void* data;                   /* device base of layer 0 (16-byte aligned) */
} bsdmrg_family_desc;

/* Exact size in bytes of the stream of n families (host arithmetic only). */
int bsdmrg_serialized_size_desc(int n, const bsdmrg_family_desc* fams, size_t* bytes);
/* Serialize families into dst_dev (device, 256-byte aligned, cap bytes).
 * ENOMEM if cap is smaller than the exact size.  Synchronizes `stream`. */
int bsdmrg_pack_desc(int n, const bsdmrg_family_desc* fams, void* dst_dev, size_t cap,
                     bsdmrg_stream_t stream);
/* Deserialize src_dev (device, 256-byte aligned) into the families' memory.
 * The stream's tables must match the families' skeletons exactly, else
 * ECORRUPT and no family memory is written.  Synchronizes `stream`. */
int bsdmrg_unpack_desc(int n, const bsdmrg_family_desc* fams, const void* src_dev, size_t bytes,
                       bsdmrg_stream_t stream);

/* bsdmrg_pack_desc for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): allocates nothing.  The descriptor tables go through a
 * file-scope host array into a file-scope device array of
 * bsdmrg_noalloc_scratch_bytes() bytes (16 MiB) that each GPU holds until the
 * process ends; EINVAL, before any launch, if the tables of the given
 * families exceed it (about 32 bytes per block plus 24 per copy task).  The
 * caller passes the families and dst_dev as for bsdmrg_pack_desc; the bytes
 * written are identical.  Every call on one GPU uses that GPU's array and
 * leaves its tables there; two calls that overlapped would race on it, so
 * calls are serialized (a mutex across host threads) and each synchronizes
 * `stream` before returning. */
int bsdmrg_pack_desc_noalloc(int n, const bsdmrg_family_desc* fams, void* dst_dev, size_t cap,
                             bsdmrg_stream_t stream);
int bsdmrg_noalloc_scratch_bytes(size_t* bytes);

/* The same for all operator families of a renormalized block. */
int bsdmrg_serialized_size(bsdmrg_ctx* ctx, int side, int bond, size_t* bytes);
int bsdmrg_pack(bsdmrg_ctx* ctx, int side, int bond, void* dst_dev, size_t cap, bsdmrg_stream_t stream);
int bsdmrg_unpack(bsdmrg_ctx* ctx, int side, int bond, const void* src_dev, size_t bytes,
                  bsdmrg_stream_t stream);

/* Asynchronous offload of a block (Sec. III.A strategy 2, Sec. III.B.4):
 * pack into staging_dev on `compute` (synchronizing only the host-side
 * descriptor upload the first time), then a device-to-host copy into
 * pinned_host (allocated with hipHostMalloc) on `side`, ordered after the pack
 * by an event.  Returns immediately after enqueueing the copy.  The pack waits
 * on `compute` for the last copy or unpack that used staging_dev (the library
 * tracks each staging buffer by address).  With release != 0 the block's
 * device memory is freed by bsdmrg_offload_wait once the copy has completed
 * (the block then reports EBUSY until prefetched); products and serializer
 * descriptors of the block stay valid where the device has virtual memory
 * management (the block keeps its address range and only its physical memory
 * is returned).  staging_dev and pinned_host must hold
 * bsdmrg_serialized_size bytes; pinned_host must stay valid until
 * bsdmrg_offload_wait returns. */
int bsdmrg_offload(bsdmrg_ctx* ctx, int side, int bond, void* staging_dev, void* pinned_host,
                   size_t cap, int release, bsdmrg_stream_t compute, bsdmrg_stream_t side_stream);
/* Block until the last offload of (side, bond) has reached host memory
 * ("fetching", the blocking wait of Sec. III.B.4 when the copy is not yet
 * done), then free the device memory if the offload asked for it.  The host
 * wait in seconds goes to *waited_s (optional) and into the statistics as
 * exposed IO. */
int bsdmrg_offload_wait(bsdmrg_ctx* ctx, int side, int bond, double* waited_s);
/* Reload a block (Sec. III.B.4): validate pinned_host on the host, copy it to
 * staging_dev on `side` (after the last pack or unpack that used staging_dev),
 * then unpack on `compute` after an event (backing the block with device
 * memory again if it was released; the unpack writes every element).  Work
 * enqueued on `compute` before this call runs before the unpack and overlaps
 * the copy; work enqueued after it reads the restored block.  staging_dev and
 * pinned_host must stay valid until the unpack has run (bsdmrg_prefetch_wait,
 * or any later synchronization of `compute`).  ECORRUPT if the stream does not
 * match the block. */
int bsdmrg_prefetch(bsdmrg_ctx* ctx, int side, int bond, const void* pinned_host, void* staging_dev,
                    size_t bytes, bsdmrg_stream_t compute, bsdmrg_stream_t side_stream);
/* Block until the last prefetch of (side, bond) has been unpacked; the host
 * wait in seconds goes to *waited_s (optional) and into the exposed IO. */
int bsdmrg_prefetch_wait(bsdmrg_ctx* ctx, int side, int bond, double* waited_s);
/* Precision policy of split products (BF16X3, BF16X6): with fp64_heavy = 1
 * (the default) the channels whose right operator is the identity, the block
 * Hamiltonian H or a diagonal two-index operator Q_pp run on the float64
 * matrix cores inside every split product.  They carry the bulk of the energy
 * (the particle-number-dependent Coulomb and exchange sums of Eq. 1) and the
 * largest operator entries, so they dominate the rounding error of a split
 * product while being a small share of its work.  0 splits every channel.
 * Applies to products prepared from now on. */
int bsdmrg_set_split_policy(bsdmrg_ctx* ctx, int fp64_heavy);

/* Test hook for the fetching path of Sec. III.B.4: every later side-stream
 * copy of bsdmrg_offload / bsdmrg_prefetch is preceded by a host function that
 * sleeps `ms` milliseconds on the side stream (0 disables; at most 10 s), so
 * the copy finishes late and the blocking waits become visible. */
int bsdmrg_set_side_delay(bsdmrg_ctx* ctx, double ms);

/* Segmented offload in the synchronous small-buffer form of Sec. III.A
 * (strategy 1, Fig. 4b) with self-contained packages (Sec. III.B.3).  The
 * block's families are cut into segments of whole layers that fit half of
 * staging_dev (staging_bytes, 256-byte aligned); a segment is packed into one
 * half on `compute` while the other half is copied to pinned_host on `side`.
 * Every segment starts with a 256-byte little-endian header: bytes 0-7 magic
 * "BSDSEG01", u64 owner at 8 (the block's family tags with the low 20 bits
 * cleared), u32 family at 16, u32 family count at 20, u32 first layer at 24,
 * u32 layer count at 28, u64 payload bytes at 32, u64 skeleton fingerprint at
 * 40 (64-bit FNV-1a over the 8-byte little-endian values of dq, the layer
 * count and every block's sector, rows and cols), u64 segment index at 48,
 * zeros to 256.  Its layers follow (blocks compact row-major, as in the
 * one-stream payload), zero padded to 256 B, so segments can be stored, moved
 * and read back in any order.
 * bsdmrg_segments_size gives the exact total and the segment count for a
 * staging size (host arithmetic).  ENOMEM if half the staging area cannot hold
 * one layer of a family or cap is too small.  Synchronizing; *written gets the
 * bytes written. */
int bsdmrg_segments_size(bsdmrg_ctx* ctx, int side, int bond, size_t staging_bytes, size_t* bytes,
                         int* n_segments);
int bsdmrg_pack_segments(bsdmrg_ctx* ctx, int side, int bond, void* staging_dev, size_t staging_bytes,
                         void* pinned_host, size_t cap, size_t* written, int* n_segments,
                         bsdmrg_stream_t compute, bsdmrg_stream_t side_stream);
/* Read segments (any order, back to back in pinned_host, `bytes` in total)
 * into the block through the same double-buffered staging area, backing a
 * released block with device memory again.  Every header is checked first:
 * ECORRUPT, with nothing written, unless the segments belong to this block,
 * match its skeletons and cover every layer of every family exactly once.
 * Synchronizing. */
int bsdmrg_unpack_segments(bsdmrg_ctx* ctx, int side, int bond, const void* pinned_host, size_t bytes,
                           void* staging_dev, size_t staging_bytes, bsdmrg_stream_t compute,
                           bsdmrg_stream_t side_stream);
/* Workgroups of the serializer's copy launches for all later packs and
 * unpacks (0: one per copy task, the default).  The bytes written do not
 * depend on it (Sec. III.B.2: the serializing threads are independent). */
int bsdmrg_set_copy_workgroups(int workgroups);

/* Device bytes held by the block operators of (side, bond) (Sec. III.A: the
 * memory the offload frees). */
int bsdmrg_block_bytes(bsdmrg_ctx* ctx, int side, int bond, size_t* bytes);

/* Operator families of a renormalized block (Sec. III.B.2: operators sharing
 * one block-sparse skeleton are serialized together): *n_families families
 * holding *n_operators operators in total.  Either pointer may be NULL.
 * ESTATE if the block is not built. */
int bsdmrg_family_count(bsdmrg_ctx* ctx, int side, int bond, int* n_families, int* n_operators);

/* Running statistics of the context, in the wall-time categories of the
 * paper's profile of one DMRG sweep (Fig. 9): seconds[] is indexed by the
 * BSDMRG_PH_* constants and measured on the host around synchronizing calls
 * (asynchronous calls add their enqueue time only; H.psi products are counted
 * in hpsi_calls and hpsi_flops).  io_exposed_s is the time spent blocked in
 * bsdmrg_offload_wait (the fetch that could not be hidden, Sec. III.B.4). */
enum {
  BSDMRG_PH_TABLES = 0,   /* product plans: term lists, tile lists, operator planes */
  BSDMRG_PH_DIAG_H = 1,   /* Davidson (products and vector work) */
  BSDMRG_PH_REN_L = 2,    /* renormalization of left blocks */
  BSDMRG_PH_REN_R = 3,    /* renormalization of right blocks */
  BSDMRG_PH_SVD = 4,      /* truncation */
  BSDMRG_PH_STVEC = 5,    /* transformation of the wave function into the next guess */
  BSDMRG_PH_IO = 6,       /* pack, unpack, offload and prefetch calls */
  BSDMRG_N_PHASES = 7
};
typedef struct {
  double seconds[8];
  double io_exposed_s;
  double hpsi_flops, renorm_flops;          /* useful flops (2 m n k) */
  int64_t hpsi_calls, davidson_calls, davidson_iters, truncations, renorm_steps;
  int64_t bytes_packed, bytes_unpacked, bytes_d2h, bytes_h2d;
} bsdmrg_stats_t;
/* Copy the statistics into *out; reset != 0 clears them afterwards. */
int bsdmrg_stats(bsdmrg_ctx* ctx, bsdmrg_stats_t* out, int reset);

#ifdef __cplusplus
}
#endif

#endif /* BSDMRG_H */
