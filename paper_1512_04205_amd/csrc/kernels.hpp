// Launchers of the cDMD HIP kernels (gfx950).  Every launcher enqueues on `stream`
// and returns the hipError_t of the launch.  Shapes are validated by the caller
// (api.cpp); the launchers assume them.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cdmd {
namespace k {

// ----- sketch, sparse / single-pixel, uint8 video (exact integer sums) -------------
// Triples (pixel, row | sign bit 31) grouped by segment; each segment covers rows
// [seg_r0, seg_r0 + seg_nrows) and triple range [seg_begin, seg_end), its triples
// sorted by pixel.  seg[4*s + 0..3] = begin, end, r0, nrows; part[s] is the partial
// slot of the segment inside its row block (0 .. nslot-1).
// Output: Ypart[slot][t][r] int32 (t < m, r < p) when nslot > 1, else Y directly.
hipError_t sketch_sparse_u8(const uint8_t* D, int64_t ld, int64_t m, const int32_t* tri_pix,
                            const uint32_t* tri_rs, const int32_t* seg, int nseg, int p,
                            int max_rows, int fpb, int32_t* Yout, int nslot,
                            hipStream_t stream);
// Streaming form (16-byte aligned frames): grid (nrange pixel ranges, frame groups of F,
// nblk row blocks).  Triples of row block b are sorted by pixel; chunk_off[b*(nchunk+1) + c]
// is the first triple of b with pixel >= c * chunk (chunk = sketch_stream_chunk()), and
// rblk[2b], rblk[2b+1] its first row and row count.  Output Ypart[range][t][r] (every
// range writes all its rows); LDS F * (4 max_rows + V chunk) bytes.
// V: 16-byte vectors per thread and frame (chunk V * sketch_stream_chunk() bytes);
// (F, V) in {(4,1), (2,1), (2,2), (1,1), (1,2), (1,4)} with sketch_stream_fits.
bool sketch_stream_fits(int F, int V, int max_rows);
hipError_t sketch_stream_u8(const uint8_t* D, int64_t ld, int64_t n, int64_t m, const int32_t* tri_pix,
                            const uint32_t* tri_rs, const int32_t* chunk_off, int nchunk, const int32_t* rblk,
                            int nblk, int nrange, int p, int max_rows, int F, int V, int32_t* Ypart,
                            hipStream_t stream);
int sketch_stream_chunk();
// Y[t][r] = sum_s Ypart[s][t][r]
hipError_t reduce_slots_i32(const int32_t* Ypart, int nslot, int64_t count, int32_t* Y,
                            hipStream_t stream);

// ----- sketch, sparse / single-pixel, float32 video (row order, float64 sums) ------
// Y[t][r] = sum_j sign_rj * D[t][idx_rj], j in row order.
hipError_t sketch_sparse_f32(const float* D, int64_t ld, int64_t m, const int32_t* idx,
                             const int8_t* sign, int p, int nnz, double* Y,
                             hipStream_t stream);

// ----- sketch, dense Gaussian (entries drawn on the fly) --------------------------
// prec 0: FP32 form (float64 Box-Muller rounded to float32, FP32 MFMA; dtype 0 uint8 or
// 1 float32 video); prec 1: BF16 form (float32 Box-Muller rounded to bfloat16, BF16
// MFMA); prec 2: FP8 form (rounded to e4m3, pixel bytes split into two exact e4m3
// operands, FP8 MFMA).  BF16 and FP8: uint8 video with 16-byte aligned frames only.  part: nsplit * m * p floats of
// per-slice partial sums; Y[t][r] = (1/sqrt(p)) * sum over slices (float64, m x p).
struct GaussPlan {
  int nrt, nft, nsplit, frames, rows;  // row tiles of `rows` sketch rows, frame tiles of `frames`
  int64_t pps, blocks;
};
// target: about how many workgroups to spread over (pixel slices are added until then)
GaussPlan gauss_plan(int64_t n, int64_t m, int p, int prec, int target);
// Cm: the stored C of gauss_fill for the FP8 form, or null to draw the entries (the BF16
// form refuses a stored C: that goes to the library GEMM); ldc its row stride in entries.
hipError_t sketch_gauss(const void* D, int dtype, int64_t ld, int64_t n, int64_t m, int p,
                        uint64_t seed, int prec, const GaussPlan& g, const void* Cm, int64_t ldc, float* part,
                        double* Y, hipStream_t stream);
// Row stride (entries) of a stored C for n pixels, and its fill: the entries of the FP8 form
// (prec 2: e4m3 codes; other forms are refused), p rows of ldc, zero past n.
int64_t gauss_ldc(int64_t n);
// SRFT sketch (the FP32 form's kernel with the entries of C = R F D): g = gauss_plan(n, m,
// 2 p, FP32), freq[p] the DFT rows kept; Y (m x 2p float64, frame-major) holds the real and
// imaginary part of each complex row r at 2r, 2r + 1, scaled by 1/sqrt(p).  gram_cplx: the
// Hermitian Gram Y^H Y of that sketch, real part to Gr and imaginary part to Gi (m x m).
hipError_t sketch_srft(const void* D, int dtype, int64_t ld, int64_t n, int64_t m, int p, uint64_t seed,
                       const GaussPlan& g, const int32_t* freq, float* part, double* Y, hipStream_t stream);
hipError_t gram_cplx(const double* Y, int p, int64_t m, double* Gr, double* Gi, hipStream_t stream);
// The BF16 form with a stored C as S batched library GEMMs over pixel slices of Ks
// (a multiple of 64; S Ks >= n): gauss_fill_t writes C pixel-major, Ct[j][r] (p
// contiguous per pixel, rows n..jn-1 zero), bit for bit the drawn form's entries;
// video_bf16_split writes the video as exact bfloat16 in slices, Xs[s][t][i] = x(t, s Ks + i)
// (zero past n); reduce_gauss sums the S float32 partials part[s][t][r] in order into
// Y[t][r] (float64) times scale.
hipError_t gauss_fill_t(void* Ct, int64_t jn, int64_t n, int p, uint64_t seed, hipStream_t stream);
hipError_t video_bf16_split(const void* D, int64_t ld, int64_t n, int64_t m, int64_t Ks, int S, void* Xs,
                            hipStream_t stream);
hipError_t reduce_gauss(const float* part, int nsplit, int64_t count, double scale, double* Y, hipStream_t stream);
// The FP8 form's counterparts: C pixel-major as e4m3 codes (the drawn form's, bit for bit),
// and each video byte u = 16 hi + lo as the two exact e4m3 codes of 16 hi (Xh) and lo (Xl)
// in the same split layout.
hipError_t gauss_fill_fp8_t(void* Ct, int64_t jn, int64_t n, int p, uint64_t seed, hipStream_t stream);
hipError_t video_fp8_split(const void* D, int64_t ld, int64_t n, int64_t m, int64_t Ks, int S, void* Xh, void* Xl,
                           hipStream_t stream);
hipError_t gauss_fill(void* Cm, int64_t ldc, int64_t n, int p, uint64_t seed, int prec, hipStream_t stream);

// ----- learned selector (mlp.hip) -------------------------------------------------
int mlp_nparts(int batch);
// grad / loss (either may be null) of the mean loss over nb samples (rows idx[q], or q)
hipError_t mlp_grad(const float* th, const float* X, const float* y, const int32_t* idx, int nb, float* part,
                    float* lpart, float* grad, float* loss, hipStream_t stream);
hipError_t mlp_train(float* th, float* am, float* av, const float* X, const float* y, int64_t nsamp,
                     const int32_t* idx, int batch, int steps, float lr, int64_t t0, float* part, float* lpart,
                     float* losses, hipStream_t stream);
// mlp_train with the partials in the library's static device scratch (no allocation);
// batch <= CDMD_MLP_NOALLOC_MAX_BATCH.  Calls that overlap on one device race.
hipError_t mlp_train_noalloc(float* th, float* am, float* av, const float* X, const float* y, int64_t nsamp,
                             const int32_t* idx, int batch, int steps, float lr, int64_t t0, float* losses,
                             hipStream_t stream);
hipError_t mlp_forward(const float* th, const float* X, int n, int round_bf16, float* logits, hipStream_t stream);
hipError_t mode_features(const double* lam, const double* b, const double* phin, double x1n2, int64_t m, int k,
                         float* F, hipStream_t stream);

// ----- Gram of the sketch: Gr[a][b] = sum_r Y[a][r] Y[b][r] (m x m, float64) ------
hipError_t gram_i32(const int32_t* Y, int p, int64_t m, double* Gr, hipStream_t stream);
hipError_t gram_f64(const double* Y, int p, int64_t m, double* Gr, hipStream_t stream);

// ----- lift: Phi = X' G (fp32) with fused per-block partial Gram of Phi -----------
// G is (m-1) x NC float row-major (columns >= nc are zero).  Per block, partial sums
// over its pixels: entries e < npair of Phi[:, pa]^T Phi[:, pb] (pairs[e] = pa | pb<<16),
// then nc entries Phi[:, a]^T x_1, then ||x_1||^2.  part: [grid][ne] float64.
// phi (optional): complex64 mode-contiguous store, phi[2*(j*n + i) + 0/1] =
// Phi[i, j] / Phi[i, k + j] for j < kmodes.
hipError_t lift_fp32(const void* D, int dtype, int64_t ld, int64_t n, int64_t m, const float* G,
                     int NC, int nc, const uint32_t* pairs, int npair, double* part,
                     int grid, float* phi, int kmodes, float xscale, hipStream_t stream);
int lift_grid(int64_t n);
// ----- lift on MFMA (uint8 video, 16-byte aligned frames) -------------------------
// Gp: B operands pre-arranged as [kstep][nb][split][lane][8 bf16] (kstep = 16 frames of
// X', nb = 32-column block, split = bf16 term of G), nksteps = ceil((m-1)/16).
// Column nc of Phi_ext is replaced by x_1 * xscale.  part: [grid][NP*16*64] float64,
// NP = nb(nb+1)/2 column-block pairs (a <= b); entry (q, j, lane) of pair q = (a, b) is
// P[32a + 8(j/4) + 4(lane/32) + j%4][32b + lane%32].  nb in {1,2,3}, nsplit in {1,3}.
hipError_t lift_mfma(const uint8_t* D, int64_t ld, int64_t n, int64_t m, const void* Gp, int nb,
                     int nsplit, int nksteps, int nc, float xscale, double* part, int grid,
                     float* phi, int kmodes, hipStream_t stream);
int lift_mfma_grid(int64_t n);
// out[e] = sum_b part[b][e]
hipError_t reduce_partials(const double* part, int grid, int ne, double* out,
                           hipStream_t stream);

// ----- fused background reconstruction + foreground threshold --------------------
// T = X' Gs (Gs: (m-1) x NS float, NS = 2|S| padded), then per frame t
// L_t = sum_c T[:, c] Vc[t][c]; mask = |x_t - L_t| > tau.
// mode 0: bit-packed mask (uint32 words, ceil(n/32) per frame)
// mode 1: uint8 mask (n per frame)
// mode 2: write L (float, frames t0..t1-1 at (t - t0) * ldL)
hipError_t bgfg(const void* D, int dtype, int64_t ld, int64_t n, int64_t m, const float* Gs,
                int NS, const float* Vc, float tau, float xscale, int mode, void* out,
                int64_t t0, int64_t t1, int64_t ldL, hipStream_t stream);
// Single-read form on MFMA (uint8 video, 16-byte aligned frames, |S| <= 16): 128-pixel
// tiles whose frames stay in LDS.  Gp, Vp: the operands recon_prep writes (KS =
// recon_ksteps(m) k-steps plus 4 zero ones, NFB = recon_frame_blocks(m) frame blocks plus
// a zero one).  nsg/ntv: (2, 3) float32-class L,
// (1, 2) bfloat16 form.
struct ReconArgs {
  const uint8_t* D;
  int64_t ld, n, m;
  const uint4* Gp;
  const uint4* Vp;
  int KS, NFB, ns;
  float tau, xscale;
  int mode;
  void* out;
  int64_t t0, t1, ldL;
};
hipError_t recon_mfma(const ReconArgs& a, int nsg, int ntv, hipStream_t stream);
// Pixels per workgroup tile of recon_mfma.
int recon_tile_pixels();
// One entry of a work list of reconstructions: tiles tile0 .. tile0 + ntiles - 1 of a are
// tiles start .. start + ntiles - 1 of the launch.
struct ReconWork {
  ReconArgs a;
  int64_t tile0, start;
};
// recon_mfma of up to 64 reconstructions in one launch over the tiles of all of them
// (list in device memory, starts increasing from 0, total = the last start + its tile
// count; every entry of the same NSG/NTV form and mode, already checked by the caller with
// recon_mfma's rules; ragged: every entry is the one partial tile past its n).  lds: the
// largest recon_lds_bytes over the entries.
hipError_t recon_mfma_list(const ReconWork* list, int nw, int64_t total, size_t lds, int nsg, int ntv, int mode,
                           bool ragged, hipStream_t stream);
int recon_ksteps(int64_t m);        // 4 ceil(m / 64)
int recon_frame_blocks(int64_t m);  // ceil(m / 32)
// LDS bytes of one workgroup of recon_mfma (the form applies while this is <= 160 KiB).
size_t recon_lds_bytes(int64_t m);
// Column of the reconstruction operands holding part (0 Re, 1 Im) of selected mode s.
int recon_column(int s, int part);
// The operands of recon_mfma from G (N x k complex float64): ns <= 16 selected modes in
// columns col[s], amplitudes beta and eigenvalues lam (re, im); Gp holds KS * NSG, Vp
// NFB * 2 * NTV fragments of 64 x 16 bytes.
struct ReconPrep {
  int ns, NSG, NTV, KS, NFB, N, k, static_bg;
  double xscale;
  int col[16];
  double beta[32], lam[32];
};
hipError_t recon_prep(const double* G, const ReconPrep& rp, void* Gp, void* Vp, hipStream_t stream);
// counts[t] = number of set bits of frame t of a bit-packed mask
hipError_t mask_counts(const uint32_t* mask, int64_t words, int64_t m, int64_t* counts,
                       hipStream_t stream);
// 3x3 median (majority, edges replicated) of m binary H x W masks, bit-packed (uint32
// words, ceil(H W / 32) per frame) or uint8; in and out must not overlap.
hipError_t mask_median3(const void* in, void* out, int64_t H, int64_t W, int64_t m, int bitpacked,
                        hipStream_t stream);

// ----- small float64 linear algebra on the device ---------------------------------
// From the m x m Gram Gr of the unscaled sketch: out = [status, J, mu[k], sigma[k],
// lam[2k], W[2k*k], G[2(m-1)k]] (team_la.hpp small_la_out_layout), in three parts:
// head: Lanczos, V and M12 V; after_lanczos, if given, is recorded once the Lanczos kernel
// is queued.
// gp (after the head): the lift's bf16 operands of the real basis V S^-1 * xscale in Gp
// (NB column blocks, NS terms, KS 16-row steps).
// tail (after the head, beside gp and the lift): eig(A~), W and G.
// groups: Lanczos row groups (workgroups), 0 = as many as the rows call for.  Needs
// m - 1 <= 1024 and Jmax <= 320.  scratch: small_la_scratch_doubles(m, k, Jmax).
hipError_t small_la_head(const double* Gr, int m, int k, double rtol, int Jmax, double sketch_scale,
                         double xscale, double* scratch, double* out, void* Gp, int NB, int NS, int KS,
                         int groups, hipStream_t stream, hipEvent_t after_lanczos = nullptr);
hipError_t small_la_gp(const double* Gr, int m, int k, double rtol, int Jmax, double sketch_scale,
                       double xscale, double* scratch, double* out, void* Gp, int NB, int NS, int KS,
                       int groups, hipStream_t stream);
hipError_t small_la_tail(const double* Gr, int m, int k, double rtol, int Jmax, double sketch_scale,
                         double xscale, double* scratch, double* out, void* Gp, int NB, int NS, int KS,
                         int groups, hipStream_t stream);
int64_t small_la_scratch_doubles(int m, int k, int Jmax);
// After the head (beside the tail): the compressed modes' Gram (Remark 3) from the sketch
// Gram, as block partials part[small_la_py_blocks(m)][k^2 + k + 1] (k_la_py): B^T Gr' B
// (k x k), B^T g0 and Gr[0][0], with B = V diag(1/(nu s)) the normalised real basis of
// G = B W.  k <= 64.
hipError_t small_la_py(const double* Gr, int m, int k, double rtol, int Jmax, double sketch_scale,
                       double* scratch, double* out, double* part, hipStream_t stream);
int small_la_py_blocks(int m);
// A batch of independent solves in one set of launches (a grid row each); d_descs is
// device memory holding `count` descriptors, each valid for small_la_head (small_la_fits).
struct SLADesc {
  const double* Gr;
  double* scratch;
  double* out;
  uint16_t* Gp;
  double rtol, sketch_scale, xscale;
  int m, k, Jmax, NB, NS, KS;
  int groups;  // Lanczos row groups (workgroups); 0: as many as the rows call for
};
bool small_la_fits(int m, int k, int Jmax);
// nmax: the largest m - 1 of the batch; gmax: the largest max(m - 1, 16 KS).
// ngroups: the grid's Lanczos workgroups per solve, at least the groups any solve uses.
hipError_t small_la_batch_head(const SLADesc* d_descs, int count, int nmax, int ngroups, hipStream_t stream);
hipError_t small_la_batch_gp(const SLADesc* d_descs, int count, int gmax, hipStream_t stream);
hipError_t small_la_batch_tail(const SLADesc* d_descs, int count, int nmax, int kmax, hipStream_t stream);
int64_t small_la_out_doubles(int m, int k);

}  // namespace k
}  // namespace cdmd
