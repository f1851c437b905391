// C ABI of the cDMD library: validation, device workspace, kernel orchestration and
// the float64 host stages of the fit.  The calls and their meaning are documented in
// include/cdmd.h.
#include "cdmd.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "sketch_gemm.hpp"
#include "smallla.hpp"
#include "team_la.hpp"
#include "team_la_host.hpp"

using cplx = std::complex<double>;

namespace {

thread_local std::string g_err;
constexpr int kMaxRank = 40;  // the largest target rank the kernels are built for

cdmd_status fail(cdmd_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(_e == hipErrorOutOfMemory ? CDMD_E_OUT_OF_MEMORY : CDMD_E_DEVICE,    \
                  std::string(#expr) + ": " + hipGetErrorString(_e));                  \
  } while (0)

// rank test on the Gram eigenvalues: sigma_k <= 1e-6 sigma_1  <=>  mu_k <= 1e-12 mu_1
constexpr double kRankTol2 = 1e-12;
constexpr double kOmpStopRel = 1e-12;
constexpr double kVanderMax = 1e30;
constexpr double kLanczosTol = 1e-13;

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

int pad_nc(int v) {  // lift column padding: multiple of 8, 8..80
  int r = ((v + 7) / 8) * 8;
  return r < 8 ? 8 : r;
}

int pad_ns(int v) {  // reconstruction column padding: one of the instantiated widths
  static const int w[] = {4, 8, 12, 16, 20, 24, 32, 40, 48, 64, 80};
  for (int x : w)
    if (v <= x) return x;
  return -1;
}

}  // namespace

struct cdmd_model {
  cdmd_config cfg{};
  int device = -1;
  int64_t n = 0, m = 0, ld = 0;
  int N = 0, k = 0, p = 0;
  int nc = 0, NC = 0, npair = 0, ne = 0;
  float xscale = 1.f;
  double sketch_scale = 1.0;  // Y^ = sketch_scale * (integer or float64 sums)
  // sparse plan (uint8)
  int nseg = 0, nslot = 1, max_rows = 0, fpb = 1;
  int32_t* d_tri_pix = nullptr;
  uint32_t* d_tri_rs = nullptr;
  int32_t* d_seg = nullptr;
  // sparse table (float32 video)
  int32_t* d_idx = nullptr;
  int8_t* d_sign = nullptr;
  // sketch and Gram
  int32_t* d_Yint = nullptr;
  int32_t* d_Ypart = nullptr;
  double* d_Yd = nullptr;
  bool gauss = false;               // dense Gaussian sketch
  bool srft = false;                // SRFT sketch: complex rows, (re, im) interleaved in d_Yd
  int32_t* d_freq = nullptr;        // SRFT: the DFT row kept by each sketch row
  double* d_gram_im = nullptr;      // SRFT: imaginary part of the Hermitian Gram
  double* h_gram_im = nullptr;
  cdmd::k::GaussPlan gplan{};
  float* d_gpart = nullptr;         // per-slice partial sketches
  void* d_Cm = nullptr;             // the stored C (cdmd_store_measurement), or null: drawn
  int64_t Cm_ldc = 0;
  // BF16 / FP8 form with a stored C through the library GEMM: C pixel-major in d_Cm, the
  // video converted into slices in d_Xs (bfloat16, or the two e4m3 parts of each byte), the
  // sketch as gm_S batched library GEMMs over slices of gm_Ks pixels
  cdmd::blas::SketchGemm* sgemm = nullptr;
  void* d_Xs = nullptr;
  int gm_S = 0;
  int64_t gm_Ks = 0;
  // streaming sparse sketch (16-byte aligned frames)
  int32_t* d_chunk_off = nullptr;   // [row block][chunk + 1] first triple of each chunk
  int32_t* d_rblk = nullptr;        // [row block] (first row, rows)
  int sk_nchunk = 0, sk_nrange = 0, sk_F = 0, sk_V = 1, sk_nblk = 0;
  int sk_slots_cap = 0;             // partial slots allocated at d_Ypart
  size_t gpart_cap = 0;             // floats allocated at d_gpart
  double* d_gram = nullptr;
  // lift
  bool lift_mfma = false;   // MFMA path (uint8 video, 16-byte aligned frames)
  int lm_nb = 0, lm_nsplit = 0, lm_nksteps = 0, lm_grid = 0, lm_ne = 0;
  int lm_grid_max = 0;            // largest lift grid the partial buffer holds
  // real-basis lift grid: many short workgroups, so that the dispatcher balances them
  // around the compute unit the A~ eigen-solve holds
  int lr_grid = 0;
  // real-basis lift (device small LA): Phi' = X' V S^-1, k columns + x_1; W applied on the host
  bool lift_real = false;
  int lr_nb = 0, lr_ne = 0;
  hipStream_t st2 = nullptr;      // the A~ eigen-solve beside the lift
  hipEvent_t e_fork = nullptr, e_join = nullptr;
  uint16_t* h_Gp = nullptr;
  void* d_Gp = nullptr;
  float* d_G = nullptr;
  uint32_t* d_pairs = nullptr;
  double* d_part = nullptr;
  double* d_red = nullptr;
  int lgrid = 0;
  // reconstruction
  void* d_Gsp = nullptr;     // reconstruction operands: G~' fragments
  void* d_Rv = nullptr;      // and V~ fragments
  double* d_Gd = nullptr;    // G (N x k complex) of a host solve, for the operand kernel
  double* h_Gd = nullptr;
  int rc_nsg = 0, rc_ntv = 0, rc_ks = 0, rc_nfb = 0;
  bool recon_mfma = false;
  hipEvent_t e_stage = nullptr;   // the H2D copies of the reconstruction staging
  bool stage_pending = false;
  float* d_Gs = nullptr;
  float* d_Vc = nullptr;
  int64_t* d_counts = nullptr;
  double* d_modes = nullptr;   // lam[2k], b[2k], phi norms[k] for the feature kernel
  float* d_feats = nullptr;    // k x 6
  float* d_logits = nullptr;   // k
  // pinned host staging
  double* h_gram = nullptr;
  float* h_G = nullptr;
  double* h_red = nullptr;
  float* h_Gs = nullptr;
  float* h_Vc = nullptr;
  int64_t* h_counts = nullptr;
  // results (canonical order)
  bool fitted = false, selected = false, g_canonical_on_device = false;
  std::vector<cplx> lam, W, G, H, c, b;
  std::vector<double> sigma, phinorm;
  std::vector<int> perm;  // canonical index -> device column
  double x1n2 = 0.0;
  std::vector<int> S;
  std::vector<cplx> beta;
  cdmd_info info{};
  // kernel-group timing (HIP events on the call's stream)
  bool timing = false, recon_pending = false;
  bool force_valu_lift = false;  // test hook: use the float32 VALU lift for uint8 video
  bool force_host_la = false;    // test hook: float64 small LA on the host
  int la_groups = 0;             // test hook: Lanczos row groups of the device solve (0: auto)
  double la_phase_ms[16] = {};
  // device small LA (one workgroup)
  bool device_la_ok = false;     // sized at create
  bool device_la = false;        // used by the last fit
  int la_jmax = 0;
  double* d_la_scratch = nullptr;
  double* d_la_out = nullptr;
  double* h_la_out = nullptr;
  int64_t la_out_n = 0;
  hipEvent_t ev[8] = {};
  // amplitudes and selection on the compressed modes (Remark 3): no lift in the fit
  bool amp_compressed = false;
  double* d_py = nullptr;   // k_la_py block partials, then their sum
  double* d_pyred = nullptr;
  double* h_py = nullptr;

  bool capturing = false;         // inside a graph capture: no timing events
  bool force_gather_sketch = false;  // test hook: gather form of the sparse sketch
  bool tuned = false;             // autotuner choices applied
  uint64_t stamp = 0;             // bumped by every change of configuration after create
  void mark(int i, hipStream_t st) {
    if (timing && !capturing) (void)hipEventRecord(ev[i], st);
  }
  double span(int a, int b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev[a], ev[b]) != hipSuccess) return -1.0;
    return (double)ms;
  }

  ~cdmd_model() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (e_fork) (void)hipEventDestroy(e_fork);
    if (e_join) (void)hipEventDestroy(e_join);
    if (e_stage) {
      if (stage_pending) (void)hipEventSynchronize(e_stage);
      (void)hipEventDestroy(e_stage);
    }
    if (st2) (void)hipStreamDestroy(st2);
    if (sgemm) cdmd::blas::sketch_gemm_free(sgemm);
    void* dev[] = {d_tri_pix, d_tri_rs, d_seg, d_idx, d_sign, d_Yint, d_Ypart, d_Yd, d_gpart, d_Cm, d_chunk_off, d_rblk,
                   d_gram, d_G, d_Gp, d_pairs, d_part, d_red, d_Gs, d_Gsp, d_Rv, d_Gd, d_Vc, d_counts, d_modes,
                   d_feats, d_logits,
                   d_la_scratch, d_la_out, d_py, d_pyred, d_freq, d_gram_im, d_Xs};
    for (void* q : dev)
      if (q) (void)hipFree(q);
    void* host[] = {h_gram, h_G, h_Gp, h_red, h_Gs, h_Gd, h_Vc, h_counts, h_la_out, h_py, h_gram_im};
    for (void* q : host)
      if (q) (void)hipHostFree(q);
  }
};

namespace {

template <typename T>
cdmd_status dalloc(T** p, size_t count) {
  if (count == 0) count = 1;
  HIPCHK(hipMalloc((void**)p, count * sizeof(T)));
  return CDMD_OK;
}
template <typename T>
cdmd_status halloc(T** p, size_t count) {
  if (count == 0) count = 1;
  HIPCHK(hipHostMalloc((void**)p, count * sizeof(T), hipHostMallocDefault));
  return CDMD_OK;
}

#define TRY(expr)                      \
  do {                                 \
    cdmd_status _s = (expr);           \
    if (_s != CDMD_OK) return _s;      \
  } while (0)

// Gaussian sketch form for the kernels: 0 FP32, 1 BF16, 2 FP8.
int gauss_prec(const cdmd_config& c) {
  return c.sketch_prec == CDMD_PREC_BF16 ? 1 : c.sketch_prec == CDMD_PREC_FP8 ? 2 : 0;
}

cdmd_status validate(const cdmd_config* c) {
  if (!c) return fail(CDMD_E_INVALID_ARG, "config is NULL");
  if (c->m < 2) return fail(CDMD_E_INVALID_ARG, "need m >= 2 frames");
  if (c->n < c->m) return fail(CDMD_E_INVALID_ARG, "need n >= m (pixels >= frames)");
  if (c->ld < c->n) return fail(CDMD_E_INVALID_ARG, "need ld >= n");
  if (c->p < 1 || c->k < 1) return fail(CDMD_E_INVALID_ARG, "need k, p >= 1");
  if (c->p < c->k) return fail(CDMD_E_INVALID_ARG, "need p >= k");
  if ((int64_t)c->k > c->m - 1) return fail(CDMD_E_INVALID_ARG, "need k <= m - 1");
  if (c->dtype != CDMD_U8 && c->dtype != CDMD_F32) return fail(CDMD_E_INVALID_ARG, "unknown dtype");
  if (c->sketch < CDMD_SKETCH_GAUSSIAN || c->sketch > CDMD_SKETCH_SRFT)
    return fail(CDMD_E_INVALID_ARG, "unknown sketch");
  // single-pixel and SRFT: one distinct index per row (a pixel, or the DFT row kept by R)
  const bool one_per_row = c->sketch == CDMD_SKETCH_SPIXEL || c->sketch == CDMD_SKETCH_SRFT;
  if (c->sketch_prec < CDMD_PREC_FP32 || c->sketch_prec > CDMD_PREC_FP8 ||
      c->lift_prec < CDMD_PREC_FP32 || c->lift_prec > CDMD_PREC_FP8)
    return fail(CDMD_E_INVALID_ARG, "unknown precision");
  if (c->lift_prec == CDMD_PREC_FP8)
    return fail(CDMD_E_INVALID_ARG, "FP8 is a sketch precision only");
  if (c->sketch != CDMD_SKETCH_GAUSSIAN) {
    if (!c->sparse_idx) return fail(CDMD_E_INVALID_ARG, "sparse, single-pixel and SRFT sketches need sparse_idx");
    if (c->nnz < 1 || c->nnz > 32) return fail(CDMD_E_INVALID_ARG, "nnz must be in [1, 32]");
    if (one_per_row && c->nnz != 1)
      return fail(CDMD_E_INVALID_ARG, "single-pixel and SRFT sketches have nnz = 1");
    if (one_per_row && (int64_t)c->p > c->n)
      return fail(CDMD_E_INVALID_ARG, "single-pixel and SRFT sketches need p <= n");
    if ((int64_t)c->nnz > c->n) return fail(CDMD_E_INVALID_ARG, "nnz must not exceed n");
  }
  if (c->k > kMaxRank) return fail(CDMD_E_UNSUPPORTED, "k > 40 is not built");
  if (c->n >= (int64_t)1 << 31) return fail(CDMD_E_UNSUPPORTED, "n >= 2^31 pixels is not built");
  if (c->sketch == CDMD_SKETCH_GAUSSIAN) {
    if (c->sketch_prec != CDMD_PREC_FP32 && (c->dtype != CDMD_U8 || c->ld % 16 != 0))
      return fail(CDMD_E_UNSUPPORTED, "the BF16 / FP8 Gaussian sketch needs a uint8 video with ld % 16 == 0");
    if ((int64_t)c->p * c->m > ((int64_t)1 << 31))
      return fail(CDMD_E_UNSUPPORTED, "p * m >= 2^31 is not built");
  } else if (c->sketch == CDMD_SKETCH_SRFT) {
    if (c->sketch_prec != CDMD_PREC_FP32) return fail(CDMD_E_UNSUPPORTED, "the SRFT sketch has the FP32 form only");
    if (2 * (int64_t)c->p * c->m > ((int64_t)1 << 31))
      return fail(CDMD_E_UNSUPPORTED, "2 p * m >= 2^31 is not built");
  } else if (c->sketch_prec != CDMD_PREC_FP32) {
    return fail(CDMD_E_UNSUPPORTED, "sparse and single-pixel sketches are exact: sketch precision must be FP32");
  }
  if (c->lift_prec == CDMD_PREC_BF16 && (c->dtype != CDMD_U8 || c->ld % 16 != 0))
    return fail(CDMD_E_UNSUPPORTED, "the BF16 lift needs a uint8 video with ld % 16 == 0");
  // table contents
  if (c->sketch != CDMD_SKETCH_GAUSSIAN) {
    const int64_t p = c->p, z = c->nnz;
    for (int64_t r = 0; r < p; ++r) {
      for (int64_t j = 0; j < z; ++j) {
        const int32_t v = c->sparse_idx[r * z + j];
        if (v == -1 && c->sketch == CDMD_SKETCH_SPARSE) continue;  // empty slot of a shorter row
        if (v < 0 || (int64_t)v >= c->n) return fail(CDMD_E_INVALID_ARG, "sparse_idx out of range");
        if (c->sparse_sign) {
          const int8_t sg = c->sparse_sign[r * z + j];
          if (sg != 1 && sg != -1) return fail(CDMD_E_INVALID_ARG, "sparse_sign must be +1 or -1");
          if (one_per_row && sg != 1)
            return fail(CDMD_E_INVALID_ARG, "single-pixel and SRFT weights are +1");
        }
        for (int64_t q = 0; q < j; ++q)
          if (c->sparse_idx[r * z + q] == v)
            return fail(CDMD_E_INVALID_ARG, "sparse_idx repeats a pixel within a row");
      }
    }
    if (std::find_if(c->sparse_idx, c->sparse_idx + p * z, [](int32_t v) { return v >= 0; }) ==
        c->sparse_idx + p * z)
      return fail(CDMD_E_INVALID_ARG, "sparse table has no nonzeros");
    if (one_per_row) {
      std::vector<int32_t> s(c->sparse_idx, c->sparse_idx + p);
      std::sort(s.begin(), s.end());
      if (std::adjacent_find(s.begin(), s.end()) != s.end())
        return fail(CDMD_E_INVALID_ARG, "single-pixel and SRFT rows must be distinct indices");
    }
  }
  return CDMD_OK;
}

cdmd_status check_device(int* dev) {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count < 1) return fail(CDMD_E_DEVICE, "no HIP device available");
  HIPCHK(hipGetDevice(dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, *dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(CDMD_E_DEVICE, std::string("device is ") + prop.gcnArchName + ", library is built for gfx950");
  return CDMD_OK;
}

// Build the pixel-sorted triple table of a sparse / single-pixel C for the uint8 sketch.
// Pixel ranges of the streaming sketch: about 1024 workgroups in all.
int stream_nrange(const cdmd_model* M, int F, int V) {
  const int64_t fgroups = (M->m + F - 1) / F;
  const int64_t nck = (M->sk_nchunk + V - 1) / V;
  return (int)std::max<int64_t>(1, std::min<int64_t>(nck, (1024 + fgroups * M->sk_nblk - 1) / (fgroups * M->sk_nblk)));
}

cdmd_status build_sparse_plan(cdmd_model* M) {
  const cdmd_config& c = M->cfg;
  const int p = c.p, z = c.nnz;
  const int max_rows = std::min(p, 8192);
  int fpb = 1;
  while (fpb < 4 && (size_t)(fpb * 2) * max_rows * 4 <= 65536) fpb *= 2;
  const int nb = (p + max_rows - 1) / max_rows;
  const int64_t groups = (M->m + fpb - 1) / fpb;
  int nslot = (int)std::max<int64_t>(1, std::min<int64_t>(16, (1024 + nb * groups - 1) / (nb * groups)));
  const int64_t T = (int64_t)p * z;
  if (T / nb / nslot < 512) nslot = (int)std::max<int64_t>(1, T / nb / 512);
  std::vector<int32_t> pix;
  std::vector<uint32_t> rs;
  std::vector<int32_t> seg;
  pix.reserve(T);
  rs.reserve(T);
  std::vector<std::pair<int32_t, uint32_t>> tri;
  std::vector<int64_t> blk_base(nb), blk_cnt(nb);  // triples of each row block (empty slots skipped)
  for (int b = 0; b < nb; ++b) {
    const int r0 = b * max_rows, r1 = std::min(p, r0 + max_rows);
    tri.clear();
    for (int r = r0; r < r1; ++r)
      for (int j = 0; j < z; ++j) {
        const int32_t v = c.sparse_idx[(int64_t)r * z + j];
        if (v < 0) continue;  // empty slot
        const bool neg = c.sparse_sign && c.sparse_sign[(int64_t)r * z + j] < 0;
        tri.emplace_back(v, (uint32_t)(r - r0) | (neg ? 0x80000000u : 0u));
      }
    std::stable_sort(tri.begin(), tri.end(),
                     [](const std::pair<int32_t, uint32_t>& a, const std::pair<int32_t, uint32_t>& b2) {
                       return a.first < b2.first;
                     });
    const int64_t base = (int64_t)pix.size(), cnt = (int64_t)tri.size();
    blk_base[b] = base;
    blk_cnt[b] = cnt;
    for (auto& t : tri) {
      pix.push_back(t.first);
      rs.push_back(t.second);
    }
    for (int s = 0; s < nslot; ++s) {
      seg.push_back((int32_t)(base + cnt * s / nslot));
      seg.push_back((int32_t)(base + cnt * (s + 1) / nslot));
      seg.push_back(r0);
      seg.push_back(r1 - r0);
      seg.push_back(s);
    }
  }
  M->nseg = nb * nslot;
  M->nslot = nslot;
  M->max_rows = max_rows;
  M->fpb = fpb;
  // streaming form: per row block, the first triple of every chunk of pixels
  const int CH = cdmd::k::sketch_stream_chunk();
  const int nchunk = (int)((M->n + CH - 1) / CH);
  std::vector<int32_t> coff((size_t)nb * (nchunk + 1)), rblk(2 * (size_t)nb);
  for (int b = 0; b < nb; ++b) {
    const int r0 = b * max_rows, r1 = std::min(p, r0 + max_rows);
    rblk[2 * b] = r0;
    rblk[2 * b + 1] = r1 - r0;
    const int64_t base = blk_base[b], cnt = blk_cnt[b];
    int64_t e = base;
    for (int c = 0; c <= nchunk; ++c) {
      const int64_t lim = (int64_t)c * CH;
      while (e < base + cnt && pix[e] < lim) ++e;
      coff[(size_t)b * (nchunk + 1) + c] = (int32_t)e;
    }
  }
  int F = 4;
  while (F > 1 && !cdmd::k::sketch_stream_fits(F, 1, max_rows)) F /= 2;
  M->sk_nchunk = nchunk;
  M->sk_nblk = nb;
  M->sk_F = F;
  M->sk_V = 1;
  M->sk_nrange = stream_nrange(M, F, 1);
  M->sk_slots_cap = std::max(M->nslot, M->sk_nrange);
  TRY(dalloc(&M->d_chunk_off, coff.size()));
  TRY(dalloc(&M->d_rblk, rblk.size()));
  HIPCHK(hipMemcpy(M->d_chunk_off, coff.data(), coff.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(M->d_rblk, rblk.data(), rblk.size() * 4, hipMemcpyHostToDevice));
  TRY(dalloc(&M->d_tri_pix, pix.size()));
  TRY(dalloc(&M->d_tri_rs, rs.size()));
  TRY(dalloc(&M->d_seg, seg.size()));
  HIPCHK(hipMemcpy(M->d_tri_pix, pix.data(), pix.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(M->d_tri_rs, rs.data(), rs.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(M->d_seg, seg.data(), seg.size() * 4, hipMemcpyHostToDevice));
  return CDMD_OK;
}

// Eigenvector normalisation: unit 2-norm, largest-modulus entry (lowest index on ties)
// real and positive.
void normalise_columns(std::vector<cplx>& W, int k) {
  for (int j = 0; j < k; ++j) {
    cplx* w = &W[(size_t)j * k];
    double nr = 0.0;
    for (int i = 0; i < k; ++i) nr += std::norm(w[i]);
    nr = std::sqrt(nr);
    int piv = 0;
    double best = -1.0;
    for (int i = 0; i < k; ++i)
      if (std::abs(w[i]) > best) best = std::abs(w[i]), piv = i;
    const cplx ph = w[piv] / std::abs(w[piv]);
    for (int i = 0; i < k; ++i) w[i] = w[i] / (ph * nr);
    w[piv] = cplx(w[piv].real(), 0.0);
  }
}

// Canonical order: descending key |b_j| ||phi_j||; the members of a conjugate pair
// (lambda_b = conj(lambda_a) to 1e-12) share the larger of their keys and the member
// with Im lambda > 0 comes first; remaining ties keep the eigensolver's order.
std::vector<int> canonical_order(const std::vector<cplx>& lam, const std::vector<double>& key) {
  const int k = (int)lam.size();
  std::vector<double> pk(key);
  const std::vector<int> partner = cdmd::la::conj_partners(lam.data(), k);
  for (int a = 0; a < k; ++a)
    if (partner[a] >= 0) pk[a] = std::max(key[a], key[partner[a]]);
  std::vector<int> o(k);
  std::iota(o.begin(), o.end(), 0);
  std::stable_sort(o.begin(), o.end(), [&](int a, int b) {
    if (pk[a] != pk[b]) return pk[a] > pk[b];
    const bool pa = lam[a].imag() > 0.0, pb = lam[b].imag() > 0.0;
    if (pa != pb) return pa;
    return a < b;
  });
  return o;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Sketch + Gram + D2H of the Gram.
// The dense sketch with a stored C through the library GEMM: the video converted into the
// split layout (exact bfloat16, or the two e4m3 parts of each byte), the batched products
// (for FP8: 16 hi, then lo added), and the float64 sum over the slices.
cdmd_status gemm_sketch(cdmd_model* M, const void* d_video, hipStream_t st) {
  const size_t half = (size_t)M->gm_S * M->m * M->gm_Ks;  // elements of one converted copy
  if (gauss_prec(M->cfg) == 1) {
    HIPCHK(cdmd::k::video_bf16_split(d_video, M->ld, M->n, M->m, M->gm_Ks, M->gm_S, M->d_Xs, st));
    if (!cdmd::blas::sketch_gemm_run(M->sgemm, M->d_Cm, M->d_Xs, M->d_gpart, st))
      return fail(CDMD_E_DEVICE, "the sketch GEMM failed");
  } else {
    uint8_t* xh = static_cast<uint8_t*>(M->d_Xs);
    HIPCHK(cdmd::k::video_fp8_split(d_video, M->ld, M->n, M->m, M->gm_Ks, M->gm_S, xh, xh + half, st));
    if (!cdmd::blas::sketch_gemm_run(M->sgemm, M->d_Cm, xh, M->d_gpart, st) ||
        !cdmd::blas::sketch_gemm_run(M->sgemm, M->d_Cm, xh + half, M->d_gpart, st, true))
      return fail(CDMD_E_DEVICE, "the sketch GEMM failed");
  }
  HIPCHK(cdmd::k::reduce_gauss(M->d_gpart, M->gm_S, M->m * (int64_t)M->p, 1.0 / std::sqrt((double)M->p), M->d_Yd,
                               st));
  return CDMD_OK;
}

cdmd_status run_sketch(cdmd_model* M, const void* d_video, hipStream_t st, bool to_host) {
  const cdmd_config& c = M->cfg;
  M->mark(0, st);
  if (M->srft) {
    HIPCHK(cdmd::k::sketch_srft(d_video, c.dtype == CDMD_U8 ? 0 : 1, M->ld, M->n, M->m, M->p, c.seed, M->gplan,
                                M->d_freq, M->d_gpart, M->d_Yd, st));
    M->mark(1, st);
    HIPCHK(cdmd::k::gram_cplx(M->d_Yd, M->p, M->m, M->d_gram, M->d_gram_im, st));
  } else if (M->gauss) {
    if (c.sketch_prec != CDMD_PREC_FP32 && (reinterpret_cast<uintptr_t>(d_video) & 15) != 0)
      return fail(CDMD_E_UNSUPPORTED, "the BF16 / FP8 Gaussian sketch needs a 16-byte aligned video");
    if (M->sgemm) {
      TRY(gemm_sketch(M, d_video, st));
    } else {
      HIPCHK(cdmd::k::sketch_gauss(d_video, c.dtype == CDMD_U8 ? 0 : 1, M->ld, M->n, M->m, M->p, c.seed,
                                   gauss_prec(c), M->gplan, M->d_Cm, M->Cm_ldc, M->d_gpart, M->d_Yd, st));
    }
    M->mark(1, st);
    HIPCHK(cdmd::k::gram_f64(M->d_Yd, M->p, M->m, M->d_gram, st));
  } else if (c.dtype == CDMD_U8 && M->ld % 16 == 0 && (reinterpret_cast<uintptr_t>(d_video) & 15) == 0 &&
             !M->force_gather_sketch) {
    HIPCHK(cdmd::k::sketch_stream_u8((const uint8_t*)d_video, M->ld, M->n, M->m, M->d_tri_pix, M->d_tri_rs,
                                     M->d_chunk_off, M->sk_nchunk, M->d_rblk, M->sk_nblk, M->sk_nrange, M->p,
                                     M->max_rows, M->sk_F, M->sk_V, M->d_Ypart, st));
    HIPCHK(cdmd::k::reduce_slots_i32(M->d_Ypart, M->sk_nrange, (int64_t)M->m * M->p, M->d_Yint, st));
    M->mark(1, st);
    HIPCHK(cdmd::k::gram_i32(M->d_Yint, M->p, M->m, M->d_gram, st));
  } else if (c.dtype == CDMD_U8) {
    int32_t* out = M->nslot > 1 ? M->d_Ypart : M->d_Yint;
    HIPCHK(cdmd::k::sketch_sparse_u8((const uint8_t*)d_video, M->ld, M->m, M->d_tri_pix, M->d_tri_rs,
                                     M->d_seg, M->nseg, M->p, M->max_rows, M->fpb, out, M->nslot, st));
    if (M->nslot > 1)
      HIPCHK(cdmd::k::reduce_slots_i32(M->d_Ypart, M->nslot, (int64_t)M->m * M->p, M->d_Yint, st));
    M->mark(1, st);
    HIPCHK(cdmd::k::gram_i32(M->d_Yint, M->p, M->m, M->d_gram, st));
  } else {
    HIPCHK(cdmd::k::sketch_sparse_f32((const float*)d_video, M->ld, M->m, M->d_idx, M->d_sign, M->p,
                                      c.nnz, M->d_Yd, st));
    M->mark(1, st);
    HIPCHK(cdmd::k::gram_f64(M->d_Yd, M->p, M->m, M->d_gram, st));
  }
  M->mark(2, st);
  if (!to_host) return CDMD_OK;
  HIPCHK(hipMemcpyAsync(M->h_gram, M->d_gram, sizeof(double) * M->m * M->m, hipMemcpyDeviceToHost, st));
  if (M->srft)
    HIPCHK(hipMemcpyAsync(M->h_gram_im, M->d_gram_im, sizeof(double) * M->m * M->m, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (M->timing) {
    M->info.gpu_ms_sketch = M->span(0, 1);
    M->info.gpu_ms_gram = M->span(1, 2);
  }
  return CDMD_OK;
}

// The same for the complex sketch of the SRFT: the Hermitian Gram Y^H Y (upper triangle as
// computed, lower triangle its conjugate), its top-k eigenpairs by complex Lanczos (V
// complex), A~ = S^-1 V^H (Y^H Y') V S^-1 complex, its eigenpairs by the complex Schur
// form, G = V S^-1 W.
cdmd_status small_la_complex(cdmd_model* M) {
  const int N = M->N, k = M->k;
  const int64_t m = M->m;
  const double* Gr = M->h_gram;
  const double* Gi = M->h_gram_im;
  for (int64_t i = 0; i < m * m; ++i)
    if (!std::isfinite(Gr[i]) || !std::isfinite(Gi[i])) return fail(CDMD_E_NUMERIC, "non-finite value in the sketch Gram");
  auto g = [&](int64_t a, int64_t b) {
    return a <= b ? cplx(Gr[a * m + b], Gi[a * m + b]) : std::conj(cplx(Gr[b * m + a], Gi[b * m + a]));
  };
  std::vector<cplx> M11((size_t)N * N);
  for (int a = 0; a < N; ++a)
    for (int b2 = 0; b2 < N; ++b2) M11[(size_t)a * N + b2] = g(a, b2);
  std::vector<cplx> V((size_t)N * k);
  std::vector<double> mu(k, 0.0);
  const int J = cdmd::la::herm_topk(M11.data(), N, k, kLanczosTol, mu.data(), V.data());
  if (J < 0) return fail(CDMD_E_NUMERIC, "Hermitian eigensolver failed");
  M->info.lanczos_steps = J;
  if (!(mu[0] > 0.0) || !(mu[k - 1] > kRankTol2 * mu[0]))
    return fail(CDMD_E_RANK_DEFICIENT, "sigma_k <= 1e-6 sigma_1: target rank exceeds the numerical rank of Y");
  std::vector<double> s(k);
  for (int i = 0; i < k; ++i) s[i] = std::sqrt(mu[i]);
  M->info.sigma_ratio = s[k - 1] / s[0];
  M->sigma.resize(k);
  for (int i = 0; i < k; ++i) M->sigma[i] = s[i] * M->sketch_scale;
  std::vector<cplx> T((size_t)N * k);  // T = (Y^H Y') V, N x k
  for (int a = 0; a < N; ++a)
    for (int j = 0; j < k; ++j) {
      const cplx* v = &V[(size_t)j * N];
      cplx acc = 0.0;
      for (int b2 = 0; b2 < N; ++b2) acc += g(a, b2 + 1) * v[b2];
      T[(size_t)a * k + j] = acc;
    }
  std::vector<cplx> At((size_t)k * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      const cplx* v = &V[(size_t)i * N];
      cplx acc = 0.0;
      for (int a = 0; a < N; ++a) acc += std::conj(v[a]) * T[(size_t)a * k + j];
      At[(size_t)i * k + j] = acc / (s[i] * s[j]);
    }
  M->lam.assign(k, 0.0);
  M->W.assign((size_t)k * k, 0.0);
  if (!cdmd::la::eig_complex(At.data(), k, M->lam.data(), M->W.data()))
    return fail(CDMD_E_NUMERIC, "eigensolver of A~ failed");
  normalise_columns(M->W, k);
  M->G.assign((size_t)N * k, 0.0);
  for (int t = 0; t < N; ++t)
    for (int j = 0; j < k; ++j) {
      cplx acc = 0.0;
      for (int i = 0; i < k; ++i) acc += (V[(size_t)i * N + t] / M->sigma[i]) * M->W[(size_t)j * k + i];
      M->G[(size_t)t * k + j] = acc;
    }
  return CDMD_OK;
}

// Truncated SVD (eq. svd), A~ and eig(A~) (Section 3.2) and G = V S^-1 W on the host in float64.
cdmd_status small_la(cdmd_model* M, std::vector<double>& V, std::vector<double>& mu) {
  if (M->srft) return small_la_complex(M);
  const int N = M->N, k = M->k;
  const int64_t m = M->m;
  const double* Gr = M->h_gram;
  for (int64_t i = 0; i < m * m; ++i)
    if (!std::isfinite(Gr[i])) return fail(CDMD_E_NUMERIC, "non-finite value in the sketch Gram");
  std::vector<double> M11((size_t)N * N);
  for (int a = 0; a < N; ++a)
    for (int b2 = 0; b2 < N; ++b2) M11[(size_t)a * N + b2] = Gr[(size_t)a * m + b2];
  V.assign((size_t)N * k, 0.0);
  mu.assign(k, 0.0);
  const int J = cdmd::la::sym_topk(M11.data(), N, k, kLanczosTol, mu.data(), V.data());
  if (J < 0) return fail(CDMD_E_NUMERIC, "symmetric eigensolver failed");
  M->info.lanczos_steps = J;
  if (!(mu[0] > 0.0) || !(mu[k - 1] > kRankTol2 * mu[0]))
    return fail(CDMD_E_RANK_DEFICIENT, "sigma_k <= 1e-6 sigma_1: target rank exceeds the numerical rank of Y");
  std::vector<double> s(k);
  for (int i = 0; i < k; ++i) s[i] = std::sqrt(mu[i]);
  M->info.sigma_ratio = s[k - 1] / s[0];
  M->sigma.resize(k);
  for (int i = 0; i < k; ++i) M->sigma[i] = s[i] * M->sketch_scale;
  // A~ = S^-1 V^T (Y^T Y') V S^-1 with Y^T Y' = Gram[0:N, 1:m]
  std::vector<double> T((size_t)N * k, 0.0);  // T = M12 V (N x k, row-major)
  for (int a = 0; a < N; ++a) {
    const double* row = Gr + (size_t)a * m + 1;
    for (int j = 0; j < k; ++j) {
      const double* v = &V[(size_t)j * N];
      double acc = 0.0;
      for (int b2 = 0; b2 < N; ++b2) acc += row[b2] * v[b2];
      T[(size_t)a * k + j] = acc;
    }
  }
  std::vector<double> At((size_t)k * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      const double* v = &V[(size_t)i * N];
      double acc = 0.0;
      for (int a = 0; a < N; ++a) acc += v[a] * T[(size_t)a * k + j];
      At[(size_t)i * k + j] = acc / (s[i] * s[j]);
    }
  M->lam.assign(k, 0.0);
  M->W.assign((size_t)k * k, 0.0);
  if (!cdmd::la::eig_general(At.data(), k, M->lam.data(), M->W.data()))
    return fail(CDMD_E_NUMERIC, "eigensolver of A~ failed");
  normalise_columns(M->W, k);
  // G = V S^-1 W for the scaled sketch: sigma_scaled = s * sketch_scale
  M->G.assign((size_t)N * k, 0.0);
  for (int t = 0; t < N; ++t)
    for (int j = 0; j < k; ++j) {
      cplx acc = 0.0;
      for (int i = 0; i < k; ++i) acc += (V[(size_t)i * N + t] / M->sigma[i]) * M->W[(size_t)j * k + i];
      M->G[(size_t)t * k + j] = acc;
    }
  return CDMD_OK;
}

// bfloat16 bits of a float64, round to nearest even (one rounding step)
uint16_t bf16_bits(double x) {
  if (x == 0.0) return std::signbit(x) ? 0x8000 : 0;
  int e;
  const double f = std::frexp(std::fabs(x), &e);  // |x| = f 2^e, f in [0.5, 1)
  double q = std::ldexp(std::nearbyint(std::ldexp(f, 8)), e - 8);  // 8 significant bits
  const float qf = (float)q;                       // exact
  uint32_t u;
  std::memcpy(&u, &qf, 4);
  u >>= 16;
  return (uint16_t)(u | (x < 0 ? 0x8000u : 0u));
}
double bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

// Read the device small-LA output block into the model (after the stream sync).
cdmd_status take_device_la(cdmd_model* M) {
  const int k = M->k, N = M->N;
  const double* o = M->h_la_out;
  const cdmd::tla::SmallLAOutLayout L = cdmd::tla::small_la_out_layout(N, k);
  const int st = (int)o[L.status];
  M->info.lanczos_steps = (int)o[L.J];
  if (st == CDMD_E_RANK_DEFICIENT)
    return fail(CDMD_E_RANK_DEFICIENT, "sigma_k <= 1e-6 sigma_1: target rank exceeds the numerical rank of Y");
  if (st != 0) return fail(CDMD_E_NUMERIC, "device small linear algebra failed (non-finite Gram or no convergence)");
  M->sigma.assign(o + L.sigma, o + L.sigma + k);
  M->info.sigma_ratio = M->sigma[k - 1] / M->sigma[0];
  M->lam.resize(k);
  M->W.resize((size_t)k * k);
  M->G.resize((size_t)N * k);
  for (int j = 0; j < k; ++j) M->lam[j] = cplx(o[L.lam + 2 * j], o[L.lam + 2 * j + 1]);
  for (int64_t e = 0; e < (int64_t)k * k; ++e) M->W[e] = cplx(o[L.W + 2 * e], o[L.W + 2 * e + 1]);
  for (int64_t e = 0; e < (int64_t)N * k; ++e) M->G[e] = cplx(o[L.G + 2 * e], o[L.G + 2 * e + 1]);
  // phase times in ms (wall clock at 100 MHz): lanczos incl. checks, of which the
  // tridiagonal checks, A~, eigenvalues, eigenvectors, G, operand write; Lanczos matvec,
  // orthogonalisation, rest of the step (norm, check, next vector), multisection, check
  // vectors, Ritz vectors Q Z, exchange reads, final orthonormalisation
  const double* tt = o + L.timing;
  const double f = 1e-5;
  M->la_phase_ms[0] = (tt[3] - tt[2]) * f;
  M->la_phase_ms[1] = tt[0] * f;
  M->la_phase_ms[2] = (tt[4] - tt[3]) * f;
  M->la_phase_ms[3] = (tt[5] - tt[4]) * f;
  M->la_phase_ms[4] = (tt[6] - tt[5]) * f;
  M->la_phase_ms[5] = (tt[7] - tt[6]) * f;
  M->la_phase_ms[6] = tt[8] * f;
  M->la_phase_ms[7] = tt[10] * f;
  M->la_phase_ms[8] = tt[11] * f;
  M->la_phase_ms[9] = tt[12] * f;
  M->la_phase_ms[10] = tt[13] * f;
  M->la_phase_ms[11] = tt[14] * f;
  M->la_phase_ms[12] = tt[15] * f;
  M->la_phase_ms[13] = tt[9] * f;
  M->la_phase_ms[14] = tt[1] * f;
  return CDMD_OK;
}

// Upload G (columns in `order`) for the lift, scaled to raw pixel units.
cdmd_status upload_G(cdmd_model* M, const std::vector<int>& order, hipStream_t st) {
  const int N = M->N, k = M->k, NC = M->NC;
  if (M->lift_mfma) {
    // B operands [kstep][nb][split][lane][8]: element i of lane l is G row
    // 16 kstep + 8 (l / 32) + i, column 32 nb + l % 32, split term s.
    const int NB = M->lm_nb, NS = M->lm_nsplit, KS = M->lm_nksteps;
    for (int ks = 0; ks < KS; ++ks)
      for (int nb = 0; nb < NB; ++nb)
        for (int l = 0; l < 64; ++l) {
          const int col = 32 * nb + (l & 31);
          for (int i = 0; i < 8; ++i) {
            const int row = 16 * ks + 8 * (l >> 5) + i;
            double g = 0.0;
            if (row < N && col < 2 * k) {
              const cplx z = M->G[(size_t)row * k + order[col % k]] * (double)M->xscale;
              g = col < k ? z.real() : z.imag();
            }
            double rem = g;
            for (int sp = 0; sp < NS; ++sp) {
              const uint16_t bits = bf16_bits(rem);
              rem -= bf16_value(bits);
              M->h_Gp[((((size_t)ks * NB + nb) * NS + sp) * 64 + l) * 8 + i] = bits;
            }
          }
        }
    HIPCHK(hipMemcpyAsync(M->d_Gp, M->h_Gp, (size_t)KS * NB * NS * 64 * 16, hipMemcpyHostToDevice, st));
    return CDMD_OK;
  }
  for (int t = 0; t < N; ++t) {
    float* row = M->h_G + (size_t)t * NC;
    for (int c = 0; c < NC; ++c) row[c] = 0.f;
    for (int j = 0; j < k; ++j) {
      const cplx g = M->G[(size_t)t * k + order[j]] * (double)M->xscale;
      row[j] = (float)g.real();
      row[k + j] = (float)g.imag();
    }
  }
  HIPCHK(hipMemcpyAsync(M->d_G, M->h_G, sizeof(float) * N * NC, hipMemcpyHostToDevice, st));
  return CDMD_OK;
}

// real: the operands in d_Gp are those of the real basis V S^-1 (k columns; no modes are
// written), else of the complex G (2k columns).
cdmd_status launch_lift(cdmd_model* M, const void* d_video, float* d_phi, hipStream_t st, bool real) {
  if (M->lift_mfma)
    HIPCHK(cdmd::k::lift_mfma((const uint8_t*)d_video, M->ld, M->n, M->m, M->d_Gp, real ? M->lr_nb : M->lm_nb,
                              M->lm_nsplit, M->lm_nksteps, real ? M->k : M->nc, M->xscale, M->d_part,
                              real ? M->lr_grid : M->lm_grid, real ? nullptr : d_phi, M->k, st));
  else
    HIPCHK(cdmd::k::lift_fp32(d_video, M->cfg.dtype, M->ld, M->n, M->m, M->d_G, M->NC, M->nc,
                              M->d_pairs, M->npair, M->d_part, M->lgrid, d_phi, M->k, M->xscale, st));
  return CDMD_OK;
}

// Lift, reduction of its partials and the copy of the reduced partials to pinned host
// memory, enqueued without waiting (with the device small LA, the operands of the real
// basis V S^-1 are already on the device).
cdmd_status enqueue_lift(cdmd_model* M, const void* d_video, float* d_phi, hipStream_t st) {
  if (M->cfg.lift_prec == CDMD_PREC_BF16 && !M->lift_mfma)
    return fail(CDMD_E_INVALID_ARG, "the BF16 lift needs a 16-byte aligned uint8 video");
  if (!M->device_la) {
    std::vector<int> ident(M->k);
    std::iota(ident.begin(), ident.end(), 0);
    TRY(upload_G(M, ident, st));
  }
  M->mark(3, st);
  TRY(launch_lift(M, d_video, d_phi, st, M->lift_real));
  const int grid = M->lift_mfma ? (M->lift_real ? M->lr_grid : M->lm_grid) : M->lgrid;
  const int ne = M->lift_mfma ? (M->lift_real ? M->lr_ne : M->lm_ne) : M->ne;
  HIPCHK(cdmd::k::reduce_partials(M->d_part, grid, ne, M->d_red, st));
  M->mark(4, st);
  HIPCHK(hipMemcpyAsync(M->h_red, M->d_red, sizeof(double) * ne, hipMemcpyDeviceToHost, st));
  return CDMD_OK;
}

// The tail of the device small LA and the copy of its results to pinned memory, on `st`.
cdmd_status enqueue_la_tail(cdmd_model* M, hipStream_t st) {
  HIPCHK(cdmd::k::small_la_tail(M->d_gram, (int)M->m, M->k, kLanczosTol, M->la_jmax, M->sketch_scale,
                                (double)M->xscale, M->d_la_scratch, M->d_la_out, M->d_Gp, M->lr_nb,
                                M->lm_nsplit, M->lm_nksteps, M->la_groups, st));
  HIPCHK(hipMemcpyAsync(M->h_la_out, M->d_la_out, sizeof(double) * M->la_out_n, hipMemcpyDeviceToHost, st));
  return CDMD_OK;
}

cdmd_status run_lift(cdmd_model* M, const void* d_video, float* d_phi, hipStream_t st) {
  TRY(enqueue_lift(M, d_video, d_phi, st));
  if (M->device_la) HIPCHK(hipStreamWaitEvent(st, M->e_join, 0));
  HIPCHK(hipStreamSynchronize(st));
  if (M->timing) {
    M->info.gpu_ms_lift = M->span(3, 4);
    if (M->device_la) {
      M->info.gpu_ms_sketch = M->span(0, 1);
      M->info.gpu_ms_gram = M->span(1, 2);
      M->info.ms_small_la = M->span(2, 3);
      M->info.gpu_ms_lanczos = M->span(2, 7);
    }
  }
  return CDMD_OK;
}

// H = Phi^H Phi, c = Phi^H x_1.  Real-basis lift: from the partial Gram of
// [Phi' | x_1] with Phi' = X' V S^-1, as H = W^H (Phi'^T Phi') W and c = W^H Phi'^T x_1
// (Phi = Phi' W).
void assemble_H_real(cdmd_model* M, std::vector<cplx>& H, std::vector<cplx>& cvec) {
  const int k = M->k, ne1 = k + 1, NB = M->lr_nb;
  std::vector<double> P((size_t)ne1 * ne1, 0.0);
  int q = 0;
  for (int a = 0; a < NB; ++a)
    for (int b2 = a; b2 < NB; ++b2, ++q)
      for (int j = 0; j < 16; ++j)
        for (int l = 0; l < 64; ++l) {
          const int r = 32 * a + 8 * (j >> 2) + 4 * (l >> 5) + (j & 3);
          const int c = 32 * b2 + (l & 31);
          if (r < ne1 && c < ne1) {
            const double v = M->h_red[((size_t)q * 16 + j) * 64 + l];
            P[(size_t)r * ne1 + c] = v;
            P[(size_t)c * ne1 + r] = v;
          }
        }
  // T = (Phi'^T Phi') W, then H = W^H T; W column j at j*k
  const std::vector<cplx>& W = M->W;
  std::vector<cplx> T((size_t)k * k);
  for (int p2 = 0; p2 < k; ++p2)
    for (int l = 0; l < k; ++l) {
      cplx s = 0.0;
      for (int q2 = 0; q2 < k; ++q2) s += P[(size_t)p2 * ne1 + q2] * W[(size_t)l * k + q2];
      T[(size_t)p2 * k + l] = s;
    }
  H.assign((size_t)k * k, 0.0);
  cvec.assign(k, 0.0);
  for (int j = 0; j < k; ++j) {
    for (int l = j; l < k; ++l) {  // upper triangle, mirrored: H is Hermitian
      cplx s = 0.0;
      for (int p2 = 0; p2 < k; ++p2) s += std::conj(W[(size_t)j * k + p2]) * T[(size_t)p2 * k + l];
      H[(size_t)j * k + l] = l == j ? cplx(s.real(), 0.0) : s;
      H[(size_t)l * k + j] = l == j ? cplx(s.real(), 0.0) : std::conj(s);
    }
    cplx c = 0.0;
    for (int p2 = 0; p2 < k; ++p2) c += std::conj(W[(size_t)j * k + p2]) * P[(size_t)p2 * ne1 + k];
    cvec[j] = c;
  }
  M->x1n2 = P[(size_t)k * ne1 + k];
}

// Remark 3: H = Phi_Y^H Phi_Y, c = Phi_Y^H y_1 and ||y_1||^2 for the compressed modes
// Phi_Y = Y' B W (B the normalised real basis, G = B W), from the k_la_py sums of the
// unscaled sketch: P = B^T Gr' B, q = B^T g0, g00 = Gr[0][0].  Phi_Y does not depend on
// the scale of the sketch; y_1 scales with it.
void assemble_H_compressed(cdmd_model* M, std::vector<cplx>& H, std::vector<cplx>& cvec) {
  const int k = M->k;
  const double* P = M->h_py;
  const double* q = M->h_py + (size_t)k * k;
  const double sc = M->sketch_scale;
  const std::vector<cplx>& W = M->W;  // column j at j*k
  std::vector<cplx> T((size_t)k * k);
  for (int p2 = 0; p2 < k; ++p2)
    for (int l = 0; l < k; ++l) {
      cplx s = 0.0;
      for (int q2 = 0; q2 < k; ++q2) s += P[(size_t)p2 * k + q2] * W[(size_t)l * k + q2];
      T[(size_t)p2 * k + l] = s;
    }
  H.assign((size_t)k * k, 0.0);
  cvec.assign(k, 0.0);
  for (int j = 0; j < k; ++j) {
    for (int l = j; l < k; ++l) {
      cplx s = 0.0;
      for (int p2 = 0; p2 < k; ++p2) s += std::conj(W[(size_t)j * k + p2]) * T[(size_t)p2 * k + l];
      H[(size_t)j * k + l] = l == j ? cplx(s.real(), 0.0) : s;
      H[(size_t)l * k + j] = l == j ? cplx(s.real(), 0.0) : std::conj(s);
    }
    cplx c = 0.0;
    for (int p2 = 0; p2 < k; ++p2) c += std::conj(W[(size_t)j * k + p2]) * q[p2];
    cvec[j] = c * sc;
  }
  M->x1n2 = M->h_py[(size_t)k * k + k] * sc * sc;
}

// H = Phi^H Phi, c = Phi^H x_1 from the real partial Gram of [Re Phi | Im Phi].
void assemble_H(cdmd_model* M, std::vector<cplx>& H, std::vector<cplx>& cvec) {
  if (M->amp_compressed && M->device_la) {
    assemble_H_compressed(M, H, cvec);
    return;
  }
  if (M->lift_real) {
    assemble_H_real(M, H, cvec);
    return;
  }
  const int k = M->k, nc = M->nc, ne1 = nc + 1;
  // P: (nc+1) x (nc+1) Gram of [Re Phi | Im Phi | x_1]
  std::vector<double> P((size_t)ne1 * ne1, 0.0);
  if (M->lift_mfma) {
    const int NB = M->lm_nb;
    int q = 0;
    for (int a = 0; a < NB; ++a)
      for (int b2 = a; b2 < NB; ++b2, ++q)
        for (int j = 0; j < 16; ++j)
          for (int l = 0; l < 64; ++l) {
            const int r = 32 * a + 8 * (j >> 2) + 4 * (l >> 5) + (j & 3);
            const int c = 32 * b2 + (l & 31);
            if (r < ne1 && c < ne1) {
              const double v = M->h_red[((size_t)q * 16 + j) * 64 + l];
              P[(size_t)r * ne1 + c] = v;
              P[(size_t)c * ne1 + r] = v;
            }
          }
  } else {
    int e = 0;
    for (int a = 0; a < nc; ++a)
      for (int b2 = a; b2 < nc; ++b2, ++e) {
        P[(size_t)a * ne1 + b2] = M->h_red[e];
        P[(size_t)b2 * ne1 + a] = M->h_red[e];
      }
    for (int a = 0; a < nc; ++a) P[(size_t)a * ne1 + nc] = P[(size_t)nc * ne1 + a] = M->h_red[M->npair + a];
    P[(size_t)nc * ne1 + nc] = M->h_red[M->npair + nc];
  }
  H.assign((size_t)k * k, 0.0);
  cvec.assign(k, 0.0);
  for (int j = 0; j < k; ++j)
    for (int l = 0; l < k; ++l) {
      const double re = P[(size_t)j * ne1 + l] + P[(size_t)(k + j) * ne1 + (k + l)];
      const double im = P[(size_t)j * ne1 + (k + l)] - P[(size_t)(k + j) * ne1 + l];
      H[(size_t)j * k + l] = cplx(re, im);
    }
  for (int j = 0; j < k; ++j) cvec[j] = cplx(P[(size_t)j * ne1 + nc], -P[(size_t)(k + j) * ne1 + nc]);
  M->x1n2 = P[(size_t)nc * ne1 + nc];
}

}  // namespace

extern "C" {

int32_t cdmd_abi_version(void) { return CDMD_ABI_VERSION; }

const char* cdmd_last_error(void) { return g_err.c_str(); }

cdmd_status cdmd_create(const cdmd_config* cfg, cdmd_model** out) {
  g_err.clear();
  if (!out) return fail(CDMD_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  TRY(validate(cfg));
  int dev = -1;
  TRY(check_device(&dev));
  cdmd_model* M = new (std::nothrow) cdmd_model();
  if (!M) return fail(CDMD_E_OUT_OF_MEMORY, "host allocation failed");
  struct Guard {
    cdmd_model*& m;
    bool keep = false;
    ~Guard() {
      if (!keep) delete m;
    }
  } guard{M};
  M->cfg = *cfg;
  M->device = dev;
  M->n = cfg->n;
  M->m = cfg->m;
  M->ld = cfg->ld;
  M->k = cfg->k;
  M->p = cfg->p;
  M->N = (int)(cfg->m - 1);
  M->nc = 2 * cfg->k;
  M->NC = pad_nc(M->nc);
  M->npair = M->nc * (M->nc + 1) / 2;
  M->ne = M->npair + M->nc + 1;
  M->xscale = cfg->dtype == CDMD_U8 ? 1.0f / 255.0f : 1.0f;
  M->sketch_scale = cfg->dtype == CDMD_U8 ? 1.0 / 255.0 : 1.0;
  M->info.warn_few_samples =
      (double)cfg->p < (double)cfg->k * std::log((double)cfg->n / (double)cfg->k) ? 1 : 0;
  const int64_t m = M->m, p = M->p;
  if (cfg->sketch == CDMD_SKETCH_SRFT) {
    // 2p real rows: the real and imaginary parts of the p complex rows
    M->srft = true;
    M->gplan = cdmd::k::gauss_plan(M->n, m, 2 * (int)p, 0, 1024);
    M->gpart_cap = (size_t)M->gplan.nsplit * m * 2 * p;
    TRY(dalloc(&M->d_gpart, M->gpart_cap));
    TRY(dalloc(&M->d_Yd, (size_t)m * 2 * p));
    TRY(dalloc(&M->d_freq, (size_t)p));
    HIPCHK(hipMemcpy(M->d_freq, cfg->sparse_idx, (size_t)p * 4, hipMemcpyHostToDevice));
    TRY(dalloc(&M->d_gram_im, (size_t)m * m));
    TRY(halloc(&M->h_gram_im, (size_t)m * m));
  } else if (cfg->sketch == CDMD_SKETCH_GAUSSIAN) {
    M->gauss = true;
    M->gplan = cdmd::k::gauss_plan(M->n, m, (int)p, gauss_prec(*cfg), 1024);
    M->gpart_cap = (size_t)M->gplan.nsplit * m * p;
    TRY(dalloc(&M->d_gpart, M->gpart_cap));
    TRY(dalloc(&M->d_Yd, (size_t)m * p));
  } else if (cfg->dtype == CDMD_U8) {
    TRY(build_sparse_plan(M));
    TRY(dalloc(&M->d_Yint, (size_t)m * p));
    TRY(dalloc(&M->d_Ypart, (size_t)M->sk_slots_cap * m * p));
  } else {
    const size_t T = (size_t)p * cfg->nnz;
    TRY(dalloc(&M->d_idx, T));
    TRY(dalloc(&M->d_sign, T));
    std::vector<int8_t> sg(T, 1);
    if (cfg->sparse_sign) std::memcpy(sg.data(), cfg->sparse_sign, T);
    HIPCHK(hipMemcpy(M->d_idx, cfg->sparse_idx, T * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(M->d_sign, sg.data(), T, hipMemcpyHostToDevice));
    TRY(dalloc(&M->d_Yd, (size_t)m * p));
  }
  M->cfg.sparse_idx = nullptr;
  M->cfg.sparse_sign = nullptr;
  TRY(dalloc(&M->d_gram, (size_t)m * m));
  TRY(halloc(&M->h_gram, (size_t)m * m));
  TRY(dalloc(&M->d_G, (size_t)M->N * M->NC));
  TRY(halloc(&M->h_G, (size_t)M->N * M->NC));
  std::vector<uint32_t> pairs;
  for (int a = 0; a < M->nc; ++a)
    for (int b2 = a; b2 < M->nc; ++b2) pairs.push_back((uint32_t)a | ((uint32_t)b2 << 16));
  TRY(dalloc(&M->d_pairs, pairs.size()));
  HIPCHK(hipMemcpy(M->d_pairs, pairs.data(), pairs.size() * 4, hipMemcpyHostToDevice));
  M->lgrid = cdmd::k::lift_grid(M->n);
  size_t part_sz = (size_t)M->lgrid * M->ne, red_sz = (size_t)M->ne;
  if (cfg->dtype == CDMD_U8) {
    M->lm_nb = (M->nc + 1 + 31) / 32;
    M->lm_nsplit = cfg->lift_prec == CDMD_PREC_BF16 ? 1 : 3;
    M->lm_nksteps = (M->N + 15) / 16;
    M->lm_grid = cdmd::k::lift_mfma_grid(M->n);
    M->lm_grid_max = (int)std::min<int64_t>((M->n + 255) / 256, 1024);
    M->lm_ne = M->lm_nb * (M->lm_nb + 1) / 2 * 16 * 64;
    const size_t gp = (size_t)M->lm_nksteps * M->lm_nb * M->lm_nsplit * 64 * 8;
    TRY(dalloc((uint16_t**)&M->d_Gp, gp));
    TRY(halloc(&M->h_Gp, gp));
    // single-read reconstruction operands: G~' (KS = ceil(m/16) k-steps) and V~ (ceil(m/32)
    // frame blocks), in (2, 3) bf16 terms for the float32 form and (1, 2) for bfloat16
    M->rc_nsg = cfg->lift_prec == CDMD_PREC_BF16 ? 1 : 2;
    M->rc_ntv = cfg->lift_prec == CDMD_PREC_BF16 ? 2 : 3;
    M->rc_ks = cdmd::k::recon_ksteps(M->m);
    M->rc_nfb = cdmd::k::recon_frame_blocks(M->m);
    TRY(dalloc((uint16_t**)&M->d_Gsp, (size_t)(M->rc_ks + 4) * M->rc_nsg * 64 * 8));
    TRY(dalloc((uint16_t**)&M->d_Rv, (size_t)(M->rc_nfb + 1) * 2 * M->rc_ntv * 64 * 8));
    TRY(dalloc(&M->d_Gd, (size_t)2 * M->N * M->k));
    TRY(halloc(&M->h_Gd, (size_t)2 * M->N * M->k));
    M->lr_nb = (M->k + 1 + 31) / 32;
    M->lr_ne = M->lr_nb * (M->lr_nb + 1) / 2 * 16 * 64;
    if (M->N <= 1024 && cfg->ld % 16 == 0 && !M->srft) {  // (the SRFT solve is complex, on the host)
      HIPCHK(hipStreamCreateWithFlags(&M->st2, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&M->e_fork, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&M->e_join, hipEventDisableTiming));
      M->la_jmax = std::min(M->N, 320);
      TRY(dalloc(&M->d_la_scratch, (size_t)cdmd::k::small_la_scratch_doubles((int)M->m, M->k, M->la_jmax)));
      M->la_out_n = cdmd::k::small_la_out_doubles((int)M->m, M->k);
      TRY(dalloc(&M->d_la_out, (size_t)M->la_out_n));
      TRY(halloc(&M->h_la_out, (size_t)M->la_out_n));
      M->device_la_ok = true;
    }
    M->lr_grid = (int)std::min<int64_t>((M->n + 255) / 256, 2048);
    part_sz = std::max(part_sz, (size_t)std::max(M->lm_grid, M->lm_grid_max) * M->lm_ne);
    part_sz = std::max(part_sz, (size_t)M->lr_grid * M->lr_ne);
    red_sz = std::max(red_sz, (size_t)M->lm_ne);
  }
  TRY(dalloc(&M->d_part, part_sz));
  TRY(dalloc(&M->d_red, red_sz));
  TRY(halloc(&M->h_red, red_sz));
  TRY(dalloc(&M->d_Gs, (size_t)M->N * 80));
  TRY(halloc(&M->h_Gs, (size_t)M->N * 80));
  TRY(dalloc(&M->d_Vc, (size_t)m * 80));
  TRY(halloc(&M->h_Vc, (size_t)m * 80));
  TRY(dalloc(&M->d_counts, (size_t)m));
  HIPCHK(hipEventCreateWithFlags(&M->e_stage, hipEventDisableTiming));
  TRY(dalloc(&M->d_modes, (size_t)5 * M->k));
  TRY(dalloc(&M->d_feats, (size_t)6 * M->k));
  TRY(dalloc(&M->d_logits, (size_t)M->k));
  TRY(halloc(&M->h_counts, (size_t)m));
  guard.keep = true;
  *out = M;
  return CDMD_OK;
}

void cdmd_free(cdmd_model* mdl) { delete mdl; }

// Which path a fit of d_video takes: the MFMA lift needs 16-byte aligned uint8 frames;
// the device small LA needs the MFMA lift (it writes the lift operands).
void plan_fit(cdmd_model* M, const void* d_video) {
  M->lift_mfma = M->cfg.dtype == CDMD_U8 && M->ld % 16 == 0 &&
                 (reinterpret_cast<uintptr_t>(d_video) & 15) == 0 &&
                 (M->cfg.lift_prec == CDMD_PREC_BF16 || !M->force_valu_lift);
  M->device_la = M->device_la_ok && M->lift_mfma && !M->force_host_la;
  M->lift_real = M->device_la;
}

cdmd_status post_fit(cdmd_model* M, double t0, double t1, double t2);

cdmd_status cdmd_fit(cdmd_model* M, const void* d_video, void* stream) {
  g_err.clear();
  if (!M || !d_video) return fail(CDMD_E_INVALID_ARG, "NULL model or video");
  hipStream_t st = as_stream(stream);
  M->fitted = M->selected = false;
  M->g_canonical_on_device = false;
  plan_fit(M, d_video);
  double t0 = now_ms(), t1, t2;
  if (M->amp_compressed) {
    if (!M->device_la)
      return fail(CDMD_E_UNSUPPORTED, "amplitudes on the compressed modes need the device small linear algebra "
                                      "(uint8 video with 16-byte aligned frames)");
    // two passes over the video: the sketch here, the background / mask later; after the
    // solve's head, the compressed-mode Gram on the call's stream beside the tail
    TRY(run_sketch(M, d_video, st, false));
    HIPCHK(cdmd::k::small_la_head(M->d_gram, (int)M->m, M->k, kLanczosTol, M->la_jmax, M->sketch_scale,
                                  (double)M->xscale, M->d_la_scratch, M->d_la_out, M->d_Gp, M->lr_nb,
                                  M->lm_nsplit, M->lm_nksteps, M->la_groups, st,
                                  M->timing && !M->capturing ? M->ev[7] : nullptr));
    HIPCHK(hipEventRecord(M->e_fork, st));
    HIPCHK(hipStreamWaitEvent(M->st2, M->e_fork, 0));
    TRY(enqueue_la_tail(M, M->st2));
    HIPCHK(hipEventRecord(M->e_join, M->st2));
    const int nblk = cdmd::k::small_la_py_blocks((int)M->m);
    const int ne = M->k * M->k + M->k + 1;
    HIPCHK(cdmd::k::small_la_py(M->d_gram, (int)M->m, M->k, kLanczosTol, M->la_jmax, M->sketch_scale,
                                M->d_la_scratch, M->d_la_out, M->d_py, st));
    HIPCHK(cdmd::k::reduce_partials(M->d_py, nblk, ne, M->d_pyred, st));
    HIPCHK(hipMemcpyAsync(M->h_py, M->d_pyred, sizeof(double) * ne, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamWaitEvent(st, M->e_join, 0));
    M->mark(3, st);
    M->mark(4, st);
    HIPCHK(hipStreamSynchronize(st));
    if (M->timing) {
      M->info.gpu_ms_lift = 0.0;
      M->info.gpu_ms_sketch = M->span(0, 1);
      M->info.gpu_ms_gram = M->span(1, 2);
      M->info.ms_small_la = M->span(2, 3);
      M->info.gpu_ms_lanczos = M->span(2, 7);
    }
    t1 = t2 = now_ms();
    return post_fit(M, t0, t1, t2);
  }
  if (M->device_la) {
    TRY(run_sketch(M, d_video, st, false));
    HIPCHK(cdmd::k::small_la_head(M->d_gram, (int)M->m, M->k, kLanczosTol, M->la_jmax, M->sketch_scale,
                                  (double)M->xscale, M->d_la_scratch, M->d_la_out, M->d_Gp, M->lr_nb,
                                  M->lm_nsplit, M->lm_nksteps, M->la_groups, st,
                                  M->timing && !M->capturing ? M->ev[7] : nullptr));
    // the A~ eigen-solve and G on the side stream, queued before the lift's operands so
    // that its workgroup is resident before the lift fills the device
    HIPCHK(hipEventRecord(M->e_fork, st));
    HIPCHK(hipStreamWaitEvent(M->st2, M->e_fork, 0));
    TRY(enqueue_la_tail(M, M->st2));
    HIPCHK(hipEventRecord(M->e_join, M->st2));
    HIPCHK(cdmd::k::small_la_gp(M->d_gram, (int)M->m, M->k, kLanczosTol, M->la_jmax, M->sketch_scale,
                                (double)M->xscale, M->d_la_scratch, M->d_la_out, M->d_Gp, M->lr_nb,
                                M->lm_nsplit, M->lm_nksteps, M->la_groups, st));
    t1 = t2 = now_ms();
  } else {
    TRY(run_sketch(M, d_video, st, true));
    t1 = now_ms();
    std::vector<double> V, mu;
    TRY(small_la(M, V, mu));
    t2 = now_ms();
  }
  TRY(run_lift(M, d_video, nullptr, st));
  return post_fit(M, t0, t1, t2);
}

// Host part of a fit once its device results are in pinned memory: the device small-LA
// results, H = Phi^H Phi and c, the amplitudes (eq. (eq:b)) and the canonical mode order.
cdmd_status post_fit(cdmd_model* M, double t0, double t1, double t2) {
  if (M->device_la) TRY(take_device_la(M));
  double t3 = now_ms();
  std::vector<cplx> H, cv;
  assemble_H(M, H, cv);
  const int k = M->k;
  std::vector<cplx> b(k);
  if (!cdmd::la::herm_pd_solve(H.data(), k, k, cv.data(), b.data()))
    if (!cdmd::la::lu_solve(H.data(), k, cv.data(), b.data()))
      return fail(CDMD_E_NUMERIC, "amplitude least squares failed (singular Phi^H Phi)");
  std::vector<double> nrm(k), key(k);
  for (int j = 0; j < k; ++j) {
    nrm[j] = std::sqrt(std::max(H[(size_t)j * k + j].real(), 0.0));
    key[j] = std::abs(b[j]) * nrm[j];
  }
  std::vector<int> o = canonical_order(M->lam, key);
  M->perm = o;
  std::vector<cplx> lam(k), W((size_t)k * k), G((size_t)M->N * k), Hc((size_t)k * k), cc(k), bc(k);
  std::vector<double> pn(k);
  for (int j = 0; j < k; ++j) {
    const int s = o[j];
    lam[j] = M->lam[s];
    for (int i = 0; i < k; ++i) W[(size_t)j * k + i] = M->W[(size_t)s * k + i];
    for (int t = 0; t < M->N; ++t) G[(size_t)t * k + j] = M->G[(size_t)t * k + s];
    for (int l = 0; l < k; ++l) Hc[(size_t)j * k + l] = H[(size_t)s * k + o[l]];
    cc[j] = cv[s];
    bc[j] = b[s];
    pn[j] = nrm[s];
  }
  M->lam.swap(lam);
  M->W.swap(W);
  M->G.swap(G);
  M->H.swap(Hc);
  M->c.swap(cc);
  M->b.swap(bc);
  M->phinorm.swap(pn);
  double t4 = now_ms();
  M->info.ms_sketch = t1 - t0;
  if (!M->device_la) M->info.ms_small_la = t2 - t1;  // device path: HIP-event time (run_lift)
  M->info.ms_lift = t3 - t2;
  M->info.ms_host_post = t4 - t3;
  M->info.x1_norm2 = M->x1n2;
  M->fitted = true;
  M->info.fitted = 1;
  M->info.selected = 0;
  return CDMD_OK;
}

// Remark 2's rank for the video, with a model of rank 1 of its shape (only its sketch and
// Gram are used).
static cdmd_status rank_with_model(cdmd_model* M, const void* d_video, hipStream_t st, int32_t* k_out,
                                   double* tau_out, double* sigma_out) {
  plan_fit(M, d_video);
  TRY(run_sketch(M, d_video, st, true));
  // the spectrum of Y = Y^[:, :m-1] from its Gram: sigma_i = scale sqrt(mu_i), the min(p, m-1)
  // largest eigenvalues.  A complex (SRFT) sketch's Hermitian Gram G = Gr + i Gi enters as
  // the real symmetric [[Gr, -Gi], [Gi, Gr]] of twice the order, which has every eigenvalue
  // of G twice: its 2r largest have the same median, and twice the count above it.
  const int N = M->N;
  const double* A = M->h_gram;
  int nA = N, ldA = (int)M->m, mult = 1;
  std::vector<double> R2;
  if (M->srft) {
    const int64_t m = M->m;
    nA = 2 * N;
    ldA = nA;
    mult = 2;
    R2.assign((size_t)nA * nA, 0.0);
    for (int a = 0; a < N; ++a)
      for (int b2 = 0; b2 < N; ++b2) {
        // upper triangle as computed, lower triangle its conjugate
        const double gr = a <= b2 ? M->h_gram[a * m + b2] : M->h_gram[b2 * m + a];
        const double gi = a <= b2 ? M->h_gram_im[a * m + b2] : -M->h_gram_im[b2 * m + a];
        R2[(size_t)a * nA + b2] = gr;
        R2[(size_t)(a + N) * nA + b2 + N] = gr;
        R2[(size_t)a * nA + b2 + N] = -gi;
        R2[(size_t)(a + N) * nA + b2] = gi;
      }
    A = R2.data();
  }
  const int r = std::min(N, M->p);
  if (!sigma_out) {  // the median and one count are enough
    const double beta = (double)r / (double)std::max(N, M->p);
    int k = 0;
    double tau = 0.0;
    if (!cdmd::la::sym_rank_threshold(A, nA, ldA, mult * r, M->sketch_scale, cdmd::la::gd_omega(beta), &k, &tau))
      return fail(CDMD_E_NUMERIC, "non-finite Gram");
    *k_out = (k + mult - 1) / mult;
    if (tau_out) *tau_out = tau;
    return CDMD_OK;
  }
  std::vector<double> ev;
  if (!cdmd::la::sym_eigvals(A, nA, ldA, ev)) return fail(CDMD_E_NUMERIC, "non-finite Gram");
  std::vector<double> sig(r);
  for (int i = 0; i < r; ++i) sig[i] = M->sketch_scale * std::sqrt(std::max(ev[nA - 1 - mult * i], 0.0));
  // the median of the r singular values (the mean of the middle two for even r)
  const double med = (r & 1) ? sig[r / 2] : 0.5 * (sig[r / 2 - 1] + sig[r / 2]);
  const double beta = (double)r / (double)std::max(N, M->p);
  const double tau = cdmd::la::gd_omega(beta) * med;
  int k = 0;
  while (k < r && sig[k] > tau) ++k;
  *k_out = k;
  if (tau_out) *tau_out = tau;
  if (sigma_out) std::memcpy(sigma_out, sig.data(), sizeof(double) * r);
  return CDMD_OK;
}

cdmd_status cdmd_optimal_rank(const cdmd_config* cfg, const void* d_video, void* stream, int32_t* k_out,
                              double* tau_out, double* sigma_out) {
  g_err.clear();
  if (!cfg || !d_video || !k_out) return fail(CDMD_E_INVALID_ARG, "NULL argument");
  cdmd_config c = *cfg;
  c.k = 1;  // the sketch and its Gram do not depend on k
  cdmd_model* M = nullptr;
  TRY(cdmd_create(&c, &M));
  std::unique_ptr<cdmd_model> own(M);
  return rank_with_model(M, d_video, as_stream(stream), k_out, tau_out, sigma_out);
}

cdmd_status cdmd_modes(const cdmd_model* Mc, double* lambda, double* b, double* sigma,
                       double* phi_norm, const void* d_video, void* d_phi, void* stream) {
  g_err.clear();
  if (!Mc) return fail(CDMD_E_INVALID_ARG, "NULL model");
  cdmd_model* M = const_cast<cdmd_model*>(Mc);
  if (!M->fitted) return fail(CDMD_E_STATE, "model is not fitted");
  const int k = M->k;
  for (int j = 0; j < k; ++j) {
    if (lambda) lambda[2 * j] = M->lam[j].real(), lambda[2 * j + 1] = M->lam[j].imag();
    if (b) b[2 * j] = M->b[j].real(), b[2 * j + 1] = M->b[j].imag();
    if (sigma) sigma[j] = M->sigma[j];
    if (phi_norm) phi_norm[j] = M->phinorm[j];
  }
  if (d_phi) {
    if (!d_video) return fail(CDMD_E_INVALID_ARG, "d_phi needs the fitted video");
    hipStream_t st = as_stream(stream);
    std::vector<int> ident(k);
    std::iota(ident.begin(), ident.end(), 0);
    TRY(upload_G(M, ident, st));  // M->G is in canonical order
    // the lift reduction buffers are reused; results of the fit are kept on the host
    TRY(launch_lift(M, d_video, (float*)d_phi, st, false));
    HIPCHK(hipStreamSynchronize(st));
  }
  return CDMD_OK;
}

// ------------------------------------------------------------------ autotuner
// Tile shapes chosen by timing the candidates on the caller's video, once per size
// class (process-wide cache): the number of persistent lift workgroups, and for the dense
// Gaussian sketch the number of pixel slices.
extern "C++" {
namespace {
struct TuneKey {
  int64_t n, m;
  int k, p, sketch, sprec, lprec, dtype;
  bool operator<(const TuneKey& o) const {
    return std::tie(n, m, k, p, sketch, sprec, lprec, dtype) <
           std::tie(o.n, o.m, o.k, o.p, o.sketch, o.sprec, o.lprec, o.dtype);
  }
};
struct TuneChoice {
  int lift_grid = 0;
  int gauss_target = 0;
  int sparse_form = 0;  // 0 untuned, -1 gather, else 10 F + V (streaming)
  int gemm_algo = -1;   // the stored-C sketch GEMM's candidate, or -1 untuned
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice> g_tune;

// Size class: the frame size, frames in steps of 128, ranks in steps of 8, sketch rows by
// octave, and the sketch / precision / pixel type.
TuneKey tune_key(const cdmd_model* M) {
  const cdmd_config& c = M->cfg;
  int po = 0;
  while ((1 << (po + 1)) <= M->p) ++po;
  return TuneKey{M->n, (M->m + 127) / 128, (M->k + 7) / 8, po, (int)c.sketch, (int)c.sketch_prec,
                 (int)c.lift_prec, (int)c.dtype};
}

template <class F>
cdmd_status time_ms(hipStream_t st, int reps, F&& launch, double* ms) {
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(CDMD_E_DEVICE, "hipEventCreate failed");
  }
  cdmd_status r = launch();  // warm-up
  if (r == CDMD_OK) {
    (void)hipEventRecord(a, st);
    for (int i = 0; i < reps && r == CDMD_OK; ++i) r = launch();
    (void)hipEventRecord(b, st);
    (void)hipEventSynchronize(b);
    float t = 0.f;
    (void)hipEventElapsedTime(&t, a, b);
    *ms = t / reps;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return r;
}

cdmd_status apply_sparse_form(cdmd_model* M, int form) {
  if (form < 0) {
    M->force_gather_sketch = true;
    return CDMD_OK;
  }
  const int F = form / 10, V = form % 10;
  if (!cdmd::k::sketch_stream_fits(F, V, M->max_rows) || stream_nrange(M, F, V) > M->sk_slots_cap)
    return fail(CDMD_E_INVALID_ARG, "streaming sketch form does not fit");
  M->force_gather_sketch = false;
  M->sk_F = F;
  M->sk_V = V;
  M->sk_nrange = stream_nrange(M, F, V);
  return CDMD_OK;
}

cdmd_status apply_gauss_target(cdmd_model* M, int target) {
  cdmd::k::GaussPlan g = cdmd::k::gauss_plan(M->n, M->m, (int)M->p, gauss_prec(M->cfg), target);
  const size_t need = (size_t)g.nsplit * M->m * M->p;
  if (need > M->gpart_cap) {
    float* np = nullptr;
    TRY(dalloc(&np, need));
    (void)hipFree(M->d_gpart);
    M->d_gpart = np;
    M->gpart_cap = need;
  }
  M->gplan = g;
  return CDMD_OK;
}
}  // namespace
}  // extern "C++"

cdmd_status cdmd_autotune(cdmd_model* M, const void* d_video, void* stream) {
  g_err.clear();
  if (!M || !d_video) return fail(CDMD_E_INVALID_ARG, "NULL model or video");
  hipStream_t st = as_stream(stream);
  plan_fit(M, d_video);
  const TuneKey key = tune_key(M);
  TuneChoice ch;
  bool cached = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) ch = it->second, cached = true;
  }
  if (!cached) {
    if (M->lift_mfma && !M->lift_real) {
      double best = 1e300;
      for (int g : {128, 256, 512, 1024}) {
        if (g > M->lm_grid_max) continue;
        M->lm_grid = g;
        double ms = 0.0;
        TRY(time_ms(st, 3, [&] { return launch_lift(M, d_video, nullptr, st, M->lift_real); }, &ms));
        if (ms < best) best = ms, ch.lift_grid = g;
      }
    }
    if (M->sgemm) {
      // the library's candidate GEMM algorithms on this video (conversion, products, sum)
      double best = 1e300;
      for (int i = 0; i < cdmd::blas::sketch_gemm_candidates(M->sgemm); ++i) {
        (void)cdmd::blas::sketch_gemm_select(M->sgemm, i);
        double ms = 0.0;
        const cdmd_status r = time_ms(st, 2, [&] { return gemm_sketch(M, d_video, st); }, &ms);
        if (r == CDMD_OK && ms < best) best = ms, ch.gemm_algo = i;
      }
      g_err.clear();
      if (ch.gemm_algo < 0) return fail(CDMD_E_DEVICE, "no sketch GEMM candidate ran");
    }
    if (M->gauss && !M->sgemm) {
      double best = 1e300;
      for (int target : {512, 1024, 2048}) {
        TRY(apply_gauss_target(M, target));
        double ms = 0.0;
        TRY(time_ms(st, 1, [&] {
          HIPCHK(cdmd::k::sketch_gauss(d_video, M->cfg.dtype == CDMD_U8 ? 0 : 1, M->ld, M->n, M->m, M->p,
                                       M->cfg.seed, gauss_prec(M->cfg), M->gplan, M->d_Cm, M->Cm_ldc,
                                       M->d_gpart, M->d_Yd, st));
          return CDMD_OK;
        }, &ms));
        if (ms < best) best = ms, ch.gauss_target = target;
      }
    }
    if (!M->gauss && !M->srft && M->cfg.dtype == CDMD_U8 && M->ld % 16 == 0 &&
        (reinterpret_cast<uintptr_t>(d_video) & 15) == 0) {
      // sparse sketch: the gather form, or streaming with (frames per group, vectors per thread)
      double best = 1e300;
      const int forms[] = {-1, 41, 21, 22, 11, 12, 14};
      for (int f : forms) {
        if (f > 0 && !cdmd::k::sketch_stream_fits(f / 10, f % 10, M->max_rows)) continue;
        if (f > 0 && stream_nrange(M, f / 10, f % 10) > M->sk_slots_cap) continue;
        TRY(apply_sparse_form(M, f));
        double ms = 0.0;
        TRY(time_ms(st, 3, [&] { return run_sketch(M, d_video, st, false); }, &ms));
        if (ms < best) best = ms, ch.sparse_form = f;
      }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = ch;
  }
  if (ch.sparse_form != 0) TRY(apply_sparse_form(M, ch.sparse_form));
  if (ch.lift_grid > 0) M->lm_grid = ch.lift_grid;
  if (ch.gauss_target > 0 && !M->sgemm) TRY(apply_gauss_target(M, ch.gauss_target));
  if (ch.gemm_algo >= 0 && M->sgemm) (void)cdmd::blas::sketch_gemm_select(M->sgemm, ch.gemm_algo);
  M->tuned = true;
  ++M->stamp;
  M->info.lift_grid = M->lift_real ? M->lr_grid : M->lm_grid;
  M->info.sketch_slices = M->gauss ? M->gplan.nsplit : 0;
  M->info.sparse_form = M->gauss || M->srft ? 0 : (M->force_gather_sketch ? -1 : 10 * M->sk_F + M->sk_V);
  return CDMD_OK;
}

// ------------------------------------------------------------------ batched fits
// Many models fitted by one graph launch: the sketch + Gram and the lift of every model
// run on a pool of streams (fork/join through events), and the device small LA of all
// of them is one launch with a workgroup per model.  The graph is captured on the first
// call and replayed while the videos stay the same.  Models whose fit needs the host small
// LA (float32 videos, unaligned frames, m > 1025) are fitted one after the other after the
// graph.
struct cdmd_batch {
  std::vector<cdmd_model*> models;
  std::vector<const void*> videos;  // of the captured graph
  std::vector<uint64_t> stamps;     // the members' configuration stamps at capture
  std::vector<int> dev;             // models on the graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipStream_t> pool;
  hipEvent_t fork1 = nullptr, fork2 = nullptr, fork_tail = nullptr;
  std::vector<hipEvent_t> join1, join2;
  cdmd::k::SLADesc* d_desc = nullptr;
  int la_nmax = 0, la_gmax = 0;     // grid extents of the small-LA row kernels
  int la_ngroups = 0;               // Lanczos workgroups per solve in the grid
  int la_kmax = 0;                  // largest k of the batch
  hipStream_t cap = nullptr;        // the graph's own stream (capture needs a non-null stream)
  hipEvent_t entry = nullptr;       // caller's stream -> cap
  // cdmd_batch_foreground's work lists: staged in pinned memory (rewritten once the last
  // copy from it has completed) and read by the kernels from d_rwork (rewritten after the
  // last launch that read it)
  cdmd::k::ReconWork* h_rwork = nullptr;
  cdmd::k::ReconWork* d_rwork = nullptr;
  size_t rwork_cap = 0;
  hipEvent_t rw_copied = nullptr, rw_read = nullptr;
  bool rw_pending = false;

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    videos.clear();
    stamps.clear();
  }
  ~cdmd_batch() {
    drop_graph();
    for (hipStream_t s : pool) (void)hipStreamDestroy(s);
    for (hipEvent_t e : join1) (void)hipEventDestroy(e);
    for (hipEvent_t e : join2) (void)hipEventDestroy(e);
    if (fork1) (void)hipEventDestroy(fork1);
    if (fork_tail) (void)hipEventDestroy(fork_tail);
    if (fork2) (void)hipEventDestroy(fork2);
    if (entry) (void)hipEventDestroy(entry);
    if (cap) (void)hipStreamDestroy(cap);
    if (d_desc) (void)hipFree(d_desc);
    if (rw_pending) (void)hipEventSynchronize(rw_read);
    if (rw_copied) (void)hipEventDestroy(rw_copied);
    if (rw_read) (void)hipEventDestroy(rw_read);
    if (h_rwork) (void)hipHostFree(h_rwork);
    if (d_rwork) (void)hipFree(d_rwork);
  }
};

cdmd_status cdmd_batch_create(cdmd_model* const* models, int32_t n, cdmd_batch** out) {
  g_err.clear();
  if (!models || !out || n < 1) return fail(CDMD_E_INVALID_ARG, "bad arguments");
  for (int i = 0; i < n; ++i) {
    if (!models[i]) return fail(CDMD_E_INVALID_ARG, "NULL model in the batch");
    for (int j = 0; j < i; ++j)
      if (models[j] == models[i]) return fail(CDMD_E_INVALID_ARG, "a model appears twice in the batch");
    if (models[i]->amp_compressed)
      return fail(CDMD_E_UNSUPPORTED, "batches fit on the full modes (cdmd_set_amplitudes FULL)");
    if (models[i]->srft) return fail(CDMD_E_UNSUPPORTED, "SRFT models are fitted one at a time");
    if (models[i]->sgemm)
      return fail(CDMD_E_UNSUPPORTED, "a stored C is streamed by a library GEMM, which batches do not capture");
  }
  std::unique_ptr<cdmd_batch> B(new (std::nothrow) cdmd_batch());
  if (!B) return fail(CDMD_E_OUT_OF_MEMORY, "host allocation failed");
  B->models.assign(models, models + n);
  const int P = std::min(n, 8);
  for (int i = 0; i < P; ++i) {
    hipStream_t s;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    B->pool.push_back(s);
    hipEvent_t e1, e2;
    HIPCHK(hipEventCreateWithFlags(&e1, hipEventDisableTiming));
    B->join1.push_back(e1);
    HIPCHK(hipEventCreateWithFlags(&e2, hipEventDisableTiming));
    B->join2.push_back(e2);
  }
  HIPCHK(hipEventCreateWithFlags(&B->fork1, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&B->fork_tail, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&B->fork2, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&B->entry, hipEventDisableTiming));
  HIPCHK(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
  TRY(dalloc(&B->d_desc, (size_t)n));
  // work lists of cdmd_batch_foreground: at most two entries per model (its full tiles
  // and its partial tile), room for twice that
  B->rwork_cap = 4 * (size_t)n;
  TRY(halloc(&B->h_rwork, B->rwork_cap));
  TRY(dalloc(&B->d_rwork, B->rwork_cap));
  HIPCHK(hipEventCreateWithFlags(&B->rw_copied, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&B->rw_read, hipEventDisableTiming));
  *out = B.release();
  return CDMD_OK;
}

void cdmd_batch_free(cdmd_batch* B) { delete B; }

namespace {
cdmd_status capture_batch(cdmd_batch* B, hipStream_t st) {
  const int P = (int)B->pool.size();
  HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  cdmd_status r = CDMD_OK;
  auto guard = [&](cdmd_status x) {
    if (r == CDMD_OK) r = x;
  };
  auto hip = [&](hipError_t e) {
    if (e != hipSuccess && r == CDMD_OK) r = fail(CDMD_E_DEVICE, hipGetErrorString(e));
  };
  hip(hipEventRecord(B->fork1, st));
  for (int q = 0; q < P; ++q) hip(hipStreamWaitEvent(B->pool[q], B->fork1, 0));
  for (size_t i = 0; i < B->dev.size() && r == CDMD_OK; ++i) {
    cdmd_model* M = B->models[B->dev[i]];
    guard(run_sketch(M, B->videos[B->dev[i]], B->pool[i % P], false));
  }
  for (int q = 0; q < P; ++q) {
    hip(hipEventRecord(B->join1[q], B->pool[q]));
    hip(hipStreamWaitEvent(st, B->join1[q], 0));
  }
  hip(cdmd::k::small_la_batch_head(B->d_desc, (int)B->dev.size(), B->la_nmax, B->la_ngroups, st));
  // the A~ eigen-solves and G of every model on pool stream 0, queued before the lift
  // operands so that their workgroups are resident before the lifts fill the device; the
  // lifts on the other pool streams
  hip(hipEventRecord(B->fork_tail, st));
  hip(hipStreamWaitEvent(B->pool[0], B->fork_tail, 0));
  hip(cdmd::k::small_la_batch_tail(B->d_desc, (int)B->dev.size(), B->la_nmax, B->la_kmax, B->pool[0]));
  for (size_t i = 0; i < B->dev.size() && r == CDMD_OK; ++i) {
    cdmd_model* M = B->models[B->dev[i]];
    hip(hipMemcpyAsync(M->h_la_out, M->d_la_out, sizeof(double) * M->la_out_n, hipMemcpyDeviceToHost,
                       B->pool[0]));
  }
  hip(cdmd::k::small_la_batch_gp(B->d_desc, (int)B->dev.size(), B->la_gmax, st));
  hip(hipEventRecord(B->fork2, st));
  const int PL = P > 1 ? P - 1 : 1;  // lift streams: pool[1..P-1] (pool[0] if there is one stream)
  for (int q = 0; q < P; ++q) hip(hipStreamWaitEvent(B->pool[q], B->fork2, 0));
  for (size_t i = 0; i < B->dev.size() && r == CDMD_OK; ++i) {
    cdmd_model* M = B->models[B->dev[i]];
    guard(enqueue_lift(M, B->videos[B->dev[i]], nullptr, B->pool[P > 1 ? 1 + (int)(i % PL) : 0]));
  }
  for (int q = 0; q < P; ++q) {
    hip(hipEventRecord(B->join2[q], B->pool[q]));
    hip(hipStreamWaitEvent(st, B->join2[q], 0));
  }
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(st, &g);
  if (r != CDMD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  if (ee != hipSuccess) return fail(CDMD_E_DEVICE, hipGetErrorString(ee));
  B->graph = g;
  HIPCHK(hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0));
  return CDMD_OK;
}
}  // namespace

cdmd_status cdmd_batch_fit(cdmd_batch* B, const void* const* d_videos, void* stream,
                           cdmd_status* per_model) {
  g_err.clear();
  if (!B || !d_videos) return fail(CDMD_E_INVALID_ARG, "NULL batch or videos");
  const int n = (int)B->models.size();
  for (int i = 0; i < n; ++i)
    if (!d_videos[i]) return fail(CDMD_E_INVALID_ARG, "NULL video in the batch");
  hipStream_t st = as_stream(stream);
  if (per_model)
    for (int i = 0; i < n; ++i) per_model[i] = CDMD_E_STATE;  // not attempted
  for (int i = 0; i < n; ++i) {
    if (B->models[i]->amp_compressed)
      return fail(CDMD_E_UNSUPPORTED, "amplitudes on the compressed modes are not built for batches");
    if (B->models[i]->sgemm)  // a C stored after the batch was created
      return fail(CDMD_E_UNSUPPORTED, "a stored C is streamed by a library GEMM, which batches do not capture");
  }
  bool same = B->exec && (int)B->videos.size() == n && (int)B->stamps.size() == n &&
              std::equal(B->videos.begin(), B->videos.end(), d_videos, d_videos + n);
  for (int i = 0; same && i < n; ++i) same = B->stamps[i] == B->models[i]->stamp;
  if (!same) {
    B->drop_graph();
    B->videos.assign(d_videos, d_videos + n);
    B->dev.clear();
    std::vector<cdmd::k::SLADesc> desc;
    B->la_nmax = B->la_gmax = B->la_ngroups = B->la_kmax = 0;
    for (int i = 0; i < n; ++i) {
      cdmd_model* M = B->models[i];
      plan_fit(M, d_videos[i]);
      if (!M->device_la) continue;
      if (!M->tuned) TRY(cdmd_autotune(M, d_videos[i], stream));
      plan_fit(M, d_videos[i]);
      B->dev.push_back(i);
      desc.push_back(cdmd::k::SLADesc{M->d_gram, M->d_la_scratch, M->d_la_out, (uint16_t*)M->d_Gp, kLanczosTol,
                                      M->sketch_scale, (double)M->xscale, (int)M->m, M->k, M->la_jmax,
                                      M->lr_nb, M->lm_nsplit, M->lm_nksteps, M->la_groups});
      B->la_nmax = std::max(B->la_nmax, (int)M->m - 1);
      B->la_gmax = std::max(B->la_gmax, std::max((int)M->m - 1, 16 * M->lm_nksteps));
      B->la_kmax = std::max(B->la_kmax, M->k);
      B->la_ngroups = std::max(B->la_ngroups, M->la_groups > 0 ? std::min(M->la_groups, (int)M->m - 1)
                                                                : cdmd::tla::la_groups((int)M->m - 1));
    }
    if (!desc.empty()) {
      HIPCHK(hipMemcpy(B->d_desc, desc.data(), sizeof(desc[0]) * desc.size(), hipMemcpyHostToDevice));
      for (int i : B->dev) B->models[i]->capturing = true;
      const cdmd_status r = capture_batch(B, B->cap);
      for (int i : B->dev) B->models[i]->capturing = false;
      if (r != CDMD_OK) {
        B->drop_graph();
        return r;
      }
    }
    B->stamps.resize(n);
    for (int i = 0; i < n; ++i) B->stamps[i] = B->models[i]->stamp;
  }
  cdmd_status first = CDMD_OK;
  const double t0 = now_ms();
  for (int i : B->dev) {
    B->models[i]->fitted = B->models[i]->selected = false;
    B->models[i]->g_canonical_on_device = false;
  }
  if (B->exec) {
    // the graph runs on the batch's stream after the work already on the caller's stream
    HIPCHK(hipEventRecord(B->entry, st));
    HIPCHK(hipStreamWaitEvent(B->cap, B->entry, 0));
    HIPCHK(hipGraphLaunch(B->exec, B->cap));
    HIPCHK(hipStreamSynchronize(B->cap));
  }
  const double t1 = now_ms();
  std::vector<char> on_graph(n, 0);
  for (int i : B->dev) on_graph[i] = 1;
  for (int i = 0; i < n; ++i) {
    cdmd_model* M = B->models[i];
    cdmd_status r;
    if (on_graph[i]) {
      plan_fit(M, d_videos[i]);
      r = post_fit(M, t0, t1, t1);
    } else {
      r = cdmd_fit(M, d_videos[i], stream);
    }
    if (per_model) per_model[i] = r;
    if (r != CDMD_OK && first == CDMD_OK) first = r;
  }
  if (first != CDMD_OK) return fail(first, "at least one model of the batch failed (see per_model)");
  return CDMD_OK;
}

cdmd_status cdmd_select(cdmd_model* M, int32_t selector, int32_t K, double omega_thr,
                        const int32_t* explicit_idx, int32_t n_explicit, int32_t* out_idx,
                        int32_t* out_n, double* out_beta) {
  g_err.clear();
  if (!M) return fail(CDMD_E_INVALID_ARG, "NULL model");
  if (!M->fitted) return fail(CDMD_E_STATE, "model is not fitted");
  const int k = M->k;
  std::vector<int> S;
  std::vector<cplx> beta;
  double r2 = 0.0;
  switch (selector) {
    case CDMD_SEL_OMP: {
      if (K < 1) return fail(CDMD_E_INVALID_ARG, "OMP needs K >= 1");
      if (!cdmd::la::omp_gram(M->H.data(), k, M->c.data(), M->x1n2, K, M->lam.data(), kOmpStopRel, S, beta, &r2))
        return fail(CDMD_E_NUMERIC, "OMP subsystem singular");
      break;
    }
    case CDMD_SEL_ZERO_MODE: {
      int best = 0;
      double bv = 1e300;
      for (int j = 0; j < k; ++j) {
        const double w = std::abs(std::log(M->lam[j]));
        if (w < bv) bv = w, best = j;
      }
      S.push_back(best);
      beta.push_back(M->b[best]);
      break;
    }
    case CDMD_SEL_OMEGA: {
      if (!(omega_thr > 0.0)) return fail(CDMD_E_INVALID_ARG, "omega_thr must be > 0");
      for (int j = 0; j < k; ++j)
        if (std::abs(std::log(M->lam[j])) < omega_thr) S.push_back(j), beta.push_back(M->b[j]);
      break;
    }
    case CDMD_SEL_EXPLICIT: {
      if (!explicit_idx || n_explicit < 1 || n_explicit > k)
        return fail(CDMD_E_INVALID_ARG, "explicit support needs 1..k indices");
      std::vector<char> seen(k, 0);
      for (int q = 0; q < n_explicit; ++q) {
        const int j = explicit_idx[q];
        if (j < 0 || j >= k || seen[j]) return fail(CDMD_E_INVALID_ARG, "explicit index out of range or repeated");
        seen[j] = 1;
        S.push_back(j);
      }
      const int ns = (int)S.size();
      std::vector<cplx> Hs((size_t)ns * ns), cs(ns);
      for (int a = 0; a < ns; ++a) {
        cs[a] = M->c[S[a]];
        for (int b2 = 0; b2 < ns; ++b2) Hs[(size_t)a * ns + b2] = M->H[(size_t)S[a] * k + S[b2]];
      }
      beta.assign(ns, 0.0);
      if (!cdmd::la::herm_pd_solve(Hs.data(), ns, ns, cs.data(), beta.data()))
        if (!cdmd::la::lu_solve(Hs.data(), ns, cs.data(), beta.data()))
          return fail(CDMD_E_NUMERIC, "explicit support subsystem singular");
      break;
    }
    case CDMD_SEL_ALL: {
      for (int j = 0; j < k; ++j) S.push_back(j), beta.push_back(M->b[j]);
      break;
    }
    default:
      return fail(CDMD_E_INVALID_ARG, "unknown selector");
  }
  if (selector != CDMD_SEL_OMP) {
    // ||x_1 - Phi_S beta||^2 = ||x_1||^2 - 2 Re(beta^H c_S) + beta^H H_SS beta
    const int ns = (int)S.size();
    cplx q = 0.0, hq = 0.0;
    for (int a = 0; a < ns; ++a) {
      q += std::conj(beta[a]) * M->c[S[a]];
      for (int b2 = 0; b2 < ns; ++b2) hq += std::conj(beta[a]) * M->H[(size_t)S[a] * k + S[b2]] * beta[b2];
    }
    r2 = std::max(M->x1n2 - 2.0 * q.real() + hq.real(), 0.0);
  }
  M->S = S;
  M->beta = beta;
  M->selected = true;
  M->info.selected = 1;
  M->info.n_selected = (int)S.size();
  M->info.omp_residual2 = r2;
  if (out_n) *out_n = (int32_t)S.size();
  for (size_t q = 0; q < S.size(); ++q) {
    if (out_idx) out_idx[q] = S[q];
    if (out_beta) out_beta[2 * q] = beta[q].real(), out_beta[2 * q + 1] = beta[q].imag();
  }
  return CDMD_OK;
}

namespace {

// Operands of the reconstruction.  MFMA form (16-byte aligned uint8 frames, |S| <= 16,
// the tile's frames fit in LDS): the A fragments of G~^T = [Re | Im] of G_S diag(beta)
// xscale, formed on the device from the device solve's G or here from the host G; the
// Vandermonde factors are powers the kernel forms from the eigenvalues.  VALU form:
// Gs = [Re(G_S diag beta) | Im(...)] * xscale and the Vandermonde rows Vc[t] =
// [Re lambda^t | -Im lambda^t] (t = 0..m-1, 0-based).  Host staging buffers are rewritten
// only once the copies of the previous call have completed.
cdmd_status prepare_recon(cdmd_model* M, int static_bg, int* NSout, hipStream_t st) {
  const int ns = (int)M->S.size();
  const int NS = pad_ns(std::max(2 * ns, 1));
  const int N = M->N, k = M->k;
  const int64_t m = M->m;
  for (int s = 0; s < ns; ++s) {
    const cplx l = M->lam[M->S[s]];
    if (!static_bg && std::abs(l) > 1.0 && std::pow(std::abs(l), (double)(m - 1)) > kVanderMax)
      return fail(CDMD_E_NUMERIC, "|lambda|^(m-1) overflows the Vandermonde matrix");
  }
  M->recon_mfma = M->lift_mfma && ns <= 16 && cdmd::k::recon_lds_bytes(m) <= (size_t)160 * 1024;
  if (!M->recon_mfma && NS < 0) return fail(CDMD_E_UNSUPPORTED, "more than 40 selected modes");
  if (M->stage_pending) {
    HIPCHK(hipEventSynchronize(M->e_stage));
    M->stage_pending = false;
  }
  *NSout = NS;
  if (M->recon_mfma) {
    cdmd::k::ReconPrep rp{};
    rp.ns = ns;
    rp.NSG = M->rc_nsg;
    rp.NTV = M->rc_ntv;
    rp.KS = M->rc_ks;
    rp.NFB = M->rc_nfb;
    rp.N = N;
    rp.k = k;
    rp.static_bg = static_bg ? 1 : 0;
    rp.xscale = (double)M->xscale;
    for (int s = 0; s < ns; ++s) {
      rp.beta[2 * s] = M->beta[s].real();
      rp.beta[2 * s + 1] = M->beta[s].imag();
      rp.lam[2 * s] = M->lam[M->S[s]].real();
      rp.lam[2 * s + 1] = M->lam[M->S[s]].imag();
    }
    const double* Gdev = nullptr;
    if (M->device_la) {
      // the device solve's G (column order of the solve: canonical index c is column perm[c])
      for (int s = 0; s < ns; ++s) rp.col[s] = M->perm[M->S[s]];
      Gdev = M->d_la_out + cdmd::tla::small_la_out_layout(N, k).G;
    } else {
      for (int s = 0; s < ns; ++s) rp.col[s] = M->S[s];
      std::memcpy(M->h_Gd, M->G.data(), sizeof(double) * 2 * (size_t)N * k);
      HIPCHK(hipMemcpyAsync(M->d_Gd, M->h_Gd, sizeof(double) * 2 * (size_t)N * k, hipMemcpyHostToDevice, st));
      HIPCHK(hipEventRecord(M->e_stage, st));
      M->stage_pending = true;
      Gdev = M->d_Gd;
    }
    HIPCHK(cdmd::k::recon_prep(Gdev, rp, M->d_Gsp, M->d_Rv, st));
    return CDMD_OK;
  }
  for (int t = 0; t < N; ++t) {
    float* row = M->h_Gs + (size_t)t * NS;
    for (int c = 0; c < NS; ++c) row[c] = 0.f;
    for (int s = 0; s < ns; ++s) {
      const cplx g = M->G[(size_t)t * k + M->S[s]] * M->beta[s] * (double)M->xscale;
      row[s] = (float)g.real();
      row[ns + s] = (float)g.imag();
    }
  }
  std::vector<cplx> pw(ns, cplx(1.0, 0.0));
  for (int64_t t = 0; t < m; ++t) {
    float* row = M->h_Vc + (size_t)t * NS;
    for (int c = 0; c < NS; ++c) row[c] = 0.f;
    for (int s = 0; s < ns; ++s) {
      row[s] = (float)pw[s].real();
      row[ns + s] = (float)(-pw[s].imag());
      if (!static_bg) pw[s] *= M->lam[M->S[s]];
    }
  }
  HIPCHK(hipMemcpyAsync(M->d_Gs, M->h_Gs, sizeof(float) * N * NS, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(M->d_Vc, M->h_Vc, sizeof(float) * m * NS, hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(M->e_stage, st));
  M->stage_pending = true;
  return CDMD_OK;
}

// The reconstruction kernel of the form prepare_recon chose.
cdmd_status run_recon(cdmd_model* M, const void* d_video, int static_bg, int NS, float tau, int mode,
                      void* out, int64_t t0, int64_t t1, int64_t ldL, hipStream_t st) {
  if (M->recon_mfma) {
    cdmd::k::ReconArgs a{};
    a.D = static_cast<const uint8_t*>(d_video);
    a.ld = M->ld;
    a.n = M->n;
    a.m = M->m;
    a.Gp = static_cast<const uint4*>(M->d_Gsp);
    a.Vp = static_cast<const uint4*>(M->d_Rv);
    a.KS = M->rc_ks;
    a.NFB = M->rc_nfb;
    a.ns = (int)M->S.size();
    a.tau = tau;
    a.xscale = M->xscale;
    a.mode = mode;
    a.out = out;
    a.t0 = t0;
    a.t1 = t1;
    a.ldL = ldL;
    HIPCHK(cdmd::k::recon_mfma(a, M->rc_nsg, M->rc_ntv, st));
    return CDMD_OK;
  }
  HIPCHK(cdmd::k::bgfg(d_video, M->cfg.dtype, M->ld, M->n, M->m, M->d_Gs, NS, M->d_Vc, tau, M->xscale, mode, out,
                       t0, t1, ldL, st));
  return CDMD_OK;
}

}  // namespace

cdmd_status cdmd_background(const cdmd_model* Mc, const void* d_video, int64_t t0, int64_t t1,
                            int32_t static_bg, float* d_L, int64_t ldL, void* stream) {
  g_err.clear();
  if (!Mc || !d_video || !d_L) return fail(CDMD_E_INVALID_ARG, "NULL argument");
  cdmd_model* M = const_cast<cdmd_model*>(Mc);
  if (!M->selected) return fail(CDMD_E_STATE, "select background modes first");
  if (static_bg) {
    t0 = 0;
    t1 = 1;
    ldL = M->n;
  }
  if (t0 < 0 || t1 > M->m || t0 >= t1) return fail(CDMD_E_INVALID_ARG, "need 0 <= t0 < t1 <= m");
  if (ldL < M->n) return fail(CDMD_E_INVALID_ARG, "need ldL >= n");
  hipStream_t st = as_stream(stream);
  int NS = 0;
  TRY(prepare_recon(M, static_bg, &NS, st));
  M->mark(5, st);
  TRY(run_recon(M, d_video, static_bg, NS, 0.f, 2, d_L, t0, t1, ldL, st));
  M->mark(6, st);
  M->recon_pending = M->timing;
  return CDMD_OK;
}

cdmd_status cdmd_foreground(const cdmd_model* Mc, const void* d_video, float tau,
                            int32_t static_bg, int32_t bitpacked, void* d_mask,
                            int64_t* h_counts, void* stream) {
  g_err.clear();
  if (!Mc || !d_video || !d_mask) return fail(CDMD_E_INVALID_ARG, "NULL argument");
  cdmd_model* M = const_cast<cdmd_model*>(Mc);
  if (!M->selected) return fail(CDMD_E_STATE, "select background modes first");
  if (!(tau >= 0.f)) return fail(CDMD_E_INVALID_ARG, "tau must be >= 0");
  if (h_counts && !bitpacked) return fail(CDMD_E_INVALID_ARG, "counts need the bit-packed mask");
  hipStream_t st = as_stream(stream);
  int NS = 0;
  TRY(prepare_recon(M, static_bg, &NS, st));
  M->mark(5, st);
  TRY(run_recon(M, d_video, static_bg, NS, tau, bitpacked ? 0 : 1, d_mask, 0, M->m, 0, st));
  M->mark(6, st);
  M->recon_pending = M->timing;
  if (h_counts) {
    const int64_t words = (M->n + 31) / 32;
    HIPCHK(cdmd::k::mask_counts((const uint32_t*)d_mask, words, M->m, M->d_counts, st));
    HIPCHK(hipMemcpyAsync(M->h_counts, M->d_counts, sizeof(int64_t) * M->m, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::memcpy(h_counts, M->h_counts, sizeof(int64_t) * M->m);
  }
  return CDMD_OK;
}

cdmd_status cdmd_batch_foreground(cdmd_batch* B, const void* const* d_videos, float tau, int32_t static_bg,
                                  void* const* d_masks, void* stream) {
  g_err.clear();
  if (!B || !d_videos || !d_masks) return fail(CDMD_E_INVALID_ARG, "NULL argument");
  if (!(tau >= 0.f)) return fail(CDMD_E_INVALID_ARG, "tau must be >= 0");
  const int n = (int)B->models.size();
  for (int i = 0; i < n; ++i) {
    if (!d_videos[i] || !d_masks[i]) return fail(CDMD_E_INVALID_ARG, "NULL video or mask in the batch");
    if (!B->models[i]->selected) return fail(CDMD_E_STATE, "select background modes of every model first");
  }
  hipStream_t st = as_stream(stream);
  // the staging may be rewritten once the previous call's copy has completed, and the
  // device list once the previous call's kernels have read it
  if (B->rw_pending) {
    HIPCHK(hipEventSynchronize(B->rw_copied));
    HIPCHK(hipStreamWaitEvent(st, B->rw_read, 0));
    B->rw_pending = false;
  }
  const int64_t TP = cdmd::k::recon_tile_pixels();
  // lists: q = 4 c + 2 f + r with the LDS class c (0: the tile's frames take at most
  // 80 KiB, so that two workgroups share a CU, as the registers allow; 1: more), the
  // reconstruction form f (0: NSG 2 / NTV 3, 1: NSG 1 / NTV 2) and r (0: the full tiles,
  // 1: the partial tile); a launch's LDS is its largest entry's
  constexpr int NL = 8;
  std::vector<cdmd::k::ReconWork> lists[NL];
  size_t lds[NL] = {};
  for (int i = 0; i < n; ++i) {
    cdmd_model* M = B->models[i];
    int NS = 0;
    TRY(prepare_recon(M, static_bg, &NS, st));
    const int form = M->rc_nsg == 2 && M->rc_ntv == 3 ? 0 : M->rc_nsg == 1 && M->rc_ntv == 2 ? 1 : -1;
    if (!M->recon_mfma || form < 0) {  // the VALU form, one launch per model
      TRY(run_recon(M, d_videos[i], static_bg, NS, tau, 0, d_masks[i], 0, M->m, 0, st));
      continue;
    }
    cdmd::k::ReconWork w{};
    w.a.D = static_cast<const uint8_t*>(d_videos[i]);
    w.a.ld = M->ld;
    w.a.n = M->n;
    w.a.m = M->m;
    w.a.Gp = static_cast<const uint4*>(M->d_Gsp);
    w.a.Vp = static_cast<const uint4*>(M->d_Rv);
    w.a.KS = M->rc_ks;
    w.a.NFB = M->rc_nfb;
    w.a.ns = (int)M->S.size();
    w.a.tau = tau;
    w.a.xscale = M->xscale;
    w.a.mode = 0;
    w.a.out = d_masks[i];
    w.a.t0 = 0;
    w.a.t1 = M->m;
    w.a.ldL = 0;
    const size_t b = cdmd::k::recon_lds_bytes(M->m);
    const int q0 = 4 * (b > (size_t)80 * 1024 ? 1 : 0) + 2 * form;
    const int64_t full = M->n / TP;
    if (full > 0) {
      w.tile0 = 0;
      lists[q0].push_back(w);
      lds[q0] = std::max(lds[q0], b);
    }
    if (M->n % TP) {
      w.tile0 = full;
      lists[q0 + 1].push_back(w);
      lds[q0 + 1] = std::max(lds[q0 + 1], b);
    }
  }
  // launch c of list q: entries [c0, c0 + nw) with the launch's tile starts; all staged,
  // one copy, then the launches
  struct Launch {
    int q, nw;
    size_t off;
    int64_t total;
  };
  std::vector<Launch> launches;
  size_t off = 0;
  for (int q = 0; q < NL; ++q) {
    const size_t cnt = lists[q].size();
    for (size_t c0 = 0; c0 < cnt; c0 += 64) {
      const int nw = (int)std::min<size_t>(64, cnt - c0);
      int64_t start = 0;
      for (int e = 0; e < nw; ++e) {
        cdmd::k::ReconWork w = lists[q][c0 + e];
        w.start = start;
        start += (q & 1) ? 1 : w.a.n / TP;
        B->h_rwork[off + e] = w;
      }
      launches.push_back(Launch{q, nw, off, start});
      off += nw;
    }
  }
  if (off == 0) return CDMD_OK;
  HIPCHK(hipMemcpyAsync(B->d_rwork, B->h_rwork, sizeof(cdmd::k::ReconWork) * off, hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(B->rw_copied, st));
  for (const Launch& L : launches) {
    const int q = L.q, f = (q >> 1) & 1;
    HIPCHK(cdmd::k::recon_mfma_list(B->d_rwork + L.off, L.nw, L.total, lds[q], f == 0 ? 2 : 1, f == 0 ? 3 : 2, 0,
                                    (q & 1) != 0, st));
  }
  HIPCHK(hipEventRecord(B->rw_read, st));
  B->rw_pending = true;
  return CDMD_OK;
}

// ------------------------------------------------------------------ learned selector
static cdmd_status upload_mode_features(const cdmd_model* M, hipStream_t st) {
  const int k = M->k;
  std::vector<double> h((size_t)5 * k);
  for (int j = 0; j < k; ++j) {
    h[2 * j] = M->lam[j].real();
    h[2 * j + 1] = M->lam[j].imag();
    h[2 * k + 2 * j] = M->b[j].real();
    h[2 * k + 2 * j + 1] = M->b[j].imag();
    h[4 * k + j] = M->phinorm[j];
  }
  HIPCHK(hipMemcpyAsync(M->d_modes, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, st));
  HIPCHK(cdmd::k::mode_features(M->d_modes, M->d_modes + 2 * k, M->d_modes + 4 * k, M->x1n2, M->m, k,
                                M->d_feats, st));
  // the host vector must outlive the copy
  HIPCHK(hipStreamSynchronize(st));
  return CDMD_OK;
}

cdmd_status cdmd_mode_features(const cdmd_model* M, float* d_feats, void* stream) {
  g_err.clear();
  if (!M || !d_feats) return fail(CDMD_E_INVALID_ARG, "NULL argument");
  if (!M->fitted) return fail(CDMD_E_STATE, "model is not fitted");
  hipStream_t st = as_stream(stream);
  TRY(upload_mode_features(M, st));
  HIPCHK(hipMemcpyAsync(d_feats, M->d_feats, sizeof(float) * 6 * M->k, hipMemcpyDeviceToDevice, st));
  return CDMD_OK;
}

namespace {
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};
}  // namespace

cdmd_status cdmd_mlp_grad(const float* d_params, const float* d_X, const float* d_y, int32_t n,
                          float* d_grad, float* d_loss, void* stream) {
  g_err.clear();
  if (!d_params || !d_X || !d_y || n < 1) return fail(CDMD_E_INVALID_ARG, "bad arguments");
  hipStream_t st = as_stream(stream);
  const int np = cdmd::k::mlp_nparts(n);
  DevBuf part, lpart;
  HIPCHK(hipMalloc(&part.p, sizeof(float) * (size_t)np * CDMD_MLP_NPARAM));
  HIPCHK(hipMalloc(&lpart.p, sizeof(float) * (size_t)np));
  HIPCHK(cdmd::k::mlp_grad(d_params, d_X, d_y, nullptr, n, (float*)part.p, (float*)lpart.p, d_grad, d_loss, st));
  HIPCHK(hipStreamSynchronize(st));
  return CDMD_OK;
}

cdmd_status cdmd_mlp_train(float* d_params, float* d_adam_m, float* d_adam_v, const float* d_X,
                           const float* d_y, int64_t n_samples, const int32_t* d_batch_idx,
                           int32_t batch, int32_t steps, float lr, int64_t step0, float* d_losses,
                           void* stream) {
  g_err.clear();
  if (!d_params || !d_adam_m || !d_adam_v || !d_X || !d_y || !d_batch_idx || batch < 1 || steps < 0 ||
      step0 < 0 || n_samples < 1 || !(lr > 0.0f))
    return fail(CDMD_E_INVALID_ARG, "bad arguments");
  hipStream_t st = as_stream(stream);
  const int np = cdmd::k::mlp_nparts(batch);
  DevBuf part, lpart;
  HIPCHK(hipMalloc(&part.p, sizeof(float) * (size_t)np * CDMD_MLP_NPARAM));
  HIPCHK(hipMalloc(&lpart.p, sizeof(float) * (size_t)np));
  HIPCHK(cdmd::k::mlp_train(d_params, d_adam_m, d_adam_v, d_X, d_y, n_samples, d_batch_idx, batch, steps, lr, step0,
                            (float*)part.p, (float*)lpart.p, d_losses, st));
  HIPCHK(hipStreamSynchronize(st));
  return CDMD_OK;
}

cdmd_status cdmd_mlp_train_noalloc(float* d_params, float* d_adam_m, float* d_adam_v, const float* d_X,
                                   const float* d_y, int64_t n_samples, const int32_t* d_batch_idx,
                                   int32_t batch, int32_t steps, float lr, int64_t step0, float* d_losses,
                                   void* stream) {
  g_err.clear();
  if (!d_params || !d_adam_m || !d_adam_v || !d_X || !d_y || !d_batch_idx || batch < 1 || steps < 0 ||
      step0 < 0 || n_samples < 1 || !(lr > 0.0f))
    return fail(CDMD_E_INVALID_ARG, "bad arguments");
  if (batch > CDMD_MLP_NOALLOC_MAX_BATCH)
    return fail(CDMD_E_INVALID_ARG, "batch above CDMD_MLP_NOALLOC_MAX_BATCH (the static scratch holds no more)");
  HIPCHK(cdmd::k::mlp_train_noalloc(d_params, d_adam_m, d_adam_v, d_X, d_y, n_samples, d_batch_idx, batch, steps,
                                    lr, step0, d_losses, as_stream(stream)));
  return CDMD_OK;
}

cdmd_status cdmd_mlp_forward(const float* d_params, const float* d_X, int32_t n, int32_t bf16,
                             float* d_logits, void* stream) {
  g_err.clear();
  if (!d_params || !d_X || !d_logits || n < 0) return fail(CDMD_E_INVALID_ARG, "bad arguments");
  HIPCHK(cdmd::k::mlp_forward(d_params, d_X, n, bf16 != 0, d_logits, as_stream(stream)));
  return CDMD_OK;
}

cdmd_status cdmd_select_learned(cdmd_model* M, const float* d_params, double confidence,
                                int32_t K_fallback, int32_t* out_idx, int32_t* out_n,
                                double* out_beta, double* prob, int32_t* used_fallback,
                                void* stream) {
  g_err.clear();
  if (!M || !d_params) return fail(CDMD_E_INVALID_ARG, "NULL argument");
  if (!M->fitted) return fail(CDMD_E_STATE, "model is not fitted");
  if (!(confidence >= 0.5 && confidence <= 1.0)) return fail(CDMD_E_INVALID_ARG, "confidence must be in [0.5, 1]");
  if (K_fallback < 1) return fail(CDMD_E_INVALID_ARG, "K_fallback must be >= 1");
  hipStream_t st = as_stream(stream);
  const int k = M->k;
  TRY(upload_mode_features(M, st));
  HIPCHK(cdmd::k::mlp_forward(d_params, M->d_feats, k, 1, M->d_logits, st));
  std::vector<float> z(k);
  HIPCHK(hipMemcpyAsync(z.data(), M->d_logits, sizeof(float) * k, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<int32_t> S;
  bool confident = true;
  for (int j = 0; j < k; ++j) {
    const double pj = 1.0 / (1.0 + std::exp(-(double)z[j]));
    if (prob) prob[j] = pj;
    if (std::max(pj, 1.0 - pj) < confidence) confident = false;
    if (pj >= 0.5) S.push_back(j);
  }
  const bool fb = !confident || S.empty();
  if (used_fallback) *used_fallback = fb ? 1 : 0;
  if (fb) return cdmd_select(M, CDMD_SEL_OMP, K_fallback, 0.0, nullptr, 0, out_idx, out_n, out_beta);
  return cdmd_select(M, CDMD_SEL_EXPLICIT, 0, 0.0, S.data(), (int32_t)S.size(), out_idx, out_n, out_beta);
}

cdmd_status cdmd_get_sketch(const cdmd_model* Mc, double* h_Y, int64_t* h_int) {
  g_err.clear();
  if (!Mc) return fail(CDMD_E_INVALID_ARG, "NULL model");
  const cdmd_model* M = Mc;
  if (!M->fitted) return fail(CDMD_E_STATE, "model is not fitted");
  const size_t cnt = (size_t)M->m * M->p * (M->srft ? 2 : 1);
  if (M->cfg.dtype == CDMD_U8 && !M->gauss && !M->srft) {
    std::vector<int32_t> tmp(cnt);
    HIPCHK(hipMemcpy(tmp.data(), M->d_Yint, cnt * 4, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < cnt; ++i) {
      if (h_Y) h_Y[i] = tmp[i] * M->sketch_scale;
      if (h_int) h_int[i] = tmp[i];
    }
  } else {
    if (h_int) return fail(CDMD_E_INVALID_ARG, "integer sums exist only for sparse sketches of uint8 videos");
    std::vector<double> tmp(cnt);
    HIPCHK(hipMemcpy(tmp.data(), M->d_Yd, cnt * 8, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < cnt; ++i)
      if (h_Y) h_Y[i] = tmp[i] * M->sketch_scale;
  }
  return CDMD_OK;
}

cdmd_status cdmd_info_get(const cdmd_model* Mc, cdmd_info* info) {
  g_err.clear();
  if (!Mc || !info) return fail(CDMD_E_INVALID_ARG, "NULL argument");
  cdmd_model* M = const_cast<cdmd_model*>(Mc);
  if (M->recon_pending) {
    HIPCHK(hipEventSynchronize(M->ev[6]));
    M->info.gpu_ms_recon = M->span(5, 6);
    M->recon_pending = false;
  }
  *info = M->info;
  return CDMD_OK;
}

// ------------------------------------------------------------------ long videos
// Section 4 processes a long video as consecutive batches of frames, each decomposed on its
// own.  Workers (host threads, each with its own stream and models) take the batches in
// turn, so the latency-bound small linear algebra of one batch runs beside the streaming
// kernels of another.  The executor keeps its streams, models (per batch length and rank)
// and mask buffers from one video to the next, so only the first video pays for them.
namespace {
struct VideoBatch {
  int64_t t0, m;
};

std::vector<VideoBatch> video_batches(int64_t frames, int64_t F) {
  std::vector<VideoBatch> b;
  for (int64_t t = 0; t < frames; t += F) b.push_back({t, std::min(F, frames - t)});
  if (b.size() > 1 && b.back().m < 2) {  // a single trailing frame joins the batch before it
    b[b.size() - 2].m += b.back().m;
    b.pop_back();
  }
  return b;
}

struct VideoWorker {
  hipStream_t st = nullptr;
  std::map<std::pair<int64_t, int>, std::unique_ptr<cdmd_model>> models;  // (frames, rank)
  std::map<int64_t, std::unique_ptr<cdmd_model>> rank_models;             // frames -> rank-1 model
  void* d_raw = nullptr;       // unfiltered mask of a batch (median filter only)
  size_t raw_bytes = 0;
  cdmd_status status = CDMD_OK;
  std::string err;
  ~VideoWorker() {
    if (st) (void)hipStreamSynchronize(st);  // a failed batch may have left work in flight
    models.clear();
    rank_models.clear();
    if (d_raw) (void)hipFree(d_raw);
    if (st) (void)hipStreamDestroy(st);
  }
};
}  // namespace

struct cdmd_video {
  cdmd_config base{};
  cdmd_video_plan plan{};
  std::vector<int32_t> idx;  // host copies of the sparse C (the caller's arrays may go)
  std::vector<int8_t> sign;
  int dev = 0;
  bool median = false;
  hipEvent_t ready = nullptr;
  std::vector<VideoWorker> wk;
  ~cdmd_video() {
    wk.clear();
    if (ready) (void)hipEventDestroy(ready);
  }
};

cdmd_status cdmd_video_create(const cdmd_config* base, const cdmd_video_plan* plan, cdmd_video** out) {
  g_err.clear();
  if (!base || !plan || !out) return fail(CDMD_E_INVALID_ARG, "NULL argument");
  *out = nullptr;
  const cdmd_video_plan vp = *plan;
  if (vp.batch_frames < 2) return fail(CDMD_E_INVALID_ARG, "need at least 2 frames per batch");
  if (vp.workers < 1 || vp.workers > 4) return fail(CDMD_E_INVALID_ARG, "workers must be 1..4");
  if (vp.K < 1 || vp.k < 0) return fail(CDMD_E_INVALID_ARG, "need K >= 1 and k >= 0");
  if (!(vp.tau >= 0.0)) return fail(CDMD_E_INVALID_ARG, "tau must be >= 0");
  const bool median = vp.H > 0 || vp.W > 0;
  if (median && (vp.H < 1 || vp.W < 1 || vp.H * vp.W != base->n))
    return fail(CDMD_E_INVALID_ARG, "the median filter needs H * W == n");
  if (base->p < 1 || base->nnz < 1) return fail(CDMD_E_INVALID_ARG, "need p >= 1 and nnz >= 1");
  std::unique_ptr<cdmd_video> V(new cdmd_video);
  V->base = *base;
  V->plan = vp;
  V->median = median;
  const size_t tab = (size_t)base->p * (size_t)base->nnz;
  if (base->sparse_idx) {
    V->idx.assign(base->sparse_idx, base->sparse_idx + tab);
    V->base.sparse_idx = V->idx.data();
  }
  if (base->sparse_sign) {
    V->sign.assign(base->sparse_sign, base->sparse_sign + tab);
    V->base.sparse_sign = V->sign.data();
  }
  HIPCHK(hipGetDevice(&V->dev));
  HIPCHK(hipEventCreateWithFlags(&V->ready, hipEventDisableTiming));
  V->wk = std::vector<VideoWorker>(vp.workers);
  for (auto& w : V->wk) HIPCHK(hipStreamCreateWithFlags(&w.st, hipStreamNonBlocking));
  *out = V.release();
  return CDMD_OK;
}

void cdmd_video_free(cdmd_video* V) { delete V; }

cdmd_status cdmd_video_run(cdmd_video* V, const void* d_video, int64_t frames, void* d_mask, int32_t* k_used,
                           void* stream) {
  g_err.clear();
  if (!V || !d_video || !d_mask) return fail(CDMD_E_INVALID_ARG, "NULL argument");
  if (frames < 2) return fail(CDMD_E_INVALID_ARG, "need at least 2 frames");
  const cdmd_config* base = &V->base;
  const cdmd_video_plan& vp = V->plan;
  const bool median = V->median;
  const std::vector<VideoBatch> batches = video_batches(frames, vp.batch_frames);
  const int64_t words = (base->n + 31) / 32;
  const size_t elem = base->dtype == CDMD_U8 ? 1 : 4;
  const int nw = std::min<int>((int)V->wk.size(), (int)batches.size());
  // the executor's device for this call; the caller's current device is restored on return
  int caller_dev = 0;
  HIPCHK(hipGetDevice(&caller_dev));
  HIPCHK(hipSetDevice(V->dev));
  struct Restore {
    int d;
    ~Restore() { (void)hipSetDevice(d); }
  } restore{caller_dev};
  HIPCHK(hipEventRecord(V->ready, as_stream(stream)));  // the video is ready on the caller's stream
  for (int i = 0; i < nw; ++i) {
    VideoWorker& w = V->wk[i];
    w.status = CDMD_OK;
    w.err.clear();
    HIPCHK(hipStreamWaitEvent(w.st, V->ready, 0));
  }
  const int dev = V->dev;
  auto run = [&](int wi) {
    VideoWorker& w = V->wk[wi];
    if (hipSetDevice(dev) != hipSuccess) {
      w.status = CDMD_E_DEVICE;
      w.err = "hipSetDevice failed in a worker";
      return;
    }
    auto failw = [&](cdmd_status st) {
      w.status = st;
      w.err = g_err;
    };
    for (size_t bi = wi; bi < batches.size(); bi += nw) {
      const VideoBatch& b = batches[bi];
      const uint8_t* vid = static_cast<const uint8_t*>(d_video) + (size_t)b.t0 * base->ld * elem;
      cdmd_config c = *base;
      c.m = b.m;
      int32_t k = vp.k;
      if (k == 0) {
        auto& rm = w.rank_models[b.m];
        if (!rm) {
          cdmd_config c1 = c;
          c1.k = 1;
          cdmd_model* M1 = nullptr;
          const cdmd_status st = cdmd_create(&c1, &M1);
          if (st != CDMD_OK) return failw(st);
          rm.reset(M1);
        }
        const cdmd_status st = rank_with_model(rm.get(), vid, w.st, &k, nullptr, nullptr);
        if (st != CDMD_OK) return failw(st);
        // at least 1; at most what the fit accepts
        k = std::max(1, std::min<int32_t>(k, (int32_t)std::min<int64_t>(std::min<int64_t>(b.m - 1, c.p), kMaxRank)));
      }
      if (k_used) k_used[bi] = k;
      c.k = k;
      auto& mp = w.models[{b.m, k}];
      if (!mp) {
        cdmd_model* M = nullptr;
        const cdmd_status st = cdmd_create(&c, &M);
        if (st != CDMD_OK) return failw(st);
        mp.reset(M);
      }
      cdmd_model* M = mp.get();
      cdmd_status st = cdmd_fit(M, vid, w.st);
      if (st != CDMD_OK) return failw(st);
      int32_t ns = 0;
      st = cdmd_select(M, CDMD_SEL_OMP, vp.K, 0.0, nullptr, 0, nullptr, &ns, nullptr);
      if (st != CDMD_OK) return failw(st);
      void* out = static_cast<uint8_t*>(d_mask) + (size_t)b.t0 * words * 4;
      void* raw = out;
      if (median) {
        const size_t need = (size_t)b.m * words * 4;
        if (w.raw_bytes < need) {
          // the previous video's kernels on this stream may still read the old buffer
          if (w.d_raw && hipStreamSynchronize(w.st) != hipSuccess) {
            w.status = CDMD_E_DEVICE;
            w.err = "a worker stream failed";
            return;
          }
          if (w.d_raw) (void)hipFree(w.d_raw);
          w.d_raw = nullptr;
          w.raw_bytes = 0;
          if (hipMalloc(&w.d_raw, need) != hipSuccess) {
            (void)hipGetLastError();
            w.status = CDMD_E_OUT_OF_MEMORY;
            w.err = "no device memory for a batch's unfiltered mask";
            return;
          }
          w.raw_bytes = need;
        }
        raw = w.d_raw;
      }
      st = cdmd_foreground(M, vid, (float)vp.tau, 0, 1, raw, nullptr, w.st);
      if (st != CDMD_OK) return failw(st);
      if (median) {
        st = cdmd_mask_median3(raw, out, vp.H, vp.W, b.m, 1, w.st);
        if (st != CDMD_OK) return failw(st);
      }
    }
    if (hipStreamSynchronize(w.st) != hipSuccess) {
      w.status = CDMD_E_DEVICE;
      w.err = "a worker stream failed";
    }
  };
  if (nw == 1) {
    run(0);
  } else {
    std::vector<std::thread> th;
    for (int i = 0; i < nw; ++i) th.emplace_back(run, i);
    for (auto& t : th) t.join();
  }
  for (int i = 0; i < nw; ++i)
    if (V->wk[i].status != CDMD_OK) return fail(V->wk[i].status, ("a batch failed: " + V->wk[i].err).c_str());
  return CDMD_OK;
}

cdmd_status cdmd_process_video(const cdmd_config* base, const cdmd_video_plan* plan, const void* d_video,
                               int64_t frames, void* d_mask, int32_t* k_used, void* stream) {
  g_err.clear();
  if (!base || !plan || !d_video || !d_mask) return fail(CDMD_E_INVALID_ARG, "NULL argument");
  if (frames < 2) return fail(CDMD_E_INVALID_ARG, "need at least 2 frames per batch");
  cdmd_video* V = nullptr;
  cdmd_status st = cdmd_video_create(base, plan, &V);
  if (st != CDMD_OK) return st;
  std::unique_ptr<cdmd_video> own(V);
  return cdmd_video_run(V, d_video, frames, d_mask, k_used, stream);
}

cdmd_status cdmd_mask_median3(const void* d_in, void* d_out, int64_t H, int64_t W, int64_t m, int32_t bitpacked,
                              void* stream) {
  g_err.clear();
  if (!d_in || !d_out) return fail(CDMD_E_INVALID_ARG, "NULL mask");
  if (H < 1 || W < 1 || m < 1 || m > 65535) return fail(CDMD_E_INVALID_ARG, "need H, W >= 1 and 1 <= m <= 65535");
  if (H * W >= ((int64_t)1 << 31)) return fail(CDMD_E_UNSUPPORTED, "frames of 2^31 pixels or more are not built");
  const int64_t n = H * W;
  const int64_t bytes = m * (bitpacked ? 4 * ((n + 31) / 32) : n);
  const char* a = static_cast<const char*>(d_in);
  const char* b = static_cast<const char*>(d_out);
  if (a < b + bytes && b < a + bytes) return fail(CDMD_E_INVALID_ARG, "input and output masks overlap");
  HIPCHK(cdmd::k::mask_median3(d_in, d_out, H, W, m, bitpacked ? 1 : 0, as_stream(stream)));
  return CDMD_OK;
}

cdmd_status cdmd_store_measurement(cdmd_model* M, int32_t on, void* stream) {
  g_err.clear();
  if (!M) return fail(CDMD_E_INVALID_ARG, "NULL model");
  const int prec = gauss_prec(M->cfg);
  if (!M->gauss || (prec != 1 && prec != 2))
    return fail(CDMD_E_UNSUPPORTED, "C is stored for the BF16 and FP8 forms of the Gaussian sketch only");
  hipStream_t st = as_stream(stream);
  auto release = [&]() -> cdmd_status {
    HIPCHK(hipStreamSynchronize(st));
    if (M->sgemm) cdmd::blas::sketch_gemm_free(M->sgemm);
    M->sgemm = nullptr;
    if (M->d_Xs) HIPCHK(hipFree(M->d_Xs));
    M->d_Xs = nullptr;
    if (M->d_Cm) HIPCHK(hipFree(M->d_Cm));
    M->d_Cm = nullptr;
    M->gm_S = 0;
    M->gm_Ks = 0;
    ++M->stamp;
    return CDMD_OK;
  };
  if (!on) return M->d_Cm ? release() : CDMD_OK;
  if (M->d_Cm) return CDMD_OK;
  auto grab = [&](void** d, size_t bytes) -> bool {
    if (hipMalloc(d, bytes) == hipSuccess) return true;
    (void)hipGetLastError();
    *d = nullptr;
    return false;
  };
  {
    // C pixel-major for the library GEMM, the video converted into S slices of Ks pixels per
    // fit (S up to 32 so that the products fill the device): 2 bytes per element for BF16,
    // for FP8 one byte of C and the two e4m3 parts of each video byte
    const int S = (int)std::min<int64_t>(32, std::max<int64_t>(1, (M->n + 262143) / 262144));
    const int64_t Ks = ((M->n + S - 1) / S + 63) / 64 * 64;
    const int64_t jn = S * Ks;
    const size_t need_part = (size_t)S * M->m * M->p;
    if (need_part > M->gpart_cap) {
      float* np = nullptr;
      if (!grab((void**)&np, need_part * sizeof(float))) return fail(CDMD_E_OUT_OF_MEMORY, "no device memory for the GEMM partials");
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(hipFree(M->d_gpart));
      M->d_gpart = np;
      M->gpart_cap = need_part;
    }
    if (!grab(&M->d_Cm, (size_t)jn * M->p * (prec == 1 ? 2 : 1)) || !grab(&M->d_Xs, (size_t)jn * M->m * 2)) {
      (void)release();
      return fail(CDMD_E_OUT_OF_MEMORY, "no device memory for the stored C and the converted video");
    }
    M->gm_S = S;
    M->gm_Ks = Ks;
    const hipError_t e = prec == 1 ? cdmd::k::gauss_fill_t(M->d_Cm, jn, M->n, M->p, M->cfg.seed, st)
                                   : cdmd::k::gauss_fill_fp8_t(M->d_Cm, jn, M->n, M->p, M->cfg.seed, st);
    if (e != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
      (void)release();
      return fail(CDMD_E_DEVICE, "filling the stored C failed");
    }
    std::string err;
    M->sgemm = cdmd::blas::sketch_gemm_create(M->p, Ks, M->m, S, prec == 1 ? 0 : 1, &err);
    if (M->sgemm) {
      M->Cm_ldc = 0;
      ++M->stamp;
      return CDMD_OK;
    }
    (void)release();
    if (prec == 1) return fail(CDMD_E_UNSUPPORTED, err.c_str());
    // FP8 without a library GEMM for the shape: the sketch kernel streams a row-major copy
  }
  const int64_t ldc = cdmd::k::gauss_ldc(M->n);
  const size_t bytes = (size_t)M->p * (size_t)ldc;
  void* d = nullptr;
  if (!grab(&d, bytes)) return fail(CDMD_E_OUT_OF_MEMORY, "no device memory for the stored C");
  const hipError_t e = cdmd::k::gauss_fill(d, ldc, M->n, M->p, M->cfg.seed, prec, st);
  if (e == hipSuccess && hipStreamSynchronize(st) == hipSuccess) {
    M->d_Cm = d;
    M->Cm_ldc = ldc;
    ++M->stamp;
    return CDMD_OK;
  }
  (void)hipFree(d);
  return fail(CDMD_E_DEVICE, "filling the stored C failed");
}

cdmd_status cdmd_set_amplitudes(cdmd_model* M, int32_t space) {
  g_err.clear();
  if (!M) return fail(CDMD_E_INVALID_ARG, "NULL model");
  if (space != CDMD_AMP_FULL && space != CDMD_AMP_COMPRESSED) return fail(CDMD_E_INVALID_ARG, "unknown amplitude space");
  if (space == CDMD_AMP_COMPRESSED) {
    if (!M->device_la_ok)
      return fail(CDMD_E_UNSUPPORTED, "amplitudes on the compressed modes need the device small linear algebra");
    const int ne = M->k * M->k + M->k + 1;
    if (!M->d_py) {
      TRY(dalloc(&M->d_py, (size_t)cdmd::k::small_la_py_blocks((int)M->m) * ne));
      TRY(dalloc(&M->d_pyred, (size_t)ne));
      TRY(halloc(&M->h_py, (size_t)ne));
    }
  }
  M->amp_compressed = space == CDMD_AMP_COMPRESSED;
  ++M->stamp;
  M->fitted = M->selected = false;
  M->info.fitted = M->info.selected = 0;
  return CDMD_OK;
}

cdmd_status cdmd_set_timing(cdmd_model* M, int32_t enable) {
  g_err.clear();
  if (!M) return fail(CDMD_E_INVALID_ARG, "NULL model");
  if (enable && !M->ev[0]) {
    for (hipEvent_t& e : M->ev) HIPCHK(hipEventCreate(&e));
  }
  M->timing = enable != 0;
  M->info.timing = M->timing ? 1 : 0;
  return CDMD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// host-only test entry points (include/cdmd_debug.h)
#include "cdmd_debug.h"

extern "C" {

cdmd_status cdmd_dbg_team_small_la(const double* Gr, int32_t m, int32_t k, double rtol,
                                   double sketch_scale, int32_t groups, double* mu, double* sigma,
                                   double* lam, double* W, double* G, int32_t* steps) {
  g_err.clear();
  if (!Gr || !mu || !sigma || !lam || !W || !G || m < 2 || k < 1 || k > m - 1 || groups < 1 ||
      groups > 32)
    return fail(CDMD_E_INVALID_ARG, "bad arguments");
  int J = 0;
  const int st = cdmd::team_small_la_host(Gr, m, k, rtol, std::min(m - 1, 320), sketch_scale, groups, mu,
                                          sigma, lam, W, G, &J);
  if (steps) *steps = J;
  if (st != 0) return fail((cdmd_status)st, "team small LA failed");
  return CDMD_OK;
}

cdmd_status cdmd_dbg_la_phases(const cdmd_model* M, double* ms16) {
  g_err.clear();
  if (!M || !ms16) return fail(CDMD_E_INVALID_ARG, "NULL argument");
  for (int i = 0; i < 16; ++i) ms16[i] = M->la_phase_ms[i];
  return CDMD_OK;
}

cdmd_status cdmd_dbg_force_gather_sketch(cdmd_model* M, int32_t on) {
  g_err.clear();
  if (!M) return fail(CDMD_E_INVALID_ARG, "NULL model");
  M->force_gather_sketch = on != 0;
  ++M->stamp;
  return CDMD_OK;
}

cdmd_status cdmd_dbg_sparse_form(cdmd_model* M, int32_t form) {
  g_err.clear();
  if (!M) return fail(CDMD_E_INVALID_ARG, "NULL model");
  if (M->gauss || M->srft || M->cfg.dtype != CDMD_U8)
    return fail(CDMD_E_UNSUPPORTED, "the form applies to uint8 sparse sketches");
  if (form != -1) {
    const int F = form / 10, V = form % 10;
    if (form < 11 || !cdmd::k::sketch_stream_fits(F, V, M->max_rows))
      return fail(CDMD_E_INVALID_ARG, "unknown or unfitting streaming form");
    if (stream_nrange(M, F, V) > M->sk_slots_cap) return fail(CDMD_E_INVALID_ARG, "form needs more partial slots");
  }
  TRY(apply_sparse_form(M, form));
  M->info.sparse_form = form < 0 ? -1 : 10 * M->sk_F + M->sk_V;
  ++M->stamp;
  return CDMD_OK;
}

cdmd_status cdmd_dbg_force_host_la(cdmd_model* M, int32_t on) {
  g_err.clear();
  if (!M) return fail(CDMD_E_INVALID_ARG, "NULL model");
  M->force_host_la = on != 0;
  ++M->stamp;
  return CDMD_OK;
}

cdmd_status cdmd_dbg_la_groups(cdmd_model* M, int32_t groups) {
  g_err.clear();
  if (!M || groups < 0 || groups > 32) return fail(CDMD_E_INVALID_ARG, "groups must be in [0, 32]");
  M->la_groups = groups;
  ++M->stamp;
  return CDMD_OK;
}

cdmd_status cdmd_dbg_force_valu_lift(cdmd_model* M, int32_t on) {
  g_err.clear();
  if (!M) return fail(CDMD_E_INVALID_ARG, "NULL model");
  M->force_valu_lift = on != 0;
  ++M->stamp;
  return CDMD_OK;
}

cdmd_status cdmd_dbg_sym_topk(const double* M, int32_t n, int32_t k, double rtol, double* evals,
                              double* evecs, int32_t* steps) {
  g_err.clear();
  if (!M || !evals || !evecs || n < 1 || k < 1 || k > n) return fail(CDMD_E_INVALID_ARG, "bad arguments");
  const int J = cdmd::la::sym_topk(M, n, k, rtol, evals, evecs);
  if (J < 0) return fail(CDMD_E_NUMERIC, "symmetric eigensolver failed");
  if (steps) *steps = J;
  return CDMD_OK;
}

cdmd_status cdmd_dbg_eig_general(const double* A, int32_t k, double* lam, double* W) {
  g_err.clear();
  if (!A || !lam || !W || k < 1) return fail(CDMD_E_INVALID_ARG, "bad arguments");
  if (!cdmd::la::eig_general(A, k, reinterpret_cast<cplx*>(lam), reinterpret_cast<cplx*>(W)))
    return fail(CDMD_E_NUMERIC, "eigensolver failed");
  return CDMD_OK;
}

cdmd_status cdmd_dbg_herm_topk(const double* M, int32_t n, int32_t k, double rtol, double* evals,
                               double* evecs, int32_t* steps) {
  g_err.clear();
  if (!M || !evals || !evecs || n < 1 || k < 1 || k > n) return fail(CDMD_E_INVALID_ARG, "bad arguments");
  const int J = cdmd::la::herm_topk(reinterpret_cast<const cplx*>(M), n, k, rtol, evals,
                                    reinterpret_cast<cplx*>(evecs));
  if (J < 0) return fail(CDMD_E_NUMERIC, "Hermitian eigensolver failed");
  if (steps) *steps = J;
  return CDMD_OK;
}

cdmd_status cdmd_dbg_eig_complex(const double* A, int32_t k, double* lam, double* W) {
  g_err.clear();
  if (!A || !lam || !W || k < 1) return fail(CDMD_E_INVALID_ARG, "bad arguments");
  if (!cdmd::la::eig_complex(reinterpret_cast<const cplx*>(A), k, reinterpret_cast<cplx*>(lam),
                             reinterpret_cast<cplx*>(W)))
    return fail(CDMD_E_NUMERIC, "eigensolver failed");
  return CDMD_OK;
}

cdmd_status cdmd_dbg_sym_eigvals(const double* A, int32_t n, double* ev) {
  g_err.clear();
  if (!A || !ev || n < 1) return fail(CDMD_E_INVALID_ARG, "bad arguments");
  std::vector<double> v;
  if (!cdmd::la::sym_eigvals(A, n, n, v)) return fail(CDMD_E_NUMERIC, "non-finite input");
  std::memcpy(ev, v.data(), sizeof(double) * n);
  return CDMD_OK;
}

cdmd_status cdmd_dbg_rank_threshold(const double* A, int32_t n, int32_t r, double scale, double omega, int32_t* k,
                                    double* tau) {
  g_err.clear();
  if (!A || !k || !tau || n < 1 || r < 1 || r > n || !(scale > 0.0)) return fail(CDMD_E_INVALID_ARG, "bad arguments");
  int kk = 0;
  if (!cdmd::la::sym_rank_threshold(A, n, n, r, scale, omega, &kk, tau)) return fail(CDMD_E_NUMERIC, "non-finite input");
  *k = kk;
  return CDMD_OK;
}

cdmd_status cdmd_dbg_gd_threshold(double beta, double* lambda_star, double* mp_median, double* omega) {
  g_err.clear();
  if (!(beta > 0.0 && beta <= 1.0)) return fail(CDMD_E_INVALID_ARG, "beta must be in (0, 1]");
  if (lambda_star) *lambda_star = cdmd::la::gd_lambda_star(beta);
  if (mp_median) *mp_median = cdmd::la::mp_median(beta);
  if (omega) *omega = cdmd::la::gd_omega(beta);
  return CDMD_OK;
}

cdmd_status cdmd_dbg_omp_gram(const double* H, int32_t k, const double* c, double x1n2, int32_t K,
                              const double* lam, int32_t* S, double* beta, int32_t* ns, double* resid2) {
  g_err.clear();
  if (!H || !c || !S || !beta || !ns || k < 1 || K < 1) return fail(CDMD_E_INVALID_ARG, "bad arguments");
  std::vector<int> sv;
  std::vector<cplx> bv;
  double r2 = 0.0;
  if (!cdmd::la::omp_gram(reinterpret_cast<const cplx*>(H), k, reinterpret_cast<const cplx*>(c), x1n2, K,
                          reinterpret_cast<const cplx*>(lam), kOmpStopRel, sv, bv, &r2))
    return fail(CDMD_E_NUMERIC, "OMP subsystem singular");
  *ns = (int32_t)sv.size();
  for (size_t q = 0; q < sv.size(); ++q) {
    S[q] = sv[q];
    beta[2 * q] = bv[q].real();
    beta[2 * q + 1] = bv[q].imag();
  }
  if (resid2) *resid2 = r2;
  return CDMD_OK;
}

}  // extern "C"
