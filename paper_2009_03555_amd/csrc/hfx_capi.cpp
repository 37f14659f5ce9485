// C ABI of the exchange builder: validation, host plan (normalisation,
// pattern, shell-pair and primitive-pair tables, block lookup, Boys table),
// device upload, and the build sequence (density -> screen -> ERI -> K).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/hfx.h"
#include "coop.hpp"
#include "launchers.hpp"

using namespace hfx;

namespace {

thread_local std::string g_err;

hfx_status fail(hfx_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(expr)                                                                                   \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess)                                                                              \
      return fail(e_ == hipErrorOutOfMemory ? HFX_ERR_OOM : HFX_ERR_DEVICE,                            \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                                 \
  } while (0)

constexpr uint32_t kMagic = 0x48465850u;  // "HFXP"
constexpr double kPrimDrop = 1e-20;      // primitive-pair bound below which the ERI path skips it
// quartets a list holds at once unless hfx_set_list_limit says otherwise
// (64 GiB of list, under a quarter of the device's 288 GB); longer lists
// are evaluated in chunks
constexpr int64_t kDefaultMaxList = (int64_t)1 << 33;

bool lexpos(int a, int b, int c) { return a > 0 || (a == 0 && (b > 0 || (b == 0 && c >= 0))); }

double dfact(int n) {
  double r = 1.0;
  for (int k = n; k > 1; k -= 2) r *= k;
  return r;
}

int nfunc_host(int l, int sph) { return (l == 2 && sph) ? 5 : (l + 1) * (l + 2) / 2; }

// Boys table: F_m(T_i) by the everywhere-convergent series
// F_m(T) = e^-T sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)) at the top order,
// downward recursion below it, all in long double.
std::vector<double> boys_table() {
  std::vector<double> t((size_t)kBoysRows * kBoysCols);
  const int mtop = kBoysCols - 2;  // 15
  for (int i = 0; i < kBoysRows; ++i) {
    long double T = (long double)i * (long double)kBoysStep;
    long double et = expl(-T);
    long double term = 1.0L / (2 * mtop + 1), sum = term;
    for (int k = 1; k < 100000; ++k) {
      term *= 2.0L * T / (2 * mtop + 2 * k + 1);
      sum += term;
      if (term < sum * 1e-22L) break;
    }
    long double F[kBoysCols];
    F[mtop] = et * sum;
    for (int m = mtop - 1; m >= 0; --m) F[m] = (2.0L * T * F[m + 1] + et) / (2 * m + 1);
    for (int m = 0; m <= mtop; ++m) t[(size_t)i * kBoysCols + m] = (double)F[m];
    t[(size_t)i * kBoysCols + kBoysCols - 1] = (double)et;
  }
  return t;
}

// One Boys table per device, shared by every plan on it: a file-scope
// device array, filled once per device (with the device current) and
// reached through the address hipGetSymbolAddress gives for that device.
// Plans with their own copies made a fused build of many plans slower than
// the plans' separate builds (512 clusters: 56.8 s against 48.3 s; 47.0 s
// with the shared table): waves of different plans on a compute unit evicted
// each other's table rows from its L1.
constexpr int kMaxBoysDevices = 64;
__device__ double boys_shared[kBoysRows * kBoysCols];
std::mutex g_boys_mu;
double *g_boys_ptr[kMaxBoysDevices] = {};

hfx_status shared_boys(double **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(HFX_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxBoysDevices) return fail(HFX_ERR_UNSUPPORTED, "device index beyond the Boys table list");
  std::lock_guard<std::mutex> lk(g_boys_mu);
  if (!g_boys_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(boys_shared));
    if (e != hipSuccess || !ptr)
      return fail(HFX_ERR_DEVICE, std::string("hipGetSymbolAddress(boys_shared): ") + hipGetErrorString(e));
    const std::vector<double> t = boys_table();
    e = hipMemcpy(ptr, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(HFX_ERR_DEVICE, std::string("Boys table upload: ") + hipGetErrorString(e));
    g_boys_ptr[dev] = static_cast<double *>(ptr);
  }
  *out = g_boys_ptr[dev];
  return HFX_OK;
}

struct DevMem {
  std::vector<void *> ptrs;
  size_t total = 0;
  template <typename T>
  hipError_t alloc(T **p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void **)p, n * sizeof(T));
    if (e == hipSuccess) {
      ptrs.push_back((void *)*p);
      total += n * sizeof(T);
    }
    return e;
  }
  void release() {
    for (void *p : ptrs) (void)hipFree(p);
    ptrs.clear();
    total = 0;
  }
};

// device bytes of a one-plan batch's work arrays for nitems screening work
// items (counts, offsets, scan block sums, segment bounds, flags, counters;
// each array 256-byte aligned), lists excluded
size_t work_bytes(int64_t nitems) {
  auto a = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return a(4 * (size_t)(nitems + 1)) + a(8 * (size_t)(nitems + 1)) + a(8 * (size_t)((nitems + 1023) / 1024 + 2)) +
         2 * a(8 * (size_t)kNQuartetClass * 2) + a(8) + a(8 * (size_t)kNQuartetClass);
}

}  // namespace

struct hfx_plan_s {
  uint32_t magic = kMagic;
  // ---- system
  int n_atoms = 0, nsh = 0;
  std::vector<double> atom_xyz, sh_xyz;
  std::vector<int32_t> sh_atom, sh_l, sh_np, sh_poff;
  std::vector<double> ex, cn;  // exponents, normalised coefficients
  bool periodic = false;
  double lat[9] = {0}, rec[9] = {0}, recn[3] = {0};
  double cutoff = 0.0;
  int op = 0;
  double omega = 0.0, tau = 0.0;
  int precision = 0;
  double fp32_cutoff = 0.0;
  int sph = 1;
  // ---- pattern
  std::vector<hfx_block> blocks;
  std::vector<int2> blk_IJ;
  std::vector<int64_t> blk_off, blk_coff;
  std::vector<int32_t> partner, block_pair;
  std::vector<uint8_t> canon;
  int64_t nnz = 0, nnz_c = 0;
  int imgR[3] = {0, 0, 0};
  int nimg = 1;
  std::vector<int32_t> lut;
  // ---- unique pairs
  std::vector<int4> pr_info;
  std::vector<double> pr_geom;
  std::vector<int2> pr_pp;
  std::vector<int32_t> pr_npp;
  std::vector<double> pp;
  int32_t class_start[kNPairClass + 1] = {0};
  // ---- device
  hipStream_t stream = nullptr;
  DevMem mem;
  DevSys ds{};
  double *d_sh_xyz = nullptr;
  int32_t *d_sh_l = nullptr;
  int4 *d_pr_info = nullptr;
  double *d_pr_geom = nullptr;
  int2 *d_pr_pp = nullptr;
  int32_t *d_pr_npp = nullptr;
  double *d_pr_Q = nullptr;
  double *d_pp = nullptr;
  int32_t *d_lut = nullptr;
  int2 *d_blk_IJ = nullptr;
  int64_t *d_blk_off = nullptr, *d_blk_coff = nullptr;
  int32_t *d_partner = nullptr;
  uint8_t *d_canon = nullptr;
  double *d_pmax = nullptr;
  unsigned long long *d_pglob = nullptr;
  double *d_Dc = nullptr, *d_K4 = nullptr;
  double *d_boys = nullptr;
  DevSys *d_sys1 = nullptr;  // device copy of ds (one-plan launches)
  bool schwarz_done = false;
  // ---- ERI kernel per class: kern for the FP64 list, kern32 for the FP32
  // list of mixed precision (a K_* variant); coop holds the op lists of the
  // classes whose kernels take them (cooperative VRR, HRR of both)
  int kern[kNQuartetClass] = {0};
  int kern32[kNQuartetClass] = {0};
  int64_t grid[kNQuartetClass] = {0};    // grid caps (0: the kernel's default)
  int64_t grid32[kNQuartetClass] = {0};
  bool have_tables[kNQuartetClass] = {false};
  CoopDev coop[kNQuartetClass] = {};
  // ---- cached one-plan batch (hfx_build_K)
  struct Batch *self_batch = nullptr;
  int64_t max_list = kDefaultMaxList;  // quartets a build's list holds at once
  int device = -1;                     // device current at hfx_plan
  // collinear-spin builds: both spins' D_cart and K4 (allocated on the
  // first such build) and their one-plan batch
  double *d_Dc_spin = nullptr, *d_K4_spin = nullptr;
  struct Batch *spin_batch = nullptr;
  // k-space assembly (made on its first call): shell pairs of the pattern
  // with their block ranges, packed block images, shell function offsets,
  // and room for the k-points
  int4 *d_kpairs = nullptr;
  int n_kpairs = 0;
  int32_t *d_blk_img = nullptr, *d_func_off = nullptr;
  int64_t nbf = 0;
  double *d_kpts = nullptr;
  int kpts_cap = 0;
  // progress report of chunked builds (hfx_set_progress)
  hfx_progress_fn progress = nullptr;
  void *progress_user = nullptr;
};

// the plan's own one-plan batch, and the scratch address of its device
hfx_status plan_attach(hfx_plan_s *P);

namespace hfx {
// status with a message for hfx_last_error, for the other host units
hfx_status report_error(hfx_status st, const char *msg) { return fail(st, msg); }
}  // namespace hfx

namespace {

bool finite(double x) { return std::isfinite(x); }

hfx_status validate(const hfx_system *s) {
  if (!s) return fail(HFX_ERR_INVALID, "system is NULL");
  if (s->n_atoms <= 0 || !s->atom_xyz) return fail(HFX_ERR_INVALID, "no atoms");
  if (s->n_shells <= 0 || !s->shell_atom || !s->shell_l || !s->shell_nprim || !s->prim_exp || !s->prim_coef)
    return fail(HFX_ERR_INVALID, "no shells or NULL shell arrays");
  for (int i = 0; i < 3 * s->n_atoms; ++i)
    if (!finite(s->atom_xyz[i])) return fail(HFX_ERR_INVALID, "non-finite atom coordinate");
  int64_t np = 0;
  for (int i = 0; i < s->n_shells; ++i) {
    if (s->shell_atom[i] < 0 || s->shell_atom[i] >= s->n_atoms) return fail(HFX_ERR_INVALID, "shell_atom out of range");
    if (s->shell_l[i] < 0) return fail(HFX_ERR_INVALID, "negative angular momentum");
    if (s->shell_l[i] > HFX_MAX_L) return fail(HFX_ERR_UNSUPPORTED, "angular momentum above d is not implemented");
    if (s->shell_nprim[i] < 1 || s->shell_nprim[i] > HFX_MAX_PRIM)
      return fail(HFX_ERR_INVALID, "shell_nprim outside 1..HFX_MAX_PRIM");
    np += s->shell_nprim[i];
  }
  for (int64_t k = 0; k < np; ++k) {
    if (!(s->prim_exp[k] > 0.0) || !finite(s->prim_exp[k])) return fail(HFX_ERR_INVALID, "exponent must be positive and finite");
    if (!finite(s->prim_coef[k])) return fail(HFX_ERR_INVALID, "non-finite contraction coefficient");
  }
  if (s->lattice) {
    for (int i = 0; i < 9; ++i)
      if (!finite(s->lattice[i])) return fail(HFX_ERR_INVALID, "non-finite lattice");
    const double *a = s->lattice;
    double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) + a[2] * (a[3] * a[7] - a[4] * a[6]);
    double n1 = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    double n2 = std::sqrt(a[3] * a[3] + a[4] * a[4] + a[5] * a[5]);
    double n3 = std::sqrt(a[6] * a[6] + a[7] * a[7] + a[8] * a[8]);
    if (!(std::fabs(det) > 1e-8 * n1 * n2 * n3)) return fail(HFX_ERR_INVALID, "singular lattice");
    if (!(s->pair_cutoff > 0.0)) return fail(HFX_ERR_INVALID, "a periodic system needs pair_cutoff > 0");
  }
  if (!finite(s->pair_cutoff)) return fail(HFX_ERR_INVALID, "non-finite pair_cutoff");
  if (s->op != HFX_OP_COULOMB && s->op != HFX_OP_ERFC) return fail(HFX_ERR_INVALID, "unknown operator");
  if (s->op == HFX_OP_ERFC && !(s->omega > 0.0 && finite(s->omega))) return fail(HFX_ERR_INVALID, "erfc needs omega > 0");
  if (!(s->tau >= 0.0) || !finite(s->tau)) return fail(HFX_ERR_INVALID, "tau must be >= 0");
  if (s->precision != HFX_FP64 && s->precision != HFX_MIXED) return fail(HFX_ERR_INVALID, "unknown precision");
  if (!(s->fp32_cutoff >= 0.0) || !finite(s->fp32_cutoff)) return fail(HFX_ERR_INVALID, "fp32_cutoff must be >= 0");
  return HFX_OK;
}

// Contraction normalisation: primitive x^l normalisation
// N = (2a/pi)^(3/4) (4a)^(l/2) / sqrt((2l-1)!!) folded into c, then c scaled
// so that the x^l component of the contracted shell has unit self-overlap.
void normalise(int l, int n, const double *ex, const double *c, double *out) {
  const double pi = 3.14159265358979323846;
  double N[HFX_MAX_PRIM];
  for (int k = 0; k < n; ++k) N[k] = std::pow(2.0 * ex[k] / pi, 0.75) * std::pow(4.0 * ex[k], 0.5 * l) / std::sqrt(dfact(2 * l - 1));
  double S = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double p = ex[i] + ex[j];
      S += c[i] * N[i] * c[j] * N[j] * std::pow(pi / p, 1.5) * dfact(2 * l - 1) / std::pow(2.0 * p, l);
    }
  for (int k = 0; k < n; ++k) out[k] = c[k] * N[k] / std::sqrt(S);
}

void lattice_vec(const hfx_plan_s &P, int a, int b, int c, double *t) {
  for (int k = 0; k < 3; ++k) t[k] = a * P.lat[k] + b * P.lat[3 + k] + c * P.lat[6 + k];
}

hfx_status build_host(hfx_plan_s &P, const hfx_system *s) {
  P.n_atoms = s->n_atoms;
  P.nsh = s->n_shells;
  P.atom_xyz.assign(s->atom_xyz, s->atom_xyz + 3 * s->n_atoms);
  P.sh_atom.assign(s->shell_atom, s->shell_atom + P.nsh);
  P.sh_l.assign(s->shell_l, s->shell_l + P.nsh);
  P.sh_np.assign(s->shell_nprim, s->shell_nprim + P.nsh);
  P.sh_poff.resize(P.nsh + 1);
  int tot = 0;
  for (int i = 0; i < P.nsh; ++i) {
    P.sh_poff[i] = tot;
    tot += P.sh_np[i];
  }
  P.sh_poff[P.nsh] = tot;
  P.ex.assign(s->prim_exp, s->prim_exp + tot);
  P.cn.resize(tot);
  for (int i = 0; i < P.nsh; ++i)
    normalise(P.sh_l[i], P.sh_np[i], &P.ex[P.sh_poff[i]], s->prim_coef + P.sh_poff[i], &P.cn[P.sh_poff[i]]);
  P.sh_xyz.resize(3 * P.nsh);
  for (int i = 0; i < P.nsh; ++i)
    for (int k = 0; k < 3; ++k) P.sh_xyz[3 * i + k] = P.atom_xyz[3 * P.sh_atom[i] + k];
  P.periodic = s->lattice != nullptr;
  P.cutoff = s->pair_cutoff;
  P.op = s->op;
  P.omega = s->omega;
  P.tau = s->tau;
  P.precision = s->precision;
  P.fp32_cutoff = s->fp32_cutoff;
  P.sph = s->spherical_d ? 1 : 0;

  // ---- lattice and image search box
  int box[3] = {0, 0, 0};
  if (P.periodic) {
    std::memcpy(P.lat, s->lattice, sizeof(P.lat));
    const double *a = P.lat;
    double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) + a[2] * (a[3] * a[7] - a[4] * a[6]);
    // b_i (rows) with b_i . a_j = delta_ij: b = (A^-1)^T
    double inv[9] = {(a[4] * a[8] - a[5] * a[7]) / det, (a[2] * a[7] - a[1] * a[8]) / det, (a[1] * a[5] - a[2] * a[4]) / det,
                     (a[5] * a[6] - a[3] * a[8]) / det, (a[0] * a[8] - a[2] * a[6]) / det, (a[2] * a[3] - a[0] * a[5]) / det,
                     (a[3] * a[7] - a[4] * a[6]) / det, (a[1] * a[6] - a[0] * a[7]) / det, (a[0] * a[4] - a[1] * a[3]) / det};
    for (int i = 0; i < 3; ++i) {
      for (int k = 0; k < 3; ++k) P.rec[3 * i + k] = inv[3 * k + i];
      P.recn[i] = std::sqrt(P.rec[3 * i] * P.rec[3 * i] + P.rec[3 * i + 1] * P.rec[3 * i + 1] + P.rec[3 * i + 2] * P.rec[3 * i + 2]);
    }
    for (int i = 0; i < 3; ++i) {
      double fmin = 1e300, fmax = -1e300;
      for (int at = 0; at < P.n_atoms; ++at) {
        double f = P.rec[3 * i] * P.atom_xyz[3 * at] + P.rec[3 * i + 1] * P.atom_xyz[3 * at + 1] + P.rec[3 * i + 2] * P.atom_xyz[3 * at + 2];
        fmin = std::min(fmin, f);
        fmax = std::max(fmax, f);
      }
      box[i] = (int)std::ceil(P.cutoff * P.recn[i] + (fmax - fmin)) + 1;
      if (box[i] > 100) return fail(HFX_ERR_UNSUPPORTED, "pair cutoff spans too many lattice images");
      // ket translations of kept quartets: a pair's midpoint lies within
      // cutoff/2 of its home-cell atom and the screening box adds both pair
      // half-lengths and the cutoff, so |G_i| <= span of the atoms'
      // fractional coordinates + 3 cutoff |b_i|; the quartet encoding holds
      // -16..15
      const int gmax = (int)std::ceil((fmax - fmin) + 3.0 * P.cutoff * P.recn[i]) + 1;
      if (gmax > 15)
        return fail(HFX_ERR_UNSUPPORTED, "pair cutoff too long for the cell: ket translations could exceed 15 cells");
    }
  }

  // ---- pattern: atom pairs within the cutoff, expanded to shells
  std::vector<std::vector<int>> atom_shells(P.n_atoms);
  for (int i = 0; i < P.nsh; ++i) atom_shells[P.sh_atom[i]].push_back(i);
  struct Key {
    int32_t I, J, a, b, c;
  };
  std::vector<Key> keys;
  const double rc2 = P.cutoff * P.cutoff;
  for (int ia = 0; ia < P.n_atoms; ++ia)
    for (int ib = 0; ib < P.n_atoms; ++ib)
      for (int a = -box[0]; a <= box[0]; ++a)
        for (int b = -box[1]; b <= box[1]; ++b)
          for (int c = -box[2]; c <= box[2]; ++c) {
            double t[3] = {0, 0, 0};
            if (P.periodic) lattice_vec(P, a, b, c, t);
            double d2 = 0.0;
            for (int k = 0; k < 3; ++k) {
              double d = P.atom_xyz[3 * ia + k] - P.atom_xyz[3 * ib + k] - t[k];
              d2 += d * d;
            }
            if (P.cutoff > 0.0 && d2 > rc2) continue;
            for (int I : atom_shells[ia])
              for (int J : atom_shells[ib]) keys.push_back({I, J, a, b, c});
          }
  std::sort(keys.begin(), keys.end(), [](const Key &x, const Key &y) {
    if (x.I != y.I) return x.I < y.I;
    if (x.J != y.J) return x.J < y.J;
    if (x.a != y.a) return x.a < y.a;
    if (x.b != y.b) return x.b < y.b;
    return x.c < y.c;
  });
  const int64_t nb = (int64_t)keys.size();
  if (nb >= (int64_t)INT32_MAX) return fail(HFX_ERR_UNSUPPORTED, "too many pattern blocks");
  for (auto &k : keys) {
    P.imgR[0] = std::max(P.imgR[0], std::abs(k.a));
    P.imgR[1] = std::max(P.imgR[1], std::abs(k.b));
    P.imgR[2] = std::max(P.imgR[2], std::abs(k.c));
  }
  P.nimg = (2 * P.imgR[0] + 1) * (2 * P.imgR[1] + 1) * (2 * P.imgR[2] + 1);
  const int64_t lut_n = (int64_t)P.nsh * P.nsh * P.nimg;
  if (lut_n > (int64_t)1 << 31) return fail(HFX_ERR_UNSUPPORTED, "block lookup table too large");
  P.lut.assign(lut_n, -1);
  auto imgidx = [&](int a, int b, int c) {
    if (std::abs(a) > P.imgR[0] || std::abs(b) > P.imgR[1] || std::abs(c) > P.imgR[2]) return -1;
    return ((a + P.imgR[0]) * (2 * P.imgR[1] + 1) + (b + P.imgR[1])) * (2 * P.imgR[2] + 1) + (c + P.imgR[2]);
  };
  P.blocks.resize(nb);
  P.blk_IJ.resize(nb);
  P.blk_off.resize(nb + 1);
  P.blk_coff.resize(nb + 1);
  int64_t off = 0, coff = 0;
  for (int64_t i = 0; i < nb; ++i) {
    const Key &k = keys[i];
    hfx_block &b = P.blocks[i];
    b.I = k.I;
    b.J = k.J;
    b.img[0] = k.a;
    b.img[1] = k.b;
    b.img[2] = k.c;
    b.pad = 0;
    b.offset = off;
    P.blk_IJ[i] = make_int2(k.I, k.J);
    P.blk_off[i] = off;
    P.blk_coff[i] = coff;
    off += nfunc_host(P.sh_l[k.I], P.sph) * nfunc_host(P.sh_l[k.J], P.sph);
    coff += ncart(P.sh_l[k.I]) * ncart(P.sh_l[k.J]);
    P.lut[((int64_t)k.I * P.nsh + k.J) * P.nimg + imgidx(k.a, k.b, k.c)] = (int32_t)i;
  }
  P.blk_off[nb] = off;
  P.blk_coff[nb] = coff;
  P.nnz = off;
  P.nnz_c = coff;
  P.partner.resize(nb);
  P.canon.resize(nb);
  for (int64_t i = 0; i < nb; ++i) {
    const Key &k = keys[i];
    int pi = imgidx(-k.a, -k.b, -k.c);
    P.partner[i] = pi < 0 ? -1 : P.lut[((int64_t)k.J * P.nsh + k.I) * P.nimg + pi];
    if (P.partner[i] < 0) return fail(HFX_ERR_DEVICE, "internal: pattern is not symmetric");
    P.canon[i] = (k.I < k.J || (k.I == k.J && lexpos(k.a, k.b, k.c))) ? 1 : 0;
  }

  // ---- unique pairs in evaluation orientation (la >= lb), class-sorted
  struct PairRec {
    int A, B, a, b, c, cls, blk, nsig;
  };
  std::vector<PairRec> prs;
  for (int64_t i = 0; i < nb; ++i) {
    if (!P.canon[i]) continue;
    const Key &k = keys[i];
    PairRec r;
    if (P.sh_l[k.I] >= P.sh_l[k.J]) {
      r = {k.I, k.J, k.a, k.b, k.c, 0, (int)i, 0};
    } else {
      r = {k.J, k.I, -k.a, -k.b, -k.c, 0, (int)P.partner[i], 0};
    }
    r.cls = pair_class(P.sh_l[r.A], P.sh_l[r.B]);
    prs.push_back(r);
  }
  if (prs.size() >= kMaxPairs) return fail(HFX_ERR_UNSUPPORTED, "too many shell pairs for the quartet encoding");
  // primitive pairs per unique pair, sorted by a magnitude bound
  struct PPRec {
    double v[kPP];
    double bound;
  };
  std::vector<std::vector<PPRec>> ppr(prs.size());
  const double pi = 3.14159265358979323846;
  for (size_t q = 0; q < prs.size(); ++q) {
    PairRec &r = prs[q];
    double RA[3], RB[3], t[3] = {0, 0, 0};
    if (P.periodic) lattice_vec(P, r.a, r.b, r.c, t);
    for (int k = 0; k < 3; ++k) {
      RA[k] = P.sh_xyz[3 * r.A + k];
      RB[k] = P.sh_xyz[3 * r.B + k] + t[k];
    }
    double AB2 = 0.0;
    for (int k = 0; k < 3; ++k) AB2 += (RA[k] - RB[k]) * (RA[k] - RB[k]);
    const int la = P.sh_l[r.A], lb = P.sh_l[r.B];
    for (int ia = 0; ia < P.sh_np[r.A]; ++ia)
      for (int ib = 0; ib < P.sh_np[r.B]; ++ib) {
        const double al = P.ex[P.sh_poff[r.A] + ia], be = P.ex[P.sh_poff[r.B] + ib];
        const double z = al + be;
        PPRec e;
        e.v[0] = z;
        double PA = 0.0, PB = 0.0;
        for (int k = 0; k < 3; ++k) {
          const double Pk = (al * RA[k] + be * RB[k]) / z;
          e.v[1 + k] = Pk;
          e.v[4 + k] = Pk - RA[k];
          PA += (Pk - RA[k]) * (Pk - RA[k]);
          PB += (Pk - RB[k]) * (Pk - RB[k]);
        }
        e.v[7] = P.cn[P.sh_poff[r.A] + ia] * P.cn[P.sh_poff[r.B] + ib] * std::exp(-al * be / z * AB2);
        // sqrt of the s-type self-repulsion of the product, widened by the
        // polynomial prefactors of the angular parts
        const double rz = 1.0 / std::sqrt(z);
        e.bound = std::fabs(e.v[7]) * std::pow(pi, 1.25) * std::pow(2.0, 0.25) * std::pow(z, -1.25) *
                  std::pow(1.0 + std::sqrt(PA) + rz, la) * std::pow(1.0 + std::sqrt(PB) + rz, lb);
        ppr[q].push_back(e);
      }
    // device form of the pair factor: sqrt(2 pi^(5/2)) K / zeta, and 1/(2 zeta)
    for (auto &e : ppr[q]) {
      e.v[7] = kSqrt2Pi52 * e.v[7] / e.v[0];
      e.v[8] = 0.5 / e.v[0];
      e.v[9] = e.bound;
    }
    std::stable_sort(ppr[q].begin(), ppr[q].end(), [](const PPRec &x, const PPRec &y) { return x.bound > y.bound; });
    int ns = 0;
    for (auto &e : ppr[q]) ns += e.bound >= kPrimDrop;
    r.nsig = ns;
  }
  std::vector<int> order(prs.size());
  for (size_t q = 0; q < prs.size(); ++q) order[q] = (int)q;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    if (prs[x].cls != prs[y].cls) return prs[x].cls < prs[y].cls;
    return prs[x].nsig > prs[y].nsig;
  });
  const int npairs = (int)prs.size();
  P.pr_info.resize(npairs);
  P.pr_geom.assign((size_t)npairs * 8, 0.0);
  P.pr_pp.resize(npairs);
  P.pr_npp.resize(npairs);
  P.block_pair.assign(nb, -1);
  for (int c = 0; c <= kNPairClass; ++c) P.class_start[c] = 0;
  int64_t ppoff = 0;
  for (int q = 0; q < npairs; ++q) {
    const PairRec &r = prs[order[q]];
    const bool self = (r.A == r.B && r.a == 0 && r.b == 0 && r.c == 0);
    P.pr_info[q] = make_int4(r.A, r.B, pack_img8(r.a, r.b, r.c), self ? 1 : 0);
    double t[3] = {0, 0, 0};
    if (P.periodic) lattice_vec(P, r.a, r.b, r.c, t);
    double ab2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double RA = P.sh_xyz[3 * r.A + k], RB = P.sh_xyz[3 * r.B + k] + t[k];
      P.pr_geom[8 * q + k] = RA - RB;
      P.pr_geom[8 * q + 3 + k] = 0.5 * (RA + RB);
      ab2 += (RA - RB) * (RA - RB);
    }
    P.pr_geom[8 * q + 6] = 0.5 * std::sqrt(ab2);
    const auto &v = ppr[order[q]];
    P.pr_pp[q] = make_int2((int)ppoff, r.nsig);
    P.pr_npp[q] = (int)v.size();
    for (auto &e : v)
      for (int k = 0; k < kPP; ++k) P.pp.push_back(e.v[k]);
    ppoff += (int64_t)v.size();
    P.block_pair[r.blk] = q;
    P.block_pair[P.partner[r.blk]] = q;
    P.class_start[r.cls + 1]++;
  }
  if (ppoff >= (int64_t)INT32_MAX) return fail(HFX_ERR_UNSUPPORTED, "too many primitive pairs");
  for (int c = 0; c < kNPairClass; ++c) P.class_start[c + 1] += P.class_start[c];

  return HFX_OK;
}

template <typename T>
hipError_t upload(hfx_plan_s &P, T **dst, const std::vector<T> &src) {
  hipError_t e = P.mem.alloc(dst, src.size());
  if (e != hipSuccess) return e;
  if (!src.empty()) e = hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, P.stream);
  return e;
}

// ERI kernel variants of a class
enum { K_REG = 0, K_COOP = 1, K_LANE = 2, K_REG32 = 3, K_LANE32 = 4, K_NVARIANT = 5 };
const char *const kKernName[K_NVARIANT] = {"reg", "coop", "lane", "reg32", "lane32"};

bool variant_available(int cb, int ck, int v) {
  switch (v) {
    case K_REG:
    case K_REG32: return register_available(cb, ck);
    case K_COOP: return coop_available(cb, ck);
    case K_LANE:
    case K_LANE32: return lane_available(cb, ck);
    default: return false;
  }
}
bool variant_fp32(int v) { return v == K_REG32 || v == K_LANE32; }

// Classes kept on the FP64 list at any cutoff: those whose one-lane kernel
// gains nothing from the FP32 recursion (measured on the 64-atom diamond
// recipe: (ss|ss), (ps|ss), (ps|ps), (pp|ps), (ds|ss), (dd|ss) are Boys- and
// latency-bound, FP32 within 1% or slower; this also saves a launch), and
// (dd|dd), whose four HRR transfer steps scale the FP32 intermediates by
// |AB|^2 |CD|^2 before they cancel: 46 of its quartets below Q_IJ Q_KL =
// 1e-6 moved K by 1.0e-7 in a 25-atom cluster of the batch recipe (2.2e-9
// with them in FP64).
bool fp32_gains(int cb, int ck) {
  const int r = region_of(cb, ck);
  return !(r == region_of(0, 0) || r == region_of(1, 0) || r == region_of(1, 1) || r == region_of(2, 1) ||
           r == region_of(3, 0) || r == region_of(5, 0) || r == region_of(5, 5));
}

// FP32-list kernel that goes with FP64-list kernel k64 (an FP64 variant:
// the class does not split, see fp32_gains)
int default_kern32(int cb, int ck, int k64) {
  if (k64 == K_REG && variant_available(cb, ck, K_REG32) && fp32_gains(cb, ck)) return K_REG32;
  if (k64 == K_LANE && fp32_gains(cb, ck)) return K_LANE32;
  return k64;
}

// HFX_KERNELS="<cb><ck>=<name>,<cb><ck>/32=<name>,...": per-class kernel
// choice for experiments (names as in kKernName)
hfx_status apply_kernel_overrides(hfx_plan_s &P) {
  const char *env = std::getenv("HFX_KERNELS");
  if (!env) return HFX_OK;
  std::string all(env);
  size_t pos = 0;
  while (pos < all.size()) {
    size_t end = all.find(',', pos);
    if (end == std::string::npos) end = all.size();
    const std::string tok = all.substr(pos, end - pos);
    pos = end + 1;
    if (tok.empty()) continue;
    const size_t eq = tok.find('=');
    if (eq == std::string::npos || eq < 2 || tok[0] < '0' || tok[0] > '5' || tok[1] < '0' || tok[1] > tok[0])
      return fail(HFX_ERR_INVALID, "HFX_KERNELS: bad entry " + tok);
    const int cb = tok[0] - '0', ck = tok[1] - '0';
    const bool f32 = tok.compare(2, eq - 2, "/32") == 0;
    if (!f32 && eq != 2) return fail(HFX_ERR_INVALID, "HFX_KERNELS: bad entry " + tok);
    const std::string name = tok.substr(eq + 1);
    int v = -1;
    for (int k = 0; k < K_NVARIANT; ++k)
      if (name == kKernName[k]) v = k;
    if (v < 0 || !variant_available(cb, ck, v) || (!f32 && variant_fp32(v)))
      return fail(HFX_ERR_INVALID, "HFX_KERNELS: unavailable kernel in " + tok);
    const int r = region_of(cb, ck);
    if (f32) {
      P.kern32[r] = v;
    } else {
      P.kern[r] = v;
      P.kern32[r] = default_kern32(cb, ck, v);
    }
  }
  return HFX_OK;
}

hfx_status upload_plan(hfx_plan_s &P) {
  HIPCHK(upload(P, &P.d_sh_xyz, P.sh_xyz));
  HIPCHK(upload(P, &P.d_sh_l, P.sh_l));
  HIPCHK(upload(P, &P.d_pr_info, P.pr_info));
  HIPCHK(upload(P, &P.d_pr_geom, P.pr_geom));
  HIPCHK(upload(P, &P.d_pr_pp, P.pr_pp));
  HIPCHK(upload(P, &P.d_pr_npp, P.pr_npp));
  HIPCHK(P.mem.alloc(&P.d_pr_Q, P.pr_info.size()));
  HIPCHK(upload(P, &P.d_pp, P.pp));
  HIPCHK(upload(P, &P.d_lut, P.lut));
  HIPCHK(upload(P, &P.d_blk_IJ, P.blk_IJ));
  HIPCHK(upload(P, &P.d_blk_off, P.blk_off));
  HIPCHK(upload(P, &P.d_blk_coff, P.blk_coff));
  HIPCHK(upload(P, &P.d_partner, P.partner));
  HIPCHK(upload(P, &P.d_canon, P.canon));
  HIPCHK(P.mem.alloc(&P.d_pmax, P.blocks.size()));
  HIPCHK(P.mem.alloc(&P.d_pglob, 1));
  HIPCHK(P.mem.alloc(&P.d_Dc, (size_t)P.nnz_c));
  HIPCHK(P.mem.alloc(&P.d_K4, (size_t)P.nnz_c));
  {
    const hfx_status st = shared_boys(&P.d_boys);  // not owned by the plan
    if (st != HFX_OK) return st;
  }
  // op lists of the classes served by the cooperative or the lane kernel
  for (int cb = 0; cb < kNPairClass; ++cb)
    for (int ck = 0; ck <= cb; ++ck) {
      const int r = region_of(cb, ck);
      const int Lt = class_la(cb) + class_lb(cb) + class_la(ck) + class_lb(ck);
      if (!coop_available(cb, ck) && !lane_available(cb, ck)) continue;
      CoopHost h;
      coop_build(cb, ck, coop_available(cb, ck) ? 64 / coop_parallel(cb, ck) : 64, h);
      if (h.n_vrr_levels != Lt) return fail(HFX_ERR_DEVICE, "internal: cooperative level structure");
      for (int lv = 0; lv < h.n_vrr_levels; ++lv)
        if (h.levels[lv].y != coop_level_count(cb, ck, lv) || h.levels[lv].x != (lv ? h.levels[lv - 1].x + h.levels[lv - 1].y : 0))
          return fail(HFX_ERR_DEVICE, "internal: cooperative op list does not match the kernel shape");
      if (lane_available(cb, ck) && (h.out_base + h.nout > lane_hrr_capacity(cb, ck) || h.nacc > lane_hrr_capacity(cb, ck)))
        return fail(HFX_ERR_DEVICE, "internal: HRR workspace of the lane kernel too small");
      uint4 *d_ops = nullptr, *d_vops = nullptr;
      int4 *d_lv = nullptr;
      uint16_t *d_acc = nullptr;
      HIPCHK(upload(P, &d_ops, h.ops));
      HIPCHK(upload(P, &d_vops, h.vops));
      HIPCHK(upload(P, &d_lv, h.levels));
      HIPCHK(upload(P, &d_acc, h.acc_off));
      CoopDev &c = P.coop[r];
      c.ops = d_ops;
      c.vops = d_vops;
      c.levels = d_lv;
      c.acc_off = d_acc;
      c.n_vrr_levels = h.n_vrr_levels;
      c.n_hrr_levels = h.n_hrr_levels;
      c.nacc = h.nacc;
      c.nout = h.nout;
      c.nw = h.nw;
      c.out_base = h.out_base;
      c.na = ncart(h.la);
      c.nb = ncart(h.lb);
      c.nc = ncart(h.lc);
      c.nd = ncart(h.ld);
      P.have_tables[r] = true;
    }
  // default kernel per class, then any override from HFX_KERNELS
  for (int cb = 0; cb < kNPairClass; ++cb)
    for (int ck = 0; ck <= cb; ++ck) {
      const int r = region_of(cb, ck);
      // the lane kernel where the one-lane recursion spills or is absent
      // (bra dp or dd with a ket of two or more angular momentum units,
      // except (dp|ds): 96 accumulators, its one-lane kernel measured 37%
      // faster on the 64-atom diamond cell); elsewhere the one-lane kernel,
      // measured faster (the autotuner revisits the choice per plan)
      const bool heavy = cb >= 4 && class_la(ck) + class_lb(ck) >= 2 && !(cb == 4 && ck == 3);
      P.kern[r] = (heavy || !register_available(cb, ck)) ? K_LANE : K_REG;
      P.kern32[r] = default_kern32(cb, ck, P.kern[r]);
    }
  {
    hfx_status st = apply_kernel_overrides(P);
    if (st != HFX_OK) return st;
  }

  DevSys &s = P.ds;
  s.sh_xyz = P.d_sh_xyz;
  s.sh_l = P.d_sh_l;
  s.nsh = P.nsh;
  s.pr_info = P.d_pr_info;
  s.pr_geom = P.d_pr_geom;
  s.pr_pp = P.d_pr_pp;
  s.pr_npp = P.d_pr_npp;
  s.pr_Q = P.d_pr_Q;
  s.npairs = (int32_t)P.pr_info.size();
  s.pp = P.d_pp;
  s.lut = P.d_lut;
  for (int k = 0; k < 3; ++k) s.imgR[k] = P.imgR[k];
  s.nimg = P.nimg;
  s.blk_coff = P.d_blk_coff;
  s.pmax = P.d_pmax;
  s.pmax_global = P.d_pglob;
  s.periodic = P.periodic ? 1 : 0;
  std::memcpy(s.lat, P.lat, sizeof(s.lat));
  std::memcpy(s.rec, P.rec, sizeof(s.rec));
  std::memcpy(s.recn, P.recn, sizeof(s.recn));
  s.cutoff = P.cutoff;
  s.op = P.op;
  s.omega2 = P.omega * P.omega;
  s.tau = P.tau;
  // a class takes the FP32 list only if its FP32-list kernel is an FP32
  // variant (the default, an HFX_KERNELS choice)
  for (int r = 0; r < kNQuartetClass; ++r)
    s.fp32_cut[r] = (P.precision == HFX_MIXED && variant_fp32(P.kern32[r])) ? P.fp32_cutoff : 0.0;
  s.boys = P.d_boys;
  s.Dc = P.d_Dc;
  s.K4 = P.d_K4;
  s.nspin = 1;
  s.spin_stride = P.nnz_c;
  for (int c = 0; c <= kNPairClass; ++c) s.class_start[c] = P.class_start[c];
  HIPCHK(P.mem.alloc(&P.d_sys1, 1));
  HIPCHK(hipMemcpyAsync(P.d_sys1, &P.ds, sizeof(DevSys), hipMemcpyHostToDevice, P.stream));
  HIPCHK(hipStreamSynchronize(P.stream));
  return HFX_OK;
}

// live plans: a destroyed handle is rejected without being dereferenced
std::mutex g_plans_mu;
std::unordered_set<const hfx_plan_s *> g_plans;

bool valid_plan(hfx_plan_t p) {
  std::lock_guard<std::mutex> lk(g_plans_mu);
  return p && g_plans.count(p) && p->magic == kMagic;
}

hfx_status run_schwarz(hfx_plan_s &P) {
  for (int c = 0; c < kNPairClass; ++c) {
    if (c >= 4)
      launch_schwarz_coop(c, P.op, P.d_sys1, P.coop[region_of(c, c)], P.class_start[c], P.class_start[c + 1],
                          P.stream);
    else
      launch_schwarz(c, P.op, P.ds, P.class_start[c], P.class_start[c + 1], P.stream);
  }
  HIPCHK(hipGetLastError());
  P.schwarz_done = true;
  return HFX_OK;
}

// ----------------------------------------------------------------- FLOPs
// Algorithmic floating-point operations of the implemented recursions
// (FMA = 2, add/mul/div/sqrt = 1), per primitive quartet and per contracted
// quartet of a class; mirrors os_hgp.hpp term by term.
void class_flops(int la, int lb, int lc, int ld, int op, int nspin, double &per_prim, double &per_quartet) {
  const int EB = la + lb, FK = lc + ld, L = EB + FK;
  auto cart = [](int l, int c, int &x, int &y, int &z) {
    int a = 0;
    while ((a + 1) * (a + 2) / 2 <= c) ++a;
    z = c - a * (a + 1) / 2;
    x = l - a;
    y = a - z;
  };
  double f = 0.0;
  f += 34.0;                                   // prefactor, rho, T, W-P, W-Q, 1/(2 zeta) ...
  double boys = 23.0 + (L > 0 ? 22.0 + 3.0 * L : 0.0);
  f += (op == 1) ? 2 * boys + 8.0 + 4.0 * (L + 1) : boys;
  f += (L + 1);                                // G *= pref
  for (int e = 1; e <= EB; ++e)
    for (int c = 0; c < ncart(e); ++c) {
      int x, y, z;
      cart(e, c, x, y, z);
      int v[3] = {x, y, z};
      int i = x > 0 ? 0 : (y > 0 ? 1 : 2);
      int n1 = v[i] - 1;
      f += (L - e + 1) * (3.0 + (n1 > 0 ? 5.0 : 0.0));
    }
  for (int fl = 1; fl <= FK; ++fl) {
    int elo = std::max(0, la - (FK - fl));
    for (int d = 0; d < ncart(fl); ++d) {
      int x, y, z;
      cart(fl, d, x, y, z);
      int w[3] = {x, y, z};
      int i = x > 0 ? 0 : (y > 0 ? 1 : 2);
      int nf = w[i] - 1;
      for (int e = elo; e <= EB; ++e)
        for (int c = 0; c < ncart(e); ++c) {
          int ux, uy, uz;
          cart(e, c, ux, uy, uz);
          int u[3] = {ux, uy, uz};
          f += (FK - fl + 1) * (3.0 + (nf > 0 ? 5.0 : 0.0) + (u[i] > 0 ? 3.0 : 0.0));
        }
    }
  }
  const int NE = noff(EB + 1) - noff(la), NF = noff(FK + 1) - noff(lc);
  f += NE * NF;  // accumulate
  per_prim = f;
  double g = 0.0;
  // HRR: one FMA per transferred element
  for (int b = 1; b <= lb; ++b) g += 2.0 * ncart(b) * (noff(EB - b + 1) - noff(la)) * NF;
  for (int d = 1; d <= ld; ++d) g += 2.0 * ncart(d) * (noff(FK - d + 1) - noff(lc)) * ncart(la) * ncart(lb);
  const int NOUT = ncart(la) * ncart(lb) * ncart(lc) * ncart(ld);
  // four digest contractions per spin density, one FMA per integral each,
  // and the weighting of their results
  g += nspin * (8.0 * NOUT +
                2.0 * (ncart(la) * ncart(lc) + ncart(lb) * ncart(lc) + ncart(la) * ncart(ld) + ncart(lb) * ncart(ld)));
  per_quartet = g;
}

}  // namespace

// =================================================================== ABI
extern "C" {

const char *hfx_last_error(void) { return g_err.c_str(); }

hfx_status hfx_footprint(const hfx_system *sys, size_t *device_bytes, size_t *list_bytes_per_quartet) {
  hfx_status st = validate(sys);
  if (st != HFX_OK) return st;
  if (!device_bytes) return fail(HFX_ERR_INVALID, "device_bytes is NULL");
  hfx_plan_s P;
  st = build_host(P, sys);
  if (st != HFX_OK) return st;
  size_t b = 0;
  b += P.sh_xyz.size() * 8 + P.sh_l.size() * 4;
  b += P.pr_info.size() * (sizeof(int4) + 8 * 8 + sizeof(int2) + 4 + 8);
  b += P.pp.size() * 8 + P.lut.size() * 4;
  b += P.blocks.size() * (sizeof(int2) + 8 + 8 + 4 + 1 + 8) + 16;
  b += (size_t)P.nnz_c * 16;
  // screening work: one item per (class region, bra pair), with its counts,
  // offsets and the rest of a batch's work arrays, for the plan's own batch
  // and for its share of a fused multi-plan batch
  int64_t nitems = 0;
  for (int cb = 0; cb < kNPairClass; ++cb) nitems += (int64_t)(cb + 1) * (P.class_start[cb + 1] - P.class_start[cb]);
  b += 2 * ((size_t)nitems * sizeof(int4) + sizeof(DevSys) + (size_t)kNQuartetClass * 2 * 8 + work_bytes(nitems));
  *device_bytes = b;
  if (list_bytes_per_quartet) *list_bytes_per_quartet = sizeof(uint64_t);
  return HFX_OK;
}

hfx_status hfx_plan(const hfx_system *sys, void *stream, hfx_plan_t *out) {
  if (!out) return fail(HFX_ERR_INVALID, "out is NULL");
  *out = nullptr;
  hfx_status st = validate(sys);
  if (st != HFX_OK) return st;
  hfx_plan_s *P = new hfx_plan_s();
  P->stream = (hipStream_t)stream;
  st = build_host(*P, sys);
  if (st == HFX_OK) st = upload_plan(*P);
  if (st == HFX_OK) st = plan_attach(P);
  if (st != HFX_OK) {
    P->mem.release();
    P->magic = 0;
    delete P;
    return st;
  }
  {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    g_plans.insert(P);
  }
  *out = P;
  return HFX_OK;
}

hfx_status hfx_pattern(hfx_plan_t plan, int64_t *n_blocks, int64_t *nnz, const hfx_block **blocks) {
  if (!valid_plan(plan)) return fail(HFX_ERR_STATE, "invalid or destroyed plan");
  if (n_blocks) *n_blocks = (int64_t)plan->blocks.size();
  if (nnz) *nnz = plan->nnz;
  if (blocks) *blocks = plan->blocks.data();
  return HFX_OK;
}

hfx_status hfx_schwarz(hfx_plan_t plan, double *q_host, int64_t *n_pairs) {
  if (!valid_plan(plan)) return fail(HFX_ERR_STATE, "invalid or destroyed plan");
  hfx_plan_s &P = *plan;
  hfx_status st = run_schwarz(P);
  if (st != HFX_OK) return st;
  if (n_pairs) *n_pairs = (int64_t)P.pr_info.size();
  if (q_host) {
    std::vector<double> q(P.pr_info.size());
    if (!q.empty()) HIPCHK(hipMemcpyAsync(q.data(), P.d_pr_Q, q.size() * 8, hipMemcpyDeviceToHost, P.stream));
    HIPCHK(hipStreamSynchronize(P.stream));
    for (size_t b = 0; b < P.blocks.size(); ++b) q_host[b] = q[P.block_pair[b]];
  }
  return HFX_OK;
}

}  // extern "C"

// ===================================================================
// Batches: one or more plans built by fused launches.  A batch owns the
// screening work items of its plans (region, bra pair, plan), the per-build
// work arrays (counts, offsets, class-segment bounds, quartet lists, error
// flags) and an optional HIP graph of the whole build.
// ===================================================================

// Per-build device work arrays.  A batch allocates its own (lists grow to
// the screened size up to the batch's list limit).  Work arrays of fixed
// capacity (fixed = true: memory the build may not reallocate) evaluate
// every list in chunks, and list32 may alias list.
struct Work {
  int32_t *counts = nullptr;
  int64_t *offsets = nullptr;
  int64_t *tiles = nullptr;  // block sums of the scan
  int64_t *seg64 = nullptr, *seg32 = nullptr;
  int32_t *err = nullptr;
  unsigned long long *nprim = nullptr;
  uint64_t *list = nullptr, *list32 = nullptr;
  int64_t cap = 0, cap32 = 0;
  bool fixed = false;
};

struct Batch {
  std::vector<hfx_plan_s *> plans;
  int op = 0;
  bool mixed = false;
  hipStream_t stream = nullptr;
  DevMem mem;
  DevSys *d_sys = nullptr;
  int4 *d_items = nullptr;
  int64_t nitems = 0;
  std::vector<int64_t> seg_items;  // [kNQuartetClass][n + 1]
  int64_t *d_seg_items = nullptr;
  Work w;                          // the batch's own work arrays (lists allocated on demand)
  int64_t max_list = 0;            // quartets a list may hold at once (larger lists run in chunks)
  int nspin = 1;                   // densities per plan (2: collinear spin, one ERI evaluation)
  std::vector<int64_t> h_seg64, h_seg32;  // whole-list class-segment bounds of the last eager build
  int64_t nq64 = 0, nq32 = 0;
  int64_t n_chunks = 0;            // list chunks of the last eager build (0: lists whole)
  bool have_counts = false;        // an eager build has filled h_seg* / nq*
  // graph of the build for fixed (D, K) pointers
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream the build is captured on
  std::vector<const double *> g_d;
  std::vector<double *> g_k;
  ~Batch() { release(); }
  void release() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    cap_stream = nullptr;
    if (w.list) (void)hipFree(w.list);
    if (w.list32) (void)hipFree(w.list32);
    w.list = w.list32 = nullptr;
    w.cap = w.cap32 = 0;
    mem.release();
  }
  int n() const { return (int)plans.size(); }
};

namespace {

std::mutex g_batch_mu;
std::vector<Batch *> g_batches;  // multi-plan batches (one-plan batches live in their plan)

void launch_variant(int v, int cb, int ck, int op, const CoopDev &cd, const SegLaunch &L) {
  switch (v) {
    case K_REG: launch_eri(cb, ck, op, L); break;
    case K_COOP: launch_eri_coop(cb, ck, op, cd, L); break;
    case K_LANE: launch_eri_lane(cb, ck, op, false, cd, L); break;
    case K_REG32: launch_eri_f32(cb, ck, op, L); break;
    case K_LANE32: launch_eri_lane(cb, ck, op, true, cd, L); break;
    default: break;
  }
}

// bytes of the per-build work arrays other than the lists, for nitems
// screening work items and n plans
struct WorkLayout {
  size_t counts, offsets, tiles, seg, err, nprim, total;
};
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
WorkLayout work_layout(int64_t nitems, int n) {
  WorkLayout L;
  L.counts = align256(sizeof(int32_t) * (size_t)(nitems + 1));
  L.offsets = align256(sizeof(int64_t) * (size_t)(nitems + 1));
  L.tiles = align256(sizeof(int64_t) * (size_t)((nitems + 1023) / 1024 + 2));
  L.seg = align256(sizeof(int64_t) * (size_t)kNQuartetClass * (n + 1));
  L.err = align256(2 * sizeof(int32_t));
  L.nprim = align256(kNQuartetClass * sizeof(unsigned long long));
  L.total = L.counts + L.offsets + L.tiles + 2 * L.seg + L.err + L.nprim;
  return L;
}
// point w's arrays (not the lists) into base, laid out as work_layout says
void work_place(Work &w, char *base, const WorkLayout &L) {
  char *p = base;
  w.counts = (int32_t *)p;
  p += L.counts;
  w.offsets = (int64_t *)p;
  p += L.offsets;
  w.tiles = (int64_t *)p;
  p += L.tiles;
  w.seg64 = (int64_t *)p;
  p += L.seg;
  w.seg32 = (int64_t *)p;
  p += L.seg;
  w.err = (int32_t *)p;
  p += L.err;
  w.nprim = (unsigned long long *)p;
}

hfx_status batch_init(Batch &B, const std::vector<hfx_plan_s *> &plans, int nspin = 1) {
  B.plans = plans;
  B.nspin = nspin;
  B.op = plans[0]->op;
  B.stream = plans[0]->stream;
  B.mixed = false;
  B.max_list = INT64_MAX;
  for (auto *P : plans) {
    B.mixed |= P->precision == HFX_MIXED;
    B.max_list = std::min(B.max_list, P->max_list);
  }
  const int n = (int)plans.size();
  std::vector<DevSys> sys(n);
  for (int i = 0; i < n; ++i) {
    sys[i] = plans[i]->ds;
    if (nspin == 2) {
      sys[i].Dc = plans[i]->d_Dc_spin;
      sys[i].K4 = plans[i]->d_K4_spin;
      sys[i].nspin = 2;
    }
  }
  // items ordered by (region, plan, bra pair): every class segment of the
  // fused list is contiguous and holds plan 0's quartets, then plan 1's, ...
  std::vector<int4> items;
  B.seg_items.assign((size_t)kNQuartetClass * (n + 1), 0);
  for (int cb = 0; cb < kNPairClass; ++cb)
    for (int ck = 0; ck <= cb; ++ck) {
      const int r = region_of(cb, ck);
      for (int i = 0; i < n; ++i) {
        B.seg_items[(size_t)r * (n + 1) + i] = (int64_t)items.size();
        const hfx_plan_s &P = *plans[i];
        if (P.class_start[ck + 1] == P.class_start[ck]) continue;
        for (int p = P.class_start[cb]; p < P.class_start[cb + 1]; ++p) items.push_back(make_int4(r, p, i, 0));
      }
      B.seg_items[(size_t)r * (n + 1) + n] = (int64_t)items.size();
    }
  B.nitems = (int64_t)items.size();
  HIPCHK(B.mem.alloc(&B.d_sys, (size_t)n));
  HIPCHK(hipMemcpyAsync(B.d_sys, sys.data(), n * sizeof(DevSys), hipMemcpyHostToDevice, B.stream));
  HIPCHK(B.mem.alloc(&B.d_items, items.size()));
  if (!items.empty())
    HIPCHK(hipMemcpyAsync(B.d_items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice, B.stream));
  HIPCHK(B.mem.alloc(&B.d_seg_items, B.seg_items.size()));
  HIPCHK(hipMemcpyAsync(B.d_seg_items, B.seg_items.data(), B.seg_items.size() * 8, hipMemcpyHostToDevice, B.stream));
  const WorkLayout L = work_layout(B.nitems, n);
  char *wbase = nullptr;
  HIPCHK(B.mem.alloc(&wbase, L.total));
  work_place(B.w, wbase, L);
  B.h_seg64.assign(B.seg_items.size(), 0);
  B.h_seg32.assign(B.seg_items.size(), 0);
  HIPCHK(hipStreamSynchronize(B.stream));
  return HFX_OK;
}

// grow a list to hold `need` entries (with headroom, at most `limit`)
hfx_status ensure_cap(uint64_t **list, int64_t *cap, int64_t need, int64_t limit) {
  if (need <= *cap && *list) return HFX_OK;
  if (*list) HIPCHK(hipFree(*list));
  *list = nullptr;
  *cap = 0;
  int64_t c = need + need / 4 + 4096;
  if (c > limit) c = limit;
  if (c < need) c = need;
  hipError_t e = hipMalloc((void **)list, (size_t)c * sizeof(uint64_t));
  if (e != hipSuccess) return fail(HFX_ERR_OOM, "quartet list allocation failed");
  *cap = c;
  return HFX_OK;
}

void drop_graph(Batch &B) {
  if (B.gexec) (void)hipGraphExecDestroy(B.gexec);
  if (B.graph) (void)hipGraphDestroy(B.graph);
  B.gexec = nullptr;
  B.graph = nullptr;
  B.g_d.clear();
  B.g_k.clear();
}

// ERI launches of every class over one list whose class-segment bounds are
// on the device at d_seg; h_seg: the same bounds on the host (grid sizes),
// or nullptr (graph: grids that drain any count).  f32: the FP32 list.
void launch_classes(Batch &B, Work &W, bool f32, const uint64_t *list, int64_t *d_seg, const int64_t *h_seg) {
  const int n = B.n();
  hfx_plan_s &P0 = *B.plans[0];
  for (int cb = kNPairClass - 1; cb >= 0; --cb)
    for (int ck = cb; ck >= 0; --ck) {
      const int r = region_of(cb, ck);
      const size_t so = (size_t)r * (n + 1);
      SegLaunch L{B.d_sys, n, d_seg + so, list, W.nprim + r, -1, B.stream, f32 ? P0.grid32[r] : P0.grid[r]};
      if (h_seg) L.nq_hint = h_seg[so + n] - h_seg[so];
      launch_variant(f32 ? P0.kern32[r] : P0.kern[r], cb, ck, B.op, P0.coop[r], L);
    }
}

// A list that does not fit its buffer, in chunks of consecutive screening
// work items (ranges of bra pairs of a class region) whose quartets fit:
// each chunk is filled, then evaluated by the ERI kernels of every class
// before the next chunk overwrites the buffer (stream order).  The offsets
// of the count pass are read back to place the chunk boundaries.
hfx_status run_chunks(Batch &B, Work &W, int mode, bool f32, uint64_t *list, int64_t cap, int64_t *d_seg) {
  const int n = B.n();
  const int64_t nit = B.nitems;
  std::vector<int64_t> off((size_t)nit + 1);
  HIPCHK(hipMemcpyAsync(off.data(), W.offsets, off.size() * sizeof(int64_t), hipMemcpyDeviceToHost, B.stream));
  HIPCHK(hipStreamSynchronize(B.stream));
  std::vector<int64_t> hs(B.seg_items.size());
  int64_t i0 = 0;
  while (i0 < nit) {
    const int64_t base = off[i0];
    const auto it = std::upper_bound(off.begin() + i0 + 1, off.end(), base + cap);
    const int64_t i1 = (int64_t)(it - off.begin()) - 1;
    if (i1 <= i0)
      return fail(HFX_ERR_OOM, "one screening work item (a bra pair against a ket class) has more quartets (" +
                                   std::to_string(off[i0 + 1] - base) + ") than the list capacity (" +
                                   std::to_string(cap) + ")");
    const int64_t end = off[i1];
    if (end > base) {
      launch_screen(B.d_sys, B.d_items + i0, i1 - i0, W.counts, W.offsets + i0, list, base, cap, W.err, true, mode,
                    B.stream);
      launch_gather_bounds(W.offsets, B.d_seg_items, d_seg, (int)B.seg_items.size(), base, end, B.stream);
      for (size_t k = 0; k < hs.size(); ++k) {
        const int64_t v = off[B.seg_items[k]];
        hs[k] = std::min(std::max(v, base), end) - base;
      }
      launch_classes(B, W, f32, list, d_seg, hs.data());
      ++B.n_chunks;
      // a plan that asked for progress reports hears of each chunk once
      // the device has finished it
      hfx_plan_s &P0 = *B.plans[0];
      if (P0.progress) {
        HIPCHK(hipStreamSynchronize(B.stream));
        P0.progress(P0.progress_user, f32 ? 1 : 0, B.n_chunks, end, off[nit]);
      }
    }
    i0 = i1;
  }
  (void)n;
  return HFX_OK;
}

// Enqueue the whole build of a batch on its stream.  graph = true: nothing
// here waits for the device (the sequence is being captured) and every list
// is whole.  Eager: each list is counted, sized on the host and either
// filled whole (its ERI launches follow all screening, class by class) or,
// when it exceeds the list limit or the work arrays are fixed, evaluated
// chunk by chunk right away.
hfx_status enqueue_build(Batch &B, Work &W, const double *const *d_dev, double *const *k_dev, bool graph,
                         hipEvent_t *ev, hipEvent_t *evc) {
  const int n = B.n();
  if (ev) HIPCHK(hipEventRecord(ev[0], B.stream));
  const int ns = B.nspin;
  for (int i = 0; i < n; ++i) {
    hfx_plan_s &P = *B.plans[i];
    double *Dc = ns == 2 ? P.d_Dc_spin : P.d_Dc;
    double *K4 = ns == 2 ? P.d_K4_spin : P.d_K4;
    launch_zero_u64(P.d_pglob, 1, B.stream);
    for (int sp = 0; sp < ns; ++sp)
      launch_density(P.ds, (int64_t)P.blocks.size(), P.d_blk_IJ, P.d_blk_off, P.d_partner, P.d_canon, P.sph,
                     d_dev[i * ns + sp], Dc + sp * P.nnz_c, sp > 0, B.stream);
    launch_zero(K4, ns * P.nnz_c, B.stream);
  }
  if (ev) HIPCHK(hipEventRecord(ev[1], B.stream));
  launch_zero_i32(W.err, 2, B.stream);
  launch_zero_u64(W.nprim, kNQuartetClass, B.stream);
  if (!graph) B.n_chunks = 0;
  bool whole[2] = {false, false};
  const int nlists = B.mixed ? 2 : 1;
  for (int li = 0; li < nlists; ++li) {
    const int mode = B.mixed ? 1 + li : 0;
    const bool f32 = li == 1;
    uint64_t **list = f32 ? &W.list32 : &W.list;
    int64_t *cap = f32 ? &W.cap32 : &W.cap;
    int64_t *d_seg = f32 ? W.seg32 : W.seg64;
    std::vector<int64_t> &h_seg = f32 ? B.h_seg32 : B.h_seg64;
    launch_screen(B.d_sys, B.d_items, B.nitems, W.counts, W.offsets, nullptr, 0, 0, W.err, false, mode, B.stream);
    HIPCHK(scan_counts(W.counts, W.offsets, B.nitems, W.tiles, B.stream));
    if (graph) {
      launch_gather_bounds(W.offsets, B.d_seg_items, d_seg, (int)B.seg_items.size(), 0, *cap, B.stream);
      launch_screen(B.d_sys, B.d_items, B.nitems, W.counts, W.offsets, *list, 0, *cap, W.err, true, mode, B.stream);
      whole[li] = true;
      continue;
    }
    launch_gather_bounds(W.offsets, B.d_seg_items, d_seg, (int)B.seg_items.size(), 0, INT64_MAX, B.stream);
    HIPCHK(hipMemcpyAsync(h_seg.data(), d_seg, h_seg.size() * 8, hipMemcpyDeviceToHost, B.stream));
    // the count pass has visited every kept translation: its error flag is
    // final here, so an eager build reports it even when nobody waits
    int32_t err[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(err, W.err, sizeof(err), hipMemcpyDeviceToHost, B.stream));
    HIPCHK(hipStreamSynchronize(B.stream));
    if (err[0] & 1) return fail(HFX_ERR_UNSUPPORTED, "a ket translation exceeds the quartet encoding range");
    const int64_t total = h_seg.empty() ? 0 : h_seg.back();
    (f32 ? B.nq32 : B.nq64) = total;
    if (!W.fixed && total <= B.max_list) {
      const uint64_t *before = *list;
      hfx_status st = ensure_cap(list, cap, total, B.max_list);
      if (st != HFX_OK) return st;
      if (*list != before) drop_graph(B);  // a captured graph holds the old list
      launch_screen(B.d_sys, B.d_items, B.nitems, W.counts, W.offsets, *list, 0, *cap, W.err, true, mode, B.stream);
      whole[li] = true;
    } else {
      if (!W.fixed) {
        hfx_status st = ensure_cap(list, cap, B.max_list, B.max_list);
        if (st != HFX_OK) return st;
        drop_graph(B);
      }
      hfx_status st = run_chunks(B, W, mode, f32, *list, *cap, d_seg);
      if (st != HFX_OK) return st;
    }
  }
  if (!B.mixed && !graph) {
    B.nq32 = 0;
    std::fill(B.h_seg32.begin(), B.h_seg32.end(), 0);
  }
  if (!graph) B.have_counts = true;
  if (ev) HIPCHK(hipEventRecord(ev[2], B.stream));
  hfx_plan_s &P0 = *B.plans[0];
  for (int cb = kNPairClass - 1; cb >= 0; --cb)
    for (int ck = cb; ck >= 0; --ck) {
      const int r = region_of(cb, ck);
      const size_t so = (size_t)r * (n + 1);
      if (evc) HIPCHK(hipEventRecord(evc[r], B.stream));
      for (int li = 0; li < nlists; ++li) {
        if (!whole[li]) continue;
        const bool f32 = li == 1;
        SegLaunch L{B.d_sys, n, (f32 ? W.seg32 : W.seg64) + so, f32 ? W.list32 : W.list, W.nprim + r, -1, B.stream,
                    f32 ? P0.grid32[r] : P0.grid[r]};
        if (!graph) {
          const std::vector<int64_t> &hs = f32 ? B.h_seg32 : B.h_seg64;
          L.nq_hint = hs[so + n] - hs[so];
        }
        launch_variant(f32 ? P0.kern32[r] : P0.kern[r], cb, ck, B.op, P0.coop[r], L);
      }
      if (evc && r == 0) HIPCHK(hipEventRecord(evc[kNQuartetClass], B.stream));
    }
  if (ev) HIPCHK(hipEventRecord(ev[3], B.stream));
  for (int i = 0; i < n; ++i) {
    hfx_plan_s &P = *B.plans[i];
    const double *K4 = ns == 2 ? P.d_K4_spin : P.d_K4;
    for (int sp = 0; sp < ns; ++sp)
      launch_finalize(P.ds, (int64_t)P.blocks.size(), P.d_blk_IJ, P.d_blk_off, P.d_partner, P.sph, K4 + sp * P.nnz_c,
                      k_dev[i * ns + sp], B.stream);
  }
  if (ev) HIPCHK(hipEventRecord(ev[4], B.stream));
  HIPCHK(hipGetLastError());
  return HFX_OK;
}

hfx_status check_err(Batch &B, Work &W, bool *overflow) {
  int32_t err[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(err, W.err, sizeof(err), hipMemcpyDeviceToHost, B.stream));
  HIPCHK(hipStreamSynchronize(B.stream));
  if (overflow) *overflow = (err[0] & 2) != 0;
  if (err[0] & 1) return fail(HFX_ERR_UNSUPPORTED, "a ket translation exceeds the quartet encoding range");
  if ((err[0] & 2) && !overflow) return fail(HFX_ERR_DEVICE, "internal: quartet list overflow in an eager build");
  return HFX_OK;
}

void fill_info(Batch &B, Work &W, hfx_build_info *info, hipEvent_t *ev, hipEvent_t *evc) {
  std::memset(info, 0, sizeof(*info));
  unsigned long long np[kNQuartetClass];
  if (hipMemcpyAsync(np, W.nprim, sizeof(np), hipMemcpyDeviceToHost, B.stream) != hipSuccess) return;
  if (hipStreamSynchronize(B.stream) != hipSuccess) return;
  const int n = B.n();
  hfx_plan_s &P0 = *B.plans[0];
  double fl = 0.0;
  for (int cb = 0; cb < kNPairClass; ++cb)
    for (int ck = 0; ck <= cb; ++ck) {
      const int r = region_of(cb, ck);
      const size_t so = (size_t)r * (n + 1);
      const int64_t q64 = B.h_seg64[so + n] - B.h_seg64[so];
      const int64_t q32 = B.mixed ? B.h_seg32[so + n] - B.h_seg32[so] : 0;
      info->n_quartets_class[r] = q64 + q32;
      info->n_quartets += q64 + q32;
      if (variant_fp32(P0.kern32[r])) info->n_fp32_quartets += q32;
      info->n_prim_quartets += (int64_t)np[r];
      double fp, fq;
      class_flops(class_la(cb), class_lb(cb), class_la(ck), class_lb(ck), B.op, B.nspin, fp, fq);
      info->flops_class[r] = fp * (double)np[r] + fq * (double)info->n_quartets_class[r];
      fl += info->flops_class[r];
    }
  info->flops = fl;
  info->n_chunks = B.n_chunks;
  if (ev) {
    float ms;
    if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) info->ms_density = ms;
    if (hipEventElapsedTime(&ms, ev[1], ev[2]) == hipSuccess) info->ms_screen = ms;
    if (hipEventElapsedTime(&ms, ev[2], ev[3]) == hipSuccess) info->ms_eri = ms;
    if (hipEventElapsedTime(&ms, ev[3], ev[4]) == hipSuccess) info->ms_finalize = ms;
    if (hipEventElapsedTime(&ms, ev[0], ev[4]) == hipSuccess) info->ms_total = ms;
  }
  if (evc) {
    int order[kNQuartetClass], k = 0;
    for (int cb = kNPairClass - 1; cb >= 0; --cb)
      for (int ck = cb; ck >= 0; --ck) order[k++] = region_of(cb, ck);
    for (int i = 0; i < kNQuartetClass; ++i) {
      hipEvent_t end = (i + 1 < kNQuartetClass) ? evc[order[i + 1]] : evc[kNQuartetClass];
      float ms;
      if (hipEventElapsedTime(&ms, evc[order[i]], end) == hipSuccess) info->ms_class[order[i]] = ms;
    }
  }
}

// Run a batch build: eager, or through a captured graph (HFX_GRAPH) that is
// re-captured when the D/K pointers change and re-run eagerly when the
// screened list outgrows the capacity fixed at capture time.  Builds whose
// lists were chunked run eagerly.
hfx_status run_batch(Batch &B, Work &W, const double *const *d_dev, double *const *k_dev, uint32_t flags,
                     hfx_build_info *info) {
  const int n = B.n() * B.nspin;  // D and K arrays: plan-major, spin-minor
  for (int i = 0; i < n; ++i)
    if (!d_dev[i] || !k_dev[i]) return fail(HFX_ERR_INVALID, "D or K pointer is NULL");
  for (auto *P : B.plans)
    if (!P->schwarz_done) {
      hfx_status st = run_schwarz(*P);
      if (st != HFX_OK) return st;
    }
  const bool timing = (flags & HFX_TIMING) != 0;
  const bool use_graph = (flags & HFX_GRAPH) != 0 && !timing && !W.fixed;
  if (use_graph && B.have_counts && B.n_chunks == 0) {
    bool same = B.gexec && (int)B.g_d.size() == n;
    for (int i = 0; same && i < n; ++i) same = B.g_d[i] == d_dev[i] && B.g_k[i] == k_dev[i];
    if (!same) {
      drop_graph(B);
      // headroom for the density-dependent list size of later SCF steps
      hfx_status st = ensure_cap(&W.list, &W.cap, B.nq64, B.max_list);
      if (st == HFX_OK && B.mixed) st = ensure_cap(&W.list32, &W.cap32, B.nq32, B.max_list);
      if (st != HFX_OK) return st;
      // capture on a private stream (the plan's stream may be the null
      // stream, which cannot be captured); the graph is launched on the
      // plan's stream
      if (!B.cap_stream) HIPCHK(hipStreamCreateWithFlags(&B.cap_stream, hipStreamNonBlocking));
      HIPCHK(hipStreamSynchronize(B.stream));
      HIPCHK(hipStreamBeginCapture(B.cap_stream, hipStreamCaptureModeThreadLocal));
      const hipStream_t user = B.stream;
      B.stream = B.cap_stream;
      st = enqueue_build(B, W, d_dev, k_dev, true, nullptr, nullptr);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(B.cap_stream, &g);
      B.stream = user;
      if (st != HFX_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return fail(HFX_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
      B.graph = g;
      HIPCHK(hipGraphInstantiate(&B.gexec, B.graph, nullptr, nullptr, 0));
      B.g_d.assign(d_dev, d_dev + n);
      B.g_k.assign(k_dev, k_dev + n);
    }
    HIPCHK(hipGraphLaunch(B.gexec, B.stream));
    HIPCHK(hipStreamSynchronize(B.stream));
    bool overflow = false;
    hfx_status st = check_err(B, W, &overflow);
    if (st != HFX_OK) return st;
    if (!overflow) {
      // counts of this build for the report
      HIPCHK(hipMemcpy(B.h_seg64.data(), W.seg64, B.h_seg64.size() * 8, hipMemcpyDeviceToHost));
      if (B.mixed) HIPCHK(hipMemcpy(B.h_seg32.data(), W.seg32, B.h_seg32.size() * 8, hipMemcpyDeviceToHost));
      B.nq64 = B.h_seg64.back();
      B.nq32 = B.mixed ? B.h_seg32.back() : 0;
      if (info) fill_info(B, W, info, nullptr, nullptr);
      return HFX_OK;
    }
    // the list outgrew the captured capacity: rebuild eagerly, recapture next time
    drop_graph(B);
  }
  hipEvent_t ev[5], evc[kNQuartetClass + 1];
  if (timing) {
    for (auto &e : ev) HIPCHK(hipEventCreate(&e));
    for (auto &e : evc) HIPCHK(hipEventCreate(&e));
  }
  hfx_status st = enqueue_build(B, W, d_dev, k_dev, false, timing ? ev : nullptr, timing ? evc : nullptr);
  if (st == HFX_OK && ((flags & (HFX_SYNC | HFX_TIMING)) || info)) {
    HIPCHK(hipStreamSynchronize(B.stream));
    st = check_err(B, W, nullptr);
    if (st == HFX_OK && info) fill_info(B, W, info, timing ? ev : nullptr, timing ? evc : nullptr);
  }
  if (timing) {
    for (auto &e : ev) (void)hipEventDestroy(e);
    for (auto &e : evc) (void)hipEventDestroy(e);
  }
  return st;
}

// graphs of every batch that contains P (its kernel choice has changed)
void drop_graphs_of(const hfx_plan_s *P) {
  if (P->self_batch) drop_graph(*P->self_batch);
  if (P->spin_batch) drop_graph(*P->spin_batch);
  std::lock_guard<std::mutex> lk(g_batch_mu);
  for (Batch *B : g_batches)
    if (std::find(B->plans.begin(), B->plans.end(), P) != B->plans.end()) drop_graph(*B);
}

// grid caps tried per kernel family (0 = default)
const int64_t kTuneGridReg[] = {0, 256 * 16, 256 * 64};  // one-wave blocks: 262k and 1M threads
const int64_t kTuneGridWave[] = {0, 256 * 8, 256 * 64};
// smallest prefix the autotuner times: several times the threads of the
// largest one-lane grid (256 * 256 one-wave blocks), so that a prefix does
// not under-fill a grid that the whole segment fills
constexpr int64_t kTuneMinPrefix = 4ll * 256 * 256 * 64;

hfx_status tune_class(Batch &B, int cb, int ck, bool f32, int64_t max_q, int64_t *d_seg2, hfx_tune_report *rep) {
  hfx_plan_s &P = *B.plans[0];
  Work &W = B.w;
  const int r = region_of(cb, ck);
  const std::vector<int64_t> &hs = f32 ? B.h_seg32 : B.h_seg64;
  const int64_t s0 = hs[(size_t)r * 2], s1 = hs[(size_t)r * 2 + 1];
  const int64_t nq = s1 - s0;
  if (nq <= 0) return HFX_OK;
  if (max_q > 0 && max_q < kTuneMinPrefix) max_q = kTuneMinPrefix;
  const int64_t take = (max_q > 0 && max_q < nq) ? max_q : nq;
  const int64_t seg2[2] = {s0, s0 + take};
  HIPCHK(hipMemcpyAsync(d_seg2, seg2, sizeof(seg2), hipMemcpyHostToDevice, B.stream));
  std::vector<std::pair<int, int64_t>> cands;
  const int vars64[] = {K_REG, K_COOP, K_LANE};
  const int vars32[] = {K_REG32, K_LANE32, K_REG, K_COOP, K_LANE};
  const int *vars = f32 ? vars32 : vars64;
  const int nv = f32 ? 5 : 3;
  for (int k = 0; k < nv; ++k) {
    const int v = vars[k];
    if (!variant_available(cb, ck, v)) continue;
    const bool wave = (v == K_COOP || v == K_LANE || v == K_LANE32);
    for (int64_t g : (wave ? kTuneGridWave : kTuneGridReg))
      if ((int)cands.size() < HFX_TUNE_MAX_CAND) cands.emplace_back(v, g);
  }
  if (cands.empty()) return HFX_OK;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  std::vector<float> ms(cands.size(), 0.0f);
  for (size_t c = 0; c < cands.size(); ++c) {
    SegLaunch L{B.d_sys, 1, d_seg2, f32 ? W.list32 : W.list, W.nprim + r, take, B.stream, cands[c].second};
    // first run loads the code object and warms the caches; the second is timed
    launch_variant(cands[c].first, cb, ck, B.op, P.coop[r], L);
    (void)hipEventRecord(e0, B.stream);
    launch_variant(cands[c].first, cb, ck, B.op, P.coop[r], L);
    (void)hipEventRecord(e1, B.stream);
    hipError_t e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return fail(HFX_ERR_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
    }
    (void)hipEventElapsedTime(&ms[c], e0, e1);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  size_t best = 0;
  for (size_t c = 1; c < cands.size(); ++c)
    if (ms[c] < ms[best]) best = c;
  if (f32) {
    P.kern32[r] = cands[best].first;
    P.grid32[r] = cands[best].second;
  } else {
    P.kern[r] = cands[best].first;
    P.grid[r] = cands[best].second;
  }
  if (rep) {
    int base = rep->n_candidates[r];
    for (size_t c = 0; c < cands.size() && base < HFX_TUNE_MAX_CAND; ++c, ++base) {
      hfx_tune_candidate &t = rep->cand[r][base];
      t.variant = cands[c].first;
      t.fp32_list = f32 ? 1 : 0;
      t.max_blocks = cands[c].second;
      t.ms = ms[c];
      if (c == best) (f32 ? rep->chosen32[r] : rep->chosen[r]) = base;
    }
    rep->n_candidates[r] = base;
    (f32 ? rep->sample_quartets32[r] : rep->sample_quartets[r]) = take;
  }
  return HFX_OK;
}

void delete_batch_locked(size_t i) {
  Batch *B = g_batches[i];
  (void)hipStreamSynchronize(B->stream);
  delete B;
  g_batches.erase(g_batches.begin() + (ptrdiff_t)i);
}

void drop_batches_of(const hfx_plan_s *P) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  for (size_t i = 0; i < g_batches.size();) {
    Batch *B = g_batches[i];
    if (std::find(B->plans.begin(), B->plans.end(), P) != B->plans.end())
      delete_batch_locked(i);
    else
      ++i;
  }
}

// ------------------------------------------------------ static scratch
// Device memory of the allocation-free build (hfx_build_K_noalloc): the
// screening counts and offsets, class-segment bounds, error flags,
// primitive-quartet counters and one quartet-list buffer, in one file-scope
// array.  Each device holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns for the
// device (recorded by hfx_plan, once per device, with the device current).
constexpr size_t kScratchBytes = (size_t)256 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

hfx_status scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(HFX_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return HFX_OK;
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(HFX_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[dev] = ptr;
  return HFX_OK;
}

}  // namespace

hfx_status plan_attach(hfx_plan_s *P) {
  HIPCHK(hipGetDevice(&P->device));
  hfx_status st = scratch_setup(P->device);
  if (st != HFX_OK) return st;
  Batch *B = new Batch();
  st = batch_init(*B, {P});
  if (st != HFX_OK) {
    delete B;
    return st;
  }
  P->self_batch = B;
  return HFX_OK;
}

extern "C" {

hfx_status hfx_build_K(hfx_plan_t plan, const double *d_dev, double *k_dev, uint32_t flags, hfx_build_info *info) {
  if (!valid_plan(plan)) return fail(HFX_ERR_STATE, "invalid or destroyed plan");
  hfx_plan_s &P = *plan;
  return run_batch(*P.self_batch, P.self_batch->w, &d_dev, &k_dev, flags, info);
}

hfx_status hfx_build_K_spin(hfx_plan_t plan, const double *d_alpha, const double *d_beta, double *k_alpha,
                            double *k_beta, uint32_t flags, hfx_build_info *info) {
  if (!valid_plan(plan)) return fail(HFX_ERR_STATE, "invalid or destroyed plan");
  hfx_plan_s &P = *plan;
  if (!P.spin_batch) {
    if (!P.d_Dc_spin) HIPCHK(P.mem.alloc(&P.d_Dc_spin, 2 * (size_t)P.nnz_c));
    if (!P.d_K4_spin) HIPCHK(P.mem.alloc(&P.d_K4_spin, 2 * (size_t)P.nnz_c));
    Batch *B = new Batch();
    hfx_status st = batch_init(*B, {&P}, 2);
    if (st != HFX_OK) {
      delete B;
      return st;
    }
    P.spin_batch = B;
  }
  const double *d[2] = {d_alpha, d_beta};
  double *k[2] = {k_alpha, k_beta};
  return run_batch(*P.spin_batch, P.spin_batch->w, d, k, flags, info);
}

hfx_status hfx_kspace(hfx_plan_t plan, const double *k_dev, int32_t nk, const double *kpts_host, double alpha,
                      double *h_dev) {
  if (!valid_plan(plan)) return fail(HFX_ERR_STATE, "invalid or destroyed plan");
  if (nk < 0 || (nk > 0 && (!kpts_host || !k_dev || !h_dev))) return fail(HFX_ERR_INVALID, "bad arguments");
  if (!std::isfinite(alpha)) return fail(HFX_ERR_INVALID, "alpha must be finite");
  for (int i = 0; i < 3 * nk; ++i)
    if (!std::isfinite(kpts_host[i])) return fail(HFX_ERR_INVALID, "non-finite k-point");
  hfx_plan_s &P = *plan;
  if (!P.d_kpairs) {
    std::vector<int4> kp;
    std::vector<int32_t> img(P.blocks.size()), foff(P.nsh);
    for (size_t b = 0; b < P.blocks.size(); ++b) {
      const hfx_block &x = P.blocks[b];
      img[b] = pack_img8(x.img[0], x.img[1], x.img[2]);
      if (kp.empty() || kp.back().x != x.I || kp.back().y != x.J)
        kp.push_back(make_int4(x.I, x.J, (int)b, 0));
      kp.back().w++;
    }
    int64_t f = 0;
    for (int i = 0; i < P.nsh; ++i) {
      foff[i] = (int32_t)f;
      f += nfunc_host(P.sh_l[i], P.sph);
    }
    HIPCHK(upload(P, &P.d_kpairs, kp));
    HIPCHK(upload(P, &P.d_blk_img, img));
    HIPCHK(upload(P, &P.d_func_off, foff));
    P.n_kpairs = (int)kp.size();
    P.nbf = f;
  }
  if (nk > P.kpts_cap) {
    // k-points are read by the kernel after the copy below; a larger set
    // replaces the buffer once the stream has drained
    HIPCHK(hipStreamSynchronize(P.stream));
    double *d = nullptr;
    HIPCHK(P.mem.alloc(&d, 3 * (size_t)nk));
    P.d_kpts = d;
    P.kpts_cap = nk;
  }
  if (nk == 0) return HFX_OK;
  HIPCHK(hipMemcpyAsync(P.d_kpts, kpts_host, 3 * (size_t)nk * sizeof(double), hipMemcpyHostToDevice, P.stream));
  launch_kspace(P.ds, P.d_kpairs, P.n_kpairs, P.d_blk_img, P.d_blk_off, P.d_func_off, P.sph, k_dev, P.d_kpts, nk, P.nbf,
                -0.5 * alpha, h_dev, P.stream);
  HIPCHK(hipGetLastError());
  // the k-points were copied from pageable host memory: wait so that the
  // caller may reuse them at once
  HIPCHK(hipStreamSynchronize(P.stream));
  return HFX_OK;
}

hfx_status hfx_set_progress(hfx_plan_t plan, hfx_progress_fn fn, void *user) {
  if (!valid_plan(plan)) return fail(HFX_ERR_STATE, "invalid or destroyed plan");
  plan->progress = fn;
  plan->progress_user = user;
  return HFX_OK;
}

hfx_status hfx_set_list_limit(hfx_plan_t plan, int64_t max_quartets) {
  if (!valid_plan(plan)) return fail(HFX_ERR_STATE, "invalid or destroyed plan");
  if (max_quartets < 0) return fail(HFX_ERR_INVALID, "max_quartets must be >= 0");
  hfx_plan_s &P = *plan;
  P.max_list = max_quartets > 0 ? max_quartets : kDefaultMaxList;
  // batches holding the plan pick the new limit up; a longer list than the
  // limit is dropped at the next build (and any graph holding it)
  std::vector<Batch *> bs{P.self_batch};
  if (P.spin_batch) bs.push_back(P.spin_batch);
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (Batch *B : g_batches)
      if (std::find(B->plans.begin(), B->plans.end(), &P) != B->plans.end()) bs.push_back(B);
  }
  for (Batch *B : bs) {
    (void)hipStreamSynchronize(B->stream);
    drop_graph(*B);
    B->max_list = INT64_MAX;
    for (auto *Q : B->plans) B->max_list = std::min(B->max_list, Q->max_list);
    if (B->w.cap > B->max_list || B->w.cap32 > B->max_list) {
      if (B->w.list) (void)hipFree(B->w.list);
      if (B->w.list32) (void)hipFree(B->w.list32);
      B->w.list = B->w.list32 = nullptr;
      B->w.cap = B->w.cap32 = 0;
    }
  }
  return HFX_OK;
}

hfx_status hfx_build_K_noalloc(hfx_plan_t plan, const double *d_dev, double *k_dev, uint32_t flags,
                               hfx_build_info *info) {
  if (!valid_plan(plan)) return fail(HFX_ERR_STATE, "invalid or destroyed plan");
  if (flags & ~HFX_SYNC) return fail(HFX_ERR_INVALID, "hfx_build_K_noalloc takes HFX_SYNC only");
  hfx_plan_s &P = *plan;
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    base = (P.device >= 0 && P.device < kMaxDevices) ? g_scratch_ptr[P.device] : nullptr;
  }
  if (!base) return fail(HFX_ERR_STATE, "no scratch address recorded for the plan's device");
  Batch &B = *P.self_batch;
  const WorkLayout L = work_layout(B.nitems, 1);
  // at least a list of 65536 quartets beside the other arrays
  if (L.total + (size_t)65536 * sizeof(uint64_t) > kScratchBytes)
    return fail(HFX_ERR_INVALID, "the plan's screening work items need " + std::to_string(L.total) +
                                     " bytes of scratch, more than the " + std::to_string(kScratchBytes >> 20) +
                                     " MiB the allocation-free build has");
  Work W;
  work_place(W, (char *)base, L);
  W.fixed = true;
  W.list = W.list32 = (uint64_t *)((char *)base + L.total);
  W.cap = W.cap32 = std::min<int64_t>((int64_t)((kScratchBytes - L.total) / sizeof(uint64_t)), B.max_list);
  return run_batch(B, W, &d_dev, &k_dev, flags, info);
}

hfx_status hfx_build_K_subset(hfx_plan_t plan, const double *d_dev, double *k_dev, const uint64_t *quartets_host,
                              int64_t n) {
  if (!valid_plan(plan)) return fail(HFX_ERR_STATE, "invalid or destroyed plan");
  if (!d_dev || !k_dev || n < 0 || (n > 0 && !quartets_host)) return fail(HFX_ERR_INVALID, "bad arguments");
  hfx_plan_s &P = *plan;
  if (!P.schwarz_done) {
    hfx_status st = run_schwarz(P);
    if (st != HFX_OK) return st;
  }
  // class segments on the host
  const int64_t npairs = (int64_t)P.pr_info.size();
  std::vector<std::vector<uint64_t>> by(kNQuartetClass);
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t q = quartets_host[i];
    const int64_t bra = (int64_t)(q & 0xFFFFFFull), ket = (int64_t)((q >> 24) & 0xFFFFFFull);
    if (bra >= npairs || ket >= npairs) return fail(HFX_ERR_INVALID, "quartet pair index out of range");
    const int cb = pair_class(P.sh_l[P.pr_info[bra].x], P.sh_l[P.pr_info[bra].y]);
    const int ck = pair_class(P.sh_l[P.pr_info[ket].x], P.sh_l[P.pr_info[ket].y]);
    if (cb < ck) return fail(HFX_ERR_INVALID, "quartet with bra pair class below its ket pair class");
    by[region_of(cb, ck)].push_back(q);
  }
  // mixed precision: a quartet whose Schwarz product is below the class's
  // FP32 cutoff goes to the class's FP32 kernel, as in a full build
  std::vector<double> Q;
  if (P.precision == HFX_MIXED) {
    Q.resize(npairs);
    HIPCHK(hipMemcpyAsync(Q.data(), P.d_pr_Q, npairs * sizeof(double), hipMemcpyDeviceToHost, P.stream));
    HIPCHK(hipStreamSynchronize(P.stream));
  }
  std::vector<uint64_t> list;
  std::vector<int64_t> seg(4 * kNQuartetClass);  // [region][FP64 part, FP32 part] bounds
  for (int r = 0; r < kNQuartetClass; ++r)
    for (int part = 0; part < 2; ++part) {
      seg[4 * r + 2 * part] = (int64_t)list.size();
      for (uint64_t q : by[r]) {
        bool f32 = false;
        if (!Q.empty()) {
          const double qq = Q[q & 0xFFFFFFull] * Q[(q >> 24) & 0xFFFFFFull];
          f32 = qq < P.ds.fp32_cut[r];
        }
        if (f32 == (part == 1)) list.push_back(q);
      }
      seg[4 * r + 2 * part + 1] = (int64_t)list.size();
    }
  DevMem mem;
  uint64_t *d_list = nullptr;
  int64_t *d_seg = nullptr;
  unsigned long long *d_np = nullptr;
  HIPCHK(mem.alloc(&d_list, list.size() + 1));
  HIPCHK(mem.alloc(&d_seg, seg.size()));
  HIPCHK(mem.alloc(&d_np, kNQuartetClass));
  const hipStream_t st = P.stream;
  if (!list.empty()) HIPCHK(hipMemcpyAsync(d_list, list.data(), list.size() * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_seg, seg.data(), seg.size() * 8, hipMemcpyHostToDevice, st));
  launch_zero_u64(d_np, kNQuartetClass, st);
  launch_zero_u64(P.d_pglob, 1, st);
  launch_density(P.ds, (int64_t)P.blocks.size(), P.d_blk_IJ, P.d_blk_off, P.d_partner, P.d_canon, P.sph, d_dev, P.d_Dc, false,
                 st);
  launch_zero(P.d_K4, P.nnz_c, st);
  for (int cb = 0; cb < kNPairClass; ++cb)
    for (int ck = 0; ck <= cb; ++ck) {
      const int r = region_of(cb, ck);
      for (int part = 0; part < 2; ++part) {
        const int64_t cnt = seg[4 * r + 2 * part + 1] - seg[4 * r + 2 * part];
        if (cnt == 0) continue;
        SegLaunch L{P.d_sys1, 1, d_seg + 4 * r + 2 * part, d_list, d_np + r, cnt, st,
                    part ? P.grid32[r] : P.grid[r]};
        launch_variant(part ? P.kern32[r] : P.kern[r], cb, ck, P.op, P.coop[r], L);
      }
    }
  launch_finalize(P.ds, (int64_t)P.blocks.size(), P.d_blk_IJ, P.d_blk_off, P.d_partner, P.sph, P.d_K4, k_dev, st);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  mem.release();
  HIPCHK(e);
  return HFX_OK;
}

hfx_status hfx_screen_count(hfx_plan_t plan, const double *d_dev, int64_t *n64, int64_t *n32) {
  if (!valid_plan(plan)) return fail(HFX_ERR_STATE, "invalid or destroyed plan");
  if (!d_dev || !n64) return fail(HFX_ERR_INVALID, "NULL argument");
  hfx_plan_s &P = *plan;
  if (!P.schwarz_done) {
    hfx_status st = run_schwarz(P);
    if (st != HFX_OK) return st;
  }
  Batch &B = *P.self_batch;
  Work &W = B.w;
  launch_zero_u64(P.d_pglob, 1, B.stream);
  launch_density(P.ds, (int64_t)P.blocks.size(), P.d_blk_IJ, P.d_blk_off, P.d_partner, P.d_canon, P.sph, d_dev, P.d_Dc, false,
                 B.stream);
  launch_zero_i32(W.err, 2, B.stream);
  int64_t tot[2] = {0, 0};
  for (int pass = 0; pass < (B.mixed ? 2 : 1); ++pass) {
    const int mode = B.mixed ? 1 + pass : 0;
    launch_screen(B.d_sys, B.d_items, B.nitems, W.counts, W.offsets, nullptr, 0, 0, W.err, false, mode, B.stream);
    HIPCHK(scan_counts(W.counts, W.offsets, B.nitems, W.tiles, B.stream));
    HIPCHK(hipMemcpyAsync(&tot[pass], W.offsets + B.nitems, sizeof(int64_t), hipMemcpyDeviceToHost, B.stream));
  }
  HIPCHK(hipStreamSynchronize(B.stream));
  hfx_status st = check_err(B, W, nullptr);
  if (st != HFX_OK) return st;
  *n64 = tot[0];
  if (n32) *n32 = tot[1];
  return HFX_OK;
}

hfx_status hfx_autotune(hfx_plan_t plan, const double *d_dev, double *k_dev, int64_t max_quartets,
                        hfx_tune_report *report) {
  if (!valid_plan(plan)) return fail(HFX_ERR_STATE, "invalid or destroyed plan");
  if (!d_dev || !k_dev) return fail(HFX_ERR_INVALID, "D or K pointer is NULL");
  hfx_plan_s &P = *plan;
  if (report) {
    std::memset(report, 0, sizeof(*report));
    for (int r = 0; r < kNQuartetClass; ++r) report->chosen[r] = report->chosen32[r] = -1;
  }
  // an eager build fills the lists the candidates are timed on
  hfx_status st = hfx_build_K(plan, d_dev, k_dev, HFX_SYNC, nullptr);
  if (st != HFX_OK) return st;
  Batch &B = *P.self_batch;
  if (B.n_chunks > 0)
    return fail(HFX_ERR_UNSUPPORTED, "autotune needs the whole quartet list: raise the plan's list limit");
  int64_t *d_seg2 = nullptr;
  HIPCHK(hipMalloc((void **)&d_seg2, 2 * sizeof(int64_t)));
  for (int cb = 0; cb < kNPairClass && st == HFX_OK; ++cb)
    for (int ck = 0; ck <= cb && st == HFX_OK; ++ck) {
      st = tune_class(B, cb, ck, false, max_quartets, d_seg2, report);
      if (st == HFX_OK && B.mixed) st = tune_class(B, cb, ck, true, max_quartets, d_seg2, report);
    }
  (void)hipStreamSynchronize(B.stream);
  (void)hipFree(d_seg2);
  if (st != HFX_OK) return st;
  drop_graphs_of(&P);
  // the timed launches accumulated into K4: one clean build with the choices
  return hfx_build_K(plan, d_dev, k_dev, HFX_SYNC, nullptr);
}

hfx_status hfx_build_K_multi(int32_t n, const hfx_plan_t *plans, const double *const *d_dev, double *const *k_dev,
                             uint32_t flags, hfx_build_info *info) {
  if (n < 0 || (n > 0 && (!plans || !d_dev || !k_dev))) return fail(HFX_ERR_INVALID, "bad arguments");
  if (info) std::memset(info, 0, sizeof(*info));
  if (n == 0) return HFX_OK;
  for (int i = 0; i < n; ++i) {
    if (!valid_plan(plans[i])) return fail(HFX_ERR_STATE, "invalid or destroyed plan");
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return fail(HFX_ERR_INVALID, "a plan appears twice in one multi build");
  }
  // one fused batch per operator (the ERI kernels are specialised on it)
  for (int op = 0; op <= 1; ++op) {
    std::vector<hfx_plan_s *> ps;
    std::vector<const double *> ds;
    std::vector<double *> ks;
    for (int i = 0; i < n; ++i)
      if (plans[i]->op == op) {
        ps.push_back(plans[i]);
        ds.push_back(d_dev[i]);
        ks.push_back(k_dev[i]);
      }
    if (ps.empty()) continue;
    Batch *B = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_batch_mu);
      for (Batch *b : g_batches)
        if (b->plans == ps) B = b;
    }
    if (!B) {
      B = new Batch();
      hfx_status st = batch_init(*B, ps);
      if (st != HFX_OK) {
        delete B;
        return st;
      }
      std::lock_guard<std::mutex> lk(g_batch_mu);
      // a plan belongs to at most one cached batch: a new plan list (the
      // serving mix changes from step to step) replaces every cached batch
      // it shares a plan with, so their lists do not pile up on the device
      for (size_t i = 0; i < g_batches.size();) {
        bool shares = false;
        for (auto *P : ps) shares |= std::find(g_batches[i]->plans.begin(), g_batches[i]->plans.end(), P) !=
                                     g_batches[i]->plans.end();
        if (shares)
          delete_batch_locked(i);
        else
          ++i;
      }
      g_batches.push_back(B);
    }
    hfx_build_info sub;
    hfx_status st = run_batch(*B, B->w, ds.data(), ks.data(), flags, info ? &sub : nullptr);
    if (st != HFX_OK) return st;
    if (info) {
      info->n_quartets += sub.n_quartets;
      info->n_prim_quartets += sub.n_prim_quartets;
      info->n_fp32_quartets += sub.n_fp32_quartets;
      info->flops += sub.flops;
      info->ms_density += sub.ms_density;
      info->ms_screen += sub.ms_screen;
      info->ms_eri += sub.ms_eri;
      info->ms_finalize += sub.ms_finalize;
      info->ms_total += sub.ms_total;
      info->n_chunks += sub.n_chunks;
      for (int r = 0; r < HFX_N_CLASSES; ++r) {
        info->n_quartets_class[r] += sub.n_quartets_class[r];
        info->ms_class[r] += sub.ms_class[r];
        info->flops_class[r] += sub.flops_class[r];
      }
    }
  }
  return HFX_OK;
}

hfx_status hfx_export(hfx_plan_t plan, int32_t what, void *host, int64_t *n) {
  if (!valid_plan(plan)) return fail(HFX_ERR_STATE, "invalid or destroyed plan");
  if (!n) return fail(HFX_ERR_INVALID, "n is NULL");
  hfx_plan_s &P = *plan;
  Batch *B = P.self_batch;
  switch (what) {
    case 0:
      *n = (int64_t)P.blocks.size();
      if (host && *n) {
        HIPCHK(hipStreamSynchronize(P.stream));
        HIPCHK(hipMemcpy(host, P.d_pmax, *n * 8, hipMemcpyDeviceToHost));
      }
      return HFX_OK;
    case 1:
    case 5: {
      const bool f32 = what == 5;
      if (B->have_counts && B->n_chunks > 0)
        return fail(HFX_ERR_STATE, "the last build evaluated its quartet list in chunks: no whole list to export");
      *n = B->have_counts ? (f32 ? B->nq32 : B->nq64) : 0;
      if (host && *n) {
        HIPCHK(hipStreamSynchronize(P.stream));
        HIPCHK(hipMemcpy(host, f32 ? B->w.list32 : B->w.list, *n * 8, hipMemcpyDeviceToHost));
      }
      return HFX_OK;
    }
    case 2: {
      *n = (int64_t)P.pr_info.size();
      if (host) {
        int32_t *o = (int32_t *)host;
        for (int64_t q = 0; q < *n; ++q) {
          int a, b, c;
          unpack_img8(P.pr_info[q].z, a, b, c);
          const int cls = pair_class(P.sh_l[P.pr_info[q].x], P.sh_l[P.pr_info[q].y]);
          int32_t row[6] = {P.pr_info[q].x, P.pr_info[q].y, a, b, c, cls};
          std::memcpy(o + 6 * q, row, sizeof(row));
        }
      }
      return HFX_OK;
    }
    case 3:
      *n = (int64_t)P.pr_info.size();
      if (host && *n) {
        HIPCHK(hipStreamSynchronize(P.stream));
        HIPCHK(hipMemcpy(host, P.d_pr_Q, *n * 8, hipMemcpyDeviceToHost));
      }
      return HFX_OK;
    default:
      return fail(HFX_ERR_INVALID, "unknown export");
  }
}

hfx_status hfx_plan_destroy(hfx_plan_t plan) {
  if (!valid_plan(plan)) return fail(HFX_ERR_STATE, "invalid or destroyed plan");
  {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    g_plans.erase(plan);
  }
  drop_batches_of(plan);
  (void)hipStreamSynchronize(plan->stream);
  delete plan->self_batch;
  plan->self_batch = nullptr;
  delete plan->spin_batch;
  plan->spin_batch = nullptr;
  plan->mem.release();
  plan->magic = 0;
  delete plan;
  return HFX_OK;
}

}  // extern "C"
