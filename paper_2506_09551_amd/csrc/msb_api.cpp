// C ABI of the multi-shift BiCG library: context, operators, ground state,
// the multi-shift solve, the coherent site sum and the continued-fraction
// spectrum.  Host code only; every vector operation runs in the HIP kernels of
// the k_*.hip files.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <limits>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "msb_internal.h"

namespace msb {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
msb_status fail(msb_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

// Grow-only device arena owned by the context; carved per call.
class Arena {
 public:
  explicit Arena(msb_ctx* c) : ctx_(c) {}
  void reserve(size_t bytes) { need_ += align(bytes); }
  hipError_t commit() {
    if (ctx_->ws_size < need_) {
      if (ctx_->ws) {
        hipError_t e = hipFree(ctx_->ws);
        if (e != hipSuccess) return e;
        ctx_->ws = nullptr;
        ctx_->ws_size = 0;
      }
      hipError_t e = hipMalloc(&ctx_->ws, need_);
      if (e != hipSuccess) return e;
      ctx_->ws_size = need_;
    }
    off_ = 0;
    return hipSuccess;
  }
  template <typename T>
  T* take(size_t bytes) {
    if (off_ + align(bytes) > ctx_->ws_size) {   // a reserve/take mismatch: never hand out memory past the end
      overflow_ = true;
      return nullptr;
    }
    T* p = reinterpret_cast<T*>(static_cast<char*>(ctx_->ws) + off_);
    off_ += align(bytes);
    return p;
  }
  size_t needed() const { return need_; }
  bool overflow() const { return overflow_; }
  static size_t align(size_t b) { return (b + 255) & ~size_t(255); }

 private:
  msb_ctx* ctx_;
  size_t need_ = 0;
  size_t off_ = 0;
  bool overflow_ = false;
};

static size_t elem_bytes(Elem e) { return e == Elem::C128 ? 16 : (e == Elem::C64 ? 8 : 8); }

static bool valid_prec(msb_prec p) { return p == MSB_C128 || p == MSB_C64; }

static msb_status make_sysdev(const msb_ctx* ctx, const msb_system& s, double d_re, double d_im,
                              bool with_core, SysDev& out) {
  out = SysDev();
  out.U = std::isnan(s.U) ? ctx->U : s.U;
  out.Uc = with_core ? s.Uc : 0.0;
  out.core = with_core ? s.core_site : -1;
  if (with_core && (s.core_site < -1 || s.core_site >= ctx->L))
    return fail(MSB_EINVAL, "core_site out of range");
  out.d_re = d_re;
  out.d_im = d_im;
  if (s.n_amp < 0 || s.n_amp > MSB_MAX_BOND_TYPES) return fail(MSB_EINVAL, "n_amp out of range");
  for (int t = 0; t < MSB_MAX_BOND_TYPES; ++t)
    out.amp[t] = (t < s.n_amp) ? s.t_amp[t] : ctx->type_amp[t];
  if (!std::isfinite(out.U) || !std::isfinite(out.Uc) || !std::isfinite(d_re) || !std::isfinite(d_im))
    return fail(MSB_EINVAL, "non-finite system parameter");
  return MSB_OK;
}

// A system's A is symmetric unless a directed bond type and its reverse have
// different amplitudes.
static bool sysdev_symmetric(const msb_ctx* ctx, const SysDev& s) {
  for (int t = 0; t < ctx->n_types; ++t)
    if (s.amp[t] != s.amp[ctx->type_partner[t]]) return false;
  return true;
}
// The same system with every directed type's amplitude swapped with its
// reverse: the apply then computes A^T x.
static SysDev sysdev_transpose(const msb_ctx* ctx, const SysDev& s) {
  SysDev t = s;
  for (int q = 0; q < ctx->n_types; ++q) t.amp[q] = s.amp[ctx->type_partner[q]];
  return t;
}

// ---- apply launch-shape autotuner -------------------------------------------
// Shapes are tuned per system count up to kTuneMaxSys (the grid and the L2
// footprint change with it); larger batches share the kTuneMaxSys entry.
constexpr int kTuneMaxSys = 16;
static int shape_class(int nsys) { return std::max(1, std::min(nsys, kTuneMaxSys)); }

struct DevBuf {               // scratch device memory released on scope exit
  void* p = nullptr;
  ~DevBuf() { if (p) (void)hipFree(p); }
};

static ApplyArgs apply_args(const msb_ctx* ctx, const SysDev* sys, int nsys, const void* x, void* v);
// up-spin rows of the LDS panel pass for element type e (0: not available)
static int pan_rows(const msb_ctx* ctx, Elem e) {
  return (e != Elem::R64 && ctx->d_ell_up && ctx->up.n < 32768) ? ctx->up.n : 0;
}
constexpr int kMaxCand = 192;   // compiled shapes x passes x row orders
constexpr int kSeedParts = 2;   // streams a recurred seed batch is split over (at most 4; 2 measured best)
constexpr int kSeedPartMin = 4; // systems per part at least

// Times every usable shape for (e, shape_class(nsys), mode) on constant vectors
// and keeps the fastest in the context.  `table` (optional) receives every
// measurement.
static msb_status tune_shapes(msb_ctx* ctx, Elem e, int nsys, hipStream_t st,
                              std::vector<std::pair<ApplyShape, double>>* table, int mode = kModePlain) {
  const int n = shape_class(nsys);
  const size_t eb = elem_bytes(e);
  ApplyShape cand[kMaxCand];
  int nc = apply_candidates(ctx->dn.n, eb, n, ctx->lds_max, ctx->up.max_hops, pan_rows(ctx, e), eb, cand, kMaxCand);
  if (mode == kModeResid) {      // the residual check runs single-pass shapes only
    int k = 0;
    for (int i = 0; i < nc; ++i)
      if (cand[i].passes == 1) cand[k++] = cand[i];
    nc = k;
  }
  if (nc == 0) return fail(MSB_EINVAL, "autotune: no compiled apply shape covers a row");
  const size_t vb = (size_t)n * ctx->D * eb;
  const int nbx = apply_nbx(ctx->up.n, n);
  const bool self = mode == kModeSelf;
  DevBuf x, y, ds, aux, part, red, zi, bt;
  bool ok = hipMalloc(&x.p, vb) == hipSuccess && hipMalloc(&y.p, vb) == hipSuccess &&
            hipMalloc(&ds.p, n * sizeof(SysDev)) == hipSuccess;
  if (ok && self)
    ok = hipMalloc(&zi.p, (size_t)n * sizeof(int)) == hipSuccess &&
         hipMalloc(&bt.p, (size_t)n * 2 * sizeof(double)) == hipSuccess;
  if (ok && mode != kModePlain)
    ok = hipMalloc(&part.p, (size_t)n * nbx * 4 * sizeof(double)) == hipSuccess &&
         hipMalloc(&red.p, (size_t)n * 4 * sizeof(double)) == hipSuccess;
  if (ok && mode == kModeResid) ok = hipMalloc(&aux.p, (size_t)n * ctx->D * 16) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    return fail(MSB_ENOMEM, "autotune: scratch vectors do not fit");
  }
  msb_system dflt;
  std::memset(&dflt, 0, sizeof(dflt));
  dflt.core_site = -1;
  dflt.U = std::numeric_limits<double>::quiet_NaN();
  SysDev hs;
  msb_status r = make_sysdev(ctx, dflt, 0.0, -1.0, false, hs);
  if (r != MSB_OK) return r;
  std::vector<SysDev> h(n, hs);
  MSB_HIP(hipMemcpyAsync(ds.p, h.data(), n * sizeof(SysDev), hipMemcpyHostToDevice, st));
  // nonzero, finite operands (every float64 0x3F3F... = 4.8e-4, every float32
  // 0x3F3F3F3F = 0.75): the timing then sees ordinary data
  MSB_HIP(hipMemsetAsync(x.p, 0x3F, vb, st));
  if (aux.p) MSB_HIP(hipMemsetAsync(aux.p, 0x3F, (size_t)n * ctx->D * 16, st));
  ApplyArgs a = apply_args(ctx, (const SysDev*)ds.p, n, x.p, y.p);
  if (mode != kModePlain) {
    a.partials = (double*)part.p;
    a.red = (double*)red.p;
    a.aux = (mode == kModeResid) ? aux.p : x.p;     // sigma reads a residual, the check reads E
    // the check runs over the shifts of a system, which share E
    if (mode == kModeResid) a.aux_div = n;
  }
  if (self) {
    // a one-slot bank (x itself), every system active at iteration 0, and a
    // nonzero beta so the old v is read and added as in the solve
    MSB_HIP(hipMemsetAsync(zi.p, 0, (size_t)n * sizeof(int), st));
    MSB_HIP(hipMemsetAsync(bt.p, 0x3F, (size_t)n * 2 * sizeof(double), st));
    MSB_HIP(hipMemsetAsync(y.p, 0x3F, vb, st));
    a.beta = (const double*)bt.p;
    a.beta_stride = 2;
    a.aux_m = (const int*)zi.p;
    a.aux_base = (const int*)zi.p;
    a.aux_cap = 1;
    a.status = (const int*)zi.p;
    a.status_stride = 1;
  }
  hipEvent_t e0, e1;
  MSB_HIP(hipEventCreate(&e0));
  MSB_HIP(hipEventCreate(&e1));
  ApplyShape best{0, 0, 0, 0, 0};
  double best_ms = 0;
  hipError_t err = hipSuccess;
  // one warm-up launch, one timed launch; a shape 1.5x slower than the best
  // so far stops there, the others are timed over four more launches
  auto timed = [&](int reps, double* out) -> hipError_t {
    hipError_t r = hipEventRecord(e0, st);
    for (int k = 0; k < reps && r == hipSuccess; ++k) r = launch_apply(e, mode, a, st);
    if (r == hipSuccess) r = hipEventRecord(e1, st);
    if (r == hipSuccess) r = hipEventSynchronize(e1);
    float ms = 0;
    if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
    *out = ms / reps;
    return r;
  };
  for (int i = 0; i < nc && err == hipSuccess; ++i) {
    a.shape = cand[i];
    err = launch_apply(e, mode, a, st);
    double m = 0;
    if (err == hipSuccess) err = timed(1, &m);
    if (err == hipSuccess && !(best.blk != 0 && m > 1.5 * best_ms)) err = timed(4, &m);
    if (err != hipSuccess) break;
    if (table) table->push_back({cand[i], m});
    if (best.blk == 0 || m < best_ms) {
      best = cand[i];
      best_ms = m;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  MSB_HIP(err);
  ctx->shapes[std::make_tuple((int)e, n, mode)] = best;
  return MSB_OK;
}

// Shape to use for an apply of nsys systems: the tuned or pinned one, tuning
// now if allowed; {0,0,0} (the default shape) if tuning is off or failed.
static ApplyShape shape_for(msb_ctx* ctx, Elem e, int nsys, hipStream_t st, bool tune,
                            int mode = kModePlain) {
  const auto key = std::make_tuple((int)e, shape_class(nsys), mode);
  auto it = ctx->shapes.find(key);
  if (it != ctx->shapes.end()) return it->second;
  if (!tune || tune_shapes(ctx, e, nsys, st, nullptr, mode) != MSB_OK) {
    (void)hipGetLastError();
    return ApplyShape{0, 0, 0, 0, 0};
  }
  return ctx->shapes[key];
}

static ApplyArgs apply_args(const msb_ctx* ctx, const SysDev* sys, int nsys, const void* x, void* v) {
  ApplyArgs a;
  std::memset(&a, 0, sizeof(a));
  a.T = ctx->tables();
  a.sys = sys;
  a.x = x;
  a.v = v;
  a.aux = nullptr;
  a.aux_div = 1;
  a.status = nullptr;
  a.status_stride = 0;
  a.D = ctx->D;
  a.lds_max = ctx->lds_max;
  a.rows_per_xcd = apply_rows_per_xcd(ctx->up.n);
  a.nbx = apply_nbx(ctx->up.n, nsys);
  a.nsys = nsys;
  return a;
}

}  // namespace msb

using namespace msb;

// ---- the fixed staging array of msb_apply_noalloc ---------------------------
// The per-system parameters of an allocation-free apply are staged here: one
// copy of the array per GPU, kept until the process ends.  Host code never
// passes the array's name to a kernel or a copy; it uses the device address
// looked up once per device (scratch_setup, called by msb_create with that
// device current).
static __device__ __align__(256) SysDev scratch[MSB_NOALLOC_MAX_SYS];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

static void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

// =============================================================================
extern "C" const char* msb_last_error(void) { return g_err.c_str(); }

extern "C" int msb_device_ok(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return 0;
  return std::strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
}

extern "C" msb_status msb_stream_create(void** out) {
  if (!out) return fail(MSB_EINVAL, "msb_stream_create: null argument");
  *out = nullptr;
  hipStream_t s = nullptr;
  MSB_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  *out = (void*)s;
  return MSB_OK;
}

extern "C" msb_status msb_stream_destroy(void* stream) {
  if (!stream) return fail(MSB_EINVAL, "msb_stream_destroy: null stream");
  MSB_HIP(hipStreamSynchronize((hipStream_t)stream));
  MSB_HIP(hipStreamDestroy((hipStream_t)stream));
  return MSB_OK;
}

// Padded, transposed copy of one spin's hop lists, one table per bond type,
// four hops to a 64-bit word: ell[t][g][c] holds hops 4g .. 4g+3 of state c,
// each 16 bits = target | (even parity ? 0x8000 : 0); padding = n (the zero
// element after every staged row or panel).  k_type[t] = words of type t.
static hipError_t upload_ell(const SpinTable& sp, int n_types, int* k_type, uint64_t** dst) {
  const int n = sp.n;
  std::vector<uint64_t> ell;
  for (int t = 0; t < n_types; ++t) {
    int kt = 0;
    for (int c = 0; c < n; ++c) {
      int cnt = 0;
      for (uint32_t k = sp.off[c]; k < sp.off[c + 1]; ++k) cnt += ((sp.hop[k] >> 1) & 127u) == (uint32_t)t;
      kt = std::max(kt, cnt);
    }
    const int kq = (kt + 3) / 4;
    k_type[t] = kq;
    std::vector<uint16_t> ent((size_t)kq * 4 * n, (uint16_t)n);
    for (int c = 0; c < n; ++c) {
      int j = 0;
      for (uint32_t k = sp.off[c]; k < sp.off[c + 1]; ++k) {
        const uint32_t h = sp.hop[k];
        if (((h >> 1) & 127u) != (uint32_t)t) continue;
        ent[(size_t)j * n + c] = (uint16_t)((h >> 16) | ((h & 1u) ? 0u : 0x8000u));
        ++j;
      }
    }
    for (int g = 0; g < kq; ++g)
      for (int c = 0; c < n; ++c) {
        uint64_t w = 0;
        for (int j = 0; j < 4; ++j) w |= (uint64_t)ent[(size_t)(4 * g + j) * n + c] << (16 * j);
        ell.push_back(w);
      }
  }
  const size_t bytes = std::max<size_t>(ell.size(), 1) * sizeof(uint64_t);
  hipError_t e = hipMalloc(dst, bytes);
  if (e == hipSuccess && !ell.empty())
    e = hipMemcpy(*dst, ell.data(), ell.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
  return e;
}

// The up-spin hops of the LDS panel pass in row-count order: rows sorted by
// their number of hops (descending) and dealt to wavefronts of 64 positions,
// each wavefront's hop words padded only to its own longest row.  perm[p]
// is the row at position p (n_up past the last row); woff[w] .. woff[w + 1]
// are the words of wavefront w; word q of position p holds four hops as
// 16-bit entries = target | type << 14 | (even parity ? 0x8000 : 0), padding
// n_up.  Needs n_up < 16384 and at most two bond types (else not built).
static hipError_t upload_pan_table(const SpinTable& sp, int n_types, uint32_t** d_perm, int** d_woff,
                                   uint64_t** d_ell) {
  const int n = sp.n;
  if (n >= 16384 || n_types > 2) return hipSuccess;
  std::vector<uint32_t> perm(n);
  std::iota(perm.begin(), perm.end(), 0u);
  std::stable_sort(perm.begin(), perm.end(), [&](uint32_t x, uint32_t y) {
    return sp.off[x + 1] - sp.off[x] > sp.off[y + 1] - sp.off[y];
  });
  const int n_waves = (n + kWave - 1) / kWave;
  perm.resize((size_t)n_waves * kWave, (uint32_t)n);
  std::vector<int> woff(n_waves + 1, 0);
  std::vector<uint64_t> ell;
  for (int w = 0; w < n_waves; ++w) {
    int mx = 0;
    for (int l = 0; l < kWave; ++l) {
      const uint32_t u = perm[(size_t)w * kWave + l];
      if (u < (uint32_t)n) mx = std::max<int>(mx, (int)(sp.off[u + 1] - sp.off[u]));
    }
    const int nw = (mx + 3) / 4;
    woff[w + 1] = woff[w] + nw;
    for (int q = 0; q < nw; ++q)
      for (int l = 0; l < kWave; ++l) {
        const uint32_t u = perm[(size_t)w * kWave + l];
        uint64_t word = 0;
        for (int j = 0; j < 4; ++j) {
          uint32_t ent = (uint32_t)n;
          const uint32_t k = 4 * q + j;
          if (u < (uint32_t)n && k < sp.off[u + 1] - sp.off[u]) {
            const uint32_t h = sp.hop[sp.off[u] + k];
            ent = (h >> 16) | (((h >> 1) & 127u) << 14) | ((h & 1u) ? 0u : 0x8000u);
          }
          word |= (uint64_t)ent << (16 * j);
        }
        ell.push_back(word);
      }
  }
  hipError_t e = hipMalloc(d_perm, perm.size() * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemcpy(*d_perm, perm.data(), perm.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(d_woff, woff.size() * sizeof(int));
  if (e == hipSuccess) e = hipMemcpy(*d_woff, woff.data(), woff.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(d_ell, std::max<size_t>(ell.size(), 1) * sizeof(uint64_t));
  if (e == hipSuccess && !ell.empty())
    e = hipMemcpy(*d_ell, ell.data(), ell.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
  return e;
}

extern "C" msb_status msb_create(const msb_model* m, msb_ctx** out) {
  if (!m || !out) return fail(MSB_EINVAL, "msb_create: null argument");
  *out = nullptr;
  if (m->n_sites < 2 || m->n_sites > 20) return fail(MSB_EINVAL, "n_sites must lie in [2, 20]");
  if (m->n_up < 0 || m->n_up > m->n_sites || m->n_dn < 0 || m->n_dn > m->n_sites)
    return fail(MSB_EINVAL, "electron numbers must lie in [0, n_sites]");
  if (m->n_bonds < 0 || (m->n_bonds > 0 && (!m->bond_i || !m->bond_j || !m->bond_t)))
    return fail(MSB_EINVAL, "bond arrays missing");
  if (!std::isfinite(m->U)) return fail(MSB_EINVAL, "U must be finite");
  std::vector<int> bi, bj, bt_f, bt_b;
  std::vector<double> amps;                       // amplitude of each type
  std::vector<std::pair<double, double>> classes; // directed: (t, t_rev) of class k = types 2k, 2k+1
  const bool directed = m->bond_t_rev != nullptr;
  for (int b = 0; b < m->n_bonds; ++b) {
    const int i = m->bond_i[b], j = m->bond_j[b];
    const double t = m->bond_t[b];
    const double tr = directed ? m->bond_t_rev[b] : t;
    if (i < 0 || j < 0 || i >= m->n_sites || j >= m->n_sites || i == j)
      return fail(MSB_EINVAL, "bond " + std::to_string(b) + " has invalid sites");
    if (!std::isfinite(t) || !std::isfinite(tr)) return fail(MSB_EINVAL, "bond amplitude must be finite");
    int tf = -1, tb = -1;
    if (directed) {
      int k = -1;
      for (size_t q = 0; q < classes.size(); ++q)
        if (classes[q].first == t && classes[q].second == tr) k = (int)q;
      if (k < 0) {
        if (2 * ((int)classes.size() + 1) > MSB_MAX_BOND_TYPES)
          return fail(MSB_EINVAL, "too many distinct directed bond classes");
        classes.push_back({t, tr});
        amps.push_back(t);
        amps.push_back(tr);
        k = (int)classes.size() - 1;
      }
      tf = 2 * k;
      tb = 2 * k + 1;
    } else {
      for (size_t q = 0; q < amps.size(); ++q)
        if (amps[q] == t) tf = (int)q;
      if (tf < 0) {
        if ((int)amps.size() >= MSB_MAX_BOND_TYPES) return fail(MSB_EINVAL, "too many distinct bond amplitudes");
        amps.push_back(t);
        tf = (int)amps.size() - 1;
      }
      tb = tf;
    }
    bi.push_back(i);
    bj.push_back(j);
    bt_f.push_back(tf);
    bt_b.push_back(tb);
  }
  msb_ctx* c = new msb_ctx();
  c->L = m->n_sites;
  c->n_up = m->n_up;
  c->n_dn = m->n_dn;
  c->U = m->U;
  c->n_types = (int)amps.size();
  for (size_t q = 0; q < amps.size(); ++q) c->type_amp[q] = amps[q];
  for (int q = 0; q < MSB_MAX_BOND_TYPES; ++q) c->type_partner[q] = directed ? (q ^ 1) : q;
  std::string err;
  if (!build_spin_table(m->n_sites, m->n_up, bi, bj, bt_f, bt_b, c->up, err) ||
      !build_spin_table(m->n_sites, m->n_dn, bi, bj, bt_f, bt_b, c->dn, err)) {
    delete c;
    return fail(MSB_EINVAL, err);
  }
  c->D = (int64_t)c->up.n * c->dn.n;
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) {
    int lds = 0;
    e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device);
    if (e == hipSuccess && lds > 0) c->lds_max = (size_t)lds;
  }
  if (e == hipSuccess) e = scratch_setup(c->device);   // staging array of msb_apply_noalloc
  if (e == hipSuccess && ((size_t)(c->dn.n + 1) * 8 > c->lds_max || c->dn.n >= 32768)) {
    const int c_dn_n = c->dn.n;
    delete c;
    return fail(MSB_EINVAL, "msb_create: a down-spin row of " + std::to_string(c_dn_n) +
                                " states does not fit one workgroup's LDS");
  }
  auto upload = [&](uint32_t** dst, const std::vector<uint32_t>& src) -> hipError_t {
    const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(uint32_t);
    hipError_t r = hipMalloc(dst, bytes);
    if (r != hipSuccess) return r;
    if (!src.empty()) r = hipMemcpy(*dst, src.data(), src.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    return r;
  };
  if (e == hipSuccess) e = upload(&c->d_conf_up, c->up.conf);
  if (e == hipSuccess) e = upload(&c->d_conf_dn, c->dn.conf);
  if (e == hipSuccess) e = upload(&c->d_off_up, c->up.off);
  if (e == hipSuccess) e = upload(&c->d_off_dn, c->dn.off);
  if (e == hipSuccess) e = upload(&c->d_hop_up, c->up.hop);
  if (e == hipSuccess) e = upload(&c->d_hop_dn, c->dn.hop);
  if (e == hipSuccess) e = upload_ell(c->dn, c->n_types, c->k_type_dn, &c->d_ell_dn);
  // the up-spin table of the same form feeds the column-panel pass (rows of
  // one panel staged in LDS); up-spin ranks fit its 15-bit targets
  if (e == hipSuccess && c->up.n < 32768) e = upload_ell(c->up, c->n_types, c->k_type_up, &c->d_ell_up);
  if (e == hipSuccess) e = upload_pan_table(c->up, c->n_types, &c->d_pan_perm, &c->d_pan_woff, &c->d_pan_ell);
  if (e == hipSuccess) e = upload(&c->d_order_up, c->up.order);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->solve_stream, hipStreamNonBlocking);
  for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipStreamCreateWithFlags(&c->part_stream[k], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(&c->d_small, 4096 * sizeof(double));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    msb_destroy(c);
    return fail(MSB_EHIP, std::string("msb_create: ") + hipGetErrorString(e));
  }
  *out = c;
  return MSB_OK;
}

extern "C" void msb_destroy(msb_ctx* c) {
  if (!c) return;
  (void)hipFree(c->d_conf_up);
  (void)hipFree(c->d_conf_dn);
  (void)hipFree(c->d_off_up);
  (void)hipFree(c->d_off_dn);
  (void)hipFree(c->d_hop_up);
  (void)hipFree(c->d_hop_dn);
  (void)hipFree(c->d_ell_dn);
  (void)hipFree(c->d_ell_up);
  (void)hipFree(c->d_pan_perm);
  (void)hipFree(c->d_pan_woff);
  (void)hipFree(c->d_pan_ell);
  (void)hipFree(c->d_order_up);
  if (c->solve_stream) (void)hipStreamDestroy(c->solve_stream);
  for (int k = 0; k < 3; ++k)
    if (c->part_stream[k]) (void)hipStreamDestroy(c->part_stream[k]);
  (void)hipFree(c->d_small);
  if (c->ws) (void)hipFree(c->ws);
  delete c;
}

extern "C" msb_status msb_release_workspace(msb_ctx* c) {
  (void)hipGetLastError();   // do not report an earlier call's failure
  if (!c) return fail(MSB_EINVAL, "msb_release_workspace: null context");
  MSB_HIP(hipStreamSynchronize(c->solve_stream));
  for (int k = 0; k < 3; ++k) MSB_HIP(hipStreamSynchronize(c->part_stream[k]));
  if (c->ws) MSB_HIP(hipFree(c->ws));
  c->ws = nullptr;
  c->ws_size = 0;
  return MSB_OK;
}

extern "C" int64_t msb_dim(const msb_ctx* c) { return c ? c->D : -1; }

extern "C" msb_status msb_sector_info(const msb_ctx* c, int* nu, int* nd, int* nt) {
  if (!c) return fail(MSB_EINVAL, "null context");
  if (nu) *nu = c->up.n;
  if (nd) *nd = c->dn.n;
  if (nt) *nt = c->n_types;
  return MSB_OK;
}

// =============================================================================
extern "C" msb_status msb_apply(msb_ctx* ctx, const msb_system* sys, int nsys, double shift,
                                msb_prec prec, const void* x, void* y, void* stream) {
  (void)hipGetLastError();   // do not report an earlier call's failure
  if (!ctx || !sys || !x || !y) return fail(MSB_EINVAL, "msb_apply: null argument");
  if (nsys <= 0 || nsys > 65535) return fail(MSB_EINVAL, "msb_apply: nsys out of range");
  if (!valid_prec(prec)) return fail(MSB_EINVAL, "msb_apply: invalid precision");
  hipStream_t st = (hipStream_t)stream;
  std::vector<SysDev> h(nsys);
  for (int s = 0; s < nsys; ++s) {
    msb_status r = make_sysdev(ctx, sys[s], -(sys[s].E_G + shift), -sys[s].Gamma, true, h[s]);
    if (r != MSB_OK) return r;
  }
  Arena ar(ctx);
  ar.reserve(sizeof(SysDev) * nsys);
  MSB_HIP(ar.commit());
  SysDev* dsys = ar.take<SysDev>(sizeof(SysDev) * nsys);
  MSB_HIP(hipMemcpyAsync(dsys, h.data(), sizeof(SysDev) * nsys, hipMemcpyHostToDevice, st));
  ApplyArgs a = apply_args(ctx, dsys, nsys, x, y);
  const Elem e = prec == MSB_C128 ? Elem::C128 : Elem::C64;
  a.shape = shape_for(ctx, e, nsys, st, true);
  MSB_HIP(launch_apply(e, kModePlain, a, st));
  MSB_HIP(hipStreamSynchronize(st));
  return MSB_OK;
}

extern "C" msb_status msb_apply_timed(msb_ctx* ctx, const msb_system* sys, int nsys, double shift,
                                      msb_prec prec, const void* x, void* y, int reps,
                                      double* ms_per_apply, void* stream) {
  (void)hipGetLastError();
  if (!ctx || !sys || !x || !y || !ms_per_apply) return fail(MSB_EINVAL, "msb_apply_timed: null argument");
  if (nsys <= 0 || nsys > 65535) return fail(MSB_EINVAL, "msb_apply_timed: nsys out of range");
  if (reps < 1) return fail(MSB_EINVAL, "msb_apply_timed: reps must be >= 1");
  if (!valid_prec(prec)) return fail(MSB_EINVAL, "msb_apply_timed: invalid precision");
  hipStream_t st = (hipStream_t)stream;
  std::vector<SysDev> h(nsys);
  for (int s = 0; s < nsys; ++s) {
    msb_status r = make_sysdev(ctx, sys[s], -(sys[s].E_G + shift), -sys[s].Gamma, true, h[s]);
    if (r != MSB_OK) return r;
  }
  Arena ar(ctx);
  ar.reserve(sizeof(SysDev) * nsys);
  MSB_HIP(ar.commit());
  SysDev* dsys = ar.take<SysDev>(sizeof(SysDev) * nsys);
  MSB_HIP(hipMemcpyAsync(dsys, h.data(), sizeof(SysDev) * nsys, hipMemcpyHostToDevice, st));
  ApplyArgs a = apply_args(ctx, dsys, nsys, x, y);
  const Elem e = prec == MSB_C128 ? Elem::C128 : Elem::C64;
  a.shape = shape_for(ctx, e, nsys, st, true);
  MSB_HIP(launch_apply(e, kModePlain, a, st));     // warm-up
  hipEvent_t e0, e1;
  MSB_HIP(hipEventCreate(&e0));
  MSB_HIP(hipEventCreate(&e1));
  MSB_HIP(hipEventRecord(e0, st));
  for (int i = 0; i < reps; ++i) MSB_HIP(launch_apply(e, kModePlain, a, st));
  MSB_HIP(hipEventRecord(e1, st));
  MSB_HIP(hipEventSynchronize(e1));
  float ms = 0;
  MSB_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms_per_apply = ms / reps;
  return MSB_OK;
}

extern "C" msb_status msb_apply_block(msb_ctx* ctx, const msb_system* sys, int nsys, double shift,
                                      msb_prec prec, int group, const void* x, void* y, int reps,
                                      double* ms_per_apply, void* stream) {
  (void)hipGetLastError();   // do not report an earlier call's failure
  if (!ctx || !sys || !x || !y) return fail(MSB_EINVAL, "msb_apply_block: null argument");
  if (nsys <= 0 || nsys > 65535) return fail(MSB_EINVAL, "msb_apply_block: nsys out of range");
  if (!valid_prec(prec)) return fail(MSB_EINVAL, "msb_apply_block: invalid precision");
  if (ms_per_apply && reps < 1) return fail(MSB_EINVAL, "msb_apply_block: reps must be >= 1");
  const Elem e = prec == MSB_C128 ? Elem::C128 : Elem::C64;
  const int width = apply_il_width(ctx->dn.n, elem_bytes(e), nsys, ctx->lds_max, ctx->up.max_hops);
  if (group != 2 && group != 4) return fail(MSB_EINVAL, "msb_apply_block: group must be 2 or 4");
  if (width < group)
    return fail(MSB_EINVAL, "msb_apply_block: a group of " + std::to_string(group) +
                                " rows does not fit one workgroup's LDS here (or nsys < group)");
  hipStream_t st = (hipStream_t)stream;
  std::vector<SysDev> h(nsys);
  for (int s = 0; s < nsys; ++s) {
    msb_status r = make_sysdev(ctx, sys[s], -(sys[s].E_G + shift), -sys[s].Gamma, true, h[s]);
    if (r != MSB_OK) return r;
  }
  Arena ar(ctx);
  ar.reserve(sizeof(SysDev) * nsys);
  MSB_HIP(ar.commit());
  SysDev* dsys = ar.take<SysDev>(sizeof(SysDev) * nsys);
  MSB_HIP(hipMemcpyAsync(dsys, h.data(), sizeof(SysDev) * nsys, hipMemcpyHostToDevice, st));
  ApplyArgs a = apply_args(ctx, dsys, nsys, x, y);
  MSB_HIP(launch_apply_il(e, kModePlain, group, a, st));
  if (ms_per_apply) {
    hipEvent_t e0, e1;
    MSB_HIP(hipEventCreate(&e0));
    MSB_HIP(hipEventCreate(&e1));
    MSB_HIP(hipEventRecord(e0, st));
    for (int i = 0; i < reps; ++i) MSB_HIP(launch_apply_il(e, kModePlain, group, a, st));
    MSB_HIP(hipEventRecord(e1, st));
    MSB_HIP(hipEventSynchronize(e1));
    float ms = 0;
    MSB_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_per_apply = ms / reps;
  }
  MSB_HIP(hipStreamSynchronize(st));
  return MSB_OK;
}

extern "C" msb_status msb_apply_noalloc(msb_ctx* ctx, const msb_system* sys, int nsys, double shift,
                                        msb_prec prec, const void* x, void* y, void* stream) {
  (void)hipGetLastError();   // do not report an earlier call's failure
  if (!ctx || !sys || !x || !y) return fail(MSB_EINVAL, "msb_apply_noalloc: null argument");
  if (nsys <= 0 || nsys > MSB_NOALLOC_MAX_SYS)
    return fail(MSB_EINVAL, "msb_apply_noalloc: nsys must lie in [1, " + std::to_string(MSB_NOALLOC_MAX_SYS) +
                                "] (the fixed staging array holds that many systems)");
  if (!valid_prec(prec)) return fail(MSB_EINVAL, "msb_apply_noalloc: invalid precision");
  void* const stage = scratch_address(ctx->device);
  if (!stage) return fail(MSB_EHIP, "msb_apply_noalloc: staging array of this device not set up");
  hipStream_t st = (hipStream_t)stream;
  // systems are staged in chunks through a stack buffer (no host or device
  // allocation); each chunk's copy completes before the buffer is refilled
  constexpr int kChunk = 64;
  SysDev h[kChunk];
  for (int s0 = 0; s0 < nsys; s0 += kChunk) {
    const int n = std::min(kChunk, nsys - s0);
    for (int s = 0; s < n; ++s) {
      msb_status r = make_sysdev(ctx, sys[s0 + s], -(sys[s0 + s].E_G + shift), -sys[s0 + s].Gamma, true, h[s]);
      if (r != MSB_OK) return r;
    }
    MSB_HIP(hipMemcpyAsync(static_cast<SysDev*>(stage) + s0, h, sizeof(SysDev) * n, hipMemcpyHostToDevice, st));
    MSB_HIP(hipStreamSynchronize(st));
  }
  ApplyArgs a = apply_args(ctx, static_cast<const SysDev*>(stage), nsys, x, y);
  const Elem e = prec == MSB_C128 ? Elem::C128 : Elem::C64;
  a.shape = shape_for(ctx, e, nsys, st, false);   // tuned or pinned before, else the default: no tuning
  MSB_HIP(launch_apply(e, kModePlain, a, st));
  MSB_HIP(hipStreamSynchronize(st));
  return MSB_OK;
}

extern "C" msb_status msb_number_op(msb_ctx* ctx, int site, double w_up, double w_dn, int count,
                                    int x_real, const void* x, void* y, void* stream) {
  (void)hipGetLastError();   // do not report an earlier call's failure
  if (!ctx || !x || !y) return fail(MSB_EINVAL, "msb_number_op: null argument");
  if (count <= 0 || count > 65535) return fail(MSB_EINVAL, "msb_number_op: count out of range");
  if (site >= ctx->L) return fail(MSB_EINVAL, "msb_number_op: site out of range");
  hipStream_t st = (hipStream_t)stream;
  MSB_HIP(launch_number_op(ctx->tables(), ctx->D, site, w_up, w_dn, count, x_real, x, (double*)y, st));
  MSB_HIP(hipStreamSynchronize(st));
  return MSB_OK;
}

// Electron-number-changing site operators (dipole-type O_1 / O_2 between two
// sectors): host tables of input rank and Jordan-Wigner sign, then k_dipole.
extern "C" msb_status msb_dipole(const msb_ctx* src, const msb_ctx* dst, int spin, int create,
                                 const double* coef, int nvec, int accumulate, const void* x, void* y,
                                 void* stream) {
  (void)hipGetLastError();   // do not report an earlier call's failure
  if (!src || !dst || !coef || !x || !y) return fail(MSB_EINVAL, "msb_dipole: null argument");
  if (spin != 0 && spin != 1) return fail(MSB_EINVAL, "msb_dipole: spin must be 0 (up) or 1 (down)");
  if (nvec <= 0 || nvec > 65535) return fail(MSB_EINVAL, "msb_dipole: nvec out of range");
  if (src->L != dst->L || src->L > kMaxSites) return fail(MSB_EINVAL, "msb_dipole: contexts of different lattices");
  const int dn = create ? 1 : -1;
  const bool ok = (spin == 0) ? (dst->n_up == src->n_up + dn && dst->n_dn == src->n_dn)
                              : (dst->n_dn == src->n_dn + dn && dst->n_up == src->n_up);
  if (!ok) return fail(MSB_EINVAL, "msb_dipole: destination sector does not match the operator");
  const SpinTable& S = (spin == 0) ? src->up : src->dn;
  const SpinTable& T = (spin == 0) ? dst->up : dst->dn;
  const int L = src->L;
  // orbital order: all up sites, then all down sites; a down-spin operator
  // passes every up electron (N_up is the same in both sectors)
  const int base_parity = (spin == 1) ? (src->n_up & 1) : 0;
  std::vector<int> table((size_t)L * T.n, -1);
  for (int c = 0; c < T.n; ++c) {
    const uint32_t cf = T.conf[c];
    for (int j = 0; j < L; ++j) {
      const bool occ = (cf >> j) & 1u;
      if (create != (int)occ) continue;          // c+ needs j occupied in the output, c needs it empty
      const uint32_t ci = cf ^ (1u << j);
      const auto it = std::lower_bound(S.conf.begin(), S.conf.end(), ci);
      if (it == S.conf.end() || *it != ci) continue;
      const int r = (int)(it - S.conf.begin());
      const int par = (base_parity + __builtin_popcount(cf & ((1u << j) - 1u))) & 1;
      table[(size_t)j * T.n + c] = (r << 1) | par;
    }
  }
  DipoleArgs a;
  std::memset(&a, 0, sizeof(a));
  a.x = x;
  a.y = y;
  a.D_src = src->D;
  a.D_dst = dst->D;
  a.nd_src = src->dn.n;
  a.nd_dst = dst->dn.n;
  a.n_conf = T.n;
  a.n_sites = L;
  a.spin = spin;
  a.accumulate = accumulate ? 1 : 0;
  for (int j = 0; j < L; ++j) {
    a.coef_re[j] = coef[2 * j];
    a.coef_im[j] = coef[2 * j + 1];
  }
  DevBuf tb;
  MSB_HIP(hipMalloc(&tb.p, table.size() * sizeof(int)));
  MSB_HIP(hipMemcpy(tb.p, table.data(), table.size() * sizeof(int), hipMemcpyHostToDevice));
  a.table = (const int*)tb.p;
  hipStream_t st = (hipStream_t)stream;
  MSB_HIP(launch_dipole(a, nvec, st));
  MSB_HIP(hipStreamSynchronize(st));
  return MSB_OK;
}

// =============================================================================
// Ground state: FP64 Lanczos with full reorthogonalisation (classical
// Gram-Schmidt applied twice against every stored Lanczos vector).
extern "C" msb_status msb_ground_state(msb_ctx* ctx, const msb_system* sys, const double* x0,
                                       double tol, int maxit, double* E_G, double* G, int* iters,
                                       void* stream) {
  (void)hipGetLastError();   // do not report an earlier call's failure
  if (!ctx || !sys || !x0 || !E_G || !G) return fail(MSB_EINVAL, "msb_ground_state: null argument");
  if (maxit <= 0) return fail(MSB_EINVAL, "msb_ground_state: maxit must be positive");
  if (!(tol > 0)) return fail(MSB_EINVAL, "msb_ground_state: tol must be positive");
  hipStream_t st = (hipStream_t)stream;
  const int64_t D = ctx->D;
  const int kmax = (int)std::min<int64_t>(maxit, D);
  SysDev hs;
  msb_status r = make_sysdev(ctx, *sys, 0.0, 0.0, false, hs);
  if (r != MSB_OK) return r;
  if (!sysdev_symmetric(ctx, hs))
    return fail(MSB_EINVAL, "Lanczos needs a symmetric H: give directed types equal amplitudes");
  const ApplyShape shp = shape_for(ctx, Elem::R64, 1, st, true, kModeHerm);

  const size_t part_doubles = std::max<size_t>(
      {(size_t)apply_nbx(ctx->up.n, 1) * 4, (size_t)gram_blocks(D) * (kmax + 1),
       (size_t)cocg_nbx(D, 1) * 4});
  Arena ar(ctx);
  ar.reserve(sizeof(SysDev));
  ar.reserve((size_t)(kmax + 1) * D * sizeof(double));            // Q
  ar.reserve((size_t)D * sizeof(double));                         // w
  ar.reserve(part_doubles * sizeof(double));                      // partials
  ar.reserve((size_t)(kmax + 2) * 4 * sizeof(double));            // red
  ar.reserve((size_t)(kmax + 2) * sizeof(double));                // coefficients
  size_t fr = 0, tot = 0;
  MSB_HIP(hipMemGetInfo(&fr, &tot));
  if (ar.needed() > fr + ctx->ws_size) return fail(MSB_ENOMEM, "msb_ground_state: Lanczos basis does not fit");
  MSB_HIP(ar.commit());
  SysDev* dsys = ar.take<SysDev>(sizeof(SysDev));
  double* Q = ar.take<double>((size_t)(kmax + 1) * D * sizeof(double));
  double* w = ar.take<double>((size_t)D * sizeof(double));
  double* partials = ar.take<double>(part_doubles * sizeof(double));
  double* red = ar.take<double>((size_t)(kmax + 2) * 4 * sizeof(double));
  double* coef = ar.take<double>((size_t)(kmax + 2) * sizeof(double));
  if (ar.overflow()) return fail(MSB_EINVAL, "internal: ground-state workspace layout");
  MSB_HIP(hipMemcpyAsync(dsys, &hs, sizeof(SysDev), hipMemcpyHostToDevice, st));

  auto dot = [&](const double* a, const double* b, double& outv) -> msb_status {
    MSB_HIP(launch_dot_many(a, 1, b, D, partials, red, st));
    MSB_HIP(hipMemcpyAsync(&outv, red, sizeof(double), hipMemcpyDeviceToHost, st));
    MSB_HIP(hipStreamSynchronize(st));
    return MSB_OK;
  };
  double hscal = 0.0;   // host staging value, alive for the whole call
  auto scale = [&](const double* src, double s, double* dst) -> msb_status {
    hscal = s;
    MSB_HIP(hipMemcpyAsync(coef, &hscal, sizeof(double), hipMemcpyHostToDevice, st));
    MSB_HIP(launch_scale_real(src, coef, dst, D, st));
    return MSB_OK;
  };

  double nx = 0;
  if ((r = dot(x0, x0, nx)) != MSB_OK) return r;
  if (!(nx > 0) || !std::isfinite(nx)) return fail(MSB_EINVAL, "msb_ground_state: start vector is zero or not finite");
  if ((r = scale(x0, 1.0 / std::sqrt(nx), Q)) != MSB_OK) return r;

  std::vector<double> a, b;   // b[k] couples q_k and q_{k+1}
  std::vector<double> y;
  double theta = 0.0;
  bool conv = false;
  int k = 0;
  for (k = 0; k < kmax; ++k) {
    double* qk = Q + (size_t)k * D;
    ApplyArgs aa = apply_args(ctx, dsys, 1, qk, w);
    aa.shape = shp;
    aa.partials = partials;
    aa.red = red;
    MSB_HIP(launch_apply(Elem::R64, kModeHerm, aa, st));
    double red_h[4];
    MSB_HIP(hipMemcpyAsync(red_h, red, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    MSB_HIP(hipStreamSynchronize(st));
    const double ak = red_h[0];
    a.push_back(ak);
    const double bk = (k > 0) ? b[k - 1] : 0.0;
    double ab[2] = {ak, bk};
    MSB_HIP(hipMemcpyAsync(coef, ab, 2 * sizeof(double), hipMemcpyHostToDevice, st));
    MSB_HIP(launch_lanczos_real_update(w, qk, k > 0 ? Q + (size_t)(k - 1) * D : nullptr, coef, D,
                                       partials, red, st));
    double w2 = 0;   // |w|^2 before the reorthogonalisation
    MSB_HIP(hipMemcpyAsync(&w2, red, sizeof(double), hipMemcpyDeviceToHost, st));
    // full reorthogonalisation by classical Gram-Schmidt against every q_j; a
    // second pass only if the first removed more than half of |w|^2 (the
    // criterion of Kahan and Parlett: otherwise w is orthogonal to working
    // precision after one pass)
    double bb = 0;
    for (int pass = 0; pass < 2; ++pass) {
      MSB_HIP(launch_dot_many(Q, k + 1, w, D, partials, red, st));
      MSB_HIP(launch_gemv_sub(Q, k + 1, red, w, D, st));
      if ((r = dot(w, w, bb)) != MSB_OK) return r;   // (synchronises: w2 has landed)
      if (bb >= 0.5 * w2) break;
      w2 = bb;
    }
    const double bnext = std::sqrt(bb);
    theta = tridiag_lowest(a, b, y);
    const double est = std::fabs(bnext * y.back());
    if (est <= tol * std::fabs(theta) || bnext <= 1e-14 * std::fabs(theta) || k + 1 == kmax) {
      conv = (est <= tol * std::fabs(theta)) || bnext <= 1e-14 * std::fabs(theta);
      ++k;
      break;
    }
    b.push_back(bnext);
    if ((r = scale(w, 1.0 / bnext, Q + (size_t)(k + 1) * D)) != MSB_OK) return r;
  }
  // G = Q y, normalised, sign fixed by <x0, G> >= 0
  MSB_HIP(hipMemcpyAsync(coef, y.data(), y.size() * sizeof(double), hipMemcpyHostToDevice, st));
  MSB_HIP(launch_gemv(Q, (int)y.size(), coef, G, D, st));
  double gg = 0, xg = 0;
  if ((r = dot(G, G, gg)) != MSB_OK) return r;
  if ((r = dot(x0, G, xg)) != MSB_OK) return r;
  double sc = 1.0 / std::sqrt(gg);
  if (xg < 0) sc = -sc;
  if ((r = scale(G, sc, G)) != MSB_OK) return r;
  MSB_HIP(hipStreamSynchronize(st));
  *E_G = theta;
  if (iters) *iters = k;
  if (!conv) return fail(MSB_NOT_CONVERGED, "msb_ground_state: Lanczos did not converge within maxit");
  return MSB_OK;
}

// =============================================================================
// Multi-shift solve.
namespace {

// Bump allocator over the context workspace; with a null base it only counts.
class Carver {
 public:
  explicit Carver(void* base) : base_(static_cast<char*>(base)) {}
  template <typename T>
  T* take(size_t bytes) {
    T* p = base_ ? reinterpret_cast<T*>(base_ + off_) : nullptr;
    off_ += Arena::align(bytes);
    return p;
  }
  size_t used() const { return off_; }

 private:
  char* base_;
  size_t off_ = 0;
};

struct SolveBufs {
  void* bank = nullptr;
  void* pvec = nullptr;
  void* vvec = nullptr;
  void* Pc = nullptr;
  SysDev* dsys = nullptr;
  SysState* dst = nullptr;
  double* partials = nullptr;
  size_t part_cap = 0;          // doubles in partials (the parts of a split batch take regions)
  double* red1 = nullptr;
  double* red2 = nullptr;
  int* dbase = nullptr;
  double* wshift = nullptr;
  double* zeta = nullptr;
  double* zeta_prev = nullptr;
  int* conv = nullptr;
  double* alog = nullptr;
  double* blog = nullptr;
  double* rlog = nullptr;
  int* dlist = nullptr;
  int* dlend = nullptr;
  int* dtile = nullptr;
  double* coef = nullptr;
  double* gcoef = nullptr;
  double* cscr = nullptr;
  double* ab = nullptr;
  double* xseed = nullptr;      // residual replacement: seed solution [B][D] c128
  void* psnap = nullptr;        // residual replacement, direct form: p at the last rebuild [B][D]
  double* wrep = nullptr;       // residual replacement: A_s x [B][D] c128
  double* rcoef = nullptr;      // residual replacement, recurred form: rebuild coefficients
  SysDev* tsys = nullptr;       // true-residual systems
  double* tpart = nullptr;
  double* tred = nullptr;
  void* rt = nullptr;           // dual-space form: r~, p~, A^T p~ [B][D] and the transposed systems
  void* pt = nullptr;
  void* vt = nullptr;
  SysDev* dsysT = nullptr;
  void* ozw = nullptr;          // int8 assembly engine: coefficient digit planes

  void carve(Carver& c, const msb_ctx* ctx, int B, int cap, int n_shift, int n_list, int maxit,
             size_t s_el, size_t s_out, bool carry, bool want_true, bool replace, bool dual, int engine) {
    const int64_t D = ctx->D;
    size_t part_n = 0;   // largest nsys * nbx over the batch sizes that can occur
    for (int n = 1; n <= B; ++n)
      part_n = std::max(part_n, (size_t)n * std::max(apply_nbx(ctx->up.n, n), cocg_nbx(D, n)));
    bank = c.take<void>((size_t)cap * B * D * s_el);
    const size_t Bp = ((size_t)B + 3) / 4 * 4;   // whole groups of an interleaved batch
    pvec = c.take<void>(Bp * D * s_el);
    vvec = c.take<void>(Bp * D * s_el);
    Pc = carry ? c.take<void>((size_t)B * n_shift * D * s_out) : nullptr;
    dsys = c.take<SysDev>(B * sizeof(SysDev));
    dst = c.take<SysState>(B * sizeof(SysState));
    // room for twice [nsys][nbx][4]: the parts of a split batch run at once,
    // each in a region of its own
    part_cap = part_n * 8;
    partials = c.take<double>(part_cap * sizeof(double));
    red1 = c.take<double>((size_t)B * 4 * sizeof(double));
    red2 = c.take<double>((size_t)B * 4 * sizeof(double));
    dbase = c.take<int>(4 * sizeof(int));
    wshift = c.take<double>((size_t)n_shift * sizeof(double));
    zeta = c.take<double>((size_t)B * n_shift * 2 * sizeof(double));
    zeta_prev = c.take<double>((size_t)B * n_shift * 2 * sizeof(double));
    conv = c.take<int>((size_t)B * n_shift * sizeof(int));
    alog = c.take<double>((size_t)B * maxit * 2 * sizeof(double));
    blog = c.take<double>((size_t)B * maxit * 2 * sizeof(double));
    rlog = c.take<double>((size_t)B * (maxit + 1) * sizeof(double));
    const int n_stiles = n_list;   // bound on the shift tiles of every engine (tiles hold >= 1 shift)
    dlist = c.take<int>((size_t)B * n_list * sizeof(int));
    dlend = c.take<int>((size_t)B * n_list * sizeof(int));
    dtile = c.take<int>((size_t)B * (n_stiles + 1) * sizeof(int));
    coef = c.take<double>((size_t)B * n_list * cap * 3 * sizeof(double));   // up to 3 doubles per entry
    gcoef = carry ? c.take<double>((size_t)B * n_list * cap * 3 * sizeof(double)) : nullptr;
    cscr = c.take<double>((size_t)B * n_list * cap * 4 * sizeof(double));
    ab = c.take<double>((size_t)B * n_list * 4 * sizeof(double));
    const size_t ozb = flush_work_bytes(engine, B, n_list, cap);
    ozw = ozb ? c.take<void>(ozb) : nullptr;
    if (replace) {
      xseed = c.take<double>((size_t)B * D * 16);
      psnap = c.take<void>((size_t)B * D * s_el);
      wrep = c.take<double>((size_t)B * D * 16);
      rcoef = c.take<double>((size_t)B * 2 * (cap + 1) * 2 * sizeof(double));
    }
    if (dual) {
      rt = c.take<void>((size_t)B * D * s_el);
      pt = c.take<void>((size_t)B * D * s_el);
      vt = c.take<void>((size_t)B * D * s_el);
      dsysT = c.take<SysDev>(B * sizeof(SysDev));
    }
    if (want_true) {
      const size_t nt = (size_t)B * n_shift;
      tsys = c.take<SysDev>(nt * sizeof(SysDev));
      size_t tp = 0;
      for (int n = 1; n <= B; ++n) tp = std::max(tp, (size_t)n * n_shift * apply_nbx(ctx->up.n, n * n_shift));
      tpart = c.take<double>(tp * 4 * sizeof(double));
      tred = c.take<double>(nt * 4 * sizeof(double));
    }
  }
};

}  // namespace

extern "C" msb_status msb_solve(msb_ctx* ctx, const msb_system* sys, int nsys, const void* E,
                                const double* w_in, int n_shift, double seed_shift, double tol,
                                int maxit, msb_prec prec, void* psi, msb_info* info,
                                const msb_opts* opts, void* stream) {
  (void)hipGetLastError();   // do not report an earlier call's failure
  using clk = std::chrono::steady_clock;
  const auto t_entry = clk::now();
  auto ms_since = [](clk::time_point t0) {
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  };
  if (!ctx || !sys || !E || !w_in || !psi) return fail(MSB_EINVAL, "msb_solve: null argument");
  if (nsys <= 0) return fail(MSB_EINVAL, "msb_solve: nsys must be positive");
  if (n_shift <= 0 || n_shift > 65535) return fail(MSB_EINVAL, "msb_solve: n_shift out of range");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(MSB_EINVAL, "msb_solve: tol must be positive");
  if (maxit < 0 || maxit > 1000000) return fail(MSB_EINVAL, "msb_solve: maxit out of range");
  if (!valid_prec(prec)) return fail(MSB_EINVAL, "msb_solve: invalid precision");
  if (!std::isfinite(seed_shift)) return fail(MSB_EINVAL, "msb_solve: seed_shift must be finite");
  for (int k = 0; k < n_shift; ++k)
    if (!std::isfinite(w_in[k])) return fail(MSB_EINVAL, "msb_solve: non-finite shift");
  // residual replacement (complex64 only): 0 = default period 50, < 0 = off
  int replace_every = 0;
  if (prec == MSB_C64) {
    replace_every = (opts && opts->replace_every != 0) ? opts->replace_every : 50;
    if (replace_every < 0) replace_every = 0;
  }
  int chunk = (opts && opts->chunk > 0) ? opts->chunk : 16;
  if (replace_every > 0 && !(opts && opts->chunk > 0)) chunk = std::min(replace_every, 64);
  const double memfrac = (opts && opts->mem_fraction > 0) ? std::min(opts->mem_fraction, 0.98) : 0.9;
  const Elem ev = (prec == MSB_C128) ? Elem::C128 : Elem::C64;
  const Elem eo = ev;
  const int64_t D = ctx->D;
  const int mx = std::max(maxit, 1);
  int engine = opts ? opts->assembly_engine : 0;
  if (engine < 0 || engine > kNumFlushEngines) return fail(MSB_EINVAL, "msb_solve: unknown assembly engine");
  // 0, the default: the FP64 vector engine, except for a complex64 bank with
  // many shifts, which the int8 matrix-core engine assembles faster (five
  // digit planes of 24-bit values; with few shifts per system its workgroups
  // of 256 shift slots stay mostly idle); kNumFlushEngines: the FP64 vector
  // engine in every case
  if (engine == 0 && prec == MSB_C64 && n_shift >= 128) engine = 5;
  if (engine == kNumFlushEngines) engine = 0;
  // the FP64 matrix-core engine takes complex128 banks only
  if (prec == MSB_C64 && engine == 6) engine = 0;
  // the three-product engines take complex64 slots in 16-byte units (or
  // assume them aligned so), which needs an even D; odd D takes the
  // four-product vector engine
  if (prec == MSB_C64 && (ctx->D & 1) && flush_coef_comps(engine) == 3) engine = 2;
  const int tile_s = flush_shifts_per_tile(engine);
  const int n_list = ((n_shift + tile_s - 1) / tile_s) * tile_s;
  const size_t s_el = elem_bytes(ev), s_out = elem_bytes(eo);
  const bool want_true = info && info->resid_true;

  std::vector<SysDev> hsys(nsys), hsysT;
  bool dual = opts && opts->dual == 1;
  for (int s = 0; s < nsys; ++s) {
    msb_status r = make_sysdev(ctx, sys[s], -(sys[s].E_G + seed_shift), -sys[s].Gamma, true, hsys[s]);
    if (r != MSB_OK) return r;
    dual = dual || !sysdev_symmetric(ctx, hsys[s]);
  }
  // recurred seed form (A p_m carried by recurrence; p_m formed only for the
  // seed solution of residual replacement); the dual form runs the direct one
  // complex64 carries A p_m in float storage, so the recurred product drifts
  // from A p_m: it runs recurred only on request (direct_ap = -1) and with
  // residual replacement, which resets the product to A p_{m-1} at every
  // replacement (measured: without the reset single systems stall above tol;
  // with it the final true residuals of hard systems are several times the
  // direct form's)
  const int dap = opts ? opts->direct_ap : 0;
  if (dap < 0) return fail(MSB_EINVAL, "msb_solve: direct_ap must be 0 or 1 (the recurred seed form runs in "
                                        "complex128 only)");
  const bool recur = !dual && dap != 1 && prec == MSB_C128;
  // interleaved block apply (direct seed form, two or more systems per batch)
  const bool il_ok = !recur && !dual && opts && opts->interleave > 0;
  if (dual) {
    if (prec != MSB_C128) return fail(MSB_EINVAL, "msb_solve: the dual-space form runs in complex128");
    hsysT.resize(nsys);
    for (int s = 0; s < nsys; ++s) hsysT[s] = sysdev_transpose(ctx, hsys[s]);
  }

  // apply launch shapes: tuned on first use, before the workspace is sized
  hipStream_t ust = (hipStream_t)stream;
  const bool tune = !(opts && opts->autotune < 0);
  const int seed_mode = recur ? (int)kModeSelf : (int)kModeBilinear;
  const int il_all = il_ok ? apply_il_width(ctx->dn.n, elem_bytes(ev), nsys, ctx->lds_max, ctx->up.max_hops) : 0;
  if (!il_all) (void)shape_for(ctx, ev, nsys, ust, tune, seed_mode);
  if (replace_every > 0) (void)shape_for(ctx, Elem::C128, nsys, ust, tune);
  // the residual check stages FP64 rows whatever the storage: tune it as complex128
  if (want_true)
    (void)shape_for(ctx, Elem::C128, (int)std::min<int64_t>((int64_t)nsys * n_shift, kTuneMaxSys), ust, tune,
                    kModeResid);

  // ---- plan: batch size and bank capacity from the memory that is free ----
  size_t fr = 0, tot = 0;
  MSB_HIP(hipMemGetInfo(&fr, &tot));
  size_t budget = (size_t)((double)(fr + ctx->ws_size) * memfrac);
  // Keep a workspace that already holds most of the budget: re-allocating a
  // few hundred GB costs seconds, more than a slightly smaller bank does.
  if (ctx->ws_size > 0 && (double)ctx->ws_size >= 0.85 * (double)budget) budget = ctx->ws_size;
  auto need_bytes = [&](int B, int cap, bool carry) {
    Carver c(nullptr);
    SolveBufs b;
    b.carve(c, ctx, B, cap, n_shift, n_list, mx, s_el, s_out, carry, want_true, replace_every > 0, dual, engine);
    return c.used();
  };
  int planB = 0, plancap = 0;
  bool plancarry = false;
  int Bmax = std::min(nsys, 64);
  if (opts && opts->batch > 0) Bmax = std::min(Bmax, opts->batch);
  // Default bank: 1024 residual slots (enough for the iteration counts of the
  // workloads); a fixed size keeps repeated solves on the same workspace.
  int want_cap = std::min(mx + 1, 1024);
  if (opts && opts->bank_slots > 0) want_cap = std::min(mx + 1, std::max(opts->bank_slots, 3));
  const int min_cap = std::min(want_cap, 64);
  const bool carry_full = want_cap < mx + 1;
  // largest bank below want_cap that fits B systems with a carry buffer (0:
  // not even min_cap), in whole multiples of 32 slots, so that small changes
  // of the free memory give the same plan (and the same workspace) on the
  // next call; called only when want_cap itself does not fit
  auto largest_cap = [&](int B) {
    if (need_bytes(B, min_cap, true) > budget) return 0;
    int lo = min_cap, hi = want_cap;
    while (hi - lo > 1) {
      const int mid = lo + (hi - lo) / 2;
      if (need_bytes(B, mid, true) <= budget) lo = mid; else hi = mid;
    }
    if (lo > min_cap) lo = std::max(min_cap, lo - lo % 32);
    return lo;
  };
  // Prefer the whole batch with the full bank.  When that does not fit, take
  // the largest group of systems whose banks still hold kGroupSlots slots
  // each: a flush before the last iteration also assembles every shift's
  // search direction (the carried p^w), twice the assembly work of the slots
  // it covers, while iterating more systems together saves only a few per
  // cent of the seed iterations (measured: four 4x4-cluster systems 7%),
  // because the apply's gathers are per system.  Only when no group reaches
  // that does the whole batch run with the largest smaller bank that fits.
  constexpr int kGroupSlots = 512;
  const int group_slots = std::min(want_cap, kGroupSlots);
  for (int B = Bmax; B >= 1 && planB == 0; --B) {
    if (need_bytes(B, want_cap, carry_full) <= budget) {
      planB = B; plancap = want_cap; plancarry = carry_full;
      break;
    }
    const int c = largest_cap(B);
    if (c >= group_slots) {
      planB = B; plancap = c; plancarry = true;
    }
  }
  for (int B = Bmax; B >= 1 && planB == 0; --B) {
    const int c = largest_cap(B);
    if (c > 0) {
      planB = B; plancap = c; plancarry = true;
    }
  }
  if (planB == 0) {
    for (int cap = min_cap - 1; cap >= 3; --cap) {
      if (need_bytes(1, cap, true) <= budget) {
        planB = 1; plancap = cap; plancarry = true;
        break;
      }
    }
  }
  if (planB == 0) return fail(MSB_ENOMEM, "msb_solve: workspace does not fit in device memory");

  // inputs are complete on the caller's stream; the solve runs on the
  // context's own stream (needed for graph capture) and is finished on return
  MSB_HIP(hipStreamSynchronize(ust));
  hipStream_t st = ctx->solve_stream;
  const bool use_graph = !(opts && opts->use_graph < 0);

  const int B = planB, cap = plancap;
  const int n_stiles = n_list / tile_s;

  const double t_tune_plan = ms_since(t_entry);
  const auto t_a0 = clk::now();
  Arena ar(ctx);
  ar.reserve(need_bytes(B, cap, plancarry));
  MSB_HIP(ar.commit());
  const double t_alloc = ms_since(t_a0);
  SolveBufs bf;
  {
    Carver c(ctx->ws);
    bf.carve(c, ctx, B, cap, n_shift, n_list, mx, s_el, s_out, plancarry, want_true, replace_every > 0, dual, engine);
  }
  void* bank = bf.bank;
  void* pvec = bf.pvec;
  void* vvec = bf.vvec;
  void* Pc = bf.Pc;
  SysDev* dsys = bf.dsys;
  SysState* dst = bf.dst;
  double* partials = bf.partials;
  double* red1 = bf.red1;
  double* red2 = bf.red2;
  int* dbase = bf.dbase;
  double* wshift = bf.wshift;
  double* zeta = bf.zeta;
  double* zeta_prev = bf.zeta_prev;
  int* conv = bf.conv;
  double* alog = bf.alog;
  double* blog = bf.blog;
  double* rlog = bf.rlog;
  int* dlist = bf.dlist;
  int* dlend = bf.dlend;
  int* dtile = bf.dtile;
  double* coef = bf.coef;
  double* gcoef = bf.gcoef;
  double* cscr = bf.cscr;
  double* ab = bf.ab;

  std::vector<double> hw(n_shift);
  for (int k = 0; k < n_shift; ++k) hw[k] = w_in[k] - seed_shift;
  MSB_HIP(hipMemcpyAsync(wshift, hw.data(), n_shift * sizeof(double), hipMemcpyHostToDevice, st));

  hipEvent_t ev0, ev1, eg0, eg1, fork_ev, join_ev[kSeedParts - 1];
  MSB_HIP(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming));
  for (auto& j : join_ev) MSB_HIP(hipEventCreateWithFlags(&j, hipEventDisableTiming));
  MSB_HIP(hipEventCreate(&ev0));
  MSB_HIP(hipEventCreate(&ev1));
  MSB_HIP(hipEventCreate(&eg0));
  MSB_HIP(hipEventCreate(&eg1));
  double t_iter = 0, t_flush = 0, t_true = 0, t_gemm = 0, gemm_flops = 0, gemm_bytes = 0;
  int n_gemm = 0;
  auto elapsed = [&](double& acc) -> msb_status {
    MSB_HIP(hipEventSynchronize(ev1));
    float ms = 0;
    MSB_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    acc += ms;
    return MSB_OK;
  };

  msb_status result = MSB_OK;
  int max_iters = 0, total_mvms = 0, brk_iter = -1, flushes = 0, n_replace = 0;
  ApplyShape seed_shape{0, 0, 0, 0};
  std::vector<SysState> hst(B);
  std::vector<int> hconv((size_t)B * n_shift);
  std::vector<double> hz((size_t)B * n_shift * 2);
  std::vector<double> hrlog((size_t)B * (mx + 1));

  for (int b0 = 0; b0 < nsys; b0 += B) {
    const int nb = std::min(B, nsys - b0);
    const double* Eb = (const double*)E + (size_t)b0 * D * 2;
    char* psib = (char*)psi + (size_t)b0 * n_shift * D * s_out;
    MSB_HIP(hipMemcpyAsync(dsys, hsys.data() + b0, nb * sizeof(SysDev), hipMemcpyHostToDevice, st));
    if (dual)
      MSB_HIP(hipMemcpyAsync(bf.dsysT, hsysT.data() + b0, nb * sizeof(SysDev), hipMemcpyHostToDevice, st));
    int zero = 0;
    MSB_HIP(hipMemcpyAsync(dbase, &zero, sizeof(int), hipMemcpyHostToDevice, st));

    MSB_HIP(hipEventRecord(ev0, st));
    const int il = il_ok ? apply_il_width(ctx->dn.n, elem_bytes(ev), nb, ctx->lds_max, ctx->up.max_hops) : 0;
    InitArgs ia;
    ia.il = il;
    ia.E = Eb; ia.bank = bank; ia.pvec = pvec; ia.st = dst; ia.partials = partials;
    ia.cap = cap; ia.D = D; ia.nbx = cocg_nbx(D, nb); ia.nsys = nb; ia.n_shift = n_shift; ia.zeta = zeta;
    ia.zeta_prev = zeta_prev; ia.conv_iter = conv; ia.rnorm_log = rlog; ia.maxit = mx;
    ia.xseed = bf.xseed;
    ia.psnap = recur ? nullptr : bf.psnap;
    ia.rt = dual ? bf.rt : nullptr;
    ia.pt = dual ? bf.pt : nullptr;
    MSB_HIP(launch_cocg_init(ev, ia, st));

    ApplyArgs aa = apply_args(ctx, dsys, nb, pvec, vvec);
    if (il) {
      const int nd = ctx->dn.n, blk = nd <= 1024 ? 256 : 1024;
      seed_shape = ApplyShape{blk, (nd + blk - 1) / blk, il, 2, 0};
    } else {
      aa.shape = shape_for(ctx, ev, nb, st, tune, seed_mode);
      seed_shape = apply_shape_used(ev, seed_mode, aa);
    }
    aa.aux = bank;
    aa.partials = partials;
    aa.red = red1;
    aa.status = &dst[0].status;
    aa.status_stride = (int)(sizeof(SysState) / sizeof(int));
    aa.aux_m = &dst[0].m;
    aa.aux_base = dbase;
    aa.aux_cap = cap;
    if (recur) {                 // v = A r_m + beta_{m-1} v, r_m read in place from the bank
      static_assert(sizeof(SysState) % sizeof(double) == 0, "beta stride");
      aa.x = nullptr;
      aa.beta = &dst[0].bp_re;
      aa.beta_stride = (int)(sizeof(SysState) / sizeof(double));
    }
    ApplyArgs ta = apply_args(ctx, bf.dsysT, nb, bf.pt, bf.vt);   // dual: v~ = A^T p~
    if (dual) {
      aa.aux = bf.rt;            // sigma = r~^T A p
      aa.aux_m = nullptr;
      aa.aux_base = nullptr;
      aa.aux_cap = 0;
      ta.shape = aa.shape;
      ta.status = aa.status;
      ta.status_stride = aa.status_stride;
    }

    CocgArgs ca;
    ca.il = il;
    ca.st = dst; ca.red1 = red1; ca.partials = partials; ca.red2 = red2;
    ca.bank = bank; ca.vvec = vvec; ca.pvec = pvec; ca.base = dbase; ca.cap = cap; ca.D = D;
    ca.nbx = cocg_nbx(D, nb); ca.nsys = nb; ca.n_shift = n_shift; ca.wshift = wshift; ca.zeta = zeta;
    ca.zeta_prev = zeta_prev; ca.conv_iter = conv; ca.tol = tol; ca.maxit = mx;
    ca.alpha_log = alog; ca.beta_log = blog; ca.rnorm_log = rlog;
    ca.xseed = bf.xseed;
    ca.rep_floor = std::max(tol, kReplaceFloor);
    ca.rt = dual ? bf.rt : nullptr;
    ca.pt = dual ? bf.pt : nullptr;
    ca.vt = dual ? bf.vt : nullptr;
    // x is rebuilt from the bank at each replacement, not updated every iteration
    ca.xseed = nullptr;

    int base = 0;
    bool first_flush = true;
    // flush residual slots [base, m) into psi (and the carried p^w if `carry`)
    auto flush = [&](bool carry) -> msb_status {
      MSB_HIP(hipMemcpyAsync(hst.data(), dst, nb * sizeof(SysState), hipMemcpyDeviceToHost, st));
      MSB_HIP(hipMemcpyAsync(hconv.data(), conv, (size_t)nb * n_shift * sizeof(int), hipMemcpyDeviceToHost, st));
      MSB_HIP(hipStreamSynchronize(st));
      std::vector<int> list((size_t)nb * n_list, -1), lend((size_t)nb * n_list, 0);
      std::vector<int> tile((size_t)nb * n_stiles, 0);
      int K = 0;
      for (int s = 0; s < nb; ++s) {
        const int ms = hst[s].m;
        std::vector<std::pair<int, int>> part;   // (lend, k)
        for (int k = 0; k < n_shift; ++k) {
          const int Mw = hconv[(size_t)s * n_shift + k];
          if (!(base == 0 || Mw < 0 || Mw > base)) continue;
          const int endk = (Mw < 0) ? ms : std::min(Mw, ms);
          part.push_back({std::max(endk - base, 0), k});
        }
        std::stable_sort(part.begin(), part.end(), [](const std::pair<int, int>& x, const std::pair<int, int>& y) {
          return x.first > y.first;
        });
        for (size_t j = 0; j < part.size(); ++j) {
          list[(size_t)s * n_list + j] = part[j].second;
          lend[(size_t)s * n_list + j] = part[j].first;
          K = std::max(K, part[j].first);
          int& tk = tile[(size_t)s * n_stiles + j / tile_s];
          tk = std::max(tk, part[j].first);
        }
      }
      if (K > cap) return fail(MSB_EINVAL, "internal: flush range exceeds the bank");
      const int Kc = std::max(K, 1);
      MSB_HIP(hipMemcpyAsync(dlist, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice, st));
      MSB_HIP(hipMemcpyAsync(dlend, lend.data(), lend.size() * sizeof(int), hipMemcpyHostToDevice, st));
      MSB_HIP(hipMemcpyAsync(dtile, tile.data(), tile.size() * sizeof(int), hipMemcpyHostToDevice, st));
      MSB_HIP(hipEventRecord(ev0, st));
      CoefArgs cf;
      cf.st = dst; cf.alpha_log = alog; cf.beta_log = blog; cf.wshift = wshift; cf.conv_iter = conv;
      cf.list = dlist; cf.lend = dlend; cf.coef = coef; cf.gcoef = carry ? gcoef : nullptr; cf.ab = ab;
      cf.nsys = nb; cf.n_shift = n_shift; cf.n_list = n_list; cf.maxit = mx; cf.K = Kc; cf.base = base;
      cf.ncomp = flush_coef_comps(engine);
      MSB_HIP(launch_coef(cf, cscr, st));
      FlushArgs fa;
      fa.bank = bank; fa.cap = cap; fa.coef = coef; fa.pw = nullptr; fa.ow = nullptr;
      fa.pw_stride = 4; fa.ow_stride = 4; fa.list = dlist; fa.tile_k = dtile; fa.lend = dlend; fa.out = psib;
      fa.X = nullptr; fa.D = D; fa.n_shift = n_shift; fa.n_list = n_list; fa.K = Kc; fa.nsys = nb;
      fa.n_etiles = (int)((D + flush_elems_per_tile(engine) - 1) / flush_elems_per_tile(engine));
      fa.n_stiles = n_stiles;
      fa.work = bf.ozw;
      fa.rnorm = rlog;
      fa.rn_stride = mx + 1;
      fa.rn_base = base;
      if (!first_flush && Pc) {
        fa.pw = ab;          // Psi += (bw_base S_base) p_{base-1}
        fa.X = Pc;
      }
      MSB_HIP(hipEventRecord(eg0, st));
      MSB_HIP(launch_flush(ev, eo, fa, first_flush ? 0 : 1, engine, st));
      MSB_HIP(hipEventRecord(eg1, st));
      ++n_gemm;
      // algorithmic work: every (system, shift) range reads its residual slots
      // once per tile of shifts and writes (and re-reads if accumulating) Psi
      double sum_len = 0, n_out = 0;
      for (size_t j = 0; j < lend.size(); ++j)
        if (list[j] >= 0) { sum_len += lend[j]; n_out += 1; }
      gemm_flops += 8.0 * (double)D * sum_len;
      gemm_bytes += (double)D * ((double)K * nb * s_el + n_out * s_out * (first_flush ? 1.0 : 3.0));
      if (carry) {
        FlushArgs fp = fa;
        fp.coef = gcoef;
        fp.out = Pc;
        fp.pw = nullptr;
        fp.X = nullptr;
        fp.ow = ab + 2;      // p_{end-1} = (bw_base G_base) p_{base-1} + ...
        MSB_HIP(launch_flush(ev, eo, fp, first_flush ? 0 : 2, engine, st));
      }
      MSB_HIP(hipEventRecord(ev1, st));
      msb_status r = elapsed(t_flush);
      if (r != MSB_OK) return r;
      {
        float ms = 0;
        MSB_HIP(hipEventElapsedTime(&ms, eg0, eg1));
        t_gemm += ms;
      }
      first_flush = false;
      ++flushes;
      return MSB_OK;
    };

    // one chunk of seed iterations; kernels skip systems that are not active.
    // The chunk is captured once per batch into a hipGraph and replayed.
    // Recurred form, two or more systems: the batch is split into parts of
    // consecutive systems, each captured as its own chunk graph and launched on
    // its own stream, so one part's latency-bound apply overlaps another
    // part's streaming r-update.  Each part has its own region of partials.
    // (measured: 12 systems of the L=12 ring gain 8% per iteration; 4 systems
    // of the 4x4 cluster, whose apply dominates and gathers from L2, lose 8%)
    int n_parts = (use_graph && recur && nb >= kSeedPartMin * kSeedParts) ? kSeedParts : 1;
    std::vector<ApplyArgs> aa_p;
    std::vector<CocgArgs> ca_p;
    if (n_parts > 1) {
      size_t off = 0;
      for (int p = 0; p < n_parts; ++p) {
        const int s0 = (int)((int64_t)nb * p / n_parts), s1 = (int)((int64_t)nb * (p + 1) / n_parts);
        const int n = s1 - s0;
        const size_t need = (size_t)n * std::max(apply_nbx(ctx->up.n, n), cocg_nbx(D, n)) * 4;
        if (off + need > bf.part_cap) {   // not enough room: one graph for the whole batch
          n_parts = 1;
          break;
        }
        ApplyArgs ha = aa;
        ha.sys = dsys + s0;
        ha.aux = (const char*)bank + (size_t)s0 * cap * D * s_el;
        ha.v = (char*)vvec + (size_t)s0 * D * s_el;
        ha.aux_m = &dst[s0].m;
        ha.status = &dst[s0].status;
        ha.beta = &dst[s0].bp_re;
        ha.partials = partials + off;
        ha.red = red1 + 4 * (size_t)s0;
        ha.nsys = n;
        CocgArgs hc = ca;
        hc.st = dst + s0;
        hc.red1 = red1 + 4 * (size_t)s0;
        hc.partials = partials + off;
        hc.red2 = red2 + 4 * (size_t)s0;
        hc.bank = (char*)bank + (size_t)s0 * cap * D * s_el;
        hc.vvec = (const char*)vvec + (size_t)s0 * D * s_el;
        hc.pvec = (char*)pvec + (size_t)s0 * D * s_el;
        hc.nbx = cocg_nbx(D, n);
        hc.nsys = n;
        hc.zeta = zeta + 2 * (size_t)s0 * n_shift;
        hc.zeta_prev = zeta_prev + 2 * (size_t)s0 * n_shift;
        hc.conv_iter = conv + (size_t)s0 * n_shift;
        hc.alpha_log = alog + 2 * (size_t)s0 * mx;
        hc.beta_log = blog + 2 * (size_t)s0 * mx;
        hc.rnorm_log = rlog + (size_t)s0 * (mx + 1);
        aa_p.push_back(ha);
        ca_p.push_back(hc);
        off += need;
      }
    }
    auto part_stream = [&](int p) { return p == 0 ? st : ctx->part_stream[p - 1]; };
    auto enqueue_part = [&](int p) -> hipError_t {
      for (int c = 0; c < chunk; ++c) {
        hipError_t e = launch_apply(ev, kModeSelf, aa_p[p], part_stream(p));
        if (e == hipSuccess) e = launch_cocg_r(ev, ca_p[p], part_stream(p));
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    };
    auto enqueue_chunk = [&]() -> hipError_t {
      for (int c = 0; c < chunk; ++c) {
        if (recur) {
          hipError_t e = launch_apply(ev, kModeSelf, aa, st);
          if (e == hipSuccess) e = launch_cocg_r(ev, ca, st);
          if (e != hipSuccess) return e;
          continue;
        }
        hipError_t e = launch_cocg_p(ev, ca, st);
        if (e == hipSuccess) e = il ? launch_apply_il(ev, kModeBilinear, il, aa, st) : launch_apply(ev, kModeBilinear, aa, st);
        if (e == hipSuccess && dual) e = launch_apply(ev, kModePlain, ta, st);
        if (e == hipSuccess) e = launch_cocg_r(ev, ca, st);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    };
    hipGraphExec_t gexec[kSeedParts] = {};
    struct GraphGuard {
      hipGraphExec_t* g;
      ~GraphGuard() {
        for (int p = 0; p < kSeedParts; ++p)
          if (g[p]) (void)hipGraphExecDestroy(g[p]);
      }
    } graph_guard{gexec};
    auto run_chunk = [&]() -> msb_status {
      if (!use_graph) {
        MSB_HIP(enqueue_chunk());
        return MSB_OK;
      }
      for (int p = 0; p < n_parts; ++p) {
        if (gexec[p]) continue;
        const hipStream_t s = part_stream(p);
        MSB_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const hipError_t e_launch = n_parts > 1 ? enqueue_part(p) : enqueue_chunk();
        hipGraph_t g = nullptr;
        const hipError_t e_end = hipStreamEndCapture(s, &g);
        hipError_t e_inst = hipSuccess;
        if (e_launch == hipSuccess && e_end == hipSuccess) e_inst = hipGraphInstantiate(&gexec[p], g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        MSB_HIP(e_launch);
        MSB_HIP(e_end);
        MSB_HIP(e_inst);
      }
      if (n_parts > 1) {           // every part starts after the work queued on st; st waits for all
        MSB_HIP(hipEventRecord(fork_ev, st));
        for (int p = 1; p < n_parts; ++p) MSB_HIP(hipStreamWaitEvent(part_stream(p), fork_ev, 0));
        for (int p = 0; p < n_parts; ++p) MSB_HIP(hipGraphLaunch(gexec[p], part_stream(p)));
        for (int p = 1; p < n_parts; ++p) {
          MSB_HIP(hipEventRecord(join_ev[p - 1], part_stream(p)));
          MSB_HIP(hipStreamWaitEvent(st, join_ev[p - 1], 0));
        }
      } else {
        MSB_HIP(hipGraphLaunch(gexec[0], st));
      }
      return MSB_OK;
    };

    // recurred form with replacement: fold the bank slots written since the
    // last rebuild (iterations m0 .. m_now - 1) into x and p (Alg. 1's
    // x_{j+1} = x_j + alpha_j p_j, p_j = r_j + beta_{j-1} p_{j-1} as linear
    // combinations of r_j, from the logged alpha / beta in FP64 on the host)
    int m0 = 0;
    std::vector<double> hal, hbl, hcoef;
    auto rebuild = [&](int m_now) -> msb_status {
      if (!bf.xseed) return MSB_OK;             // no residual replacement
      const int L = m_now - m0;
      if (L <= 0) return MSB_OK;
      if (m0 < base || L > cap) return fail(MSB_EINVAL, "internal: rebuild range outside the bank");
      hal.resize((size_t)nb * mx * 2);
      hbl.resize((size_t)nb * mx * 2);
      MSB_HIP(hipMemcpyAsync(hal.data(), alog, hal.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      MSB_HIP(hipMemcpyAsync(hbl.data(), blog, hbl.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      MSB_HIP(hipStreamSynchronize(st));
      using cd = std::complex<double>;
      hcoef.assign((size_t)nb * 2 * (L + 1) * 2, 0.0);
      std::vector<cd> d(L), sx(L);
      for (int s = 0; s < nb; ++s) {
        if (hst[s].status != kActive && hst[s].status != kPaused) continue;
        auto alpha = [&](int j) { return cd(hal[((size_t)s * mx + j) * 2], hal[((size_t)s * mx + j) * 2 + 1]); };
        auto beta = [&](int j) { return cd(hbl[((size_t)s * mx + j) * 2], hbl[((size_t)s * mx + j) * 2 + 1]); };
        std::fill(d.begin(), d.end(), cd(0.0));
        std::fill(sx.begin(), sx.end(), cd(0.0));
        cd e = (m0 > 0) ? beta(m0 - 1) : cd(0.0);   // p_j = sum_l d_l r_l + e p_{m0-1}
        cd sxp = 0.0;
        for (int j = m0; j < m_now; ++j) {
          if (j > m0) {
            const cd b = beta(j - 1);
            for (int l = 0; l < j - m0; ++l) d[l] *= b;
            e *= b;
          }
          d[j - m0] = 1.0;
          const cd a = alpha(j);
          for (int l = 0; l <= j - m0; ++l) sx[l] += a * d[l];
          sxp += a * e;
        }
        double* cx = hcoef.data() + (size_t)s * 2 * (L + 1) * 2;
        double* cp = cx + (size_t)(L + 1) * 2;
        for (int l = 0; l < L; ++l) {
          cx[2 * l] = sx[l].real(); cx[2 * l + 1] = sx[l].imag();
          cp[2 * l] = d[l].real(); cp[2 * l + 1] = d[l].imag();
        }
        cx[2 * L] = sxp.real(); cx[2 * L + 1] = sxp.imag();
        cp[2 * L] = e.real(); cp[2 * L + 1] = e.imag();
      }
      MSB_HIP(hipMemcpyAsync(bf.rcoef, hcoef.data(), hcoef.size() * sizeof(double), hipMemcpyHostToDevice, st));
      RebuildArgs rb;
      rb.bank = bank; rb.cap = cap; rb.slot0 = m0 - base; rb.L = L; rb.D = D; rb.nbx = cocg_nbx(D, nb);
      // the recurred form keeps no explicit p: the rebuilt p_{m-1} goes to pvec;
      // the direct form forms p every iteration and rebuilds a copy of it
      rb.nsys = nb; rb.coef = bf.rcoef; rb.x = bf.xseed; rb.p = recur ? pvec : bf.psnap; rb.st = dst;
      MSB_HIP(launch_seed_rebuild(ev, rb, st));
      MSB_HIP(hipStreamSynchronize(st));    // hcoef is reused by the next rebuild
      m0 = m_now;
      return MSB_OK;
    };

    ApplyArgs ra = apply_args(ctx, dsys, nb, bf.xseed, bf.wrep);
    ApplyArgs pa = apply_args(ctx, dsys, nb, pvec, vvec);          // recurred form: v <- A p at a replacement
    pa.shape = shape_for(ctx, ev, nb, st, tune);
    pa.status = &dst[0].status;
    pa.status_stride = (int)(sizeof(SysState) / sizeof(int));
    ra.shape = shape_for(ctx, Elem::C128, nb, st, tune);
    ra.status = &dst[0].status;
    ra.status_stride = (int)(sizeof(SysState) / sizeof(int));
    int last_rep = 0;   // iteration of the last residual replacement

    int it_done = 0;
    while (true) {
      {
        msb_status r = run_chunk();
        if (r != MSB_OK) return r;
      }
      it_done += chunk;
      MSB_HIP(hipMemcpyAsync(hst.data(), dst, nb * sizeof(SysState), hipMemcpyDeviceToHost, st));
      MSB_HIP(hipStreamSynchronize(st));
      bool any_active = false, any_paused = false;
      for (int s = 0; s < nb; ++s) {
        any_active |= hst[s].status == kActive;
        any_paused |= hst[s].status == kPaused;
      }
      if (any_active && replace_every > 0) {
        // active systems advance in step, so one iteration count serves the batch
        int m_now = 0, n_want = 0;
        for (int s = 0; s < nb; ++s)
          if (hst[s].status == kActive) {
            m_now = std::max(m_now, hst[s].m);
            if (hst[s].m > 0 && hst[s].rnorm > ca.rep_floor * hst[s].normE) ++n_want;   // as wants_replace()
          }
        if (n_want > 0 && m_now - last_rep >= replace_every) {
          // r_m <- E - A_s x_m with x_m and the product in complex128
          msb_status r = rebuild(m_now);
          if (r != MSB_OK) return r;
          if (recur) MSB_HIP(launch_apply(ev, kModePlain, pa, st));   // A p_{m-1} afresh from the rebuilt p
          MSB_HIP(launch_apply(Elem::C128, kModePlain, ra, st));
          MSB_HIP(launch_cocg_replace(ev, ca, Eb, bf.wrep, st));
          last_rep = m_now;
          n_replace += n_want;
        }
      }
      if (any_active) continue;
      if (any_paused) {
        MSB_HIP(hipEventRecord(ev1, st));
        msb_status r = elapsed(t_iter);
        if (r != MSB_OK) return r;
        if (!plancarry) return fail(MSB_EINVAL, "internal: bank full without carry buffer");
        r = flush(true);
        if (r != MSB_OK) return r;
        // restart the bank at the current residual r_m
        int m = -1;
        for (int s = 0; s < nb; ++s)
          if (hst[s].status == kPaused) {
            if (m >= 0 && hst[s].m != m) return fail(MSB_EINVAL, "internal: paused systems out of step");
            m = hst[s].m;
          }
        {
          msb_status r = rebuild(m);        // before slot 0 is overwritten
          if (r != MSB_OK) return r;
        }
        MSB_HIP(launch_copy_slot(ev, (const char*)bank + (size_t)(m - base) * D * s_el, bank, D, nb,
                                 (int64_t)cap * D, (int64_t)cap * D, st));
        base = m;
        MSB_HIP(hipMemcpyAsync(dbase, &base, sizeof(int), hipMemcpyHostToDevice, st));
        for (int s = 0; s < nb; ++s)
          if (hst[s].status == kPaused) hst[s].status = kActive;
        MSB_HIP(hipMemcpyAsync(dst, hst.data(), nb * sizeof(SysState), hipMemcpyHostToDevice, st));
        MSB_HIP(hipEventRecord(ev0, st));
        continue;
      }
      break;
    }
    MSB_HIP(hipEventRecord(ev1, st));
    {
      msb_status r = elapsed(t_iter);
      if (r != MSB_OK) return r;
    }
    {
      msb_status r = flush(false);
      if (r != MSB_OK) return r;
    }
    (void)it_done;

    // report
    MSB_HIP(hipMemcpyAsync(hst.data(), dst, nb * sizeof(SysState), hipMemcpyDeviceToHost, st));
    MSB_HIP(hipMemcpyAsync(hconv.data(), conv, (size_t)nb * n_shift * sizeof(int), hipMemcpyDeviceToHost, st));
    MSB_HIP(hipMemcpyAsync(hz.data(), zeta, (size_t)nb * n_shift * 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    MSB_HIP(hipMemcpyAsync(hrlog.data(), rlog, (size_t)nb * (mx + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
    MSB_HIP(hipStreamSynchronize(st));
    for (int s = 0; s < nb; ++s) {
      const SysState& t = hst[s];
      max_iters = std::max(max_iters, t.m);
      total_mvms += dual ? 2 * t.m : t.m;
      if (t.status == kBreakdown) {
        result = MSB_BREAKDOWN;
        if (brk_iter < 0 || t.breakdown_iter < brk_iter) brk_iter = t.breakdown_iter;
      } else if ((t.status == kMaxit || t.status == kExhausted) && (result == MSB_OK || result == MSB_FLOOR)) {
        result = MSB_NOT_CONVERGED;
      } else if (t.status == kFloor && result == MSB_OK) {
        result = MSB_FLOOR;
      }
      if (info && info->sys_iters) info->sys_iters[b0 + s] = t.m;
      if (info && info->seed_hist && info->hist_len > 0)
        for (int j = 0; j < info->hist_len; ++j)
          info->seed_hist[(size_t)(b0 + s) * info->hist_len + j] =
              (j <= t.m && j <= mx && t.normE > 0) ? hrlog[(size_t)s * (mx + 1) + j] / t.normE : NAN;
      for (int k = 0; k < n_shift; ++k) {
        const size_t idx = (size_t)s * n_shift + k;
        const size_t oidx = (size_t)(b0 + s) * n_shift + k;
        const int Mw = hconv[idx];
        if (info && info->shift_iters) info->shift_iters[oidx] = Mw;
        if (info && info->resid_rec) {
          const int mm = (Mw >= 0) ? Mw : t.m;
          const double zabs = std::hypot(hz[2 * idx], hz[2 * idx + 1]);
          info->resid_rec[oidx] = (t.normE > 0) ? hrlog[(size_t)s * (mx + 1) + mm] / zabs / t.normE : 0.0;
        }
      }
    }

    // optional FP64 true residuals |E - (A - w) Psi| / |E|
    if (info && info->resid_true) {
      const int nt = nb * n_shift;
      std::vector<SysDev> tsys(nt);
      for (int s = 0; s < nb; ++s)
        for (int k = 0; k < n_shift; ++k) {
          msb_status r = make_sysdev(ctx, sys[b0 + s], -(sys[b0 + s].E_G + w_in[k]), -sys[b0 + s].Gamma,
                                     true, tsys[(size_t)s * n_shift + k]);
          if (r != MSB_OK) return r;
        }
      const size_t need_sys = (size_t)nt * sizeof(SysDev);
      const size_t need_red = (size_t)nt * 4 * sizeof(double);
      std::vector<double> hred((size_t)nt * 4);
      MSB_HIP(hipMemcpyAsync(bf.tsys, tsys.data(), need_sys, hipMemcpyHostToDevice, st));
      MSB_HIP(hipEventRecord(ev0, st));
      ApplyArgs ta = apply_args(ctx, bf.tsys, nt, psib, nullptr);
      ta.shape = shape_for(ctx, Elem::C128, nt, st, tune, kModeResid);   // FP64 rows, as tuned above
      ta.aux = Eb;
      ta.aux_div = n_shift;
      ta.partials = bf.tpart;
      ta.red = bf.tred;
      MSB_HIP(launch_apply(ev == Elem::C128 ? Elem::C128 : Elem::C64, kModeResid, ta, st));
      MSB_HIP(hipEventRecord(ev1, st));
      MSB_HIP(hipMemcpyAsync(hred.data(), bf.tred, need_red, hipMemcpyDeviceToHost, st));
      {
        msb_status r = elapsed(t_true);
        if (r != MSB_OK) return r;
      }
      MSB_HIP(hipStreamSynchronize(st));
      for (int s = 0; s < nb; ++s)
        for (int k = 0; k < n_shift; ++k) {
          const size_t idx = (size_t)s * n_shift + k;
          const double nE = hst[s].normE;
          info->resid_true[(size_t)(b0 + s) * n_shift + k] = nE > 0 ? std::sqrt(hred[idx * 4 + 2]) / nE : 0.0;
        }
    }
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  (void)hipEventDestroy(eg0);
  (void)hipEventDestroy(eg1);
  (void)hipEventDestroy(fork_ev);
  for (auto& j : join_ev) (void)hipEventDestroy(j);
  if (info) {
    info->t_gemm_ms = t_gemm;
    info->n_gemm = n_gemm;
    info->gemm_flops = gemm_flops;
    info->gemm_bytes = gemm_bytes;
    info->iters = max_iters;
    info->mvms = total_mvms;
    info->breakdown_iter = brk_iter;
    info->flushes = flushes;
    info->replacements = n_replace;
    info->apply_threads = seed_shape.blk;
    info->apply_ept = seed_shape.ept;
    info->apply_nv = seed_shape.nv;
    info->apply_passes = seed_shape.passes;
    info->apply_order = seed_shape.order;
    info->apply_panel_width = seed_shape.passes == 3 ? seed_shape.pw : 0;
    info->group = B;
    info->bank_slots = cap;
    info->t_iter_ms = t_iter;
    info->t_flush_ms = t_flush;
    info->t_true_ms = t_true;
    info->t_setup_ms = t_tune_plan;
    info->t_alloc_ms = t_alloc;
    info->t_wall_ms = ms_since(t_entry);
  }
  if (result == MSB_BREAKDOWN) return fail(MSB_BREAKDOWN, "msb_solve: COCG breakdown (r^T A p or r^T r vanished)");
  if (result == MSB_NOT_CONVERGED) return fail(MSB_NOT_CONVERGED, "msb_solve: iteration cap reached");
  if (result == MSB_FLOOR)
    return fail(MSB_FLOOR, "msb_solve: complex64 recurrence reached its attainable accuracy before tol");
  return MSB_OK;
}

// =============================================================================
// Appendix E around msb_solve: per system, restart the failing shifts from
// the worst of them until every shift passes or max_rounds is reached.
extern "C" msb_status msb_solve_reseed(msb_ctx* ctx, const msb_system* sys, int nsys, const void* E,
                                       const double* w_in, int n_shift, double seed_shift, double tol,
                                       int maxit, msb_prec prec, double reseed_tol, int max_rounds,
                                       void* psi, double* seed_of, double* resid_true, int* rounds,
                                       const msb_opts* opts, void* stream) {
  (void)hipGetLastError();   // do not report an earlier call's failure
  if (!ctx || !sys || !E || !w_in || !psi) return fail(MSB_EINVAL, "msb_solve_reseed: null argument");
  if (nsys <= 0 || n_shift <= 0) return fail(MSB_EINVAL, "msb_solve_reseed: nsys and n_shift must be positive");
  if (!valid_prec(prec)) return fail(MSB_EINVAL, "msb_solve_reseed: invalid precision");
  if (!(reseed_tol > 0.0) || max_rounds < 1)
    return fail(MSB_EINVAL, "msb_solve_reseed: need reseed_tol > 0 and max_rounds >= 1");
  const int64_t D = ctx->D;
  const size_t es = elem_bytes(prec == MSB_C128 ? Elem::C128 : Elem::C64);
  bool all_pass = true;
  for (int s = 0; s < nsys; ++s) {
    char* psi_s = static_cast<char*>(psi) + (size_t)s * n_shift * D * es;
    const void* E_s = static_cast<const char*>(E) + (size_t)s * D * 16;
    std::vector<int> todo(n_shift);
    for (int k = 0; k < n_shift; ++k) todo[k] = k;
    std::vector<double> rt_all(n_shift, 0.0);
    double seed = seed_shift;
    int r = 0;
    for (; r < max_rounds; ++r) {
      const int n = (int)todo.size();
      std::vector<double> w(n), rr(n), rt(n);
      std::vector<int> it(n);
      int si = 0;
      for (int j = 0; j < n; ++j) w[j] = w_in[todo[j]];
      msb_info inf;
      std::memset(&inf, 0, sizeof(inf));
      inf.sys_iters = &si;
      inf.shift_iters = it.data();
      inf.resid_rec = rr.data();
      inf.resid_true = rt.data();
      // round 0 solves every shift in place; later rounds into a scratch block
      void* tmp = nullptr;
      if (r > 0 && hipMalloc(&tmp, (size_t)n * D * es) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MSB_ENOMEM, "msb_solve_reseed: no room for the restarted shifts");
      }
      const msb_status st = msb_solve(ctx, sys + s, 1, E_s, w.data(), n, seed, tol, maxit, prec,
                                      r == 0 ? (void*)psi_s : tmp, &inf, opts, stream);
      if (st == MSB_EINVAL || st == MSB_ENOMEM || st == MSB_EHIP) {
        if (tmp) (void)hipFree(tmp);
        return st;
      }
      hipError_t e = hipSuccess;
      for (int j = 0; j < n && r > 0 && e == hipSuccess; ++j)
        e = hipMemcpy(psi_s + (size_t)todo[j] * D * es, static_cast<char*>(tmp) + (size_t)j * D * es,
                      (size_t)D * es, hipMemcpyDeviceToDevice);
      if (tmp) (void)hipFree(tmp);
      MSB_HIP(e);
      std::vector<int> bad;
      for (int j = 0; j < n; ++j) {
        const int k = todo[j];
        rt_all[k] = rt[j];
        if (seed_of) seed_of[(size_t)s * n_shift + k] = seed;
        if (!(rt[j] <= reseed_tol) || it[j] < 0) bad.push_back(k);
      }
      if (bad.empty()) break;
      int worst = bad[0];
      for (int k : bad) {
        if (std::isnan(rt_all[worst])) break;              // NaN counts as worst
        if (std::isnan(rt_all[k]) || rt_all[k] > rt_all[worst]) worst = k;
      }
      seed = w_in[worst];
      todo = bad;
      if (r + 1 == max_rounds) all_pass = false;
    }
    if (rounds) rounds[s] = std::min(r + 1, max_rounds);
    if (resid_true)
      for (int k = 0; k < n_shift; ++k) resid_true[(size_t)s * n_shift + k] = rt_all[k];
  }
  if (!all_pass) return fail(MSB_NOT_CONVERGED, "msb_solve_reseed: some shifts still fail after max_rounds");
  return MSB_OK;
}

extern "C" msb_status msb_combine(msb_ctx* ctx, int nsys, int n_shift, msb_prec prec, const void* psi,
                                  const double* phase_re, const double* phase_im, const int* o1_site,
                                  const double* o1_wup, const double* o1_wdn, void* phi, void* stream) {
  (void)hipGetLastError();   // do not report an earlier call's failure
  if (!ctx || !psi || !phi || !phase_re || !phase_im) return fail(MSB_EINVAL, "msb_combine: null argument");
  if (nsys <= 0 || n_shift <= 0 || n_shift > 65535) return fail(MSB_EINVAL, "msb_combine: sizes out of range");
  if (!valid_prec(prec)) return fail(MSB_EINVAL, "msb_combine: invalid precision");
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> c((size_t)nsys * 4);
  std::vector<int> site(nsys);
  for (int s = 0; s < nsys; ++s) {
    c[4 * s] = phase_re[s];
    c[4 * s + 1] = phase_im[s];
    c[4 * s + 2] = o1_wup ? o1_wup[s] : 1.0;
    c[4 * s + 3] = o1_wdn ? o1_wdn[s] : 1.0;
    site[s] = o1_site ? o1_site[s] : -1;
    if (site[s] >= ctx->L) return fail(MSB_EINVAL, "msb_combine: site out of range");
  }
  Arena ar(ctx);
  ar.reserve(c.size() * sizeof(double));
  ar.reserve(site.size() * sizeof(int));
  MSB_HIP(ar.commit());
  double* dc = ar.take<double>(c.size() * sizeof(double));
  int* ds = ar.take<int>(site.size() * sizeof(int));
  MSB_HIP(hipMemcpyAsync(dc, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice, st));
  MSB_HIP(hipMemcpyAsync(ds, site.data(), site.size() * sizeof(int), hipMemcpyHostToDevice, st));
  MSB_HIP(launch_combine(ctx->tables(), ctx->D, nsys, n_shift, prec == MSB_C128 ? Elem::C128 : Elem::C64,
                         psi, dc, ds, (double*)phi, st));
  MSB_HIP(hipStreamSynchronize(st));
  return MSB_OK;
}

// =============================================================================
// Continued-fraction spectrum: a block of independent Hermitian Lanczos
// recurrences on H, one per vector phi_k.
// Block Lanczos continued fraction behind msb_spectrum and msb_spectrum_cf;
// coef_a / coef_b (host [n][coef_ld], optional) receive the coefficients.
static msb_status spectrum_impl(msb_ctx* ctx, const msb_system* sys, const void* phi, int n,
                                const double* w, int n_w, double eta, int lanczos_max,
                                double cf_tol, double* I, int* depth_out, double* coef_a,
                                double* coef_b, int coef_ld, void* stream) {
  (void)hipGetLastError();   // do not report an earlier call's failure
  if (!ctx || !sys || !phi || !w || !I) return fail(MSB_EINVAL, "msb_spectrum: null argument");
  if (n <= 0 || n > 65535 || n_w <= 0) return fail(MSB_EINVAL, "msb_spectrum: sizes out of range");
  if (!(eta > 0)) return fail(MSB_EINVAL, "msb_spectrum: eta must be positive");
  if (lanczos_max <= 0) return fail(MSB_EINVAL, "msb_spectrum: lanczos_max must be positive");
  hipStream_t st = (hipStream_t)stream;
  const int64_t D = ctx->D;
  const int kmax = (int)std::min<int64_t>(lanczos_max, D);
  const int ld = kmax + 1;
  SysDev hs;
  msb_status r = make_sysdev(ctx, *sys, 0.0, 0.0, false, hs);
  if (r != MSB_OK) return r;
  if (!sysdev_symmetric(ctx, hs))
    return fail(MSB_EINVAL, "Lanczos needs a symmetric H: give directed types equal amplitudes");
  const ApplyShape shp = shape_for(ctx, Elem::C128, n, st, true, kModeHerm);
  std::vector<SysDev> hsys(n, hs);
  const int nbx_l = lanczos_nbx(D, n);
  const size_t part_doubles =
      (size_t)n * std::max(apply_nbx(ctx->up.n, n), nbx_l) * 4;

  Arena ar(ctx);
  const size_t vec_bytes = (size_t)n * D * 16;
  const size_t sizes[] = {vec_bytes, vec_bytes, vec_bytes,                        // bufA, bufB, bufW
                          (size_t)n * sizeof(SysDev), part_doubles * sizeof(double),
                          (size_t)n * 4 * sizeof(double), (size_t)n * 4 * sizeof(double),   // reda, redb
                          (size_t)n * sizeof(double), (size_t)n * sizeof(double),
                          (size_t)n * sizeof(double), (size_t)n * sizeof(double),        // dzero dbcur dnorm2 dnrm
                          (size_t)n * sizeof(int), (size_t)n * sizeof(int),             // dactive ddepth
                          (size_t)n * ld * sizeof(double), (size_t)n * ld * sizeof(double),  // logs
                          (size_t)n_w * sizeof(double), (size_t)n * n_w * sizeof(double)};
  for (size_t z : sizes) ar.reserve(z);
  size_t fr = 0, tot = 0;
  MSB_HIP(hipMemGetInfo(&fr, &tot));
  if (ar.needed() > fr + ctx->ws_size) return fail(MSB_ENOMEM, "msb_spectrum: block Lanczos does not fit");
  MSB_HIP(ar.commit());
  double* bufA = ar.take<double>(vec_bytes);
  double* bufB = ar.take<double>(vec_bytes);
  double* bufW = ar.take<double>(vec_bytes);
  SysDev* dsys = ar.take<SysDev>((size_t)n * sizeof(SysDev));
  double* partials = ar.take<double>(part_doubles * sizeof(double));
  double* reda = ar.take<double>((size_t)n * 4 * sizeof(double));
  double* redb = ar.take<double>((size_t)n * 4 * sizeof(double));
  double* dzero = ar.take<double>((size_t)n * sizeof(double));
  double* dbcur = ar.take<double>((size_t)n * sizeof(double));
  double* dnorm2 = ar.take<double>((size_t)n * sizeof(double));
  double* dnrm = ar.take<double>((size_t)n * sizeof(double));
  int* dactive = ar.take<int>((size_t)n * sizeof(int));
  int* ddepth = ar.take<int>((size_t)n * sizeof(int));
  double* dalog = ar.take<double>((size_t)n * ld * sizeof(double));
  double* dblog = ar.take<double>((size_t)n * ld * sizeof(double));
  double* dw = ar.take<double>((size_t)n_w * sizeof(double));
  double* dI = ar.take<double>((size_t)n * n_w * sizeof(double));
  if (ar.overflow()) return fail(MSB_EINVAL, "internal: spectrum workspace layout");

  MSB_HIP(hipMemcpyAsync(dsys, hsys.data(), n * sizeof(SysDev), hipMemcpyHostToDevice, st));
  MSB_HIP(hipMemcpyAsync(dw, w, n_w * sizeof(double), hipMemcpyHostToDevice, st));
  MSB_HIP(hipMemsetAsync(dzero, 0, n * sizeof(double), st));
  MSB_HIP(hipMemsetAsync(bufB, 0, (size_t)n * D * 16, st));
  std::vector<int> active(n, 0);
  MSB_HIP(hipMemcpyAsync(dactive, active.data(), n * sizeof(int), hipMemcpyHostToDevice, st));

  // |phi_k|^2: w = phi, w -= 0*q + 0*qprev, partial |w|^2
  MSB_HIP(hipMemcpyAsync(bufW, phi, (size_t)n * D * 16, hipMemcpyDeviceToDevice, st));
  BlockLanczosArgs bl;
  bl.w = bufW; bl.q = bufW; bl.qprev = bufW; bl.a = reda; bl.b = dzero; bl.active = dactive;
  bl.partials = partials; bl.red = redb; bl.D = D; bl.nbx = nbx_l; bl.n = n;
  MSB_HIP(hipMemsetAsync(reda, 0, (size_t)n * 4 * sizeof(double), st));
  MSB_HIP(launch_block_lanczos_update(bl, st));
  std::vector<double> hred((size_t)n * 4), norm2(n), bcur(n, 0.0);
  MSB_HIP(hipMemcpyAsync(hred.data(), redb, n * 4 * sizeof(double), hipMemcpyDeviceToHost, st));
  MSB_HIP(hipStreamSynchronize(st));
  std::vector<double> alog((size_t)n * ld, 0.0), blog((size_t)n * ld, 0.0);
  std::vector<int> depth(n, 0);
  for (int j = 0; j < n; ++j) {
    norm2[j] = hred[4 * j];
    bcur[j] = std::sqrt(norm2[j]);
    blog[(size_t)j * ld] = bcur[j];
    if (!(norm2[j] > 0)) active[j] = 1;    // phi = 0: I = 0
  }
  MSB_HIP(hipMemcpyAsync(dnorm2, norm2.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
  MSB_HIP(hipMemcpyAsync(dbcur, bcur.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
  MSB_HIP(hipMemcpyAsync(dactive, active.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
  // u_0 = phi itself (unnormalised vectors, beta_0^2 = |phi|^2), u_{-1} = 0
  MSB_HIP(hipMemcpyAsync(dnrm, norm2.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
  MSB_HIP(hipMemsetAsync(dbcur, 0, n * sizeof(double), st));      // beta_{k-1}
  double* u = bufW;
  double* up = bufB;
  double* vv = bufA;
  std::vector<double> nrm_h = norm2;
  std::vector<double> Iprev((size_t)n * n_w, 0.0), Icur((size_t)n * n_w, 0.0);
  std::vector<int> checked(n, 0);
  const int check_every = 10;
  auto eval_cf = [&](std::vector<double>& out) -> msb_status {
    MSB_HIP(hipMemcpyAsync(dalog, alog.data(), alog.size() * sizeof(double), hipMemcpyHostToDevice, st));
    MSB_HIP(hipMemcpyAsync(dblog, blog.data(), blog.size() * sizeof(double), hipMemcpyHostToDevice, st));
    MSB_HIP(hipMemcpyAsync(ddepth, depth.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
    MSB_HIP(launch_cf_eval(dalog, dblog, ddepth, ld, dnorm2, n, dw, n_w, sys->E_G, eta, dI, st));
    MSB_HIP(hipMemcpyAsync(out.data(), dI, out.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    MSB_HIP(hipStreamSynchronize(st));
    return MSB_OK;
  };

  for (int k = 0; k < kmax; ++k) {
    bool any = false;
    for (int j = 0; j < n; ++j) any |= active[j] == 0;
    if (!any) break;
    ApplyArgs aa = apply_args(ctx, dsys, n, u, vv);
    aa.shape = shp;
    aa.partials = partials;
    aa.red = reda;
    aa.status = dactive;
    aa.status_stride = 1;
    MSB_HIP(launch_apply(Elem::C128, kModeHerm, aa, st));
    BlockStepArgs bs;
    bs.v = vv; bs.u = u; bs.up = up; bs.herm = reda; bs.nrm = dnrm; bs.bprev = dbcur; bs.active = dactive;
    bs.partials = partials; bs.red = redb; bs.D = D; bs.nbx = nbx_l; bs.n = n;
    MSB_HIP(launch_block_lanczos_step(bs, st));
    std::vector<double> ha((size_t)n * 4);
    MSB_HIP(hipMemcpyAsync(ha.data(), reda, n * 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    MSB_HIP(hipMemcpyAsync(hred.data(), redb, n * 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    MSB_HIP(hipStreamSynchronize(st));
    for (int j = 0; j < n; ++j) {
      if (active[j] != 0) continue;
      alog[(size_t)j * ld + k] = ha[4 * j] / nrm_h[j];
      depth[j] = k + 1;
      const double bn = std::sqrt(hred[4 * j]);
      nrm_h[j] = hred[4 * j];
      if (k + 1 < ld) blog[(size_t)j * ld + k + 1] = bn;
      if (!(bn > 1e-14 * std::sqrt(norm2[j]))) active[j] = 2;   // invariant subspace reached
    }
    // convergence of the continued fraction every check_every steps
    if ((k + 1) % check_every == 0) {
      r = eval_cf(Icur);
      if (r != MSB_OK) return r;
      for (int j = 0; j < n; ++j) {
        if (active[j] != 0) continue;
        if (checked[j]) {
          double dmax = 0, imax = 0;
          for (int i = 0; i < n_w; ++i) {
            dmax = std::max(dmax, std::fabs(Icur[(size_t)j * n_w + i] - Iprev[(size_t)j * n_w + i]));
            imax = std::max(imax, std::fabs(Icur[(size_t)j * n_w + i]));
          }
          if (dmax <= cf_tol * imax) active[j] = 3;
        }
        checked[j] = 1;
      }
      Iprev = Icur;
    }
    MSB_HIP(hipMemcpyAsync(dactive, active.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
    std::swap(u, up);   // up now holds u_{k+1}
  }
  r = eval_cf(Icur);
  if (r != MSB_OK) return r;
  std::memcpy(I, Icur.data(), Icur.size() * sizeof(double));
  if (depth_out)
    for (int j = 0; j < n; ++j) depth_out[j] = depth[j];
  if (coef_a && coef_b) {
    // u_0 = phi, u_{k+1} = H q_k - a_k q_k - |u_k| q_{k-1} with q_k = u_k / |u_k|:
    // the logged |u_k| are b_0 = |phi| and the normalised recurrence's b_k
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < coef_ld; ++k) {
        const bool in = k < depth[j];
        coef_a[(size_t)j * coef_ld + k] = in ? alog[(size_t)j * ld + k] : 0.0;
        coef_b[(size_t)j * coef_ld + k] = in ? blog[(size_t)j * ld + k] : 0.0;
      }
  }
  return MSB_OK;
}

extern "C" msb_status msb_spectrum(msb_ctx* ctx, const msb_system* sys, const void* phi, int n,
                                   const double* w, int n_w, double eta, int lanczos_max,
                                   double cf_tol, double* I, int* depth_out, void* stream) {
  return spectrum_impl(ctx, sys, phi, n, w, n_w, eta, lanczos_max, cf_tol, I, depth_out, nullptr, nullptr, 0,
                       stream);
}

extern "C" msb_status msb_spectrum_cf(msb_ctx* ctx, const msb_system* sys, const void* phi, int n,
                                      const double* w, int n_w, double eta, int lanczos_max,
                                      double cf_tol, double* I, int* depth, double* a, double* b, int ld,
                                      void* stream) {
  if (!a || !b || !depth || ld < 1) return fail(MSB_EINVAL, "msb_spectrum_cf: coefficient arrays missing");
  return spectrum_impl(ctx, sys, phi, n, w, n_w, eta, lanczos_max, cf_tol, I, depth, a, b, ld, stream);
}

// =============================================================================
// Apply launch-shape autotuner (public entry points).
extern "C" msb_status msb_autotune(msb_ctx* ctx, int nsys, msb_prec prec, msb_shape* out, int max_out,
                                   int* n_out, void* stream) {
  (void)hipGetLastError();   // do not report an earlier call's failure
  if (!ctx) return fail(MSB_EINVAL, "msb_autotune: null context");
  if (nsys <= 0) return fail(MSB_EINVAL, "msb_autotune: nsys must be positive");
  if (!valid_prec(prec)) return fail(MSB_EINVAL, "msb_autotune: invalid precision");
  if (max_out < 0 || (max_out > 0 && !out)) return fail(MSB_EINVAL, "msb_autotune: bad output table");
  const Elem e = prec == MSB_C128 ? Elem::C128 : Elem::C64;
  std::vector<std::pair<ApplyShape, double>> table;
  msb_status r = tune_shapes(ctx, e, nsys, (hipStream_t)stream, &table);
  if (r != MSB_OK) return r;
  const int n = std::min<int>((int)table.size(), max_out);
  for (int i = 0; i < n; ++i) {
    out[i].threads = table[i].first.blk;
    out[i].elems_per_thread = table[i].first.ept;
    out[i].vectors = table[i].first.nv;
    out[i].passes = table[i].first.passes;
    out[i].row_order = table[i].first.order;
    out[i].panel_width = table[i].first.passes == 3 ? table[i].first.pw : 0;
    out[i].ms = table[i].second;
  }
  if (n_out) *n_out = (int)table.size();
  return MSB_OK;
}

extern "C" msb_status msb_set_shape(msb_ctx* ctx, int nsys, msb_prec prec, const msb_shape* shape) {
  (void)hipGetLastError();   // do not report an earlier call's failure
  if (!ctx || !shape) return fail(MSB_EINVAL, "msb_set_shape: null argument");
  if (nsys <= 0) return fail(MSB_EINVAL, "msb_set_shape: nsys must be positive");
  if (!valid_prec(prec)) return fail(MSB_EINVAL, "msb_set_shape: invalid precision");
  const Elem e = prec == MSB_C128 ? Elem::C128 : Elem::C64;
  const int modes[] = {kModePlain, kModeBilinear, kModeHerm, kModeResid, kModeSelf};
  if (shape->threads == 0) {
    for (int md : modes) ctx->shapes.erase(std::make_tuple((int)e, shape_class(nsys), md));
    return MSB_OK;
  }
  ApplyShape cand[kMaxCand];
  const int nc = apply_candidates(ctx->dn.n, elem_bytes(e), shape_class(nsys), ctx->lds_max, ctx->up.max_hops,
                                  pan_rows(ctx, e), elem_bytes(e),
                                  cand, kMaxCand);
  for (int i = 0; i < nc; ++i)
    if (cand[i].blk == shape->threads && cand[i].ept == shape->elems_per_thread &&
        cand[i].nv == shape->vectors &&
        cand[i].passes == ((shape->passes == 2 || shape->passes == 3) ? shape->passes : 1) &&
        (cand[i].passes != 3 || cand[i].pw == shape->panel_width) &&
        cand[i].order == (shape->row_order == 1 ? 1 : 0)) {
      for (int md : modes) ctx->shapes[std::make_tuple((int)e, shape_class(nsys), md)] = cand[i];
      return MSB_OK;
    }
  return fail(MSB_EINVAL, "msb_set_shape: shape not compiled or not usable for this row length");
}
