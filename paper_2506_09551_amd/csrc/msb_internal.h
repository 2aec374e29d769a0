// Internal declarations of the MI355X multi-shift BiCG library.
//
// Layout of a many-body vector: index = rank_up(u) * n_dn + rank_dn(d); the
// Hamiltonian H = H_up (x) I + I (x) H_dn + diagonal (Sec. III, Eq. Hubbard,
// with the core-hole term of Eq. intermediate_H) is applied matrix-free from
// per-spin hopping tables.  See msb.h for the public contract.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/msb.h"

namespace msb {

constexpr int kBlock = 256;            // threads per block of the streaming kernels
constexpr int kWave = 64;              // CDNA wavefront
constexpr int kNumXcd = 8;             // MI355X: 8 XCDs, workgroups dispatched round-robin

// ---- error handling ---------------------------------------------------------
void set_error(const std::string& msg);
msb_status fail(msb_status st, const std::string& msg);
#define MSB_HIP(call)                                                             \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return ::msb::fail(MSB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---- per-spin tables (host build, tables.cpp) --------------------------------
// Hop entry: (target_rank << 16) | (bond_type << 1) | neg.  The matrix element
// <c'|H_sigma|c> = -t_type * (neg ? -1 : +1), neg from the Jordan-Wigner
// parity of the occupied sites strictly between the two hop ends.
struct SpinTable {
  int L = 0, N = 0, n = 0;
  std::vector<uint32_t> conf;   // [n] ascending configs
  std::vector<uint32_t> off;    // [n + 1] CSR offsets into hop
  std::vector<uint32_t> hop;    // packed hop entries
  std::vector<uint32_t> order;  // [n] ranks by ascending sum of occupied site indices, then rank
  int max_hops = 0;
};
// bt_fwd[b]: type of the hop i_b -> j_b, bt_bwd[b]: of j_b -> i_b (equal for
// symmetric bonds)
bool build_spin_table(int L, int N, const std::vector<int>& bi, const std::vector<int>& bj,
                      const std::vector<int>& bt_fwd, const std::vector<int>& bt_bwd, SpinTable& out,
                      std::string& err);

// ---- host tridiagonal eigensolver (tridiag.cpp) ------------------------------
// Lowest eigenvalue of the symmetric tridiagonal T (diag a[0..k), offdiag b[0..k-1))
// by Sturm-sequence bisection, and its unit eigenvector by inverse iteration.
double tridiag_lowest(const std::vector<double>& a, const std::vector<double>& b,
                      std::vector<double>& y);

// ---- device-side structures ---------------------------------------------------
struct SysDev {                 // one linear system / Hamiltonian instance
  double U;
  double Uc;
  double d_re;                  // real diagonal offset (e.g. -(E_G + shift))
  double d_im;                  // imaginary diagonal (e.g. -Gamma)
  int core;                     // core-hole site or -1
  int pad;
  double amp[MSB_MAX_BOND_TYPES];
};

struct TablesDev {
  const uint32_t* conf_up;
  const uint32_t* conf_dn;
  const uint32_t* off_up;
  const uint32_t* off_dn;
  const uint32_t* hop_up;
  const uint32_t* hop_dn;
  // down-spin hops, one padded transposed table per bond type t (types in
  // order, k_type[t] rows of n_dn words each): word g of state d holds its
  // hops 4g .. 4g+3 as 16-bit entries = target column, with bit 15 set where
  // the matrix element is -t (even parity); padding = n_dn
  const uint64_t* ell_dn;
  // up-spin hops in the same form (padding = n_up), k_type_up[t] words of
  // type t; null when the up-spin sector has 32768 states or more
  const uint64_t* ell_up;
  // up-spin hops of the LDS panel pass in row-count order (null when not
  // built: 16384 up-spin states or more, or more than two bond types):
  // pan_perm[p] = row at position p, pan_woff[w] .. pan_woff[w + 1] = words of
  // wavefront w (positions 64 w .. 64 w + 63), pan_ell[q * 64 + lane] = four
  // 16-bit hops (target | type << 14 | even-parity sign bit 15), padding n_up
  const uint32_t* pan_perm;
  const int* pan_woff;
  const uint64_t* pan_ell;
  const uint32_t* order_up;   // [n_up] up-spin rows in level order (SpinTable::order)
  int n_up, n_dn, k_dn;       // k_dn: sum of k_type (words of four hops)
  int k_up_max;               // most up-spin hops of one row
  int n_types;
  int k_type[MSB_MAX_BOND_TYPES];
  int k_type_up[MSB_MAX_BOND_TYPES];
};
constexpr uint32_t kNoHop = 0xFFFFFFFFu;

// Apply kernel modes (fused reductions).
enum ApplyMode : int {
  kModePlain = 0,       // v = A x
  kModeBilinear = 1,    // v = A x;  partial (sum aux*v, sum |v|^2)        -- COCG sigma
  kModeHerm = 2,        // v = A x;  partial (sum conj(x)*v, sum |v|^2)    -- Lanczos a_k
  kModeResid = 3,       // no v;     partial (sum |aux - A x|^2)           -- true residual
  kModeSelf = 4         // v = A x + beta v with x the aux bank slot read in place; partial
                        // (sum x*v, sum |v|^2), x from the staged row -- recurred COCG sigma
};

// Launch shape of the apply kernel: threads per workgroup, elements per
// thread, vectors (systems) per workgroup of the row kernel, whether the
// diagonal and the up-spin hops run first in a separate column-panel pass
// (passes = 2: panels gathered from one XCD's L2; passes = 3: panels of pw
// columns staged in LDS), and the order in which the XCDs walk the rows (order 0: each
// XCD one contiguous range of ranks of every system; order 1: the rows of
// all systems in level order, one contiguous eighth per XCD).  blk == 0
// selects the default.
struct ApplyShape {
  int blk, ept, nv, passes, order;
  int pw;                     // passes = 3: columns of the LDS-staged panel of the first pass
};

struct ApplyArgs {
  TablesDev T;
  const SysDev* sys;          // [nsys]
  const void* x;              // [nsys][D]
  void* v;                    // [nsys][D]  (unused in kModeResid)
  const void* aux;            // [nsys/aux_div][D] (bilinear / resid modes)
  int aux_div;
  const int* aux_m;           // optional: aux is a bank [nsys][aux_cap][D]; the slot of
  const int* aux_base;        //   system s is aux_m[s*status_stride] - *aux_base
  int aux_cap;
  const int* status;          // optional: per-system status stride, skip if != 0
  int status_stride;          // in ints
  double* partials;           // [nsys][nbx][4]
  double* red;                // [nsys][4] reduced sums
  int64_t D;
  int nbx;                    // workgroups along the rows (XCD-padded row count)
  int rows_per_xcd;
  int nsys;
  int nvec;                   // vectors (systems) per workgroup (set by the launcher)
  ApplyShape shape;           // requested launch shape ({0,0,0,0} = default)
  size_t lds_max;             // LDS bytes one workgroup may use (device limit)
  const void* vin;            // set by the launcher for the second pass: v holds diag + up-spin hops
  int ordered;                // set by the launcher: row order of the shape (ApplyShape::order)
  int x_from_aux;             // set by the launcher in kModeSelf: the operand is the aux bank
                              //   slot of each system (x unused)
  const double* beta;         // kModeSelf, optional: v = A x + beta_s v (v read in place, skipped
  int beta_stride;            //   where beta_s = 0); beta_s = beta[s * beta_stride + {0, 1}]
};

enum class Elem { R64, C128, C64 };   // real float64, complex128, complex64 storage

hipError_t launch_apply(Elem e, int mode, const ApplyArgs& a, hipStream_t st);
int apply_nbx(int n_up, int nsys);  // grid.x (workgroups per system) for the apply kernel
int apply_rows_per_xcd(int n_up);
// Compiled shapes usable for rows of nd elements (row_bytes per element of the
// staged row) and nsys systems; pan_nu > 0 adds the LDS panel first pass for
// n_up = pan_nu rows of pan_es-byte elements.  Returns how many were written.
int apply_candidates(int nd, size_t row_bytes, int nsys, size_t lds_max, int k_up_max, int pan_nu,
                     size_t pan_es, ApplyShape* out, int max_out);
// The shape launch_apply(e, mode, a) will use.
ApplyShape apply_shape_used(Elem e, int mode, const ApplyArgs& a);
// Interleaved block apply (modes plain and bilinear): x and v hold groups of
// G systems interleaved, [nsys / G][D][G] (ApplyArgs::x, v; aux, status and
// the bank slots keep one vector per system).  Two passes: column panels for
// the diagonal and H_up (x) I, then rows for I (x) H_dn.
hipError_t launch_apply_il(Elem e, int mode, int G, const ApplyArgs& a, hipStream_t st);
// Interleave width for nsys systems of elem_bytes elements (4, 2, or 0 when
// the staged rows or the panel work lists do not fit).
int apply_il_width(int nd, size_t elem_bytes, int nsys, size_t lds_max, int k_up_max);

// ---- COCG seed step kernels (k_cocg.hip) -----------------------------------
// Per-system state.  status codes:
// One iteration runs p-update, apply, r-update (+ bookkeeping) in that order,
// so a chunk boundary falls between the bookkeeping of iteration m-1 and the
// p-update of iteration m (where the residual may be replaced).
// kPaused: the bank has no slot for the next residual; the host flushes it.
// kFloor: complex64 attainable accuracy reached, seen at a residual
// replacement either as a recurrence residual more than kFloorGap times below
// the true one, or as kStallMax replacements in a row where the recurrence
// claimed to have cut the best true residual by kStall but the true residual
// did not follow.
enum : int { kActive = 0, kDone = 1, kBreakdown = 2, kMaxit = 3, kPaused = 4, kFloor = 5, kExhausted = 6 };
// kExhausted: the seed's residual fell below kSeedFloor |E| (or beta stopped
// being finite) with shifts still open; its bilinear products would leave the
// normal float64 range, so it stops and the open shifts are unconverged.
constexpr double kSeedFloor = 1e-150;
constexpr double kFloorGap = 10.0;
// Residual replacement stops once |r_m| <= max(tol, kReplaceFloor) |E|: the FP64
// product E - A x cannot resolve much less (about 1e-15 relative was measured).
constexpr double kReplaceFloor = 1e-12;
constexpr double kStall = 0.5;
constexpr int kStallMax = 3;
struct SysState {
  double rho_re, rho_im;        // rho_m = r_m^T r_m
  double ap_re, ap_im;          // alpha_{m-1}
  double bp_re, bp_im;          // beta_{m-1}
  double al_re, al_im;          // alpha_m (current)
  double be_re, be_im;          // beta_m (current)
  double rnorm;                 // |r_m|
  double normE;                 // |E|
  int m;                        // completed iterations
  int status;
  int n_active;                 // shifts still iterating
  int breakdown_iter;
  double rbest;                 // smallest true residual seen at a replacement (|E| at start)
  int n_stall;                  // replacements in a row that exposed a false improvement
  int pad;
  double rtnorm;                // |r~_m| of the dual-space form (= rnorm otherwise)
};

struct CocgArgs {
  SysState* st;                 // [nsys]
  const double* red1;           // [nsys][4] from the apply (sigma re, im, |v|^2)
  double* partials;             // [nsys][nbx][4]
  double* red2;                 // [nsys][4]
  void* bank;                   // [nsys][cap][D] residual bank
  const void* vvec;             // [nsys][D]
  void* pvec;                   // [nsys][D]
  const int* base;              // device: iteration index held in bank slot 0
  int cap;                      // bank slots per system
  int64_t D;
  int nbx;
  int nsys;
  // shift recurrences (done in the last block of the residual kernel)
  int n_shift;
  const double* wshift;         // [n_shift]  w - seed_shift
  double* zeta;                 // [nsys][n_shift][2]   zeta_m
  double* zeta_prev;            // [nsys][n_shift][2]   zeta_{m-1}
  int* conv_iter;               // [nsys][n_shift]      -1 while active
  double tol;
  int maxit;
  double* alpha_log;            // [nsys][maxit][2]
  double* beta_log;             // [nsys][maxit][2]
  double* rnorm_log;            // [nsys][maxit+1]
  double* xseed;                // optional [nsys][D] complex128 seed solution (x += alpha p)
  double rep_floor;             // residual replacement only while |r_m| > rep_floor |E|
  // dual-space form (null for the complex-symmetric one): shadow residual r~,
  // direction p~ and vt = A^T p~, each [nsys][D]
  void* rt;
  void* pt;
  const void* vt;
  int il;                       // > 0: p and v interleaved in groups of il systems ([nsys/il][D][il])
};

hipError_t launch_cocg_r(Elem e, const CocgArgs& a, hipStream_t st);   // r_{m+1} = r_m - alpha v
hipError_t launch_cocg_p(Elem e, const CocgArgs& a, hipStream_t st);   // p_m = r_m + beta_{m-1} p_{m-1}
// Recurred seed form with residual replacement: the seed solution and the
// last direction, as linear combinations of the bank slots written since the
// previous rebuild (Alg. 1: x_{j+1} = x_j + alpha_j p_j, p_j = r_j + beta_{j-1} p_{j-1}):
//   x <- x + sum_l cx[l] r_l + cx[L] p,   p <- sum_l cp[l] r_l + cp[L] p
// for systems that are active or paused.  coef: [nsys][2][L + 1] complex.
struct RebuildArgs {
  const void* bank;             // [nsys][cap][D] of the vector precision
  int cap;
  int slot0;                    // bank slot of the first residual combined
  int L;                        // residuals combined (slots slot0 .. slot0 + L - 1)
  int64_t D;
  int nbx;
  int nsys;
  const double* coef;
  double* x;                    // [nsys][D] complex128
  void* p;                      // [nsys][D] of the vector precision
  const SysState* st;
};
hipError_t launch_seed_rebuild(Elem e, const RebuildArgs& a, hipStream_t st);
// Residual replacement: r_m <- E - w (w = A_s x_m in complex128, computed by the
// apply), rho_m and |r_m| recomputed in FP64, beta_{m-1} rescaled accordingly.
hipError_t launch_cocg_replace(Elem e, const CocgArgs& a, const double* E, const double* w,
                               hipStream_t st);
int cocg_nbx(int64_t D, int nsys);

// Initialisation: bank slot 0 = p = E (converted to Elem), rho_0 = E^T E, |E|.
struct InitArgs {
  const double* E;              // [nsys][D] complex128
  void* bank;                   // slot 0 of each system
  void* pvec;
  SysState* st;
  double* partials;
  int cap;
  int64_t D;
  int nbx;
  int nsys;
  int n_shift;
  double* zeta;
  double* zeta_prev;
  int* conv_iter;
  double* rnorm_log;
  int maxit;
  double* xseed;                // optional: zeroed
  void* psnap;                  // optional: set to E (the direct form's copy of p for x rebuilds)
  void* rt;                     // optional (dual-space form): r~_0 = p~_0 = E
  void* pt;
  int il;                       // > 0: p interleaved in groups of il systems
};
hipError_t launch_cocg_init(Elem e, const InitArgs& a, hipStream_t st);

// ---- multi-shift assembly (k_shift.hip) --------------------------------------
struct CoefArgs {
  const SysState* st;
  const double* alpha_log;      // [nsys][maxit][2]
  const double* beta_log;
  const double* wshift;         // [n_shift]
  const int* conv_iter;         // [nsys][n_shift]
  const int* list;              // [nsys][n_list] shift index per sorted slot (-1 = empty)
  const int* lend;              // [nsys][n_list] end of the shift's range within the block
  double* coef;                 // [nsys][K][n_list][ncomp]   Psi coefficients of r_base+l
  double* gcoef;                // [nsys][K][n_list][ncomp]   p coefficients (carry) or null
  double* ab;                   // [nsys][n_list][4]: (a_re,a_im) = p_prev weight in Psi, (h_re,h_im) in p
  int nsys, n_shift, n_list, maxit, K, base;
  int ncomp;                    // 2: (c_re, c_im); 3: (c_re, c_re + c_im, c_im - c_re) for the
                                //   three-product assembly (flush_coef_comps(engine))
};
hipError_t launch_coef(const CoefArgs& a, double* scratch /*[nsys*n_list][K][4]*/, hipStream_t st);

struct FlushArgs {
  const void* bank;             // [nsys][cap][D]
  int cap;
  const double* coef;           // [nsys][K][n_list][flush_coef_comps(engine)] (slot-major)
  const double* pw;             // [nsys][n_list][2]: weight of X (p_prev) term, or null
  const double* ow;             // [nsys][n_list][2]: weight of old output, or null (= 0)
  int pw_stride, ow_stride;     // doubles between consecutive entries of pw / ow
  const int* list;              // [nsys][n_list]
  const int* tile_k;            // [nsys][n_tiles] K extent of each shift tile
  const int* lend;              // [nsys][n_list] slots of each listed shift (descending), or null
  void* out;                    // [nsys][n_shift][D]   (Psi, or P in place)
  const void* X;                // [nsys][n_shift][D]   p_prev (or null)
  int64_t D;
  int n_shift, n_list, K, nsys;
  int n_etiles, n_stiles;
  void* work = nullptr;         // engine 5: coefficient digit planes (flush_work_bytes)
  const double* rnorm = nullptr;  // engine 5: |r_m| log [nsys][rn_stride]; slot l is m = rn_base + l
  int rn_stride = 0, rn_base = 0;
};
// ow_mode: 0 = old output ignored, 1 = weight 1, 2 = per-shift weights from ow
// engine: 0 = FP64 vector ALU, three real products per complex product (the
// default), 1 = FP64 matrix cores, 2 = FP64 vector ALU, four real products,
// 3 = as 0 with eight wavefronts (64 shifts per workgroup), 4 = eight
// wavefronts of four shifts and 256 elements, 5 = int8 matrix cores on
// 8-bit digit planes of the FP64 operands (six planes for a complex128 bank,
// five for complex64), 6 = FP64 matrix cores, three real products
// (complex128 bank)
constexpr int kNumFlushEngines = 7;
size_t flush_work_bytes(int engine, int nsys, int n_list, int K);
// engine 5 (k_flush_oz.hip): coefficient digit planes, then the contraction
hipError_t launch_flush_oz(Elem bank, Elem out, const FlushArgs& a, dim3 grid, int ow_mode, hipStream_t st);
// engine 6 (k_flush_mf64.hip)
hipError_t launch_flush_mf64(Elem out, const FlushArgs& a, int ow_mode, hipStream_t st);
hipError_t launch_flush(Elem bank, Elem out, const FlushArgs& a, int ow_mode, int engine,
                        hipStream_t st);
int flush_shifts_per_tile(int engine);
int flush_elems_per_tile(int engine);
int flush_coef_comps(int engine);   // doubles per coefficient table entry (2 or 3)

// ---- Lanczos helpers (k_lanczos.hip) -----------------------------------------
// Generic last-block reductions and axpy-style updates used by the ground
// state and the continued fraction.
hipError_t launch_dot_many(const double* Q, int k, const double* w, int64_t D,
                           double* partials, double* out, hipStream_t st);
hipError_t launch_gemv_sub(const double* Q, int k, const double* c, double* w, int64_t D,
                           hipStream_t st);
hipError_t launch_gemv(const double* Q, int k, const double* c, double* out, int64_t D,
                       hipStream_t st);
// real FP64: w -= a q + b qprev ; partial |w|^2
hipError_t launch_lanczos_real_update(double* w, const double* q, const double* qprev,
                                      const double* ab /*host-visible device pair*/, int64_t D,
                                      double* partials, double* out,
                                      hipStream_t st);
hipError_t launch_scale_real(const double* w, const double* s, double* q, int64_t D,
                             hipStream_t st);

// Complex block Lanczos (continued fraction): per vector j
//   w_j -= a_j q_j + b_j qprev_j ; partial |w_j|^2
struct BlockLanczosArgs {
  double* w;                    // [n][D] complex128
  const double* q;
  const double* qprev;
  const double* a;              // [n]  (device)
  const double* b;              // [n]
  const int* active;            // [n]
  double* partials;             // [n][nbx][4]
  double* red;                  // [n][4]
  int64_t D;
  int nbx, n;
};
hipError_t launch_block_lanczos_update(const BlockLanczosArgs& a, hipStream_t st);
struct BlockStepArgs {
  const double* v;              // [n][D] H u_k
  const double* u;              // u_k
  double* up;                   // u_{k-1} in, u_{k+1} out
  const double* herm;           // [n][4] <u_k|H u_k> in [4 j]
  double* nrm;                  // [n] |u_k|^2, advanced to |u_{k+1}|^2
  double* bprev;                // [n] |u_{k-1}| (0: no previous vector), advanced
  const int* active;            // [n]
  double* partials;             // [n][nbx][4]
  double* red;                  // [n][4] |u_{k+1}|^2
  int64_t D;
  int nbx, n;
};
hipError_t launch_block_lanczos_step(const BlockStepArgs& a, hipStream_t st);
int lanczos_nbx(int64_t D, int n);     // workgroups per vector of the block update
int gram_blocks(int64_t D);            // partial rows of launch_dot_many
// q_prev <- w / b (per vector, active only); returns via pointer rotation by the host
hipError_t launch_block_scale(const double* w, const double* b, const int* active, double* out,
                              int64_t D, int n, hipStream_t st);
hipError_t launch_cf_eval(const double* a, const double* b, const int* depth, int ld, const double* norm2,
                          int n, const double* w, int n_w, double E_G, double eta, double* I,
                          hipStream_t st);

// ---- small utility kernels ---------------------------------------------------
// Site operator c+ / c of one spin between two sectors (k_dipole.hip).
constexpr int kMaxSites = 20;
struct DipoleArgs {
  const int* table;             // [n_sites][n_conf]: input rank << 1 | (sign < 0), or -1
  const void* x;                // [nvec][D_src] complex128
  void* y;                      // [nvec][D_dst] complex128
  int64_t D_src, D_dst;
  int nd_src, nd_dst;           // down-spin states of each sector (row lengths)
  int n_conf;                   // output configurations of the operator's spin
  int n_sites, spin;
  int accumulate;               // y += op x instead of y = op x
  double coef_re[kMaxSites], coef_im[kMaxSites];
};
hipError_t launch_dipole(const DipoleArgs& a, int nvec, hipStream_t st);

hipError_t launch_number_op(const TablesDev& T, int64_t D, int site, double w_up, double w_dn,
                            int count, int x_real, const void* x, double* y, hipStream_t st);
hipError_t launch_combine(const TablesDev& T, int64_t D, int nsys, int n, Elem e, const void* psi,
                          const double* coef /*[nsys][4]: phase re, im, w_up, w_dn*/,
                          const int* site /*[nsys]*/, double* phi, hipStream_t st);
hipError_t launch_copy_slot(Elem e, const void* src, void* dst, int64_t D, int nsys,
                            int64_t src_stride, int64_t dst_stride, hipStream_t st);

}  // namespace msb

// Context (opaque in the public header).
struct msb_ctx {
  int L = 0, n_up = 0, n_dn = 0;
  int64_t D = 0;
  int n_types = 0;
  double type_amp[MSB_MAX_BOND_TYPES] = {0};
  double U = 0;
  msb::SpinTable up, dn;
  int device = 0;
  size_t lds_max = 64 * 1024;         // LDS per workgroup (queried from the device)
  // device tables
  uint32_t* d_conf_up = nullptr;
  uint32_t* d_conf_dn = nullptr;
  uint32_t* d_off_up = nullptr;
  uint32_t* d_off_dn = nullptr;
  uint32_t* d_hop_up = nullptr;
  uint32_t* d_hop_dn = nullptr;
  uint64_t* d_ell_dn = nullptr;
  uint64_t* d_ell_up = nullptr;
  uint32_t* d_pan_perm = nullptr;
  int* d_pan_woff = nullptr;
  uint64_t* d_pan_ell = nullptr;
  uint32_t* d_order_up = nullptr;
  int k_type_dn[MSB_MAX_BOND_TYPES] = {0};   // words (four hops each) of each bond type's down-spin table
  int k_type_up[MSB_MAX_BOND_TYPES] = {0};   // the same for the up-spin table
  int type_partner[MSB_MAX_BOND_TYPES] = {0}; // type of the reverse hop (itself when symmetric)
  // private stream for the captured seed iterations (default priority)
  hipStream_t solve_stream = nullptr;
  hipStream_t part_stream[3] = {};         // the other parts of a split seed batch
  double* d_small = nullptr;          // small reduction outputs
  // growable workspace
  void* ws = nullptr;
  size_t ws_size = 0;
  // apply launch shapes chosen by the autotuner (or pinned), key (Elem,
  // min(nsys, 16), apply mode): the fused reductions change a kernel's
  // registers and occupancy, so each mode is tuned where it runs
  std::map<std::tuple<int, int, int>, msb::ApplyShape> shapes;
  msb::TablesDev tables() const {
    msb::TablesDev t;
    t.conf_up = d_conf_up; t.conf_dn = d_conf_dn;
    t.off_up = d_off_up; t.off_dn = d_off_dn;
    t.hop_up = d_hop_up; t.hop_dn = d_hop_dn;
    t.ell_dn = d_ell_dn;
    t.ell_up = d_ell_up;
    t.pan_perm = d_pan_perm;
    t.pan_woff = d_pan_woff;
    t.pan_ell = d_pan_ell;
    t.order_up = d_order_up;
    t.n_up = up.n; t.n_dn = dn.n; t.k_dn = 0;
    t.k_up_max = up.max_hops;
    t.n_types = n_types;
    for (int i = 0; i < MSB_MAX_BOND_TYPES; ++i) {
      t.k_type[i] = i < n_types ? k_type_dn[i] : 0;
      t.k_type_up[i] = i < n_types ? k_type_up[i] : 0;
      t.k_dn += t.k_type[i];
    }
    return t;
  }
};
