// C ABI of the solver: workspace layout, setup, iteration scheduling (HIP
// graphs), convergence checks and outputs.  Host code only; kernels live in
// setup.hip and sweep_sparse.hip.
#include "mmot_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <vector>

namespace mmot {
// setup.hip
void launch_validate_vals(const double*, size_t, int, int, int, int*, hipStream_t);
void launch_validate_csr(const int*, const int*, int, long long, int*, hipStream_t);
void launch_validate_mass(const double*, const double*, int, int, int*, double*, hipStream_t);
template <typename V, bool LOG> void launch_gibbs(const double*, size_t, double, V*, hipStream_t);
void launch_transpose_pattern(const int*, const int*, int, long long, int*, int*, int*, int*, int*, hipStream_t);
template <typename V> void launch_gather_vals(const V*, const int*, long long, V*, hipStream_t);
template <typename V, bool LOG> void launch_rowsum_max(const int*, const V*, int, double, uint32_t*, hipStream_t);
template <typename V> void launch_to_panel(const double*, int, int, int, int, double, V, V*, hipStream_t);
template <typename V, bool LOG> void launch_cap(const double*, int, int, int, V*, hipStream_t);
template <typename V> void launch_fill(V*, size_t, V, hipStream_t);
template <typename V, bool LOG> void launch_init_u0t(const V*, size_t, V*, hipStream_t);
void launch_init_offsets(double*, double*, double*, double*, int, int, const uint32_t*, hipStream_t);
template <typename V, bool LOG>
void launch_log_duals(const V*, const double*, const V*, const double*, const V*, int, int, int, int, double*,
                      double*, double*, hipStream_t);
template <typename V, bool LOG>
void launch_set_duals(const double*, const double*, const double*, int, int, int, int, V*, V*, V*, double*, double*,
                      hipStream_t);
template <typename V, bool LOG>
void launch_comm_duals(const V*, int, int, int, int, double*, int, const double*, V*, hipStream_t);
void launch_excess(const int*, const int*, const double*, int, double*, int*, double*, hipStream_t);
void launch_max_degree(const int*, int, int*, hipStream_t);
template <typename V> void launch_build_ell(const int*, const int*, const V*, int, int, V, int*, V*, int*, hipStream_t);
// sweep_sparse.hip
template <typename V, bool LOG> void launch_step(const StepArgs<V>&, int, int, hipStream_t);
template <typename V, bool LOG>
void launch_source(int, int, int, int, const V*, const V*, V*, uint32_t*, int, size_t, int*, unsigned long long*, int,
                   size_t, int, hipStream_t);
template <typename V, bool LOG>
void launch_check0(int, int, int, int, int, const V*, const V*, const V*, const double*, const double*, double*,
                   double*, double*, int, int, int, hipStream_t);
template <typename V, bool LOG>
void launch_sink_check(int, int, int, int, int, const V*, const V*, const V*, const double*, const double*, double*,
                       int, hipStream_t);
template <typename V, bool LOG>
void launch_flows(int, int, int, int, int, const int*, const int*, const V*, const double*, const V*, const V*,
                  const V*, const V*, const double*, const double*, double*, double*, int, hipStream_t);
template <typename V, bool LOG>
void launch_prep_bwd(int, int, const double*, double*, V*, const double*, double*, uint32_t*, int, hipStream_t);
template <typename V, bool LOG>
void launch_prep_fwd(int, int, int, const double*, double*, const double*, V*, V*, double*, double*, double*, uint32_t*,
                     int, hipStream_t);
void launch_growth(double*, const float*, int, int, int, hipStream_t);
void launch_levels(uint32_t*, float*, int, int, int, hipStream_t);
void launch_levels64(unsigned long long*, uint32_t*, float*, int, int, int, int, hipStream_t);
void launch_reduce_stats(const double*, int, int, int, int, double*, double, double*, hipStream_t);
void launch_reduce_cost(const double*, const double*, int, int, int, int, double*, double*, double*, hipStream_t);
// dense_mfma.hip
void launch_gemm(const GemmArgs&, bool, hipStream_t);
int gemm_col_tiles(int);
void launch_dense_rows(int, int, const float*, const float*, float*, int, double*, double*, const float*, uint16_t*,
                       float*, int, int, int, const double*, int, hipStream_t);
void launch_dense_sink(int, int, int, const float*, const float*, float*, int, const double*, const double*,
                       uint32_t*, int, uint32_t*, size_t, int*, double*, double*, double*, int, int, int,
                       hipStream_t);
void launch_dense_gibbs(const double*, int, int, double, float*, float*, void*, void*, hipStream_t);
void launch_dense_operand(int, int, const float*, const float*, uint16_t*, hipStream_t);
void launch_dense_operand32(int, int, int, const float*, const float*, float*, hipStream_t);
void launch_dense_rowsum_max(const float*, int, int, uint32_t*, hipStream_t);
void launch_dense_flows(int, int, int, int, const float*, const float*, const float*, const float*, const double*,
                        const double*, float*, const float*, double, double*, double*, int, hipStream_t);
void launch_dense_state_cost(int, int, int, const float*, const float*, const float*, const float*, const float*,
                             const double*, const double*, double, double*, int, hipStream_t);
void launch_dense_comm_stats(int, int, int, const float*, const float*, const float*, const float*, const float*,
                             const float*, const double*, const double*, double*, int, hipStream_t);
void launch_pool_tick(const TickArgs&, bool, hipStream_t);
bool pool_item_is_light(const PoolItem&);

// ---- recording of kernel launches into serving-pool work items ----
struct Recorder {
  std::vector<PoolItem> items;
  bool ok = true;
};
thread_local Recorder* tl_recorder = nullptr;
bool record_item(int kind, int log_domain, int nblk, const void* args, size_t bytes) {
  Recorder* r = tl_recorder;
  if (!r) return false;
  if (bytes > (size_t)kItemArgBytes) { r->ok = false; return true; }
  PoolItem it;
  std::memset(&it, 0, sizeof(it));
  it.kind = kind;
  it.log_domain = log_domain;
  it.nblk = nblk;
  std::memcpy(it.args, args, bytes);
  r->items.push_back(it);
  return true;
}
}  // namespace mmot

using namespace mmot;

namespace {

struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += std::max<size_t>(count, 1) * sizeof(T);
    return p;
  }
};

}  // namespace

struct mmot_solver {
  // problem
  int n = 0, L = 0, T = 0, kind = 0;
  long long nnz = 0;
  double eps = 0;
  bool has_kl = false;
  bool has_comm = false;          // commodity-dependent capacities D_t
  int comm_steps = 1;             // D value sets: T-1 (per step) or 1
  mmot_options opt{};
  int prec = MMOT_FP32;   // FP32 or FP64 (element type V)
  int dom = MMOT_DOMAIN_SCALED;
  hipStream_t stream = nullptr;
  // geometry
  int vsize = 4, Lp = 0, G = 64, nchunk = 1, nblk = 8, nslot = 1;
  // sparse sweep steps: 2^lwpr waves per whole-wave row, nblk_s blocks (>= nblk,
  // the block count of the row kernels); stats partials are nblk_s apart per time
  int lwpr = 0, nblk_s = 8;
  // device buffers (carved from the workspace)
  int *rp_b = nullptr, *ci_b = nullptr, *rp_f = nullptr, *ci_f = nullptr;
  int *cnt = nullptr, *cursor = nullptr, *srcpos = nullptr;
  void *kv_b = nullptr, *kv_f = nullptr;
  int steps_k = 1;                 // operator value sets: T for a time-varying network, else 1
  double* cost = nullptr;
  void *KL = nullptr, *cap = nullptr, *R01 = nullptr, *R0T = nullptr, *U01 = nullptr, *U0T = nullptr;
  void *psi = nullptr, *zh = nullptr, *u = nullptr;
  void *dcomm = nullptr, *wcomm = nullptr;   // D_t and w_t panels [n][Lp] per interior time
  void* ones = nullptr;                      // [n] u of an input time without capacity (1, log: 0)
  double *cb = nullptr, *cf = nullptr, *sigb = nullptr, *sigf = nullptr, *gauge0 = nullptr, *gaugeT = nullptr;
  void *facb = nullptr, *facf = nullptr, *wgt = nullptr;
  uint32_t *slots_b = nullptr, *slots_f = nullptr, *slotsE = nullptr, *slotsS = nullptr, *rho = nullptr;
  // log domain calibration keys (plan level, stored value), sparse path only
  unsigned long long *cslots_b = nullptr, *cslots_f = nullptr;
  int ncslot = 1;
  double *lvlT = nullptr, *lvl0 = nullptr;
  float *levb = nullptr, *levf = nullptr;
  double *part = nullptr, *tpart = nullptr, *stats_dev = nullptr, *masses = nullptr;
  double *part_flow = nullptr, *tpart_flow = nullptr;
  double* part_cc = nullptr;   // dense check pass: commodity-capacity partials of the product's blocks
  bool keep_fwd = false;       // forward messages of every time kept (see mmot_options::keep_forward)
  bool hat_valid = false;      // the kept forward messages are those of the current scalings
  bool keep_now = false;       // the forward sweep being recorded keeps every time's message
  double *exc_row = nullptr, *exc = nullptr;
  int* exc_cnt = nullptr;
  int* flags = nullptr;
  // dense operators: K and K^T row-major with leading dimension lda (FP32, and
  // BF16 copies when the solver was created with MMOT_BF16); products in BF16
  // while dense_bf16, FP32 otherwise (polish)
  int lda = 0, ntn = 0;
  bool dense_bf16 = false, has_bf16 = false;
  float *Kd = nullptr, *Ktd = nullptr, *part_s = nullptr;
  void *Kb = nullptr, *Ktb = nullptr;
  uint16_t* Bbuf[2] = {nullptr, nullptr};   // BF16 products: next operand, u-scaled, k-blocked (rows padded to 64)
  float* B32buf[2] = {nullptr, nullptr};     // FP32 products: the same in FP32, 32-row interleaved blocks
  int n8 = 0;
  // per-commodity output window of the output pass: commodities pc_lo .. pc_lo + pc_cnt - 1
  int pc_lo = 0, pc_cnt = 0;
  // ELL copies of the operators (row width ellD, 0 = use CSR)
  int ellD = 0;
  int *ell_ci_b = nullptr, *ell_ci_f = nullptr, *deg_b = nullptr, *deg_f = nullptr, *maxdeg = nullptr;
  void *ell_kv_b = nullptr, *ell_kv_f = nullptr;
  // host state
  int64_t iters = 0;
  bool psi_fresh = false, pend_b = false, pend_f = false;
  int force_calib = 0;
  bool probe_clean = false;        // the scaled domain passed the AUTO probe iteration
  hipStream_t cap_stream = nullptr;
  std::map<int, hipGraphExec_t> graphs;
  double* host_stats = nullptr;   // pinned (or the caller's pageable buffers: owns_host false)
  int* host_flags = nullptr;
  bool owns_host = false;

  size_t panel_elems() const { return (size_t)n * Lp; }
  template <typename V> V* P(void* p) const { return static_cast<V*>(p); }
};

namespace {

int next_pow2(int x) { int p = 1; while (p < x) p <<= 1; return p; }
constexpr int64_t kStepWaves = 2048;    // a sweep step of fewer waves (two per SIMD) splits its rows
constexpr int kEllMax = 16;    // widest ELL row (one gather batch); wider graphs use CSR
constexpr int kDenseCommBlocks = 256;   // blocks of a dense check pass's commodity-capacity statistics

// the kept forward messages serve the statistics of a fused check, which runs on
// dense networks and on ELL operators of a fixed sparse network, without
// per-commodity epilogues (a sparse network whose rows turn out wider than an ELL
// row keeps the room unused and checks by a forward pass)
bool keeps_forward(const mmot_problem* p, const mmot_options* o) {
  return o->keep_forward != 0 && (p->kind == MMOT_DENSE || !p->cost_per_step) && !p->state_cost && !p->cap_comm &&
         p->T >= 2;
}

void set_geometry(mmot_solver* s) {
  s->vsize = (s->prec == MMOT_FP64) ? 8 : 4;
  const int vec = 16 / s->vsize;
  s->Lp = (s->L + vec - 1) / vec * vec;
  const int lanes = s->Lp / vec;
  s->G = std::min(64, next_pow2(lanes));
  s->nchunk = (lanes + s->G - 1) / s->G;
  const int rows_per_block = kWaves * (64 / s->G);
  int nblk = (s->n + rows_per_block - 1) / rows_per_block;
  nblk = (nblk + 7) / 8 * 8;
  s->nblk = nblk;
  // Sweep steps with few rows of several column chunks (a few hundred states with
  // hundreds of commodities) would leave most SIMDs idle with one wave per row,
  // so whole-wave rows are split over two or four waves until the step has about
  // two waves per SIMD.  Steps that already fill the GPU keep one wave per row:
  // on the 10^4-row road grid, splitting its rows of eight chunks over two or
  // four waves measured 1% and 3% slower (the per-row set-up and the commodity
  // reduction are repeated per wave, and the per-chunk work does not change).
  s->lwpr = 0;
  if (s->kind == MMOT_CSR && s->G == 64) {
    while (s->lwpr < 2 && (2 << s->lwpr) <= s->nchunk && (int64_t)s->n << s->lwpr < kStepWaves) ++s->lwpr;
  }
  const int rows_per_block_s = (kWaves >> s->lwpr) * (64 / s->G);
  s->nblk_s = ((s->n + rows_per_block_s - 1) / rows_per_block_s + 7) / 8 * 8;
  s->nslot = std::max(1, std::min(32, nblk / 16));
  s->ncslot = std::min(s->nslot, 8);
  if (s->kind == MMOT_DENSE) {
    s->lda = (s->n + 63) / 64 * 64;   // K extent zero-padded to whole 64-deep product stages
    s->ntn = gemm_col_tiles(s->Lp);
  }
}

void carve(mmot_solver* s, Carver& c) {
  const bool dense = s->kind == MMOT_DENSE;
  const size_t n = s->n, Lp = s->Lp, T = s->T, nnz = dense ? 1 : (size_t)s->nnz, vs = s->vsize;
  const size_t Tm1 = T > 1 ? T - 1 : 0;
  auto takev = [&](size_t cnt) { return static_cast<void*>(c.take<char>(cnt * vs)); };
  const size_t ks = (size_t)s->steps_k;
  s->rp_b = c.take<int>(n + 1);
  s->ci_b = c.take<int>(nnz);
  s->kv_b = takev(ks * nnz);
  s->cost = c.take<double>(ks * nnz);
  s->rp_f = c.take<int>(n + 1);
  s->ci_f = c.take<int>(nnz);
  s->kv_f = takev(ks * nnz);
  s->cnt = c.take<int>(n);
  s->cursor = c.take<int>(n);
  s->srcpos = c.take<int>(nnz);
  s->KL = s->has_kl ? takev(n * Lp) : nullptr;
  s->dcomm = s->has_comm ? takev((size_t)s->comm_steps * n * Lp) : nullptr;
  s->wcomm = s->has_comm ? takev(Tm1 * n * Lp) : nullptr;
  s->cap = takev(Tm1 * n);
  s->R01 = takev(n * Lp);
  s->R0T = takev(n * Lp);
  s->U01 = takev(n * Lp);
  s->U0T = takev(n * Lp);
  s->psi = takev(T * n * Lp);
  s->zh = takev((s->keep_fwd ? T + 1 : 2) * n * Lp);
  s->u = takev(Tm1 * n);
  s->ones = takev(n);
  s->cb = c.take<double>((T + 1) * Lp);
  s->cf = c.take<double>((T + 1) * Lp);
  s->sigb = c.take<double>((T + 1) * Lp);
  s->sigf = c.take<double>((T + 1) * Lp);
  s->gauge0 = c.take<double>(Lp);
  s->gaugeT = c.take<double>(Lp);
  s->facb = takev((T + 1) * Lp);
  s->facf = takev((T + 1) * Lp);
  s->wgt = takev((T + 1) * Lp);
  s->slots_b = c.take<uint32_t>((size_t)s->nslot * (T + 1) * Lp);
  s->slots_f = c.take<uint32_t>((size_t)s->nslot * (T + 1) * Lp);
  s->slotsE = c.take<uint32_t>((size_t)s->nslot * Lp);
  s->slotsS = c.take<uint32_t>((size_t)s->nslot * Lp);
  if (!dense) {
    s->cslots_b = c.take<unsigned long long>((size_t)s->ncslot * (T + 1) * Lp);
    s->cslots_f = c.take<unsigned long long>((size_t)s->ncslot * (T + 1) * Lp);
  }
  s->lvlT = c.take<double>(Lp);
  s->lvl0 = c.take<double>(Lp);
  s->levb = c.take<float>((T + 1) * Lp);
  s->levf = c.take<float>((T + 1) * Lp);
  s->rho = c.take<uint32_t>(2);
  s->part = c.take<double>((T + 1) * (size_t)s->nblk_s * kNSt);
  s->tpart = c.take<double>((T + 1) * kNSt);
  s->part_flow = c.take<double>((T + 1) * (size_t)s->nblk_s * kNSt);
  s->tpart_flow = c.take<double>((T + 1) * kNSt);
  s->stats_dev = c.take<double>(8);
  s->masses = c.take<double>(s->L);
  s->exc_row = c.take<double>(n);
  s->exc_cnt = c.take<int>(n);
  s->exc = c.take<double>(1);
  s->flags = c.take<int>(4);
  const size_t ell = (dense || s->steps_k > 1) ? 1 : n * kEllMax;   // time-varying networks use CSR
  s->ell_ci_b = c.take<int>(ell);
  s->ell_ci_f = c.take<int>(ell);
  s->ell_kv_b = takev(ell);
  s->ell_kv_f = takev(ell);
  if (dense) {
    const size_t nn = ks * n * (size_t)s->lda;   // one K (and K^T) per move for a time-varying network
    s->Kd = c.take<float>(nn);
    s->Ktd = c.take<float>(nn);
    s->Kb = s->has_bf16 ? static_cast<void*>(c.take<uint16_t>(nn)) : nullptr;
    s->Ktb = s->has_bf16 ? static_cast<void*>(c.take<uint16_t>(nn)) : nullptr;
    s->part_s = c.take<float>((size_t)s->ntn * n);
    // commodity-capacity terms of a check-pass product, one partial per product block
    s->part_cc = s->has_comm ? c.take<double>((size_t)kDenseCommBlocks * kNSt) : nullptr;
    s->n8 = (int)((n + 63) / 64 * 64);
    for (int i = 0; i < 2; ++i)
      s->Bbuf[i] = s->has_bf16 ? c.take<uint16_t>((size_t)s->n8 * Lp) : nullptr;
    for (int i = 0; i < 2; ++i) s->B32buf[i] = c.take<float>((size_t)s->n8 * Lp);
  }
  s->deg_b = c.take<int>(n);
  s->deg_f = c.take<int>(n);
  s->maxdeg = c.take<int>(2);
}

mmot_status basic_checks(const mmot_problem* p, const mmot_options* o) {
  if (!p || !o) return MMOT_EINVAL;
  if (p->n < 1 || p->L < 1 || p->T < 1) return MMOT_EINVAL;
  if (!(p->eps > 0) || !std::isfinite(p->eps)) return MMOT_EINVAL;
  if (p->kind != MMOT_CSR && p->kind != MMOT_DENSE) return MMOT_EINVAL;
  if (p->cost_per_step != 0 && p->cost_per_step != 1) return MMOT_EINVAL;
  if (p->cap_comm_per_step != 0 && p->cap_comm_per_step != 1) return MMOT_EINVAL;
  if (o->keep_forward != 0 && o->keep_forward != 1) return MMOT_EINVAL;
  if (p->kind == MMOT_DENSE) {
    // dense products run on MFMA in the scaled domain, FP32 or BF16 (+ FP32 polish)
    if (o->precision != MMOT_FP32 && o->precision != MMOT_BF16) return MMOT_EUNSUPPORTED;
    if (o->domain == MMOT_DOMAIN_LOG) return MMOT_EUNSUPPORTED;
    if ((size_t)p->n * (size_t)p->n > ((size_t)1 << 31)) return MMOT_EINVAL;
  } else {
    if (p->nnz < 1 || p->nnz > (1LL << 31) - 1) return MMOT_EINVAL;
    if (o->precision != MMOT_FP32 && o->precision != MMOT_FP64) return MMOT_EUNSUPPORTED;
  }
  if (o->domain < MMOT_DOMAIN_AUTO || o->domain > MMOT_DOMAIN_LOG) return MMOT_EINVAL;
  if ((size_t)p->n * (size_t)p->L > (size_t)1 << 33) return MMOT_EINVAL;
  return MMOT_OK;
}

#define HIPCK(x)                                 \
  do {                                           \
    if ((x) != hipSuccess) return MMOT_EHIP;     \
  } while (0)

// ---------------------------------------------------------------------------
// typed implementation
// ---------------------------------------------------------------------------
template <typename V, bool LOG>
struct Impl {
  using value_type = V;
  static constexpr bool kLog = LOG;
  static V* pan(mmot_solver* s, void* base, size_t k) { return static_cast<V*>(base) + k * s->panel_elems(); }
  static V* psi(mmot_solver* s, int t) { return pan(s, s->psi, t); }
  // forward messages: panel k = time k in a sweep that keeps them (the last Sinkhorn
  // sweep before a check), else two rolling panels (0 and 1)
  static V* zh(mmot_solver* s, int k) { return pan(s, s->zh, s->keep_now ? k : (k & 1)); }
  static V* zh_kept(mmot_solver* s, int k) { return pan(s, s->zh, k); }
  static V* uat(mmot_solver* s, int tau) {  // u at interior time tau (1..T-1)
    return (tau >= 1 && tau <= s->T - 1) ? static_cast<V*>(s->u) + (size_t)(tau - 1) * s->n : nullptr;
  }
  // u as a sparse step reads it: the vector of ones at the end times
  static const V* uin_at(mmot_solver* s, int tau) {
    V* p = uat(s, tau);
    return p ? p : static_cast<const V*>(s->ones);
  }
  // commodity capacities at interior time tau: scaling w_tau and bound D_tau (panels)
  static V* wat(mmot_solver* s, int tau) {
    return (s->has_comm && tau >= 1 && tau <= s->T - 1) ? pan(s, s->wcomm, tau - 1) : nullptr;
  }
  static const V* dat(mmot_solver* s, int tau) {
    return s->has_comm ? pan(s, s->dcomm, s->comm_steps > 1 ? tau - 1 : 0) : nullptr;
  }
  static StepArgs<V> base_args(mmot_solver* s) {
    StepArgs<V> a;
    std::memset(&a, 0, sizeof(a));
    a.n = s->n; a.Lp = s->Lp; a.L = s->L; a.G = s->G; a.nchunk = s->nchunk; a.lwpr = s->lwpr;
    a.eps = s->eps;
    a.nslot = s->nslot;
    a.nslot_stride = (size_t)(s->T + 1) * s->Lp;
    a.ncslot = s->ncslot;
    a.cslot_stride = (size_t)(s->T + 1) * s->Lp;
    a.flags = s->flags;
    return a;
  }

  // K (and K^T) of the move t -> t+1: one of T for a time-varying network
  static size_t kofs(mmot_solver* s, int t) {
    return (s->steps_k > 1 ? (size_t)t : 0) * (size_t)s->n * s->lda;
  }
  static GemmArgs gemm_base(mmot_solver* s, bool forward_op, int t) {
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.n = s->n; g.Lp = s->Lp; g.L = s->L; g.lda = s->lda; g.n8 = s->n8;
    const size_t o = kofs(s, t);
    if (s->dense_bf16) g.A = static_cast<const uint16_t*>(forward_op ? s->Ktb : s->Kb) + o;
    else g.A = (forward_op ? s->Ktd : s->Kd) + o;
    g.nslot = s->nslot;
    return g;
  }
  // dense backward product t+1 -> t
  // BF16 products read the operand diag(u) (panel) in BF16 as prepared by the
  // producer of the panel (the previous backward product's epilogue; the forward
  // capacity update); the first product of a sweep reads U0T / U01, converted at
  // the start of the sweep (k_dense_operand)
  // FP32 products (the polish) read the operand in FP32, written by k_dense_operand32
  // after each product and capacity update and at the start of each sweep
  static uint16_t* bbuf(mmot_solver* s, int t) { return s->Bbuf[t & 1]; }
  static float* b32(mmot_solver* s, int t) { return s->B32buf[t & 1]; }
  // check: a fused check's product (t >= 1): the capacity partial sums of P_t with
  // the kept hatPsi_t, then the row statistics of time t
  static void dense_bwd(mmot_solver* s, int t, bool calib, hipStream_t st, bool check = false) {
    GemmArgs g = gemm_base(s, false, t);
    if (s->dense_bf16) {
      g.Bb = bbuf(s, t + 1);
      if (t >= 1) { g.bout = bbuf(s, t); g.uo = reinterpret_cast<const float*>(uat(s, t)); }
    } else {
      g.B32 = b32(s, t + 1);
    }
    g.fac = reinterpret_cast<const float*>(static_cast<V*>(s->facb) + (size_t)t * s->Lp);
    g.out = reinterpret_cast<float*>(psi(s, t));
    g.kl = (s->has_kl && t >= 1) ? static_cast<const float*>(s->KL) : nullptr;
    g.cw = reinterpret_cast<const float*>(wat(s, t));
    g.slots = calib ? s->slots_b + (size_t)t * s->Lp : nullptr;
    g.slot_stride = (size_t)(s->T + 1) * s->Lp;
    const bool chk = check && t >= 1;
    if (chk) {
      g.cap = 1;
      g.wpan = reinterpret_cast<const float*>(zh_kept(s, t));
      g.wgt = reinterpret_cast<const float*>(static_cast<V*>(s->wgt) + (size_t)t * s->Lp);
      g.part_s = s->part_s;
    }
    launch_gemm(g, s->dense_bf16, st);
    if (chk)
      launch_dense_rows(s->n, s->ntn, s->part_s,
                        reinterpret_cast<const float*>(static_cast<V*>(s->cap) + (size_t)(t - 1) * s->n),
                        reinterpret_cast<float*>(uat(s, t)), 0, s->part + (size_t)t * s->nblk_s * kNSt, nullptr,
                        nullptr, nullptr, nullptr, s->n8, s->Lp, s->nblk, nullptr, 0, st);
    if (!s->dense_bf16 && t >= 1)
      launch_dense_operand32(s->n, s->n8, s->Lp, reinterpret_cast<const float*>(psi(s, t)),
                             reinterpret_cast<const float*>(uat(s, t)), b32(s, t), st);
  }
  // dense forward product t -> t+1 with its epilogue kernels
  static void dense_fwd(mmot_solver* s, int t, int mode, bool calib, double* occ, double* pcomm, hipStream_t st) {
    const int T = s->T, to = t + 1;
    const size_t Lp = s->Lp, pstride = (size_t)s->nblk_s * kNSt;
    GemmArgs g = gemm_base(s, true, t);
    if (s->dense_bf16) g.Bb = bbuf(s, t);
    else g.B32 = b32(s, t);
    g.fac = reinterpret_cast<const float*>(static_cast<V*>(s->facf) + (size_t)to * Lp);
    g.out = reinterpret_cast<float*>(zh(s, to));
    g.slot_stride = (size_t)(T + 1) * Lp;
    if (to < T) {
      g.kl = s->has_kl ? static_cast<const float*>(s->KL) : nullptr;
      g.cap = 1;
      g.wpan = reinterpret_cast<const float*>(psi(s, to));
      g.wgt = reinterpret_cast<const float*>(static_cast<V*>(s->wgt) + (size_t)to * Lp);
      g.part_s = s->part_s;
      g.slots = (mode == 0 && calib) ? s->slots_f + (size_t)to * Lp : nullptr;
      if (mode == 1) {
        g.ucur = reinterpret_cast<const float*>(uat(s, to));
        g.pcomm = pcomm ? pcomm + (size_t)to * s->pc_cnt * s->n : nullptr;
        g.pc_lo = s->pc_lo;
        g.pc_cnt = s->pc_cnt;
      }
      if (s->has_comm) {
        // commodity capacities: w_to multiplied in; the update projects it with the u_to
        // of the last sweep (still in place: the row kernel after the product updates u)
        g.cw = reinterpret_cast<const float*>(wat(s, to));
        g.dc = reinterpret_cast<const float*>(dat(s, to));
        g.ucur = reinterpret_cast<const float*>(uat(s, to));
        if (mode == 0) {
          g.cc_update = 1;
          g.cwo = reinterpret_cast<float*>(wat(s, to));
        }
      }
      launch_gemm(g, s->dense_bf16, st);
      const bool comm_stats = s->has_comm && mode == 1;
      if (comm_stats)
        launch_dense_comm_stats(s->n, s->L, s->Lp, reinterpret_cast<const float*>(zh(s, to)),
                                reinterpret_cast<const float*>(psi(s, to)),
                                s->has_kl ? static_cast<const float*>(s->KL) : nullptr, g.cw, g.dc, g.ucur,
                                s->sigf + (size_t)to * Lp, s->sigb + (size_t)to * Lp, s->part_cc, kDenseCommBlocks, st);
      launch_dense_rows(s->n, s->ntn, s->part_s, reinterpret_cast<const float*>(static_cast<V*>(s->cap) + (size_t)(to - 1) * s->n),
                        reinterpret_cast<float*>(uat(s, to)), mode == 0 ? 1 : 0,
                        mode == 1 ? s->part + (size_t)to * pstride : nullptr,
                        (mode == 1 && occ) ? occ + (size_t)to * s->n : nullptr,
                        reinterpret_cast<const float*>(zh(s, to)), s->dense_bf16 ? bbuf(s, to) : nullptr,
                        s->dense_bf16 ? nullptr : b32(s, to), s->n8, s->Lp,
                        s->nblk, comm_stats ? s->part_cc : nullptr, kDenseCommBlocks, st);
    } else {
      launch_gemm(g, s->dense_bf16, st);   // hatPsi_T into the rolling buffer
      launch_dense_sink(s->n, s->Lp, s->L, g.out, reinterpret_cast<const float*>(s->R0T),
                        reinterpret_cast<float*>(s->U0T), mode == 0 ? 1 : 0, s->sigb + (size_t)T * Lp,
                        s->sigf + (size_t)T * Lp, s->slotsE, s->nslot,
                        (mode == 0 && calib) ? s->slots_f + (size_t)T * Lp : nullptr, (size_t)(T + 1) * Lp, s->flags,
                        mode == 1 ? s->part + (size_t)T * pstride : nullptr,
                        (mode == 1 && occ) ? occ + (size_t)T * s->n : nullptr,
                        (mode == 1 && pcomm) ? pcomm + (size_t)T * s->pc_cnt * s->n : nullptr, s->pc_lo, s->pc_cnt,
                        s->nblk, st);
    }
  }

  // operator values of the move t -> t+1 (one set unless the network is time-varying)
  static const V* kvat(mmot_solver* s, void* base, int t) {
    return static_cast<const V*>(base) + (s->steps_k > 1 ? (size_t)t * s->nnz : 0);
  }
  static StepArgs<V> bwd_args(mmot_solver* s, int t, bool calib) {
    const int T = s->T;
    StepArgs<V> a = base_args(s);
    a.rp = s->rp_b; a.ci = s->ci_b; a.kv = kvat(s, s->kv_b, t);
    if (s->ellD) { a.ellD = s->ellD; a.ci = s->ell_ci_b; a.kv = static_cast<const V*>(s->ell_kv_b); }
    a.xin = (t + 1 == T) ? static_cast<const V*>(s->U0T) : psi(s, t + 1);
    a.uin = uin_at(s, t + 1);
    a.fac = static_cast<const V*>(s->facb) + (size_t)t * s->Lp;
    a.out = psi(s, t);
    a.kl = (s->has_kl && t >= 1) ? static_cast<const V*>(s->KL) : nullptr;
    a.cw = wat(s, t);
    a.epi = 0;
    // log domain: the backward panels are calibrated on their values at the plan
    // peak, recorded by the forward sweep (and the source update for t = 0)
    a.slots = (calib && !LOG) ? s->slots_b + (size_t)t * s->Lp : nullptr;
    return a;
  }

  // check: a fused check (kept forward messages): the statistics of every time
  // from this sweep's Psi_t and the kept hatPsi_t (Corollary 1), no forward pass
  static void backward(mmot_solver* s, bool consume, bool calib, hipStream_t st, bool check = false) {
    const int T = s->T;
    const size_t pstride = (size_t)s->nblk_s * kNSt;
    if (consume) {
      if (LOG && s->cslots_b)
        launch_levels64(s->cslots_b, s->slots_b, s->levb, T + 1, s->Lp, s->ncslot, s->nslot, st);
      else
        launch_levels(s->slots_b, s->levb, T + 1, s->Lp, s->nslot, st);
      launch_growth(s->cb, s->levb, T, s->Lp, 0, st);
    }
    launch_prep_bwd<V, LOG>(T, s->Lp, s->cb, s->sigb, static_cast<V*>(s->facb), s->gaugeT, s->lvlT, s->slotsE,
                            s->nslot, st);
    if (check) {
      // the weights 2^(sigma_hat_t + sigma_t) with this sweep's sigma (the kept panels
      // carry the sigma_hat of their sweep, which the update-free preparation restores),
      // then time T from the kept hatPsi_T and the current U0T
      launch_prep_fwd<V, LOG>(T, s->Lp, 1, s->cf, s->sigf, s->sigb, static_cast<V*>(s->facf),
                              static_cast<V*>(s->wgt), s->gauge0, s->gaugeT, s->lvl0, s->slotsS, s->nslot, st);
      if (s->kind == MMOT_DENSE)
        launch_dense_sink(s->n, s->Lp, s->L, reinterpret_cast<const float*>(zh_kept(s, T)),
                          reinterpret_cast<const float*>(s->R0T), reinterpret_cast<float*>(s->U0T), 0,
                          s->sigb + (size_t)T * s->Lp, s->sigf + (size_t)T * s->Lp, s->slotsE, s->nslot, nullptr,
                          (size_t)(T + 1) * s->Lp, s->flags, s->part + (size_t)T * pstride, nullptr, nullptr,
                          s->pc_lo, s->pc_cnt, s->nblk, st);
      else
        launch_sink_check<V, LOG>(s->n, s->Lp, s->L, s->G, s->nchunk, zh_kept(s, T),
                                  static_cast<const V*>(s->U0T), static_cast<const V*>(s->R0T),
                                  s->sigb + (size_t)T * s->Lp, s->sigf + (size_t)T * s->Lp,
                                  s->part + (size_t)T * pstride, s->nblk_s, st);
    }
    if (s->kind == MMOT_DENSE && s->dense_bf16)
      launch_dense_operand(s->n, s->Lp, static_cast<const float*>(s->U0T), nullptr, bbuf(s, T), st);
    else if (s->kind == MMOT_DENSE)
      launch_dense_operand32(s->n, s->n8, s->Lp, static_cast<const float*>(s->U0T), nullptr, b32(s, T), st);
    for (int t = T - 1; t >= 0; --t) {
      if (s->kind == MMOT_DENSE) {
        dense_bwd(s, t, calib, st, check);
        continue;
      }
      StepArgs<V> a = bwd_args(s, t, calib);
      if (check && t >= 1) {
        a.part = s->part + (size_t)t * pstride;
        a.wpan = zh_kept(s, t);
        a.wgt = static_cast<const V*>(s->wgt) + (size_t)t * s->Lp;
        a.uout = uat(s, t);
        a.cap = static_cast<const V*>(s->cap) + (size_t)(t - 1) * s->n;
      }
      launch_step<V, LOG>(a, 0, s->nblk_s, st);
    }
    if (check)
      launch_check0<V, LOG>(s->n, s->Lp, s->L, s->G, s->nchunk, psi(s, 0), static_cast<const V*>(s->U01),
                            static_cast<const V*>(s->R01), s->sigf, s->sigb, s->part, nullptr, nullptr, s->pc_lo,
                            s->pc_cnt, s->nblk, st);
  }

  // forward product t -> t+1; mode 0 Sinkhorn update, mode 1 update-free pass
  static StepArgs<V> fwd_args(mmot_solver* s, int t, int mode, bool calib, double* occ, double* pcomm) {
    const int T = s->T;
    const size_t Lp = s->Lp, pstride = (size_t)s->nblk_s * kNSt;
    StepArgs<V> a = base_args(s);
    a.rp = s->rp_f; a.ci = s->ci_f; a.kv = kvat(s, s->kv_f, t);
    if (s->ellD) { a.ellD = s->ellD; a.ci = s->ell_ci_f; a.kv = static_cast<const V*>(s->ell_kv_f); }
    a.xin = (t == 0) ? static_cast<const V*>(s->U01) : zh(s, t);
    a.uin = uin_at(s, t);
    const int to = t + 1;
    a.fac = static_cast<const V*>(s->facf) + (size_t)to * Lp;
    a.update = (mode == 0);
    if (mode == 1) {
      a.part = s->part + (size_t)to * pstride;
      a.occ = occ ? occ + (size_t)to * s->n : nullptr;
      a.pcomm = pcomm ? pcomm + (size_t)to * s->pc_cnt * s->n : nullptr;
      a.pc_lo = s->pc_lo;
      a.pc_cnt = s->pc_cnt;
    }
    if (to < T) {
      a.epi = 1;
      a.out = zh(s, to);
      a.kl = s->has_kl ? static_cast<const V*>(s->KL) : nullptr;
      a.cw = wat(s, to);
      a.cwo = (mode == 0) ? wat(s, to) : nullptr;
      a.dc = dat(s, to);
      a.wpan = psi(s, to);
      a.wgt = static_cast<const V*>(s->wgt) + (size_t)to * Lp;
      a.cap = static_cast<const V*>(s->cap) + (size_t)(to - 1) * s->n;
      a.uout = static_cast<V*>(s->u) + (size_t)(to - 1) * s->n;
      if (mode == 0 && calib) {
        if (LOG) {
          a.cslots_b = s->cslots_b + (size_t)to * Lp;
          a.cslots_f = s->cslots_f + (size_t)to * Lp;
        } else {
          a.slots = s->slots_f + (size_t)to * Lp;
        }
      }
    } else {
      a.epi = 2;
      a.rdst = static_cast<const V*>(s->R0T);
      a.u0t = static_cast<V*>(s->U0T);
      if (mode == 0 && s->keep_now) a.hatT = zh_kept(s, T);
      a.sigT = s->sigb + (size_t)T * Lp;
      a.sighT = s->sigf + (size_t)T * Lp;
      if (mode == 0) {
        a.slots = s->slotsE;             // exact level of the new U0T panel, every iteration
        a.nslot_stride = Lp;
        a.slots_o = (calib && !LOG) ? s->slots_f + (size_t)T * Lp : nullptr;
        a.nslot_stride_o = (size_t)(T + 1) * Lp;
        if (calib && LOG) a.cslots_f = s->cslots_f + (size_t)T * Lp;
      }
    }
    return a;
  }

  // Forward sweep.  mode 0: Sinkhorn sweep (source update, capacity updates,
  // sink update).  mode 1: update-free pass computing statistics and optional
  // outputs (occupancy, per-commodity marginals, edge flows).
  static void forward(mmot_solver* s, int mode, bool consume, bool calib, double* occ, double* pcomm,
                      hipStream_t st) {
    const int T = s->T;
    const size_t Lp = s->Lp;
    if (mode == 0) {
      // source update first: its output level feeds the offsets of the sweep
      launch_source<V, LOG>(s->n, s->Lp, s->G, s->nchunk, psi(s, 0), static_cast<const V*>(s->R01),
                            static_cast<V*>(s->U01), s->slotsS, s->nslot, Lp, s->flags,
                            (LOG && calib) ? s->cslots_b : nullptr, s->ncslot, (size_t)(T + 1) * Lp, s->nblk, st);
      if (consume) {
        if (LOG && s->cslots_f)
          launch_levels64(s->cslots_f, s->slots_f, s->levf, T + 1, s->Lp, s->ncslot, s->nslot, st);
        else
          launch_levels(s->slots_f, s->levf, T + 1, s->Lp, s->nslot, st);
        launch_growth(s->cf, s->levf, T, s->Lp, 1, st);
      }
    }
    launch_prep_fwd<V, LOG>(T, s->Lp, mode, s->cf, s->sigf, s->sigb, static_cast<V*>(s->facf),
                            static_cast<V*>(s->wgt), s->gauge0, s->gaugeT, s->lvl0, s->slotsS, s->nslot, st);
    if (mode == 1) {
      launch_check0<V, LOG>(s->n, s->Lp, s->L, s->G, s->nchunk, psi(s, 0), static_cast<const V*>(s->U01),
                            static_cast<const V*>(s->R01), s->sigf, s->sigb, s->part, occ, pcomm, s->pc_lo,
                            s->pc_cnt, s->nblk, st);
    }
    if (s->kind == MMOT_DENSE && s->dense_bf16)
      launch_dense_operand(s->n, s->Lp, static_cast<const float*>(s->U01), nullptr, bbuf(s, 0), st);
    else if (s->kind == MMOT_DENSE)
      launch_dense_operand32(s->n, s->n8, s->Lp, static_cast<const float*>(s->U01), nullptr, b32(s, 0), st);
    for (int t = 0; t < T; ++t) {
      if (s->kind == MMOT_DENSE) dense_fwd(s, t, mode, calib, occ, pcomm, st);
      else launch_step<V, LOG>(fwd_args(s, t, mode, calib, occ, pcomm), mode == 0 ? 1 : 2, s->nblk_s, st);
    }
  }

  // time `reps` launches of one sweep step at the middle time, as launched in
  // the sweep (forward: with the capacity update, its u written to scratch)
  static mmot_status time_step(mmot_solver* s, int fwd, int reps, double* avg_ms) {
    // cycle through the interior times, as a sweep does (each launch reads
    // and writes other panels than the one before it)
    const int t_lo = s->T >= 3 ? 1 : 0, t_hi = std::max(t_lo, s->T - 2);
    if (fwd && s->T < 2 && s->kind != MMOT_DENSE) return MMOT_EUNSUPPORTED;   // the only product is the sink's
    hipEvent_t e0, e1;
    HIPCK(hipEventCreate(&e0));
    HIPCK(hipEventCreate(&e1));
    auto launch_at = [&](int t) {
      if (s->kind == MMOT_DENSE) {
        GemmArgs g = gemm_base(s, fwd != 0, t);
        if (s->dense_bf16) g.Bb = bbuf(s, t + 1);   // the operand form of the sweep's products
        else g.B32 = b32(s, t + 1);
        g.fac = reinterpret_cast<const float*>(static_cast<V*>(s->facb) + (size_t)t * s->Lp);
        g.out = reinterpret_cast<float*>(zh(s, t & 1));
        if (fwd) {   // forward product with the capacity partial sums, as in the sweep
          g.cap = 1;
          g.wpan = reinterpret_cast<const float*>(psi(s, t));
          g.wgt = reinterpret_cast<const float*>(s->wgt);
          g.part_s = s->part_s;
        }
        launch_gemm(g, s->dense_bf16, s->stream);
      } else {
        StepArgs<V> a = fwd ? fwd_args(s, t, 0, false, nullptr, nullptr) : bwd_args(s, t, false);
        if (fwd && a.epi == 1) { a.uout = reinterpret_cast<V*>(s->exc_row); a.cwo = nullptr; }
        launch_step<V, LOG>(a, fwd, s->nblk_s, s->stream);
      }
    };
    HIPCK(hipEventRecord(e0, s->stream));
    for (int r = 0; r < reps; ++r) launch_at(t_lo + r % (t_hi - t_lo + 1));
    HIPCK(hipEventRecord(e1, s->stream));
    HIPCK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = ms / reps;
    return MMOT_OK;
  }

  // flows need A_t from the update-free forward recursion: run the products
  // and interleave the SDDMM at each time
  static void flows_pass(mmot_solver* s, double* flow, hipStream_t st) {
    const int T = s->T;
    const size_t Lp = s->Lp, pstride = (size_t)s->nblk_s * kNSt;
    launch_prep_fwd<V, LOG>(T, s->Lp, 1, s->cf, s->sigf, s->sigb, static_cast<V*>(s->facf),
                            static_cast<V*>(s->wgt), s->gauge0, s->gaugeT, s->lvl0, s->slotsS, s->nslot, st);
    if (s->kind == MMOT_DENSE) {
      // Dense network: F_t = K (.) (A_t B_{t+1}^T) per time on MFMA, A_t from the
      // update-free forward recursion; flows as n x n per time, the move and state
      // costs as block partials (field 0 and ST_SCOST of part_flow)
      const int n = s->n, nt = (n + 127) / 128;
      const int nb = std::min(nt * nt, s->nblk_s);
      const float* ones = static_cast<const float*>(s->ones);
      float* fab = s->levf;   // [2][Lp] commodity factors (calibration scratch, free outside sweeps)
      if (s->dense_bf16)
        launch_dense_operand(n, s->Lp, static_cast<const float*>(s->U01), nullptr, bbuf(s, 0), st);
      else
        launch_dense_operand32(n, s->n8, s->Lp, static_cast<const float*>(s->U01), nullptr, b32(s, 0), st);
      for (int t = 0; t < T; ++t) {
        const int tb = t + 1;
        const float* A = reinterpret_cast<const float*>(t == 0 ? static_cast<V*>(s->U01) : zh(s, t));
        const float* ua = t == 0 ? ones : reinterpret_cast<const float*>(uat(s, t));
        const float* B = reinterpret_cast<const float*>(tb == T ? static_cast<V*>(s->U0T) : psi(s, tb));
        const float* ub = tb == T ? ones : reinterpret_cast<const float*>(uat(s, tb));
        launch_dense_flows(n, s->L, s->Lp, s->lda, A, ua, B, ub, s->sigf + (size_t)t * Lp, s->sigb + (size_t)tb * Lp,
                           fab, s->Kd + kofs(s, t), s->eps, flow + (size_t)t * n * n,
                           s->part_flow + (size_t)t * pstride, nb, st);
        if (s->has_kl && t >= 1)
          launch_dense_state_cost(n, s->L, s->Lp, reinterpret_cast<const float*>(zh(s, t)),
                                  reinterpret_cast<const float*>(psi(s, t)), static_cast<const float*>(s->KL),
                                  reinterpret_cast<const float*>(wat(s, t)), reinterpret_cast<const float*>(uat(s, t)), s->sigf + (size_t)t * Lp,
                                  s->sigb + (size_t)t * Lp, s->eps, s->part_flow + (size_t)t * pstride, nb, st);
        if (tb < T) dense_fwd(s, t, 1, false, nullptr, nullptr, st);
      }
      launch_reduce_cost(s->part_flow, s->part_flow, nb, nb, s->nblk_s, T, s->tpart_flow, s->tpart,
                         s->stats_dev + 7, st);
      return;
    }
    for (int t = 0; t < T; ++t) {
      const V* xin = (t == 0) ? static_cast<const V*>(s->U01) : zh(s, t);
      const int tb = t + 1;
      launch_flows<V, LOG>(s->n, s->Lp, s->L, s->G, s->nchunk, s->rp_b, s->ci_b, kvat(s, s->kv_b, t),
                           s->cost + (s->steps_k > 1 ? (size_t)t * s->nnz : 0), xin, uat(s, t), (tb == T) ? static_cast<const V*>(s->U0T) : psi(s, tb),
                           uat(s, tb), s->sigf + (size_t)t * Lp, s->sigb + (size_t)tb * Lp,
                           flow + (size_t)t * s->nnz, s->part_flow + (size_t)t * pstride, s->nblk, st);
      if (tb < T) launch_step<V, LOG>(fwd_args(s, t, 1, false, nullptr, nullptr), 2, s->nblk_s, st);
    }
    launch_reduce_cost(s->part_flow, s->part, s->nblk, s->nblk_s, s->nblk_s, T, s->tpart_flow, s->tpart,
                       s->stats_dev + 7, st);
  }

  static mmot_status setup(mmot_solver* s, const mmot_problem* p) {
    hipStream_t st = s->stream;
    const size_t n = s->n, L = s->L, Lp = s->Lp, T = s->T, nnz = (size_t)s->nnz;
    const size_t Tm1 = T > 1 ? T - 1 : 0;
    launch_fill<int>(s->flags, 4, 0, st);
    launch_validate_vals(p->src, n * L, 0, 0, 0, s->flags, st);
    launch_validate_vals(p->dst, n * L, 0, 0, 0, s->flags, st);
    launch_validate_vals(p->cap, p->cap_per_step ? Tm1 * n : n, 1, 1, 0, s->flags, st);
    const bool dense = s->kind == MMOT_DENSE;
    if (!dense) launch_validate_vals(p->cost, (size_t)s->steps_k * nnz, s->steps_k > 1 ? 1 : 0, 0, 1, s->flags, st);
    else launch_validate_vals(p->cost_dense, (size_t)s->steps_k * n * n, 1, 0, 1, s->flags, st);
    if (p->state_cost) launch_validate_vals(p->state_cost, n * L, 0, 0, 1, s->flags, st);
    if (p->cap_comm) launch_validate_vals(p->cap_comm, (size_t)s->comm_steps * L * n, 1, 0, 0, s->flags, st);
    if (!dense) launch_validate_csr(p->rowptr, p->colidx, s->n, s->nnz, s->flags, st);
    launch_validate_mass(p->src, p->dst, s->L, s->n, s->flags, s->masses, st);
    HIPCK(hipMemcpyAsync(s->host_flags, s->flags, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (*s->host_flags) return MMOT_EINVAL;
    launch_fill<uint32_t>(s->rho, 2, 0u, st);
    if (dense) {
      // K = exp(-C/eps) (+inf -> 0) and K^T, FP32 and optionally BF16; one per move
      // for a time-varying network (Section 3.3)
      for (int k = 0; k < s->steps_k; ++k) {
        const size_t o = kofs(s, k);
        launch_dense_gibbs(p->cost_dense + (size_t)k * n * n, s->n, s->lda, s->eps, s->Kd + o, s->Ktd + o,
                           s->Kb ? static_cast<void*>(static_cast<uint16_t*>(s->Kb) + o) : nullptr,
                           s->Ktb ? static_cast<void*>(static_cast<uint16_t*>(s->Ktb) + o) : nullptr, st);
        launch_dense_rowsum_max(s->Kd + o, s->n, s->lda, s->rho, st);
        launch_dense_rowsum_max(s->Ktd + o, s->n, s->lda, s->rho + 1, st);
      }
    } else {
      // operators: backward = rows of K (input order), forward = rows of K^T
      HIPCK(hipMemcpyAsync(s->rp_b, p->rowptr, (n + 1) * sizeof(int), hipMemcpyDeviceToDevice, st));
      HIPCK(hipMemcpyAsync(s->ci_b, p->colidx, nnz * sizeof(int), hipMemcpyDeviceToDevice, st));
      const size_t ks = (size_t)s->steps_k;
      HIPCK(hipMemcpyAsync(s->cost, p->cost, ks * nnz * sizeof(double), hipMemcpyDeviceToDevice, st));
      launch_gibbs<V, LOG>(s->cost, ks * nnz, s->eps, static_cast<V*>(s->kv_b), st);
      launch_transpose_pattern(s->rp_b, s->ci_b, s->n, s->nnz, s->cnt, s->rp_f, s->cursor, s->ci_f, s->srcpos, st);
      for (size_t k = 0; k < ks; ++k)
        launch_gather_vals<V>(static_cast<const V*>(s->kv_b) + k * nnz, s->srcpos, s->nnz,
                              static_cast<V*>(s->kv_f) + k * nnz, st);
      launch_fill<int>(s->maxdeg, 2, 0, st);
      launch_max_degree(s->rp_b, s->n, s->maxdeg, st);
      launch_max_degree(s->rp_f, s->n, s->maxdeg + 1, st);
      HIPCK(hipMemcpyAsync(s->host_flags, s->maxdeg, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCK(hipStreamSynchronize(st));
      {
        const int D = std::max(s->host_flags[0], s->host_flags[1]);
        // an ELL row is one gather batch of 4, 5, 8 or 16 entries (the smallest that
        // holds the widest row: padding entries still cost a gather and, in the log
        // domain, an exp2); wider graphs, time-varying networks and commodity
        // capacities run on the CSR operators
        const int Dp = D <= 4 ? 4 : D == 5 ? 5 : D <= 8 ? 8 : 16;
        s->ellD = (D >= 1 && D <= 16 && s->steps_k == 1 && !s->has_comm) ? Dp : 0;
      }
      if (s->ellD) {
        const V pad = LOG ? -static_cast<V>(INFINITY) : V(0);
        launch_build_ell<V>(s->rp_b, s->ci_b, static_cast<const V*>(s->kv_b), s->n, s->ellD, pad, s->ell_ci_b,
                            static_cast<V*>(s->ell_kv_b), s->deg_b, st);
        launch_build_ell<V>(s->rp_f, s->ci_f, static_cast<const V*>(s->kv_f), s->n, s->ellD, pad, s->ell_ci_f,
                            static_cast<V*>(s->ell_kv_f), s->deg_f, st);
      }
      for (size_t k = 0; k < ks; ++k) {
        launch_rowsum_max<V, LOG>(s->rp_b, static_cast<const V*>(s->kv_b) + k * nnz, s->n, 0.0, s->rho, st);
        launch_rowsum_max<V, LOG>(s->rp_f, static_cast<const V*>(s->kv_f) + k * nnz, s->n, 0.0, s->rho + 1, st);
      }
    }
    // panels
    const V zero = LOG ? -static_cast<V>(INFINITY) : V(0);
    const int vmode = LOG ? 1 : 0;
    launch_to_panel<V>(p->src, s->L, s->n, s->Lp, vmode, s->eps, zero, static_cast<V*>(s->R01), st);
    launch_to_panel<V>(p->dst, s->L, s->n, s->Lp, vmode, s->eps, zero, static_cast<V*>(s->R0T), st);
    if (s->has_kl)
      launch_to_panel<V>(p->state_cost, s->L, s->n, s->Lp, LOG ? 3 : 2, s->eps, LOG ? V(0) : V(1),
                         static_cast<V*>(s->KL), st);
    launch_cap<V, LOG>(p->cap, p->cap_per_step, s->n, (int)Tm1, static_cast<V*>(s->cap), st);
    if (s->has_comm) {
      // D_t as panels (log2 in the log domain; padding columns unconstrained), w_t = 1
      for (int k = 0; k < s->comm_steps; ++k)
        launch_to_panel<V>(p->cap_comm + (size_t)k * L * n, s->L, s->n, s->Lp, LOG ? 1 : 0, s->eps,
                           static_cast<V>(INFINITY), pan(s, s->dcomm, k), st);
      launch_fill<V>(static_cast<V*>(s->wcomm), Tm1 * n * Lp, LOG ? V(0) : V(1), st);
    }
    // initial scalings: u = 1, U0T = 1 on supp(R0T)
    launch_fill<V>(static_cast<V*>(s->u), Tm1 * n, LOG ? V(0) : V(1), st);
    launch_fill<V>(static_cast<V*>(s->ones), n, LOG ? V(0) : V(1), st);
    launch_init_u0t<V, LOG>(static_cast<const V*>(s->R0T), n * Lp, static_cast<V*>(s->U0T), st);
    launch_fill<V>(static_cast<V*>(s->U01), n * Lp, zero, st);
    launch_fill<V>(static_cast<V*>(s->psi), T * n * Lp, zero, st);
    launch_fill<V>(static_cast<V*>(s->zh), (s->keep_fwd ? T + 1 : 2) * n * Lp, zero, st);
    for (int i = 0; i < 2; ++i)   // BF16 operand buffers: padding rows must stay zero
      if (s->Bbuf[i]) launch_fill<uint32_t>(reinterpret_cast<uint32_t*>(s->Bbuf[i]), (size_t)s->n8 * Lp / 2, 0u, st);
    for (int i = 0; i < 2; ++i)   // FP32 operand buffers: padding rows must stay zero
      if (s->B32buf[i]) launch_fill<float>(s->B32buf[i], (size_t)s->n8 * Lp, 0.f, st);
    launch_fill<uint32_t>(s->slots_b, (size_t)s->nslot * (T + 1) * Lp, 0u, st);
    launch_fill<uint32_t>(s->slots_f, (size_t)s->nslot * (T + 1) * Lp, 0u, st);
    launch_fill<uint32_t>(s->slotsE, (size_t)s->nslot * Lp, 0u, st);
    launch_fill<uint32_t>(s->slotsS, (size_t)s->nslot * Lp, 0u, st);
    if (s->cslots_b) {
      launch_fill<uint32_t>(reinterpret_cast<uint32_t*>(s->cslots_b), 2 * (size_t)s->ncslot * (T + 1) * Lp, 0u, st);
      launch_fill<uint32_t>(reinterpret_cast<uint32_t*>(s->cslots_f), 2 * (size_t)s->ncslot * (T + 1) * Lp, 0u, st);
    }
    launch_fill<double>(s->lvlT, Lp, 0.0, st);
    launch_fill<double>(s->lvl0, Lp, 0.0, st);
    launch_init_offsets(s->cb, s->cf, s->gauge0, s->gaugeT, s->T, s->Lp, s->rho, st);
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(st));
    return MMOT_OK;
  }

  static void iteration(mmot_solver* s, bool runB, bool consume_b, bool calib, bool consume_f, hipStream_t st) {
    if (runB) backward(s, consume_b, calib, st);
    forward(s, 0, consume_f, calib, nullptr, nullptr, st);
  }
};

template <typename F>
auto dispatch(mmot_solver* s, F&& f) {
  if (s->prec == MMOT_FP64) {
    if (s->dom == MMOT_DOMAIN_LOG) return f(Impl<double, true>());
    return f(Impl<double, false>());
  }
  if (s->dom == MMOT_DOMAIN_LOG) return f(Impl<float, true>());
  return f(Impl<float, false>());
}

// A zero message facing a positive source or sink entry.  Reachability is a
// property of the network and T alone, and the first iteration (u = 1) shows it;
// once a scaled-domain solver has passed its probe iteration without one, a
// later zero message comes from the range of the scalings (u -> 0 underflowing
// a message), a numeric failure and not infeasibility.
mmot_status zero_message_status(const mmot_solver* s) {
  return (s->dom == MMOT_DOMAIN_SCALED && s->probe_clean) ? MMOT_ENUMERIC : MMOT_EINFEASIBLE;
}

mmot_status read_flags(mmot_solver* s) {
  HIPCK(hipMemcpyAsync(s->host_flags, s->flags, sizeof(int), hipMemcpyDeviceToHost, s->stream));
  HIPCK(hipStreamSynchronize(s->stream));
  const int f = *s->host_flags;
  if (f & FLAG_INFEASIBLE) return zero_message_status(s);
  if (f & FLAG_NONFINITE) return MMOT_ENUMERIC;
  // (after set-up, where it means invalid data: a step launched in a form the library does not run)
  if (f & FLAG_BADINPUT) return MMOT_EUNSUPPORTED;
  return MMOT_OK;
}

mmot_status run_iterations(mmot_solver* s, int n_iter) {
  for (int k = 0; k < n_iter; ++k) {
    const bool calib = s->opt.calib_every >= 0 &&
                       (s->iters < 3 || s->force_calib > 0 ||
                        (s->opt.calib_every > 0 && s->iters % s->opt.calib_every == 0));
    const bool runB = !s->psi_fresh;
    const bool cb = runB && s->pend_b, cf = s->pend_f;
    // the last sweep of the call keeps every forward message (for a fused check);
    // the others write two rolling panels, which stay resident in the last-level cache
    s->keep_now = s->keep_fwd && k == n_iter - 1;
    const int key = (runB ? 1 : 0) | (cb ? 2 : 0) | (calib ? 4 : 0) | (cf ? 8 : 0) | (s->dense_bf16 ? 16 : 0) |
                    (s->keep_now ? 32 : 0);
    if (s->opt.use_graph) {
      auto it = s->graphs.find(key);
      if (it == s->graphs.end()) {
        hipGraph_t g;
        HIPCK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed));
        dispatch(s, [&](auto impl) { decltype(impl)::iteration(s, runB, cb, calib, cf, s->cap_stream); return 0; });
        HIPCK(hipStreamEndCapture(s->cap_stream, &g));
        hipGraphExec_t ge;
        if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) { (void)hipGraphDestroy(g); return MMOT_EHIP; }
        (void)hipGraphDestroy(g);
        it = s->graphs.emplace(key, ge).first;
      }
      HIPCK(hipGraphLaunch(it->second, s->stream));
    } else {
      dispatch(s, [&](auto impl) { decltype(impl)::iteration(s, runB, cb, calib, cf, s->stream); return 0; });
      HIPCK(hipGetLastError());
    }
    // calibration sweeps leave column maxima to consume at the next prep of the
    // same direction (the sink update records those of the U0T panel)
    s->pend_b = calib ? true : (cb ? false : s->pend_b);
    s->pend_f = calib;
    s->psi_fresh = false;
    s->hat_valid = s->keep_now;
    s->keep_now = false;
    if (s->force_calib > 0) --s->force_calib;
    ++s->iters;
  }
  return MMOT_OK;
}

// fresh backward messages for the current scalings (no range update)
void ensure_fresh(mmot_solver* s) {
  if (s->psi_fresh) return;
  const bool cb = s->pend_b;
  dispatch(s, [&](auto impl) { decltype(impl)::backward(s, cb, false, s->stream); return 0; });
  s->pend_b = false;
  s->psi_fresh = true;
}

mmot_status collect_stats(mmot_solver* s, mmot_stats* out) {
  launch_reduce_stats(s->part, s->nblk, s->nblk_s, s->nblk_s, s->T + 1, s->tpart, s->eps, s->stats_dev, s->stream);
  HIPCK(hipMemcpyAsync(s->host_stats, s->stats_dev, 8 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  mmot_status fs = read_flags(s);
  if (out) {
    out->iters = (int32_t)s->iters;
    out->domain = s->dom;
    out->precision = s->dense_bf16 ? MMOT_BF16 : s->prec;
    out->dual_obj = s->host_stats[0];
    out->src_resid = s->host_stats[1];
    out->cap_viol = s->host_stats[2];
    out->mass_drift = s->host_stats[3];
    out->dual_gap = s->host_stats[4];
    out->mass = s->host_stats[5];
    out->converged = (out->src_resid <= s->opt.tol && out->cap_viol <= s->opt.tol) ? 1 : 0;
  }
  if (fs != MMOT_OK) return fs;
  if (s->host_stats[6] > 0 || !std::isfinite(s->host_stats[0])) return MMOT_ENUMERIC;
  return MMOT_OK;
}

mmot_status check_pass(mmot_solver* s, double* occ, double* pcomm, mmot_stats* out) {
  if (out && !occ && !pcomm && s->keep_fwd && s->hat_valid && !s->psi_fresh &&
      (s->kind == MMOT_DENSE || s->ellD > 0)) {
    // fused: the fresh backward sweep the check needs computes the statistics too
    const bool cb = s->pend_b;
    dispatch(s, [&](auto impl) { decltype(impl)::backward(s, cb, false, s->stream, true); return 0; });
    s->pend_b = false;
    s->psi_fresh = true;
    if (hipGetLastError() != hipSuccess) return MMOT_EHIP;
    return collect_stats(s, out);
  }
  ensure_fresh(s);
  dispatch(s, [&](auto impl) { decltype(impl)::forward(s, 1, false, false, occ, pcomm, s->stream); return 0; });
  s->hat_valid = false;   // (its rolling panels overlap the kept ones)
  if (hipGetLastError() != hipSuccess) return MMOT_EHIP;
  if (!out && !pcomm && !occ) return MMOT_OK;
  if (out) return collect_stats(s, out);
  return MMOT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
namespace {
// Items of one recorded chunk of check_every iterations plus the check pass, at
// most: per iteration a backward sweep (T steps, the offset preparation and the
// level/growth pair) and a forward sweep (T steps, source update, offsets,
// level/growth pair); the check pass a fresh backward sweep, an update-free
// forward sweep with its time-0 statistics and the two-stage reduction.
int64_t pool_prog_items(int T, int check_every) {
  const int k = check_every < 1 ? 10 : check_every;
  return (int64_t)(k + 1) * (2 * (int64_t)T + 8) + 8;
}
}  // namespace

namespace {
// Set-up of a solver object in a workspace of at least the queried size.
// host_stats / host_flags: host buffers of 16 doubles and 4 ints to use
// (pageable; the solver then runs without captured graphs), or NULL to
// allocate pinned ones and a capture stream.  On failure the caller releases
// what was made (release_solver).
mmot_status create_into(mmot_solver* s, const mmot_problem* p, const mmot_options* o, void* ws, void* stream,
                        double* host_stats, int* host_flags) {
  mmot_status st = MMOT_OK;
  s->n = p->n; s->L = p->L; s->T = p->T; s->nnz = p->nnz; s->kind = p->kind; s->eps = p->eps;
  s->steps_k = p->cost_per_step ? p->T : 1;
  s->has_kl = p->state_cost != nullptr;
  s->has_comm = p->cap_comm != nullptr && p->T > 1;
  s->comm_steps = p->cap_comm_per_step ? std::max(p->T - 1, 1) : 1;
  s->opt = *o;
  if (s->opt.check_every < 1) s->opt.check_every = 10;
  if (!(s->opt.tol > 0)) s->opt.tol = 1e-6;
  s->prec = (o->precision == MMOT_FP64) ? MMOT_FP64 : MMOT_FP32;
  s->has_bf16 = s->dense_bf16 = o->precision == MMOT_BF16;
  s->keep_fwd = keeps_forward(p, o);
  s->stream = static_cast<hipStream_t>(stream);
  set_geometry(s);
  uintptr_t b = reinterpret_cast<uintptr_t>(ws);
  b = (b + 255) & ~uintptr_t(255);
  Carver c{reinterpret_cast<char*>(b)};
  carve(s, c);
  auto fail = [&](mmot_status e) { return e; };
  if (host_stats && host_flags) {
    s->host_stats = host_stats;
    s->host_flags = host_flags;
    s->owns_host = false;
    s->opt.use_graph = 0;
  } else {
    s->owns_host = true;
    if (hipHostMalloc(reinterpret_cast<void**>(&s->host_stats), 16 * sizeof(double), 0) != hipSuccess) return fail(MMOT_EHIP);
    if (hipHostMalloc(reinterpret_cast<void**>(&s->host_flags), 4 * sizeof(int), 0) != hipSuccess) return fail(MMOT_EHIP);
    if (hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking) != hipSuccess) return fail(MMOT_EHIP);
  }
  // domain: an estimate of the within-message dynamic range R = T * mean excess move cost / eps (log2 units)
  bool auto_probe = false;
  if (o->domain == MMOT_DOMAIN_AUTO && p->kind == MMOT_DENSE) {
    s->dom = MMOT_DOMAIN_SCALED;
  } else if (o->domain == MMOT_DOMAIN_AUTO) {
    launch_excess(p->rowptr, p->colidx, p->cost, p->n, s->exc_row, s->exc_cnt, s->exc, s->stream);
    double h = 0;
    if (hipMemcpyAsync(&s->host_stats[8], s->exc, sizeof(double), hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
      return fail(MMOT_EHIP);
    h = s->host_stats[8];
    const double R = (double)p->T * h / p->eps;       // natural-log range estimate
    const double limit = (s->prec == MMOT_FP64) ? 600.0 : 60.0;
    s->dom = (R <= limit) ? MMOT_DOMAIN_SCALED : MMOT_DOMAIN_LOG;
    auto_probe = s->dom == MMOT_DOMAIN_SCALED;
  } else {
    s->dom = o->domain;
  }
  st = dispatch(s, [&](auto impl) { return decltype(impl)::setup(s, p); });
  if (st != MMOT_OK) return fail(st);
  if (auto_probe) {
    // The cost estimate above misses the path-counting part of the range (a
    // state many forced moves away from the sink sees only a few of the walks
    // that a state next to it sees), so the scaled domain is confirmed by one
    // iteration: a zero or non-finite message at a support entry means the
    // within-commodity range exceeds the element type, and the solver switches
    // to the log domain.  Either way it then restarts from the initial scalings.
    const int g = s->opt.use_graph;
    s->opt.use_graph = 0;
    st = run_iterations(s, 1);
    s->opt.use_graph = g;
    if (st != MMOT_OK) return fail(st);
    const mmot_status fs = read_flags(s);
    if (fs == MMOT_EINFEASIBLE || fs == MMOT_ENUMERIC) s->dom = MMOT_DOMAIN_LOG;
    else if (fs != MMOT_OK) return fail(fs);
    else s->probe_clean = true;
    s->iters = 0;
    s->psi_fresh = s->pend_b = s->pend_f = s->hat_valid = false;
    s->force_calib = 0;
    st = dispatch(s, [&](auto impl) { return decltype(impl)::setup(s, p); });
    if (st != MMOT_OK) return fail(st);
  }
  return MMOT_OK;
}

// what create_into made, except the solver object itself
void release_solver(mmot_solver* s) {
  for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
  s->graphs.clear();
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  s->cap_stream = nullptr;
  if (s->owns_host) {
    if (s->host_stats) (void)hipHostFree(s->host_stats);
    if (s->host_flags) (void)hipHostFree(s->host_flags);
  }
  s->host_stats = nullptr;
  s->host_flags = nullptr;
}
}  // namespace

namespace {
// Workspace of mmot_solve_static: one array per GPU, held until the process
// ends.  In host code `scratch` names a host-side stand-in, not device memory;
// the device address comes from hipGetSymbolAddress, taken once per device with
// that device current, and only that address is ever handed to kernels or copies.
constexpr size_t kStaticWorkspaceBytes = MMOT_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];
constexpr int kMaxDevices = 64;
void* g_scratch_dev[kMaxDevices] = {};
std::mutex g_scratch_mu;

mmot_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MMOT_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MMOT_EHIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return MMOT_OK;
}
}  // namespace

extern "C" {

void mmot_default_options(mmot_options* o) {
  if (!o) return;
  o->precision = MMOT_FP32;
  o->domain = MMOT_DOMAIN_AUTO;
  o->check_every = 10;
  o->calib_every = 10;
  o->polish_iters = 20;
  o->use_graph = 1;
  o->tol = 1e-6;
  o->keep_forward = 1;
}

mmot_status mmot_query_workspace(const mmot_problem* p, const mmot_options* o, size_t* bytes) {
  if (!bytes) return MMOT_EINVAL;
  mmot_status st = basic_checks(p, o);
  if (st != MMOT_OK) return st;
  mmot_solver tmp;
  tmp.n = p->n; tmp.L = p->L; tmp.T = p->T; tmp.nnz = p->nnz; tmp.kind = p->kind;
  tmp.steps_k = p->cost_per_step ? p->T : 1;
  tmp.has_kl = p->state_cost != nullptr;
  tmp.has_comm = p->cap_comm != nullptr && p->T > 1;
  tmp.comm_steps = p->cap_comm_per_step ? std::max(p->T - 1, 1) : 1;
  tmp.prec = (o->precision == MMOT_FP64) ? MMOT_FP64 : MMOT_FP32;
  tmp.has_bf16 = o->precision == MMOT_BF16;
  tmp.keep_fwd = keeps_forward(p, o);
  set_geometry(&tmp);
  Carver c{nullptr};
  carve(&tmp, c);
  *bytes = c.off + 256;
  return MMOT_OK;
}

mmot_status mmot_pool_query_workspace(const mmot_problem* p, const mmot_options* o, size_t* bytes) {
  if (!bytes || !o) return MMOT_EINVAL;
  if (o->keep_forward) return MMOT_EUNSUPPORTED;   // (as mmot_pool_submit)
  size_t need = 0;
  const mmot_status st = mmot_query_workspace(p, o, &need);
  if (st != MMOT_OK) return st;
  *bytes = need + 256 + (size_t)pool_prog_items(p->T, o->check_every) * sizeof(PoolItem);
  return MMOT_OK;
}

mmot_status mmot_create(const mmot_problem* p, const mmot_options* o, void* ws, size_t ws_bytes, void* stream,
                        mmot_solver** out) {
  if (!out) return MMOT_EINVAL;
  *out = nullptr;
  mmot_status st = basic_checks(p, o);
  if (st != MMOT_OK) return st;
  if (!p->cap || !p->src || !p->dst) return MMOT_EINVAL;
  if (p->kind == MMOT_CSR && (!p->rowptr || !p->colidx || !p->cost)) return MMOT_EINVAL;
  if (p->kind == MMOT_DENSE && !p->cost_dense) return MMOT_EINVAL;
  size_t need = 0;
  st = mmot_query_workspace(p, o, &need);
  if (st != MMOT_OK) return st;
  if (!ws || ws_bytes < need) return MMOT_ENOMEM;
  mmot_solver* s = new (std::nothrow) mmot_solver();
  if (!s) return MMOT_ENOMEM;
  st = create_into(s, p, o, ws, stream, nullptr, nullptr);
  if (st != MMOT_OK) { mmot_destroy(s); return st; }
  *out = s;
  return MMOT_OK;
}

mmot_status mmot_iterate(mmot_solver* s, int32_t n_iter, mmot_stats* stats) {
  if (!s || n_iter < 0) return MMOT_EINVAL;
  mmot_status st = run_iterations(s, n_iter);
  if (st != MMOT_OK) return st;
  if (stats) return check_pass(s, nullptr, nullptr, stats);
  return MMOT_OK;
}

mmot_status mmot_stats_now(mmot_solver* s, mmot_stats* stats) {
  if (!s || !stats) return MMOT_EINVAL;
  return check_pass(s, nullptr, nullptr, stats);
}

mmot_status mmot_solve(mmot_solver* s, int32_t max_iter, mmot_stats* stats) {
  if (!s || max_iter < 0) return MMOT_EINVAL;
  mmot_stats local{};
  int done = 0;
  mmot_status st = MMOT_OK;
  while (done < max_iter) {
    const int k = std::min(s->opt.check_every, max_iter - done);
    st = mmot_iterate(s, k, &local);
    done += k;
    if (st != MMOT_OK) break;
    if (local.converged) break;
  }
  if (done == 0) st = mmot_stats_now(s, &local);
  if (st == MMOT_OK && s->dense_bf16 && s->opt.polish_iters > 0) {
    // BF16 products converge to a slightly perturbed fixed point; finish in FP32
    s->dense_bf16 = false;
    st = mmot_iterate(s, s->opt.polish_iters, &local);
  }
  if (stats) *stats = local;
  return st;
}

mmot_status mmot_solve_static(const mmot_problem* p, const mmot_options* o, int32_t max_iter, double* occ,
                              mmot_stats* stats, void* stream) {
  if (!p || !o || max_iter < 0) return MMOT_EINVAL;
  mmot_status st = basic_checks(p, o);
  if (st != MMOT_OK) return st;
  if (!p->cap || !p->src || !p->dst) return MMOT_EINVAL;
  if (p->kind == MMOT_CSR && (!p->rowptr || !p->colidx || !p->cost)) return MMOT_EINVAL;
  if (p->kind == MMOT_DENSE && !p->cost_dense) return MMOT_EINVAL;
  size_t need = 0;
  st = mmot_query_workspace(p, o, &need);
  if (st != MMOT_OK) return st;
  if (need > kStaticWorkspaceBytes) return MMOT_ENOMEM;
  void* ws = nullptr;
  st = scratch_address(&ws);
  if (st != MMOT_OK) return st;
  // the solver object and its host buffers live on this call's stack; no
  // captured graphs (they would be instantiated, i.e. allocated)
  double host_stats[16];
  int host_flags[4];
  mmot_solver s;
  st = create_into(&s, p, o, ws, stream, host_stats, host_flags);
  if (st == MMOT_OK) st = mmot_solve(&s, max_iter, stats);
  if (st == MMOT_OK && occ) st = mmot_occupancy(&s, occ, nullptr);
  release_solver(&s);
  return st;
}

mmot_status mmot_set_precision(mmot_solver* s, int32_t precision) {
  if (!s) return MMOT_EINVAL;
  if (s->kind != MMOT_DENSE) return (precision == (s->prec == MMOT_FP64 ? MMOT_FP64 : MMOT_FP32)) ? MMOT_OK : MMOT_EUNSUPPORTED;
  if (precision == MMOT_BF16) {
    if (!s->has_bf16) return MMOT_EUNSUPPORTED;
    s->dense_bf16 = true;
  } else if (precision == MMOT_FP32) {
    s->dense_bf16 = false;
  } else {
    return MMOT_EUNSUPPORTED;
  }
  s->hat_valid = false;   // (kept forward messages of the other precision)
  return MMOT_OK;
}

mmot_status mmot_occupancy_window(mmot_solver* s, double* occ, double* per_comm, int32_t comm_first,
                                  int32_t comm_count) {
  if (!s || !occ) return MMOT_EINVAL;
  if (per_comm && (comm_first < 0 || comm_count < 1 || comm_first > s->L - comm_count)) return MMOT_EINVAL;
  s->pc_lo = per_comm ? comm_first : 0;
  s->pc_cnt = per_comm ? comm_count : 0;
  return check_pass(s, occ, per_comm, nullptr);
}

mmot_status mmot_occupancy(mmot_solver* s, double* occ, double* per_comm) {
  if (!s) return MMOT_EINVAL;
  return mmot_occupancy_window(s, occ, per_comm, 0, s->L);
}

mmot_status mmot_edge_flows(mmot_solver* s, double* flow, double* cost_host) {
  if (!s || !flow) return MMOT_EINVAL;
  ensure_fresh(s);
  dispatch(s, [&](auto impl) { decltype(impl)::flows_pass(s, flow, s->stream); return 0; });
  s->hat_valid = false;   // (its rolling panels overlap the kept ones)
  if (hipGetLastError() != hipSuccess) return MMOT_EHIP;
  if (cost_host) {
    if (hipMemcpyAsync(s->host_stats + 7, s->stats_dev + 7, sizeof(double), hipMemcpyDeviceToHost, s->stream) !=
            hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
      return MMOT_EHIP;
    *cost_host = s->host_stats[7];
  }
  return MMOT_OK;
}

mmot_status mmot_get_log_duals(mmot_solver* s, double* ls, double* ld, double* lc) {
  if (!s) return MMOT_EINVAL;
  if (s->prec == MMOT_FP64) {
    if (s->dom == MMOT_DOMAIN_LOG)
      launch_log_duals<double, true>(static_cast<double*>(s->U01), s->gauge0, static_cast<double*>(s->U0T), s->gaugeT,
                                     static_cast<double*>(s->u), s->n, s->L, s->Lp, s->T - 1, ls, ld, lc, s->stream);
    else
      launch_log_duals<double, false>(static_cast<double*>(s->U01), s->gauge0, static_cast<double*>(s->U0T), s->gaugeT,
                                      static_cast<double*>(s->u), s->n, s->L, s->Lp, s->T - 1, ls, ld, lc, s->stream);
  } else {
    if (s->dom == MMOT_DOMAIN_LOG)
      launch_log_duals<float, true>(static_cast<float*>(s->U01), s->gauge0, static_cast<float*>(s->U0T), s->gaugeT,
                                    static_cast<float*>(s->u), s->n, s->L, s->Lp, s->T - 1, ls, ld, lc, s->stream);
    else
      launch_log_duals<float, false>(static_cast<float*>(s->U01), s->gauge0, static_cast<float*>(s->U0T), s->gaugeT,
                                     static_cast<float*>(s->u), s->n, s->L, s->Lp, s->T - 1, ls, ld, lc, s->stream);
  }
  return hipGetLastError() == hipSuccess ? MMOT_OK : MMOT_EHIP;
}

mmot_status mmot_get_comm_duals(mmot_solver* s, double* log_w) {
  if (!s || !log_w || !s->has_comm) return MMOT_EINVAL;
  dispatch(s, [&](auto impl) {
    using I = decltype(impl);
    using V = typename I::value_type;
    launch_comm_duals<V, I::kLog>(static_cast<const V*>(s->wcomm), s->n, s->L, s->Lp, s->T - 1, log_w, 0, nullptr,
                                  nullptr, s->stream);
    return 0;
  });
  return hipGetLastError() == hipSuccess ? MMOT_OK : MMOT_EHIP;
}

mmot_status mmot_set_comm_duals(mmot_solver* s, const double* log_w) {
  if (!s || !log_w || !s->has_comm) return MMOT_EINVAL;
  dispatch(s, [&](auto impl) {
    using I = decltype(impl);
    using V = typename I::value_type;
    launch_comm_duals<V, I::kLog>(nullptr, s->n, s->L, s->Lp, s->T - 1, nullptr, 1, log_w,
                                  static_cast<V*>(s->wcomm), s->stream);
    return 0;
  });
  s->psi_fresh = s->hat_valid = false;
  return hipGetLastError() == hipSuccess ? MMOT_OK : MMOT_EHIP;
}

mmot_status mmot_set_log_duals(mmot_solver* s, const double* ls, const double* ld, const double* lc) {
  if (!s) return MMOT_EINVAL;
  if (s->prec == MMOT_FP64) {
    if (s->dom == MMOT_DOMAIN_LOG)
      launch_set_duals<double, true>(ls, ld, lc, s->n, s->L, s->Lp, s->T - 1, static_cast<double*>(s->U01),
                                     static_cast<double*>(s->U0T), static_cast<double*>(s->u), s->gauge0, s->gaugeT, s->stream);
    else
      launch_set_duals<double, false>(ls, ld, lc, s->n, s->L, s->Lp, s->T - 1, static_cast<double*>(s->U01),
                                      static_cast<double*>(s->U0T), static_cast<double*>(s->u), s->gauge0, s->gaugeT, s->stream);
  } else {
    if (s->dom == MMOT_DOMAIN_LOG)
      launch_set_duals<float, true>(ls, ld, lc, s->n, s->L, s->Lp, s->T - 1, static_cast<float*>(s->U01),
                                    static_cast<float*>(s->U0T), static_cast<float*>(s->u), s->gauge0, s->gaugeT, s->stream);
    else
      launch_set_duals<float, false>(ls, ld, lc, s->n, s->L, s->Lp, s->T - 1, static_cast<float*>(s->U01),
                                     static_cast<float*>(s->U0T), static_cast<float*>(s->u), s->gauge0, s->gaugeT, s->stream);
  }
  launch_fill<uint32_t>(s->slotsE, (size_t)s->nslot * s->Lp, 0u, s->stream);
  launch_fill<uint32_t>(s->slotsS, (size_t)s->nslot * s->Lp, 0u, s->stream);
  launch_fill<double>(s->lvlT, s->Lp, 0.0, s->stream);
  launch_fill<double>(s->lvl0, s->Lp, 0.0, s->stream);
  s->psi_fresh = s->hat_valid = false;
  s->force_calib = 2;
  return hipGetLastError() == hipSuccess ? MMOT_OK : MMOT_EHIP;
}

void mmot_destroy(mmot_solver* s) {
  if (!s) return;
  release_solver(s);
  delete s;
}

const char* mmot_status_str(mmot_status st) {
  switch (st) {
    case MMOT_OK: return "ok";
    case MMOT_EINVAL: return "invalid argument or problem data";
    case MMOT_ENOMEM: return "workspace too small";
    case MMOT_EINFEASIBLE: return "infeasible: a positive source/sink entry faces a zero message";
    case MMOT_ENUMERIC: return "non-finite values (range exceeded)";
    case MMOT_EHIP: return "HIP runtime error";
    case MMOT_EAGAIN: return "over the HBM budget, retry later";
    case MMOT_EUNSUPPORTED: return "unsupported option combination";
  }
  return "unknown status";
}

int64_t mmot_iterations(const mmot_solver* s) { return s ? s->iters : -1; }

// ---------------------------------------------------------------------------
// serving pool
// ---------------------------------------------------------------------------
struct mmot_pool {
  size_t budget = 0, used = 0;
  hipStream_t stream = nullptr;       // batched lane: the tick launches
  hipStream_t setup = nullptr;        // admission work (validation, operators, probe)
  // Dedicated lanes (a solve's own captured graphs on a pool stream): lane 0 for
  // solves whose steps fill the GPU alone -- one at a time, in arrival order,
  // beside the batched lane (two together would only stretch both) -- and
  // express lanes 1..kLanes-1 for small solves admitted while the batched lane
  // is nearly idle: alone, a small solve finishes sooner replaying its own
  // graphs than advancing one kernel per tick; under load it joins the ticks.
  static constexpr int kLanes = 3;
  static constexpr int kExpressBelow = 2;   // batched requests running, at most, to use an express lane
  hipStream_t lanes[kLanes] = {nullptr, nullptr, nullptr};
  std::deque<uint64_t> lane_queue;    // admitted large solves waiting for a lane
  uint64_t next_ticket = 1;
  struct Req {
    uint64_t ticket = 0;
    mmot_solver* s = nullptr;
    size_t bytes = 0;
    int32_t max_iter = 0;
    int32_t state = 0;       // 0 running, 1 done, 2 failed
    int32_t status = MMOT_OK;
    int lane = -1;           // -1: batched lane, -2: waiting for a dedicated lane, else its stream index
    // batched lane: the current chunk's program, resident on the device in the
    // program area at the end of the request's workspace (prog_cap items)
    PoolItem* d_prog = nullptr;
    std::vector<PoolItem> h_prog;   // host copy (the upload's source until the chunk has run)
    int prog_cap = 0, len = 0;
    int pc = 0;              // next item of the chunk: it advances only when a tick runs the item
    hipEvent_t up_ev = nullptr;     // the chunk's upload (on the set-up stream)
    bool upload_wait = false;       // the tick stream has yet to wait for up_ev
    bool awaiting = false;   // chunk enqueued, its statistics not yet read
    hipEvent_t ev = nullptr;
    mmot_stats stats{};
    int iters_planned = 0;
  };
  std::map<uint64_t, Req*> reqs;
  int64_t ticks = 0;
  uint64_t rr = 0;                    // round-robin start among the ready batched requests
  static constexpr int kLead = 16;    // ticks the host may run ahead of the device
  hipEvent_t lead_ev[kLead] = {};
};

namespace {

constexpr int kFillBlocks = 256;      // a step of at least this many blocks fills the GPU alone


// Batched lane: record the next chunk of a request's work -- the same calls
// mmot_solve makes (check_every iterations, then the check pass up to its
// statistics reduction) -- and upload it; it starts at the next tick.
mmot_status pool_program(mmot_pool* P, mmot_pool::Req* r) {
  mmot_solver* s = r->s;
  const int k = std::min(s->opt.check_every, r->max_iter - r->iters_planned);
  Recorder rec;
  tl_recorder = &rec;
  const int saved_graph = s->opt.use_graph;
  s->opt.use_graph = 0;
  run_iterations(s, k);
  ensure_fresh(s);
  dispatch(s, [&](auto impl) { decltype(impl)::forward(s, 1, false, false, nullptr, nullptr, s->stream); return 0; });
  launch_reduce_stats(s->part, s->nblk, s->nblk_s, s->nblk_s, s->T + 1, s->tpart, s->eps, s->stats_dev, s->stream);
  s->opt.use_graph = saved_graph;
  tl_recorder = nullptr;
  // an item whose arguments did not fit, or a chunk longer than the program area,
  // would run incomplete: refuse the request instead
  const int n = (int)rec.items.size();
  if (!rec.ok || n > r->prog_cap || n == 0) return MMOT_EUNSUPPORTED;
  r->iters_planned += k;
  // The previous chunk has run to completion (its statistics were read), so no
  // queued tick reads the program area.  The upload runs on the set-up stream
  // (its host-side staging does not wait for queued ticks); the tick stream
  // waits for it before the chunk's first item.
  r->h_prog.assign(rec.items.begin(), rec.items.end());
  if (hipMemcpyAsync(r->d_prog, r->h_prog.data(), sizeof(PoolItem) * n, hipMemcpyHostToDevice, P->setup) !=
          hipSuccess ||
      hipEventRecord(r->up_ev, P->setup) != hipSuccess)
    return MMOT_EHIP;
  r->upload_wait = true;
  r->len = n;
  r->pc = 0;
  r->awaiting = false;
  return MMOT_OK;
}

// enqueue the copy of a request's statistics and flags behind its chunk
mmot_status pool_fetch_stats(mmot_pool::Req* r, hipStream_t st) {
  mmot_solver* s = r->s;
  if (hipMemcpyAsync(s->host_stats, s->stats_dev, 8 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(s->host_flags, s->flags, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipEventRecord(r->ev, st) != hipSuccess)
    return MMOT_EHIP;
  r->awaiting = true;
  return MMOT_OK;
}

// Dedicated lane: enqueue the next chunk with the solver's own launches
// (captured iteration graphs, then the check pass) on the lane's stream.
mmot_status lane_chunk(mmot_pool::Req* r) {
  mmot_solver* s = r->s;
  const int k = std::min(s->opt.check_every, r->max_iter - r->iters_planned);
  mmot_status st = run_iterations(s, k);
  if (st != MMOT_OK) return st;
  st = check_pass(s, nullptr, nullptr, nullptr);
  if (st != MMOT_OK) return st;
  launch_reduce_stats(s->part, s->nblk, s->nblk_s, s->nblk_s, s->T + 1, s->tpart, s->eps, s->stats_dev, s->stream);
  r->iters_planned += k;
  return pool_fetch_stats(r, s->stream);
}

// a chunk whose statistics have landed: decide, and schedule the next one
mmot_status pool_finish_chunk(mmot_pool* P, mmot_pool::Req* r) {
  mmot_solver* s = r->s;
  r->awaiting = false;
  mmot_stats& o = r->stats;
  const int f = *s->host_flags;
  o.iters = (int32_t)s->iters;
  o.domain = s->dom;
  o.precision = s->prec;
  o.dual_obj = s->host_stats[0];
  o.src_resid = s->host_stats[1];
  o.cap_viol = s->host_stats[2];
  o.mass_drift = s->host_stats[3];
  o.dual_gap = s->host_stats[4];
  o.mass = s->host_stats[5];
  o.converged = (o.src_resid <= s->opt.tol && o.cap_viol <= s->opt.tol) ? 1 : 0;
  mmot_status st = MMOT_OK;
  if (f & FLAG_INFEASIBLE) st = zero_message_status(s);
  else if ((f & FLAG_NONFINITE) || s->host_stats[6] > 0 || !std::isfinite(s->host_stats[0])) st = MMOT_ENUMERIC;
  if (st == MMOT_OK && !o.converged && r->iters_planned < r->max_iter)
    return r->lane >= 0 ? lane_chunk(r) : pool_program(P, r);
  r->state = st == MMOT_OK ? 1 : 2;
  r->status = st;
  // finished: the solver's work has completed (its event fired); later output
  // calls on it run on the pool's stream, ordered with the caller's work there
  s->stream = P->stream;
  return MMOT_OK;
}

void pool_sync_all(mmot_pool* P) {
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  for (int i = 0; i < mmot_pool::kLanes; ++i)
    if (P->lanes[i]) (void)hipStreamSynchronize(P->lanes[i]);
}

}  // namespace

mmot_status mmot_pool_create(size_t hbm_budget, void* stream, mmot_pool** out) {
  if (!out || hbm_budget == 0) return MMOT_EINVAL;
  mmot_pool* P = new (std::nothrow) mmot_pool();
  if (!P) return MMOT_ENOMEM;
  P->budget = hbm_budget;
  P->stream = static_cast<hipStream_t>(stream);
  bool ok = hipStreamCreateWithFlags(&P->setup, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; ok && i < mmot_pool::kLanes; ++i)
    ok = hipStreamCreateWithFlags(&P->lanes[i], hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; ok && i < mmot_pool::kLead; ++i)
    ok = hipEventCreateWithFlags(&P->lead_ev[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) { mmot_pool_destroy(P); return MMOT_EHIP; }
  *out = P;
  return MMOT_OK;
}

mmot_status mmot_pool_submit(mmot_pool* P, const mmot_problem* prob, const mmot_options* opt, void* ws,
                             size_t ws_bytes, int32_t max_iter, uint64_t* ticket) {
  if (!P || !prob || !opt || !ticket || max_iter < 1) return MMOT_EINVAL;
  if (prob->kind != MMOT_CSR || opt->precision != MMOT_FP32) return MMOT_EUNSUPPORTED;
  if (opt->keep_forward) return MMOT_EUNSUPPORTED;   // the pool keeps two forward panels per request
  size_t need = 0, solver_need = 0;
  mmot_status st = mmot_pool_query_workspace(prob, opt, &need);
  if (st != MMOT_OK) return st;
  if (!ws || ws_bytes < need) return MMOT_ENOMEM;
  (void)mmot_query_workspace(prob, opt, &solver_need);
  if (P->used + need > P->budget) return MMOT_EAGAIN;
  // set-up runs on the pool's own set-up stream and ends synchronised, so it
  // never waits for queued ticks; the solver then moves to its lane
  mmot_solver* s = nullptr;
  st = mmot_create(prob, opt, ws, solver_need, P->setup, &s);
  if (st != MMOT_OK) return st;
  auto* r = new (std::nothrow) mmot_pool::Req();
  if (!r) { mmot_destroy(s); return MMOT_ENOMEM; }
  r->ticket = P->next_ticket++;
  r->s = s;
  r->bytes = need;
  r->max_iter = max_iter;
  // the program area: after the solver's workspace, 256-byte aligned
  uintptr_t pa = reinterpret_cast<uintptr_t>(ws) + solver_need;
  pa = (pa + 255) & ~uintptr_t(255);
  r->d_prog = reinterpret_cast<PoolItem*>(pa);
  r->prog_cap = (int)pool_prog_items(prob->T, s->opt.check_every);
  if (hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess) { mmot_destroy(s); delete r; return MMOT_EHIP; }
  if (hipEventCreateWithFlags(&r->up_ev, hipEventDisableTiming) != hipSuccess) {
    mmot_destroy(s); (void)hipEventDestroy(r->ev); delete r; return MMOT_EHIP;
  }
  int express = -1;
  if (s->nblk < kFillBlocks) {
    int batched = 0;
    bool used[mmot_pool::kLanes] = {};
    for (auto& kv : P->reqs) {
      const mmot_pool::Req* q = kv.second;
      if (q->state != 0) continue;
      if (q->lane == -1) ++batched;
      else if (q->lane > 0) used[q->lane] = true;
    }
    for (int i = 1; i < mmot_pool::kLanes && express < 0 && batched < mmot_pool::kExpressBelow; ++i)
      if (!used[i]) express = i;
  }
  if (s->nblk >= kFillBlocks) {
    r->lane = -2;                      // started by mmot_pool_run when lane 0 is free
    P->lane_queue.push_back(r->ticket);
  } else if (express > 0) {
    r->lane = express;
    s->stream = P->lanes[express];
    st = lane_chunk(r);
  } else {
    s->stream = P->stream;
    st = pool_program(P, r);
  }
  if (st != MMOT_OK) {
    if (r->lane == -2) P->lane_queue.pop_back();
    (void)hipStreamSynchronize(P->setup);
    mmot_destroy(s); (void)hipEventDestroy(r->ev); (void)hipEventDestroy(r->up_ev); delete r; return st;
  }
  P->used += need;
  P->reqs[r->ticket] = r;
  *ticket = r->ticket;
  return MMOT_OK;
}

mmot_status mmot_pool_run(mmot_pool* P, int32_t max_ticks, int32_t* n_running) {
  if (!P || max_ticks < 0) return MMOT_EINVAL;
  for (int tk = 0; tk < max_ticks; ++tk) {
    // chunks whose statistics have landed: decide and schedule the next chunk
    bool large_busy = false;
    for (auto& kv : P->reqs) {
      mmot_pool::Req* r = kv.second;
      if (r->state == 0 && r->awaiting && hipEventQuery(r->ev) == hipSuccess) {
        const mmot_status st = pool_finish_chunk(P, r);
        if (st != MMOT_OK) { r->state = 2; r->status = st; }
      }
      large_busy = large_busy || (r->state == 0 && r->lane == 0);
    }
    // start the oldest waiting large solve when lane 0 is free
    while (!large_busy && !P->lane_queue.empty()) {
      auto it = P->reqs.find(P->lane_queue.front());
      P->lane_queue.pop_front();
      if (it == P->reqs.end() || it->second->state != 0) continue;
      mmot_pool::Req* r = it->second;
      r->lane = 0;
      r->s->stream = P->lanes[0];
      const mmot_status st = lane_chunk(r);
      if (st != MMOT_OK) { r->state = 2; r->status = st; r->s->stream = P->stream; continue; }
      large_busy = true;
    }
    // one tick of the batched lane: the next item of up to kTickSlots batched
    // requests, taken round-robin among those with an item ready; a request
    // left out waits for a later tick (its program counter moves only when its
    // item runs)
    std::vector<mmot_pool::Req*> ready;
    for (auto& kv : P->reqs) {
      mmot_pool::Req* r = kv.second;
      if (r->state != 0 || r->lane >= 0 || r->awaiting || r->pc >= r->len) continue;
      ready.push_back(r);
    }
    if (ready.empty()) break;   // nothing batched to run now: let the caller admit and poll
    TickArgs ta;
    ta.nslot = 0;
    int total = 0;
    bool lean = true;   // every item of the tick is light: the leaner tick kernel
    mmot_pool::Req* in_tick[kTickSlots];
    const size_t start = (size_t)(P->rr++ % ready.size());
    for (size_t q = 0; q < ready.size() && ta.nslot < kTickSlots; ++q) {
      mmot_pool::Req* r = ready[(start + q) % ready.size()];
      if (r->upload_wait) {
        if (hipStreamWaitEvent(P->stream, r->up_ev, 0) != hipSuccess) return MMOT_EHIP;
        r->upload_wait = false;
      }
      const PoolItem& it = r->h_prog[r->pc];
      ta.prefix[ta.nslot] = total;
      ta.idx[ta.nslot] = r->pc;
      ta.prog[ta.nslot] = r->d_prog;
      lean = lean && pool_item_is_light(it);
      total += it.nblk;
      in_tick[ta.nslot++] = r;
    }
    ta.prefix[ta.nslot] = total;
    const int li = (int)(P->ticks % mmot_pool::kLead);
    if (P->ticks >= mmot_pool::kLead) (void)hipEventSynchronize(P->lead_ev[li]);
    launch_pool_tick(ta, lean, P->stream);
    if (hipEventRecord(P->lead_ev[li], P->stream) != hipSuccess) return MMOT_EHIP;
    // requests whose chunk ended with this tick: fetch their statistics
    for (int q = 0; q < ta.nslot; ++q) {
      mmot_pool::Req* r = in_tick[q];
      if (++r->pc == r->len)
        if (pool_fetch_stats(r, P->stream) != MMOT_OK) return MMOT_EHIP;
    }
    ++P->ticks;
  }
  if (n_running) {
    int c = 0;
    for (auto& kv : P->reqs) c += kv.second->state == 0;
    *n_running = c;
  }
  return MMOT_OK;
}

mmot_status mmot_pool_poll(mmot_pool* P, uint64_t ticket, int32_t* state, mmot_stats* stats) {
  if (!P || !state) return MMOT_EINVAL;
  auto it = P->reqs.find(ticket);
  if (it == P->reqs.end()) return MMOT_EINVAL;
  mmot_pool::Req* r = it->second;
  if (r->state == 0 && r->awaiting && hipEventQuery(r->ev) == hipSuccess) {
    const mmot_status st = pool_finish_chunk(P, r);
    if (st != MMOT_OK) { r->state = 2; r->status = st; }
  }
  *state = r->state;
  if (stats) *stats = r->stats;
  return r->state == 2 ? (mmot_status)r->status : MMOT_OK;
}

mmot_solver* mmot_pool_solver(mmot_pool* P, uint64_t ticket) {
  if (!P) return nullptr;
  auto it = P->reqs.find(ticket);
  return it == P->reqs.end() ? nullptr : it->second->s;
}

mmot_status mmot_pool_release(mmot_pool* P, uint64_t ticket) {
  if (!P) return MMOT_EINVAL;
  auto it = P->reqs.find(ticket);
  if (it == P->reqs.end()) return MMOT_EINVAL;
  mmot_pool::Req* r = it->second;
  if (r->state == 0) return MMOT_EAGAIN;
  (void)hipStreamSynchronize(r->s->stream);
  (void)hipStreamSynchronize(P->setup);
  mmot_destroy(r->s);
  (void)hipEventDestroy(r->ev);
  if (r->up_ev) (void)hipEventDestroy(r->up_ev);
  P->used -= r->bytes;
  delete r;
  P->reqs.erase(it);
  return MMOT_OK;
}

void mmot_pool_destroy(mmot_pool* P) {
  if (!P) return;
  pool_sync_all(P);
  for (auto& kv : P->reqs) {
    mmot_destroy(kv.second->s);
    if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
    if (kv.second->up_ev) (void)hipEventDestroy(kv.second->up_ev);
    delete kv.second;
  }
  for (int i = 0; i < mmot_pool::kLead; ++i)
    if (P->lead_ev[i]) (void)hipEventDestroy(P->lead_ev[i]);
  for (int i = 0; i < mmot_pool::kLanes; ++i)
    if (P->lanes[i]) (void)hipStreamDestroy(P->lanes[i]);
  if (P->setup) (void)hipStreamDestroy(P->setup);
  delete P;
}

mmot_status mmot_time_step(mmot_solver* s, int32_t forward, int32_t reps, double* avg_ms) {
  if (!s || reps < 1 || !avg_ms) return MMOT_EINVAL;
  mmot_status st = dispatch(s, [&](auto impl) { return decltype(impl)::time_step(s, forward ? 1 : 0, reps, avg_ms); });
  s->psi_fresh = s->hat_valid = false;   // the timed launches overwrite message buffers
  return st;
}

}  // extern "C"
