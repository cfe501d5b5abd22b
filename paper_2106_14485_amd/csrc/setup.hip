// One-time setup kernels: validation of the problem data, the Gibbs kernel
// K = exp(-C/eps) of eq. K_multicommodity on the CSR of C and of C^T, the
// state-cost kernel K_L = exp(-C_L/eps), conversion of R^(0,1), R^(0,TT), d to
// the state-major internal layout, and the initial scalings.
#include "mmot_internal.h"
#include <math.h>

namespace mmot {

// -------- validation --------
__global__ void k_validate_vals(const double* __restrict__ x, size_t cnt, int allow_inf, int strictly_pos,
                                int allow_neg, int* flags) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < cnt; i += (size_t)gridDim.x * blockDim.x) {
    const double v = x[i];
    bool bad = isnan(v) || (isinf(v) && v < 0);   // -inf is never a valid cost, mass or capacity
    if (!allow_inf && isinf(v)) bad = true;
    if (!allow_neg && v < 0) bad = true;
    if (strictly_pos && !(v > 0)) bad = true;
    if (bad) atomicOr(flags, FLAG_BADINPUT);
  }
}

__global__ void k_validate_csr(const int* __restrict__ rp, const int* __restrict__ ci, int n, long long nnz,
                               int* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  if (i == 0 && rp[0] != 0) atomicOr(flags, FLAG_BADCSR);
  if (i == n) { if ((long long)rp[n] != nnz) atomicOr(flags, FLAG_BADCSR); return; }
  const int a = rp[i], b = rp[i + 1];
  if (b < a || a < 0 || (long long)b > nnz) { atomicOr(flags, FLAG_BADCSR); return; }
  int prev = -1;
  for (int e = a; e < b; ++e) {
    const int j = ci[e];
    if (j < 0 || j >= n || j <= prev) { atomicOr(flags, FLAG_BADCSR); return; }
    prev = j;
  }
}

// per-commodity masses of src and dst must agree (mu_0, Section 3.2)
__global__ void k_validate_mass(const double* __restrict__ src, const double* __restrict__ dst, int n,
                                int* flags, double* masses) {
  const int l = blockIdx.x;
  __shared__ double rs[256], rd[256];
  double a = 0, b = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    a += src[(size_t)l * n + i];
    b += dst[(size_t)l * n + i];
  }
  rs[threadIdx.x] = a; rd[threadIdx.x] = b;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) { rs[threadIdx.x] += rs[threadIdx.x + s]; rd[threadIdx.x] += rd[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    masses[l] = rs[0];
    if (!(rs[0] > 0) || fabs(rs[0] - rd[0]) > 1e-9 * fmax(rs[0], rd[0])) atomicOr(flags, FLAG_MASS);
  }
}

// -------- Gibbs kernel on CSR --------
template <typename V, bool LOG>
__global__ void k_gibbs(const double* __restrict__ cost, size_t nnz, double eps, V* __restrict__ kv) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nnz; e += (size_t)gridDim.x * blockDim.x) {
    const double c = cost[e];
    kv[e] = LOG ? static_cast<V>(-c / eps * M_LOG2E) : static_cast<V>(exp(-c / eps));
  }
}

// -------- transpose of the CSR pattern (forward operator = K^T rows) --------
__global__ void k_count_cols(const int* __restrict__ ci, long long nnz, int* __restrict__ cnt) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nnz; e += (long long)gridDim.x * blockDim.x)
    atomicAdd(&cnt[ci[e]], 1);
}

// exclusive scan of n counts into rp[0..n], single block (setup only)
__global__ void k_scan(const int* __restrict__ cnt, int n, int* __restrict__ rp) {
  __shared__ int part[1024];
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = (n + nt - 1) / nt;
  const int a = min(n, t * per), b = min(n, a + per);
  int s = 0;
  for (int i = a; i < b; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int k = 0; k < nt; ++k) { const int v = part[k]; part[k] = acc; acc += v; }
    rp[n] = acc;
  }
  __syncthreads();
  int acc = part[t];
  for (int i = a; i < b; ++i) { rp[i] = acc; acc += cnt[i]; }
}

__global__ void k_fill_transpose(const int* __restrict__ rp, const int* __restrict__ ci, int n,
                                 const int* __restrict__ rpt, int* __restrict__ cursor, int* __restrict__ cit,
                                 int* __restrict__ srcpos) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const int j = ci[e];
    const int pos = rpt[j] + atomicAdd(&cursor[j], 1);
    cit[pos] = i;
    srcpos[pos] = e;
  }
}

// sort each transposed row by source state (insertion sort; rows are short)
__global__ void k_sort_rows(const int* __restrict__ rpt, int n, int* __restrict__ cit, int* __restrict__ srcpos) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int a = rpt[j], b = rpt[j + 1];
  for (int k = a + 1; k < b; ++k) {
    const int key = cit[k], val = srcpos[k];
    int m = k - 1;
    while (m >= a && cit[m] > key) { cit[m + 1] = cit[m]; srcpos[m + 1] = srcpos[m]; --m; }
    cit[m + 1] = key; srcpos[m + 1] = val;
  }
}

template <typename V>
__global__ void k_gather_vals(const V* __restrict__ kv, const int* __restrict__ srcpos, long long nnz, V* __restrict__ kvt) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nnz; e += (long long)gridDim.x * blockDim.x)
    kvt[e] = kv[srcpos[e]];
}

// max over rows of the row sum of K (log2), for the first-sweep range bound
template <typename V, bool LOG>
__global__ void k_rowsum_max(const int* __restrict__ rp, const V* __restrict__ kv, int n, double klmax_log2,
                             uint32_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float v = -INFINITY;
  if (i < n) {
    double s = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) s += LOG ? exp2((double)kv[e]) : (double)kv[e];
    if (s > 0) v = (float)(log2(s) + klmax_log2);
  }
  for (int m = 32; m > 0; m >>= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
  if ((threadIdx.x & 63) == 0 && v > -INFINITY) atomicMax(out, enc_f32(v));
}

// -------- ELL copy of an operator (rows padded to D entries) --------
__global__ void k_max_degree(const int* __restrict__ rp, int n, int* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int d = (i < n) ? rp[i + 1] - rp[i] : 0;
  for (int m = 32; m > 0; m >>= 1) d = max(d, __shfl_xor(d, m, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, d);
}
template <typename V>
__global__ void k_build_ell(const int* __restrict__ rp, const int* __restrict__ ci, const V* __restrict__ kv, int n,
                            int D, V pad, int* __restrict__ eci, V* __restrict__ ekv, int* __restrict__ deg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = rp[i], d = rp[i + 1] - a;
  deg[i] = d;
  for (int k = 0; k < D; ++k) {
    eci[(size_t)i * D + k] = (k < d) ? ci[a + k] : i;
    ekv[(size_t)i * D + k] = (k < d) ? kv[a + k] : pad;
  }
}

// -------- layout conversion: (L x n, l-major, double) -> panel [n][Lp] --------
// mode 0: value; 1: log2(value) (-inf for 0); 2: exp(-value/eps) (state cost -> K_L);
// 3: -value/eps*log2(e) (state cost -> log2 K_L).  Padding columns get padv.
template <typename V>
__global__ void k_to_panel(const double* __restrict__ in, int L, int n, int Lp, int mode, double eps, V padv,
                           V* __restrict__ out) {
  __shared__ double tile[32][33];
  const int i0 = blockIdx.x * 32, l0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int l = l0 + r, i = i0 + tx;
    tile[r][tx] = (l < L && i < n) ? in[(size_t)l * n + i] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + r, l = l0 + tx;
    if (i < n && l < Lp) {
      V v;
      if (l >= L) v = padv;
      else {
        const double x = tile[tx][r];
        switch (mode) {
          case 0: v = static_cast<V>(x); break;
          case 1: v = (x > 0) ? static_cast<V>(log2(x)) : -static_cast<V>(INFINITY); break;
          case 2: v = static_cast<V>(exp(-x / eps)); break;
          default: v = static_cast<V>(-x / eps * M_LOG2E); break;
        }
      }
      out[(size_t)i * Lp + l] = v;
    }
  }
}

// capacity to internal form: (T-1) x n; src either n (broadcast) or (T-1) x n
template <typename V, bool LOG>
__global__ void k_cap(const double* __restrict__ cap, int per_step, int n, int Tm1, V* __restrict__ out) {
  const size_t tot = (size_t)Tm1 * n;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < tot; k += (size_t)gridDim.x * blockDim.x) {
    const double d = per_step ? cap[k] : cap[k % n];
    out[k] = LOG ? static_cast<V>(log2(d)) : static_cast<V>(d);
  }
}

template <typename V>
__global__ void k_fill(V* __restrict__ p, size_t cnt, V v) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < cnt; k += (size_t)gridDim.x * blockDim.x) p[k] = v;
}

// initial sink scaling U0T = 1 on supp(R0T) (0 / -inf elsewhere)
template <typename V, bool LOG>
__global__ void k_init_u0t(const V* __restrict__ rdst, size_t cnt, V* __restrict__ u0t) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < cnt; k += (size_t)gridDim.x * blockDim.x) {
    const V r = rdst[k];
    if (LOG) u0t[k] = (r != -static_cast<V>(INFINITY)) ? V(0) : -static_cast<V>(INFINITY);
    else u0t[k] = (r > V(0)) ? V(1) : V(0);
  }
}

// initial range offsets: c_b[t] = rho_b (t < T), c_b[T] = 0; c_f[0] = 0, c_f[t] = rho_f
__global__ void k_init_offsets(double* cb, double* cf, double* gauge0, double* gaugeT, int T, int Lp,
                               const uint32_t* rho) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= Lp) return;
  const double rb = rho[0] ? (double)dec_f32(rho[0]) : 0.0;
  const double rf = rho[1] ? (double)dec_f32(rho[1]) : 0.0;
  for (int t = 0; t <= T; ++t) {
    cb[(size_t)t * Lp + l] = (t < T) ? rb : 0.0;
    cf[(size_t)t * Lp + l] = (t > 0) ? rf : 0.0;
  }
  gauge0[l] = 0.0;
  gaugeT[l] = 0.0;
}

// log duals out: natural logs in the paper's L x n layout
template <typename V, bool LOG>
__global__ void k_log_duals_panel(const V* __restrict__ pan, const double* __restrict__ sig, int n, int L, int Lp,
                                  double* __restrict__ out) {
  const size_t tot = (size_t)L * n;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < tot; k += (size_t)gridDim.x * blockDim.x) {
    const int l = (int)(k / n), i = (int)(k % n);
    const V x = pan[(size_t)i * Lp + l];
    const double sg = sig ? sig[l] : 0.0;
    double r;
    if (LOG) r = (x == -static_cast<V>(INFINITY)) ? -INFINITY : ((double)x + sg) * M_LN2;
    else r = (x > V(0)) ? (log2((double)x) + sg) * M_LN2 : -INFINITY;
    out[k] = r;
  }
}
template <typename V, bool LOG>
__global__ void k_log_duals_u(const V* __restrict__ u, size_t cnt, double* __restrict__ out) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < cnt; k += (size_t)gridDim.x * blockDim.x)
    out[k] = LOG ? (double)u[k] * M_LN2 : log((double)u[k]);
}
// warm start: per-commodity gauge g = max_i log2 U[l, i]; panel = 2^(log2 U - g)
// (log2 U - g in the log domain).  One block per commodity.
template <typename V, bool LOG>
__global__ void k_set_panel(const double* __restrict__ in, int n, int L, int Lp, V* __restrict__ pan,
                            double* __restrict__ gauge) {
  const int l = blockIdx.x;
  __shared__ double red[256];
  double m = -INFINITY;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, in[(size_t)l * n + i] * M_LOG2E);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double g = isfinite(red[0]) ? red[0] : 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double lv = in[(size_t)l * n + i] * M_LOG2E - g;
    pan[(size_t)i * Lp + l] = LOG ? static_cast<V>(lv) : static_cast<V>(exp2(lv));
  }
  if (threadIdx.x == 0) gauge[l] = g;
}
template <typename V, bool LOG>
__global__ void k_set_u(const double* __restrict__ in, size_t cnt, V* __restrict__ u) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < cnt; k += (size_t)gridDim.x * blockDim.x)
    u[k] = LOG ? static_cast<V>(fmin(in[k], 0.0) * M_LOG2E) : static_cast<V>(exp(fmin(in[k], 0.0)));
}

// commodity-capacity scalings w_t in (0, 1] from natural logs (clamped at 0)
template <typename V, bool LOG>
__global__ void k_set_wpanel(const double* __restrict__ in, int n, int L, int Lp, V* __restrict__ pan) {
  const size_t tot = (size_t)L * n;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < tot; k += (size_t)gridDim.x * blockDim.x) {
    const int l = (int)(k / n), i = (int)(k % n);
    const double x = fmin(in[k], 0.0);
    pan[(size_t)i * Lp + l] = LOG ? static_cast<V>(x * M_LOG2E) : static_cast<V>(exp(x));
  }
}

// range estimate for the domain choice: per row, sum over off-diagonal moves
// of max(C_ij - C_ii, 0) and their count (deterministic per-row values)
__global__ void k_excess_rows(const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ cost,
                              int n, double* __restrict__ rowsum, int* __restrict__ rowcnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double wait = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) if (ci[e] == i) wait = cost[e];
  double s = 0.0; int c = 0;
  // (moves closed at this step, +inf, carry no range)
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (ci[e] != i && isfinite(cost[e])) { s += fmax(cost[e] - wait, 0.0); ++c; }
  rowsum[i] = s; rowcnt[i] = c;
}
__global__ void k_excess_total(const double* __restrict__ rowsum, const int* __restrict__ rowcnt, int n,
                               double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0; long long c = 0;
  for (int i = 0; i < n; ++i) { s += rowsum[i]; c += rowcnt[i]; }
  out[0] = c ? s / (double)c : 0.0;
}

// -------- launchers --------
static inline int gs(size_t cnt) { return (int)((cnt + 255) / 256 > 4096 ? 4096 : (cnt + 255) / 256 ? (cnt + 255) / 256 : 1); }

void launch_max_degree(const int* rp, int n, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_max_degree, dim3((n + 255) / 256), dim3(256), 0, s, rp, n, out);
}
template <typename V>
void launch_build_ell(const int* rp, const int* ci, const V* kv, int n, int D, V pad, int* eci, V* ekv, int* deg,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_build_ell<V>, dim3((n + 255) / 256), dim3(256), 0, s, rp, ci, kv, n, D, pad, eci, ekv, deg);
}
template void launch_build_ell<float>(const int*, const int*, const float*, int, int, float, int*, float*, int*, hipStream_t);
template void launch_build_ell<double>(const int*, const int*, const double*, int, int, double, int*, double*, int*,
                                       hipStream_t);

void launch_validate_vals(const double* x, size_t cnt, int allow_inf, int strictly_pos, int allow_neg, int* flags,
                          hipStream_t s) {
  if (cnt) hipLaunchKernelGGL(k_validate_vals, dim3(gs(cnt)), dim3(256), 0, s, x, cnt, allow_inf, strictly_pos, allow_neg, flags);
}
void launch_validate_csr(const int* rp, const int* ci, int n, long long nnz, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_validate_csr, dim3((n + 1 + 255) / 256), dim3(256), 0, s, rp, ci, n, nnz, flags);
}
void launch_validate_mass(const double* src, const double* dst, int L, int n, int* flags, double* masses,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_validate_mass, dim3(L), dim3(256), 0, s, src, dst, n, flags, masses);
}
template <typename V, bool LOG>
void launch_gibbs(const double* cost, size_t nnz, double eps, V* kv, hipStream_t s) {
  if (nnz) hipLaunchKernelGGL((k_gibbs<V, LOG>), dim3(gs(nnz)), dim3(256), 0, s, cost, nnz, eps, kv);
}
void launch_transpose_pattern(const int* rp, const int* ci, int n, long long nnz, int* cnt, int* rpt, int* cursor,
                              int* cit, int* srcpos, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<int>, dim3(gs(n)), dim3(256), 0, s, cnt, (size_t)n, 0);
  hipLaunchKernelGGL(k_fill<int>, dim3(gs(n)), dim3(256), 0, s, cursor, (size_t)n, 0);
  hipLaunchKernelGGL(k_count_cols, dim3(gs(nnz)), dim3(256), 0, s, ci, nnz, cnt);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, cnt, n, rpt);
  hipLaunchKernelGGL(k_fill_transpose, dim3((n + 255) / 256), dim3(256), 0, s, rp, ci, n, rpt, cursor, cit, srcpos);
  hipLaunchKernelGGL(k_sort_rows, dim3((n + 255) / 256), dim3(256), 0, s, rpt, n, cit, srcpos);
}
template <typename V>
void launch_gather_vals(const V* kv, const int* srcpos, long long nnz, V* kvt, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_vals<V>, dim3(gs(nnz)), dim3(256), 0, s, kv, srcpos, nnz, kvt);
}
template <typename V, bool LOG>
void launch_rowsum_max(const int* rp, const V* kv, int n, double klmax_log2, uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL((k_rowsum_max<V, LOG>), dim3((n + 255) / 256), dim3(256), 0, s, rp, kv, n, klmax_log2, out);
}
template <typename V>
void launch_to_panel(const double* in, int L, int n, int Lp, int mode, double eps, V padv, V* out, hipStream_t s) {
  dim3 grid((n + 31) / 32, (Lp + 31) / 32);
  hipLaunchKernelGGL(k_to_panel<V>, grid, dim3(256), 0, s, in, L, n, Lp, mode, eps, padv, out);
}
template <typename V, bool LOG>
void launch_cap(const double* cap, int per_step, int n, int Tm1, V* out, hipStream_t s) {
  if (Tm1 > 0) hipLaunchKernelGGL((k_cap<V, LOG>), dim3(gs((size_t)Tm1 * n)), dim3(256), 0, s, cap, per_step, n, Tm1, out);
}
template <typename V>
void launch_fill(V* p, size_t cnt, V v, hipStream_t s) {
  if (cnt) hipLaunchKernelGGL(k_fill<V>, dim3(gs(cnt)), dim3(256), 0, s, p, cnt, v);
}
template <typename V, bool LOG>
void launch_init_u0t(const V* rdst, size_t cnt, V* u0t, hipStream_t s) {
  hipLaunchKernelGGL((k_init_u0t<V, LOG>), dim3(gs(cnt)), dim3(256), 0, s, rdst, cnt, u0t);
}
void launch_init_offsets(double* cb, double* cf, double* g0, double* gT, int T, int Lp, const uint32_t* rho,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_init_offsets, dim3((Lp + 255) / 256), dim3(256), 0, s, cb, cf, g0, gT, T, Lp, rho);
}
template <typename V, bool LOG>
void launch_log_duals(const V* u01, const double* sig01, const V* u0t, const double* sig0t, const V* u, int n, int L,
                      int Lp, int Tm1, double* ls, double* ld, double* lc, hipStream_t s) {
  const size_t tot = (size_t)L * n;
  if (ls) hipLaunchKernelGGL((k_log_duals_panel<V, LOG>), dim3(gs(tot)), dim3(256), 0, s, u01, sig01, n, L, Lp, ls);
  if (ld) hipLaunchKernelGGL((k_log_duals_panel<V, LOG>), dim3(gs(tot)), dim3(256), 0, s, u0t, sig0t, n, L, Lp, ld);
  if (lc && Tm1 > 0)
    hipLaunchKernelGGL((k_log_duals_u<V, LOG>), dim3(gs((size_t)Tm1 * n)), dim3(256), 0, s, u, (size_t)Tm1 * n, lc);
}
template <typename V, bool LOG>
void launch_set_duals(const double* ls, const double* ld, const double* lc, int n, int L, int Lp, int Tm1, V* u01,
                      V* u0t, V* u, double* g0, double* gT, hipStream_t s) {
  if (ls) hipLaunchKernelGGL((k_set_panel<V, LOG>), dim3(L), dim3(256), 0, s, ls, n, L, Lp, u01, g0);
  if (ld) hipLaunchKernelGGL((k_set_panel<V, LOG>), dim3(L), dim3(256), 0, s, ld, n, L, Lp, u0t, gT);
  if (lc && Tm1 > 0)
    hipLaunchKernelGGL((k_set_u<V, LOG>), dim3(gs((size_t)Tm1 * n)), dim3(256), 0, s, lc, (size_t)Tm1 * n, u);
}
template <typename V, bool LOG>
void launch_comm_duals(const V* w, int n, int L, int Lp, int Tm1, double* out, int set, const double* in,
                       V* wout, hipStream_t s) {
  const size_t tot = (size_t)L * n;
  for (int t = 0; t < Tm1; ++t) {
    if (set)
      hipLaunchKernelGGL((k_set_wpanel<V, LOG>), dim3(gs(tot)), dim3(256), 0, s, in + (size_t)t * tot, n, L, Lp,
                         wout + (size_t)t * n * Lp);
    else
      hipLaunchKernelGGL((k_log_duals_panel<V, LOG>), dim3(gs(tot)), dim3(256), 0, s, w + (size_t)t * n * Lp,
                         nullptr, n, L, Lp, out + (size_t)t * tot);
  }
}
void launch_excess(const int* rp, const int* ci, const double* cost, int n, double* rowsum, int* rowcnt, double* out,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_excess_rows, dim3((n + 255) / 256), dim3(256), 0, s, rp, ci, cost, n, rowsum, rowcnt);
  hipLaunchKernelGGL(k_excess_total, dim3(1), dim3(64), 0, s, rowsum, rowcnt, n, out);
}

#define MMOT_SETUP_INST(V, LOG)                                                                                    \
  template void launch_gibbs<V, LOG>(const double*, size_t, double, V*, hipStream_t);                            \
  template void launch_rowsum_max<V, LOG>(const int*, const V*, int, double, uint32_t*, hipStream_t);            \
  template void launch_cap<V, LOG>(const double*, int, int, int, V*, hipStream_t);                               \
  template void launch_init_u0t<V, LOG>(const V*, size_t, V*, hipStream_t);                                      \
  template void launch_log_duals<V, LOG>(const V*, const double*, const V*, const double*, const V*, int, int,   \
                                         int, int, double*, double*, double*, hipStream_t);                      \
  template void launch_set_duals<V, LOG>(const double*, const double*, const double*, int, int, int, int, V*,    \
                                         V*, V*, double*, double*, hipStream_t);                                 \
  template void launch_comm_duals<V, LOG>(const V*, int, int, int, int, double*, int, const double*, V*,         \
                                          hipStream_t);
MMOT_SETUP_INST(float, false)
MMOT_SETUP_INST(float, true)
MMOT_SETUP_INST(double, false)
MMOT_SETUP_INST(double, true)
template void launch_gather_vals<float>(const float*, const int*, long long, float*, hipStream_t);
template void launch_gather_vals<double>(const double*, const int*, long long, double*, hipStream_t);
template void launch_to_panel<float>(const double*, int, int, int, int, double, float, float*, hipStream_t);
template void launch_to_panel<double>(const double*, int, int, int, int, double, double, double*, hipStream_t);
template void launch_fill<float>(float*, size_t, float, hipStream_t);
template void launch_fill<double>(double*, size_t, double, hipStream_t);
template void launch_fill<uint32_t>(uint32_t*, size_t, uint32_t, hipStream_t);
template void launch_fill<int>(int*, size_t, int, hipStream_t);

}  // namespace mmot
