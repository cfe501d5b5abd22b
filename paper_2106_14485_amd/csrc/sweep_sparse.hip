// Sparse sweep kernels of the graph-structured multi-commodity Sinkhorn scheme.
//
// One launch = one product of Theorem 5 (eqs. psi_hat / psi) over all
// commodities: out[j, :] = sum_{i in N(j)} K(i -> j) u_tau[i] in[i, :], read as
// a CSR SpMM whose operands are state-major panels (see mmot_internal.h).
// Forward steps fuse the capacity update of Algorithm 2 / Corollary 1
// (u_t = min(d / (hatPsi_t (.) Psi_t (.) K_L)^T 1, 1)) and, at the last time,
// the sink update U^(0,TT) = R^(0,TT) ./ hatPsi_TT into the epilogue.  The
// log domain replaces multiply-add by log-sum-exp (base 2).
//
// Mapping: a "row group" of G lanes (G = 64 when Lp >= 256 floats) owns one
// output state; each lane holds 16 bytes (4 floats / 2 doubles) of the row per
// 64*16-byte chunk.  Neighbour rows are gathered with coalesced 16-byte loads;
// the commodity reduction is a shuffle reduction inside the group.  Four
// wavefronts per block, blocks ordered XCD-contiguously.
#include "mmot_internal.h"
#include <math.h>

namespace mmot {

template <typename V> struct VT;
template <> struct VT<float> { static constexpr int N = 4; };
template <> struct VT<double> { static constexpr int N = 2; };

__device__ __forceinline__ void vld(const float* p, float (&r)[4]) {
  float4 t = *reinterpret_cast<const float4*>(p);
  r[0] = t.x; r[1] = t.y; r[2] = t.z; r[3] = t.w;
}
__device__ __forceinline__ void vld(const double* p, double (&r)[2]) {
  double2 t = *reinterpret_cast<const double2*>(p);
  r[0] = t.x; r[1] = t.y;
}
__device__ __forceinline__ void vst(float* p, const float (&r)[4]) {
  *reinterpret_cast<float4*>(p) = make_float4(r[0], r[1], r[2], r[3]);
}
__device__ __forceinline__ void vst(double* p, const double (&r)[2]) {
  *reinterpret_cast<double2*>(p) = make_double2(r[0], r[1]);
}

template <typename V> __device__ __forceinline__ V ninf() { return -static_cast<V>(INFINITY); }
__device__ __forceinline__ float xexp2(float x) { return exp2f(x); }
__device__ __forceinline__ double xexp2(double x) { return exp2(x); }
__device__ __forceinline__ float xlog2(float x) { return log2f(x); }
__device__ __forceinline__ double xlog2(double x) { return log2(x); }

template <typename V>
__device__ __forceinline__ V shfl_xor(V v, int m) { return __shfl_xor(v, m, 64); }

// sum over the G lanes of a row group (G power of two)
template <typename V>
__device__ __forceinline__ V group_sum(V v, int G) {
  for (int m = G >> 1; m > 0; m >>= 1) v += shfl_xor(v, m);
  return v;
}
// log-sum-exp combine over the group: (m, s) represents s * 2^m
template <typename V>
__device__ __forceinline__ void group_lse(V& m, V& s, int G) {
  for (int k = G >> 1; k > 0; k >>= 1) {
    V om = shfl_xor(m, k), os = shfl_xor(s, k);
    V nm = fmax(m, om);
    V base = (nm == ninf<V>()) ? V(0) : nm;
    s = s * xexp2(m - base) + os * xexp2(om - base);
    m = nm;
  }
}
__device__ __forceinline__ double wave_sum_d(double v) {
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
  for (int m = 32; m > 0; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
  return v;
}

// Block reduction of kNSt doubles (sum, except ST_CAP_VIOL: max) -> part[blk]
__device__ void block_stats(double (&st)[kNSt], double* part, int blk) {
  __shared__ double red[kWaves][kNSt];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kNSt; ++k) {
    double v = (k == ST_CAP_VIOL) ? wave_max_d(st[k]) : wave_sum_d(st[k]);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < kNSt) {
    const int k = threadIdx.x;
    double v = red[0][k];
    for (int w = 1; w < kWaves; ++w) v = (k == ST_CAP_VIOL) ? fmax(v, red[w][k]) : v + red[w][k];
    part[(size_t)blk * kNSt + k] = v;
  }
}

// Column maxima of a chunk of the stored panel -> encoded atomicMax into one
// calibration slot.  cal holds, per lane, the value to calibrate on (the max
// over this lane's rows; identity for invalid lanes).
template <typename V, bool LOG>
__device__ void calib_chunk(const V (&val)[VT<V>::N], int G, int chunk_col0, int Lp, uint32_t* slot) {
  constexpr int NV = VT<V>::N;
  __shared__ float cm[kWaves][64 * 4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gl = lane & (G - 1);
  float c[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    V x = val[v];
    for (int m = G; m < 64; m <<= 1) x = fmax(x, shfl_xor(x, m));
    if (LOG) c[v] = static_cast<float>(x);
    else c[v] = (x > V(0)) ? static_cast<float>(xlog2(x)) : -INFINITY;
  }
  if (lane < G) {
#pragma unroll
    for (int v = 0; v < NV; ++v) cm[wave][gl * NV + v] = c[v];
  }
  __syncthreads();
  const int ncol = G * NV;
  for (int k = threadIdx.x; k < ncol; k += kBlock) {
    float m = cm[0][k];
    for (int w = 1; w < kWaves; ++w) m = fmaxf(m, cm[w][k]);
    const int col = chunk_col0 + k;
    if (col < Lp && m > -INFINITY) atomicMax(slot + col, enc_f32(m));
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// the sweep step
// ---------------------------------------------------------------------------
template <typename V, bool LOG, bool FWD>
__global__ __launch_bounds__(kBlock) void k_step(StepArgs<V> a) {
  constexpr int NV = VT<V>::N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int G = a.G;
  const int grp = lane / G, gl = lane & (G - 1);
  const int rpw = 64 / G;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int row = (lb * kWaves + wave) * rpw + grp;
  const bool valid = row < a.n;
  int e0 = 0, e1 = 0;
  if (valid) { e0 = a.rp[row]; e1 = a.rp[row + 1]; }
  if (G == 64) { e0 = __builtin_amdgcn_readfirstlane(e0); e1 = __builtin_amdgcn_readfirstlane(e1); }
  const size_t Lp = (size_t)a.Lp;

  V ssum = 0;                       // scaled: capacity column sum (lane partial)
  V lm = ninf<V>(), ls = 0;         // log: running LSE of the column sum
  double st[kNSt] = {0, 0, 0, 0, 0, 0, 0, 0};
  double occ_row = 0.0;             // sink / output: occupancy of this row

  for (int ch = 0; ch < a.nchunk; ++ch) {
    const int col = (ch * G + gl) * NV;
    const bool cv = valid && col < a.Lp;
    V o[NV];
    // ---------------- product ----------------
    if (!LOG) {
      V acc[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] = 0;
      if (cv) {
        int e = e0;
        for (; e + 4 <= e1; e += 4) {
          const int i0 = a.ci[e], i1 = a.ci[e + 1], i2 = a.ci[e + 2], i3 = a.ci[e + 3];
          V c0 = a.kv[e], c1 = a.kv[e + 1], c2 = a.kv[e + 2], c3 = a.kv[e + 3];
          if (a.uin) { c0 *= a.uin[i0]; c1 *= a.uin[i1]; c2 *= a.uin[i2]; c3 *= a.uin[i3]; }
          V x0[NV], x1[NV], x2[NV], x3[NV];
          vld(a.xin + i0 * Lp + col, x0);
          vld(a.xin + i1 * Lp + col, x1);
          vld(a.xin + i2 * Lp + col, x2);
          vld(a.xin + i3 * Lp + col, x3);
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            acc[v] = fma(c0, x0[v], acc[v]);
            acc[v] = fma(c1, x1[v], acc[v]);
            acc[v] = fma(c2, x2[v], acc[v]);
            acc[v] = fma(c3, x3[v], acc[v]);
          }
        }
        for (; e < e1; ++e) {
          const int i0 = a.ci[e];
          V c0 = a.kv[e];
          if (a.uin) c0 *= a.uin[i0];
          V x0[NV];
          vld(a.xin + i0 * Lp + col, x0);
#pragma unroll
          for (int v = 0; v < NV; ++v) acc[v] = fma(c0, x0[v], acc[v]);
        }
        V f[NV];
        vld(a.fac + col, f);
#pragma unroll
        for (int v = 0; v < NV; ++v) o[v] = acc[v] * f[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) o[v] = 0;
      }
    } else {
      V m[NV], s[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) { m[v] = ninf<V>(); s[v] = 0; }
      if (cv) {
        int e = e0;
        for (; e + 4 <= e1; e += 4) {
          const int i0 = a.ci[e], i1 = a.ci[e + 1], i2 = a.ci[e + 2], i3 = a.ci[e + 3];
          V c0 = a.kv[e], c1 = a.kv[e + 1], c2 = a.kv[e + 2], c3 = a.kv[e + 3];
          if (a.uin) { c0 += a.uin[i0]; c1 += a.uin[i1]; c2 += a.uin[i2]; c3 += a.uin[i3]; }
          V x0[NV], x1[NV], x2[NV], x3[NV];
          vld(a.xin + i0 * Lp + col, x0);
          vld(a.xin + i1 * Lp + col, x1);
          vld(a.xin + i2 * Lp + col, x2);
          vld(a.xin + i3 * Lp + col, x3);
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const V y0 = c0 + x0[v], y1 = c1 + x1[v], y2 = c2 + x2[v], y3 = c3 + x3[v];
            const V nm = fmax(m[v], fmax(fmax(y0, y1), fmax(y2, y3)));
            const V b = (nm == ninf<V>()) ? V(0) : nm;
            s[v] = s[v] * xexp2(m[v] - b) + xexp2(y0 - b) + xexp2(y1 - b) + xexp2(y2 - b) + xexp2(y3 - b);
            m[v] = nm;
          }
        }
        for (; e < e1; ++e) {
          const int i0 = a.ci[e];
          V c0 = a.kv[e];
          if (a.uin) c0 += a.uin[i0];
          V x0[NV];
          vld(a.xin + i0 * Lp + col, x0);
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const V y0 = c0 + x0[v];
            const V nm = fmax(m[v], y0);
            const V b = (nm == ninf<V>()) ? V(0) : nm;
            s[v] = s[v] * xexp2(m[v] - b) + xexp2(y0 - b);
            m[v] = nm;
          }
        }
        V f[NV];
        vld(a.fac + col, f);
#pragma unroll
        for (int v = 0; v < NV; ++v) o[v] = (s[v] > V(0)) ? m[v] + xlog2(s[v]) + f[v] : ninf<V>();
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) o[v] = ninf<V>();
      }
    }

    // ---------------- epilogue ----------------
    V z[NV];   // value stored into the output panel (and calibrated on)
    if (FWD && a.epi == 2) {
      // sink: U0T = R0T ./ hatPsi_T (Algorithm 2), zero off the support
      if (cv) {
        V r[NV], f[NV], cur[NV];
        vld(a.rdst + row * Lp + col, r);
        vld(a.facT + col, f);
        if (a.update) {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            if (!LOG) {
              if (r[v] > V(0)) {
                if (!(o[v] > V(0))) atomicOr(a.flags, FLAG_INFEASIBLE);
                z[v] = r[v] / o[v] * f[v];
              } else z[v] = 0;
            } else {
              if (r[v] != ninf<V>()) {
                if (o[v] == ninf<V>()) atomicOr(a.flags, FLAG_INFEASIBLE);
                z[v] = r[v] - o[v] + f[v];
              } else z[v] = ninf<V>();
            }
          }
          vst(a.u0t + row * Lp + col, z);
        } else {
          vld(a.u0t + row * Lp + col, cur);
#pragma unroll
          for (int v = 0; v < NV; ++v) z[v] = cur[v];
        }
        if (a.part || a.occ || a.pcomm) {
          // P_{0,T} = U0T (.) hatPsi_T, the sink marginal of the current plan
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const int l = col + v;
            if (l >= a.L) continue;
            const double sg = a.sigT[l] + a.sighT[l];
            double P, lnU, R;
            if (!LOG) {
              P = (double)z[v] * (double)o[v] * exp2(sg);
              lnU = (z[v] > V(0)) ? (log2((double)z[v]) + a.sigT[l]) * M_LN2 : 0.0;
              R = (double)r[v];
            } else {
              P = (z[v] == ninf<V>() || o[v] == ninf<V>()) ? 0.0 : exp2((double)z[v] + (double)o[v] + sg);
              lnU = (z[v] != ninf<V>()) ? ((double)z[v] + a.sigT[l]) * M_LN2 : 0.0;
              R = (r[v] == ninf<V>()) ? 0.0 : exp2((double)r[v]);
            }
            st[ST_MASS] += P;
            st[ST_DUAL] += R * lnU;
            st[ST_GAP] += lnU * (P - R);
            occ_row += P;
            if (a.pcomm) a.pcomm[(size_t)l * a.n + row] = P;
          }
        }
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) z[v] = LOG ? ninf<V>() : V(0);
      }
    } else {
      if (FWD && cv && a.epi == 1) {
        V w[NV], g[NV];
        vld(a.wpan + row * Lp + col, w);
        vld(a.wgt + col, g);
        if (!LOG) {
#pragma unroll
          for (int v = 0; v < NV; ++v) ssum = fma(o[v] * w[v], g[v], ssum);
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const V y = o[v] + w[v] + g[v];
            const V nm = fmax(lm, y);
            const V b = (nm == ninf<V>()) ? V(0) : nm;
            ls = ls * xexp2(lm - b) + xexp2(y - b);
            lm = nm;
          }
        }
        if (a.pcomm) {
          // output pass: u is final, P_{0,t} = hatPsi (.) Psi (.) K_L u_t (eq. proj_0t)
          const V ur = a.uout[row];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const int l = col + v;
            if (l >= a.L) continue;
            double P = LOG ? ((o[v] == ninf<V>() || w[v] == ninf<V>()) ? 0.0
                                : exp2((double)o[v] + (double)w[v] + (double)g[v] + (double)ur))
                           : (double)o[v] * (double)w[v] * (double)g[v] * (double)ur;
            a.pcomm[(size_t)l * a.n + row] = P;
          }
        }
      }
      if (cv && a.kl) {
        V k[NV];
        vld(a.kl + row * Lp + col, k);
#pragma unroll
        for (int v = 0; v < NV; ++v) z[v] = LOG ? o[v] + k[v] : o[v] * k[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) z[v] = o[v];
      }
      if (cv && a.out) vst(a.out + row * Lp + col, z);
      if (!cv) {
#pragma unroll
        for (int v = 0; v < NV; ++v) z[v] = LOG ? ninf<V>() : V(0);
      }
    }
    if (a.slots) calib_chunk<V, LOG>(z, G, ch * G * NV, a.Lp, a.slots + (size_t)(blockIdx.x % a.nslot) * a.nslot_stride);
  }

  // ---------------- capacity update (Corollary 1 + Proposition 1) ----------------
  if (FWD && a.epi == 1) {
    V sv;
    if (!LOG) sv = group_sum(ssum, G);
    else { group_lse(lm, ls, G); sv = (ls > V(0)) ? lm + xlog2(ls) : ninf<V>(); }
    if (valid && gl == 0) {
      const V d = a.cap[row];
      V u;
      if (a.update) {
        if (!LOG) u = (sv <= d) ? V(1) : d / sv;
        else u = fmin(V(0), d - sv);
        a.uout[row] = u;
      } else {
        u = a.uout[row];
      }
      if (a.part || a.occ) {
        double occ, dd, lnu;
        if (!LOG) { occ = (double)u * (double)sv; dd = (double)d; lnu = log((double)u); }
        else {
          occ = (sv == ninf<V>()) ? 0.0 : exp2((double)u + (double)sv);
          dd = exp2((double)d); lnu = (double)u * M_LN2;
        }
        st[ST_MASS] += occ;
        if (isfinite(dd)) {
          st[ST_CAP_VIOL] = fmax(st[ST_CAP_VIOL], fmax(occ - dd, 0.0) / dd);
          st[ST_DUAL] += dd * lnu;
          st[ST_GAP] += lnu * (occ - dd);
        }
        if (!isfinite(occ)) st[ST_NONFINITE] += 1.0;
        if (a.occ) a.occ[row] = occ;
      }
    }
  }
  if (FWD && a.epi == 2 && (a.part || a.occ)) {
    // gather the row's occupancy across the group lanes for the output
    double t = occ_row;
    for (int m = G >> 1; m > 0; m >>= 1) t += __shfl_xor(t, m, 64);
    if (valid && gl == 0 && a.occ) a.occ[row] = t;
  }
  if (FWD && a.part) block_stats(st, a.part, blockIdx.x);
}

// ---------------------------------------------------------------------------
// source update: U01 = R01 ./ Psi_1 (Algorithm 2), stored scaled by fac
// ---------------------------------------------------------------------------
template <typename V, bool LOG>
__global__ __launch_bounds__(kBlock) void k_source(int n, int Lp, int G, int nchunk, const V* __restrict__ psi0,
                                                   const V* __restrict__ rsrc, const V* __restrict__ fac,
                                                   V* __restrict__ u01, uint32_t* slots, int nslot,
                                                   size_t slot_stride, int* flags) {
  constexpr int NV = VT<V>::N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / G, gl = lane & (G - 1);
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int row = (lb * kWaves + wave) * (64 / G) + grp;
  const bool valid = row < n;
  for (int ch = 0; ch < nchunk; ++ch) {
    const int col = (ch * G + gl) * NV;
    const bool cv = valid && col < Lp;
    V z[NV];
    if (cv) {
      V x[NV], r[NV], f[NV];
      vld(psi0 + (size_t)row * Lp + col, x);
      vld(rsrc + (size_t)row * Lp + col, r);
      vld(fac + col, f);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (!LOG) {
          if (r[v] > V(0)) {
            if (!(x[v] > V(0))) atomicOr(flags, FLAG_INFEASIBLE);
            z[v] = r[v] / x[v] * f[v];
          } else z[v] = 0;
        } else {
          if (r[v] != ninf<V>()) {
            if (x[v] == ninf<V>()) atomicOr(flags, FLAG_INFEASIBLE);
            z[v] = r[v] - x[v] + f[v];
          } else z[v] = ninf<V>();
        }
      }
      vst(u01 + (size_t)row * Lp + col, z);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) z[v] = LOG ? ninf<V>() : V(0);
    }
    if (slots) calib_chunk<V, LOG>(z, G, ch * G * NV, Lp, slots + (size_t)(blockIdx.x % nslot) * slot_stride);
  }
}

// ---------------------------------------------------------------------------
// statistics at time 0: P_{0,1} = U01 (.) Psi_1 against R01 (check / output pass)
// ---------------------------------------------------------------------------
template <typename V, bool LOG>
__global__ __launch_bounds__(kBlock) void k_check0(int n, int Lp, int L, int G, int nchunk, const V* __restrict__ psi0,
                                                   const V* __restrict__ u01, const V* __restrict__ rsrc,
                                                   const double* __restrict__ sigf0, const double* __restrict__ sigb0,
                                                   double* part, double* occ, double* pcomm) {
  constexpr int NV = VT<V>::N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / G, gl = lane & (G - 1);
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int row = (lb * kWaves + wave) * (64 / G) + grp;
  const bool valid = row < n;
  double st[kNSt] = {0, 0, 0, 0, 0, 0, 0, 0};
  double occ_row = 0.0;
  for (int ch = 0; ch < nchunk; ++ch) {
    const int col = (ch * G + gl) * NV;
    if (!(valid && col < Lp)) continue;
    V x[NV], u[NV], r[NV];
    vld(psi0 + (size_t)row * Lp + col, x);
    vld(u01 + (size_t)row * Lp + col, u);
    vld(rsrc + (size_t)row * Lp + col, r);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int l = col + v;
      if (l >= L) continue;
      const double sg = sigf0[l] + sigb0[l];
      double P, lnU, R;
      if (!LOG) {
        P = (double)u[v] * (double)x[v] * exp2(sg);
        lnU = (u[v] > V(0)) ? (log2((double)u[v]) + sigf0[l]) * M_LN2 : 0.0;
        R = (double)r[v];
      } else {
        P = (u[v] == ninf<V>() || x[v] == ninf<V>()) ? 0.0 : exp2((double)u[v] + (double)x[v] + sg);
        lnU = (u[v] != ninf<V>()) ? ((double)u[v] + sigf0[l]) * M_LN2 : 0.0;
        R = (r[v] == ninf<V>()) ? 0.0 : exp2((double)r[v]);
      }
      st[ST_SRC_ABS] += fabs(P - R);
      st[ST_SRC_MASS] += R;
      st[ST_MASS] += P;
      st[ST_DUAL] += R * lnU;
      st[ST_GAP] += lnU * (P - R);
      if (!isfinite(P)) st[ST_NONFINITE] += 1.0;
      occ_row += P;
      if (pcomm) pcomm[(size_t)l * n + row] = P;
    }
  }
  if (occ) {
    double t = occ_row;
    for (int m = G >> 1; m > 0; m >>= 1) t += __shfl_xor(t, m, 64);
    if (valid && gl == 0) occ[row] = t;
  }
  if (part) block_stats(st, part, blockIdx.x);
}

// ---------------------------------------------------------------------------
// aggregate edge flows (SDDMM) between times t and t+1 on the CSR of K:
//   F[e = (i -> j)] = K_ij u_t[i] u_{t+1}[j] sum_l A[i, l] B[j, l] 2^(sigma_hat_t + sigma_{t+1})
// with A = hatPsi_t (.) K_L (U01 at t = 0) and B = Psi_{t+1} (.) K_L (U0T at T).
// Also accumulates sum_e C_e F[e] into part (transport cost).
// ---------------------------------------------------------------------------
template <typename V, bool LOG>
__global__ __launch_bounds__(kBlock) void k_flows(int n, int Lp, int L, int G, int nchunk, const int* __restrict__ rp,
                                                  const int* __restrict__ ci, const V* __restrict__ kv,
                                                  const double* __restrict__ cost, const V* __restrict__ A,
                                                  const V* __restrict__ ua, const V* __restrict__ B,
                                                  const V* __restrict__ ub, const double* __restrict__ siga,
                                                  const double* __restrict__ sigb, double* __restrict__ flow,
                                                  double* part) {
  constexpr int NV = VT<V>::N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / G, gl = lane & (G - 1);
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int row = (lb * kWaves + wave) * (64 / G) + grp;
  const bool valid = row < n;
  double st[kNSt] = {0, 0, 0, 0, 0, 0, 0, 0};
  int e0 = 0, e1 = 0;
  if (valid) { e0 = rp[row]; e1 = rp[row + 1]; }
  // all lanes of a group walk the same edges; groups of a wave may have different counts
  int emax = e1 - e0;
  for (int m = 32; m > 0; m >>= 1) emax = max(emax, __shfl_xor(emax, m, 64));
  const size_t Lpz = (size_t)Lp;
  for (int k = 0; k < emax; ++k) {
    const int e = e0 + k;
    const bool ev = valid && e < e1;
    const int j = ev ? ci[e] : 0;
    double acc = 0.0;
    double lm = -INFINITY, ls = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) {
      const int col = (ch * G + gl) * NV;
      if (!(ev && col < Lp)) continue;
      V x[NV], y[NV];
      vld(A + row * Lpz + col, x);
      vld(B + (size_t)j * Lpz + col, y);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int l = col + v;
        if (l >= L) continue;
        const double sg = siga[l] + sigb[l];
        if (!LOG) acc += (double)x[v] * (double)y[v] * exp2(sg);
        else if (x[v] != ninf<V>() && y[v] != ninf<V>()) {
          const double t = (double)x[v] + (double)y[v] + sg;
          const double nm = fmax(lm, t);
          ls = ls * exp2(lm - nm) + 1.0 * exp2(t - nm);
          lm = nm;
        }
      }
    }
    double val;
    if (!LOG) {
      val = acc;
      for (int m = G >> 1; m > 0; m >>= 1) val += __shfl_xor(val, m, 64);
    } else {
      for (int m = G >> 1; m > 0; m >>= 1) {
        const double om = __shfl_xor(lm, m, 64), os = __shfl_xor(ls, m, 64);
        const double nm = fmax(lm, om);
        const double b = (nm == -INFINITY) ? 0.0 : nm;
        ls = ls * exp2(lm - b) + os * exp2(om - b);
        lm = nm;
      }
      val = 0.0;
    }
    if (ev) {
      double F;
      if (!LOG) {
        F = (double)kv[e] * (ua ? (double)ua[row] : 1.0) * (ub ? (double)ub[j] : 1.0) * val;
      } else {
        const double lg = (double)kv[e] + (ua ? (double)ua[row] : 0.0) + (ub ? (double)ub[j] : 0.0) + lm;
        F = (ls > 0.0) ? ls * exp2(lg) : 0.0;
      }
      if (gl == 0) {
        flow[e] = F;
        st[0] += cost[e] * F;
      }
    }
  }
  if (part) block_stats(st, part, blockIdx.x);
}

// ---------------------------------------------------------------------------
// range-offset bookkeeping (one thread per commodity column)
// ---------------------------------------------------------------------------
// c[t][l] += max over calibration slots (log2 of the column max of the stored
// panel), slots cleared.  Thread per (t, l).
__global__ void k_consume(uint32_t* slots, double* c, int T1, int Lp, int nslot) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= T1 * Lp) return;
  float m = -INFINITY;
  for (int p = 0; p < nslot; ++p) {
    uint32_t* s = slots + (size_t)p * T1 * Lp + idx;
    const uint32_t e = *s;
    if (e) m = fmaxf(m, dec_f32(e));
    *s = 0u;
  }
  if (m > -INFINITY && isfinite(m)) c[idx] += (double)m;
}

template <typename V, bool LOG>
__device__ __forceinline__ V to_fac(double c) {
  return LOG ? static_cast<V>(-c) : static_cast<V>(exp2(-c));
}
template <typename V, bool LOG>
__device__ __forceinline__ V to_wgt(double s) {
  return LOG ? static_cast<V>(s) : static_cast<V>(exp2(s));
}

// Backward-sweep offsets: sigma_b[T] = gauge of U0T, sigma_b[t] = sigma_b[t+1] + c_b[t].
template <typename V, bool LOG>
__global__ void k_prep_bwd(int T, int Lp, const double* __restrict__ cb, double* __restrict__ sigb,
                           V* __restrict__ facb, const double* __restrict__ gaugeT) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= Lp) return;
  double s = gaugeT[l];
  sigb[(size_t)T * Lp + l] = s;
  facb[(size_t)T * Lp + l] = to_fac<V, LOG>(cb[(size_t)T * Lp + l]);
  for (int t = T - 1; t >= 0; --t) {
    const double c = cb[(size_t)t * Lp + l];
    s += c;
    sigb[(size_t)t * Lp + l] = s;
    facb[(size_t)t * Lp + l] = to_fac<V, LOG>(c);
  }
}

// Forward-sweep offsets.  mode 0 (Sinkhorn sweep): the source update writes a
// new U01 panel, sigma_hat_0 = c_f[0] - sigma_b[0]; mode 1 (check / output
// pass): U01 is kept, sigma_hat_0 = gauge0.  Then sigma_hat_t = sigma_hat_{t-1}
// + c_f[t]; weights wgt[t] = 2^(sigma_hat_t + sigma_b[t]); in mode 0 the gauge
// of the U0T panel the sink update will write is c_b[T] - sigma_hat_T.
template <typename V, bool LOG>
__global__ void k_prep_fwd(int T, int Lp, int mode, const double* __restrict__ cf, const double* __restrict__ cb,
                           double* __restrict__ sigf, const double* __restrict__ sigb, V* __restrict__ facf,
                           V* __restrict__ wgt, double* __restrict__ gauge0, double* __restrict__ gaugeT) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= Lp) return;
  double s = (mode == 0) ? cf[l] - sigb[l] : gauge0[l];
  if (mode == 0) gauge0[l] = s;
  sigf[l] = s;
  facf[l] = to_fac<V, LOG>(cf[l]);
  wgt[l] = to_wgt<V, LOG>(s + sigb[l]);
  for (int t = 1; t <= T; ++t) {
    const double c = cf[(size_t)t * Lp + l];
    s += c;
    sigf[(size_t)t * Lp + l] = s;
    facf[(size_t)t * Lp + l] = to_fac<V, LOG>(c);
    wgt[(size_t)t * Lp + l] = to_wgt<V, LOG>(s + sigb[(size_t)t * Lp + l]);
  }
  if (mode == 0) gaugeT[l] = cb[(size_t)T * Lp + l] - s;
}

// ---------------------------------------------------------------------------
// deterministic two-stage reduction of the stats partials
// ---------------------------------------------------------------------------
// stage 1: one block per time slot, sums its nblk partials in block order
__global__ void k_reduce_stats1(const double* __restrict__ part, int nblk, double* __restrict__ tpart) {
  const int t = blockIdx.x;
  const double* p = part + (size_t)t * nblk * kNSt;
  __shared__ double red[kBlock][kNSt];
  double acc[kNSt] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblk; b += kBlock) {
#pragma unroll
    for (int k = 0; k < kNSt; ++k) {
      const double v = p[(size_t)b * kNSt + k];
      acc[k] = (k == ST_CAP_VIOL) ? fmax(acc[k], v) : acc[k] + v;
    }
  }
#pragma unroll
  for (int k = 0; k < kNSt; ++k) red[threadIdx.x][k] = acc[k];
  __syncthreads();
  if (threadIdx.x < kNSt) {
    const int k = threadIdx.x;
    double v = red[0][k];
    for (int i = 1; i < kBlock; ++i) v = (k == ST_CAP_VIOL) ? fmax(v, red[i][k]) : v + red[i][k];
    tpart[(size_t)t * kNSt + k] = v;
  }
}

// stage 2: combine the T+1 time slots into the stats record
//   out[0] dual_obj, [1] src_resid, [2] cap_viol, [3] mass_drift, [4] dual_gap, [5] mass, [6] nonfinite
__global__ void k_reduce_stats2(const double* __restrict__ tpart, int T1, double eps, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double dual = 0, gap = 0, viol = 0, nonfin = 0;
  for (int t = 0; t < T1; ++t) {
    const double* p = tpart + (size_t)t * kNSt;
    dual += p[ST_DUAL];
    gap += p[ST_GAP];
    viol = fmax(viol, p[ST_CAP_VIOL]);
    nonfin += p[ST_NONFINITE];
  }
  const double massT = tpart[(size_t)(T1 - 1) * kNSt + ST_MASS];
  double drift = 0;
  for (int t = 0; t < T1; ++t) drift = fmax(drift, fabs(tpart[(size_t)t * kNSt + ST_MASS] - massT));
  out[0] = eps * dual - eps * massT;
  out[1] = tpart[ST_SRC_ABS] / fmax(tpart[ST_SRC_MASS], 1e-300);
  out[2] = viol;
  out[3] = drift / fmax(massT, 1e-300);
  out[4] = eps * gap;
  out[5] = massT;
  out[6] = nonfin;
}

// transport cost = sum of the flow-kernel partials (stage-1 output of T slots)
__global__ void k_reduce_cost(const double* __restrict__ tpart, int T, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0;
  for (int t = 0; t < T; ++t) s += tpart[(size_t)t * kNSt];
  out[0] = s;
}

// ---------------------------------------------------------------------------
// host-side launchers (explicit instantiations)
// ---------------------------------------------------------------------------
template <typename V, bool LOG>
void launch_step(const StepArgs<V>& a, int fwd, int nblk, hipStream_t s) {
  if (fwd) hipLaunchKernelGGL((k_step<V, LOG, true>), dim3(nblk), dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((k_step<V, LOG, false>), dim3(nblk), dim3(kBlock), 0, s, a);
}
template <typename V, bool LOG>
void launch_source(int n, int Lp, int G, int nchunk, const V* psi0, const V* rsrc, const V* fac, V* u01,
                   uint32_t* slots, int nslot, size_t slot_stride, int* flags, int nblk, hipStream_t s) {
  hipLaunchKernelGGL((k_source<V, LOG>), dim3(nblk), dim3(kBlock), 0, s, n, Lp, G, nchunk, psi0, rsrc, fac, u01,
                     slots, nslot, slot_stride, flags);
}
template <typename V, bool LOG>
void launch_check0(int n, int Lp, int L, int G, int nchunk, const V* psi0, const V* u01, const V* rsrc,
                   const double* sigf0, const double* sigb0, double* part, double* occ, double* pcomm, int nblk,
                   hipStream_t s) {
  hipLaunchKernelGGL((k_check0<V, LOG>), dim3(nblk), dim3(kBlock), 0, s, n, Lp, L, G, nchunk, psi0, u01, rsrc,
                     sigf0, sigb0, part, occ, pcomm);
}
template <typename V, bool LOG>
void launch_flows(int n, int Lp, int L, int G, int nchunk, const int* rp, const int* ci, const V* kv,
                  const double* cost, const V* A, const V* ua, const V* B, const V* ub, const double* siga,
                  const double* sigb, double* flow, double* part, int nblk, hipStream_t s) {
  hipLaunchKernelGGL((k_flows<V, LOG>), dim3(nblk), dim3(kBlock), 0, s, n, Lp, L, G, nchunk, rp, ci, kv, cost, A,
                     ua, B, ub, siga, sigb, flow, part);
}
template <typename V, bool LOG>
void launch_prep_bwd(int T, int Lp, const double* cb, double* sigb, V* facb, const double* gaugeT, hipStream_t s) {
  hipLaunchKernelGGL((k_prep_bwd<V, LOG>), dim3((Lp + 255) / 256), dim3(256), 0, s, T, Lp, cb, sigb, facb, gaugeT);
}
template <typename V, bool LOG>
void launch_prep_fwd(int T, int Lp, int mode, const double* cf, const double* cb, double* sigf, const double* sigb,
                     V* facf, V* wgt, double* gauge0, double* gaugeT, hipStream_t s) {
  hipLaunchKernelGGL((k_prep_fwd<V, LOG>), dim3((Lp + 255) / 256), dim3(256), 0, s, T, Lp, mode, cf, cb, sigf,
                     sigb, facf, wgt, gauge0, gaugeT);
}
void launch_consume(uint32_t* slots, double* c, int T1, int Lp, int nslot, hipStream_t s) {
  const int tot = T1 * Lp;
  hipLaunchKernelGGL(k_consume, dim3((tot + 255) / 256), dim3(256), 0, s, slots, c, T1, Lp, nslot);
}
void launch_reduce_stats(const double* part, int nblk, int T1, double* tpart, double eps, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_stats1, dim3(T1), dim3(kBlock), 0, s, part, nblk, tpart);
  hipLaunchKernelGGL(k_reduce_stats2, dim3(1), dim3(64), 0, s, tpart, T1, eps, out);
}
void launch_reduce_cost(const double* part, int nblk, int T, double* tpart, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_stats1, dim3(T), dim3(kBlock), 0, s, part, nblk, tpart);
  hipLaunchKernelGGL(k_reduce_cost, dim3(1), dim3(64), 0, s, tpart, T, out);
}

#define MMOT_INST(V, LOG)                                                                                         \
  template void launch_step<V, LOG>(const StepArgs<V>&, int, int, hipStream_t);                                       \
  template void launch_source<V, LOG>(int, int, int, int, const V*, const V*, const V*, V*, uint32_t*, int,      \
                                      size_t, int*, int, hipStream_t);                                            \
  template void launch_check0<V, LOG>(int, int, int, int, int, const V*, const V*, const V*, const double*,      \
                                      const double*, double*, double*, double*, int, hipStream_t);               \
  template void launch_flows<V, LOG>(int, int, int, int, int, const int*, const int*, const V*, const double*,   \
                                     const V*, const V*, const V*, const V*, const double*, const double*,       \
                                     double*, double*, int, hipStream_t);                                        \
  template void launch_prep_bwd<V, LOG>(int, int, const double*, double*, V*, const double*, hipStream_t);       \
  template void launch_prep_fwd<V, LOG>(int, int, int, const double*, const double*, double*, const double*, V*, \
                                        V*, double*, double*, hipStream_t);
MMOT_INST(float, false)
MMOT_INST(float, true)
MMOT_INST(double, false)
MMOT_INST(double, true)

}  // namespace mmot
