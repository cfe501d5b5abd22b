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
// 64*16-byte chunk.  Neighbour rows are gathered with coalesced 16-byte loads in
// batches (an ELL row is exactly one batch of 4, 5, 8 or 16, loaded once per row; CSR
// rows take batches of 16); the commodity reduction is a shuffle reduction inside
// the group.  Four wavefronts per block, blocks ordered XCD-contiguously.
#include "mmot_internal.h"

#include <type_traits>
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
__device__ __forceinline__ float xlog2(float x) { return log2f(x); }
__device__ __forceinline__ double xlog2(double x) { return log2(x); }
// log-sum-exp terms: exp2 of an argument <= 0 (or -inf) added to a sum that holds
// a unit term, and log2 of such a sum (>= 1).  In single precision these are the
// bare v_exp_f32 / v_log_f32: the library versions differ only by the scaling that
// makes results below 2^-126 denormal instead of 0 (and accepts denormal inputs),
// which cannot change a sum of at least 1.
__device__ __forceinline__ float lexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double lexp2(double x) { return exp2(x); }
__device__ __forceinline__ float llog2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ double llog2(double x) { return log2(x); }

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
    s = s * lexp2(m - base) + os * lexp2(om - base);
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
// over this lane's rows; identity for invalid lanes).  Chunk index: the block's
// waves are in 2^lw sets (wave w in set w mod 2^lw); at loop step `it` set b
// holds column chunk it * 2^lw + b of its rows, so the maxima are taken over
// the waves of one set.
template <typename V, bool LOG>
__device__ void calib_chunk(const V (&val)[VT<V>::N], int G, int it, int lw, int Lp, uint32_t* slot) {
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
  for (int k = threadIdx.x; k < (ncol << lw); k += kBlock) {
    const int b = k / ncol, kk = k - b * ncol;
    float m = cm[b][kk];
    for (int w = b + (1 << lw); w < kWaves; w += 1 << lw) m = fmaxf(m, cm[w][kk]);
    const int col = ((it << lw) + b) * ncol + kk;
    if (col < Lp && m > -INFINITY) atomicMax(slot + col, enc_f32(m));
  }
  __syncthreads();
}

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long x, int m) {
  const unsigned hi = __shfl_xor((unsigned)(x >> 32), m, 64), lo = __shfl_xor((unsigned)x, m, 64);
  return ((unsigned long long)hi << 32) | lo;
}

// Log domain calibration: per column of the chunk, the key (plan level, value)
// maximised over this block's rows, then atomicMax into the slot, so the slot
// keeps the stored value at the state where the plan peaks.  Entries with a
// non-finite plan level or value are skipped.
template <typename V>
__device__ void corr_chunk(const V (&pl)[VT<V>::N], const V (&val)[VT<V>::N], int G, int it, int lw, int Lp,
                           unsigned long long* slot) {
  constexpr int NV = VT<V>::N;
  __shared__ unsigned long long ck[kWaves][64 * 4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gl = lane & (G - 1);
  unsigned long long kk[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const float p = static_cast<float>(pl[v]), x = static_cast<float>(val[v]);
    unsigned long long key =
        (isfinite(p) && isfinite(x)) ? (((unsigned long long)enc_f32(p) << 32) | enc_f32(x)) : 0ull;
    for (int m = G; m < 64; m <<= 1) {
      const unsigned long long y = shfl_xor_u64(key, m);
      key = y > key ? y : key;
    }
    kk[v] = key;
  }
  if (lane < G) {
#pragma unroll
    for (int v = 0; v < NV; ++v) ck[wave][gl * NV + v] = kk[v];
  }
  __syncthreads();
  const int ncol = G * NV;
  for (int k = threadIdx.x; k < (ncol << lw); k += kBlock) {
    const int b = k / ncol, kk = k - b * ncol;
    unsigned long long m = ck[b][kk];
    for (int w = b + (1 << lw); w < kWaves; w += 1 << lw) m = ck[w][kk] > m ? ck[w][kk] : m;
    const int col = ((it << lw) + b) * ncol + kk;
    if (col < Lp && m) atomicMax(slot + col, m);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// the sweep step
// ---------------------------------------------------------------------------
// KB: neighbours gathered per batch (ELL rows are padded to a multiple of it);
// CM: commodity capacities at the output time (a.cw set; CSR operators only)
template <typename V, bool LOG, bool FWD, bool CHK, bool ELL, int KB, bool CM>
__device__ __forceinline__ void step_body(const StepArgs<V>& a, int bid, int nblk) {

  constexpr int NV = VT<V>::N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int G = a.G;
  const int grp = lane / G, gl = lane & (G - 1);
  const int rpw = 64 / G;
  const int lb = xcd_block(bid, nblk);
  // 2^lw waves share a whole-wave row (lw = 0 when G < 64): wave w works on the
  // row's column chunks congruent to w mod 2^lw, so that a step with few rows
  // of many chunks still launches enough short waves to keep every SIMD busy
  const int lw = a.lwpr;
  const int rslot = wave >> lw, sub = wave & ((1 << lw) - 1);
  const int row = ((lb * kWaves >> lw) + rslot) * rpw + grp;
  const bool valid = row < a.n;
  constexpr bool ell = ELL;
  // CSR batches need the row start at once (wave-uniform for whole-wave rows);
  // ELL rows start at a fixed offset and are exactly one (padded) batch.
  const int rowc = valid ? row : 0;
  int e0 = 0, endv = 0;
  if (ELL) {
    e0 = rowc * a.ellD;
  } else {
    e0 = a.rp[rowc];
    endv = a.rp[rowc + 1];
    if (G == 64) { e0 = __builtin_amdgcn_readfirstlane(e0); endv = __builtin_amdgcn_readfirstlane(endv); }
  }

  // ELL rows are exactly one batch of KB entries (padded with the own index and a
  // zero coefficient), the same for every column chunk of the row: their entries
  // and the u values at the neighbours are loaded once per row
  int eidx[ELL ? KB : 1];
  V ecf[ELL ? KB : 1], euu[ELL ? KB : 1];
  if constexpr (ELL) {
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      eidx[k] = a.ci[e0 + k];
      ecf[k] = a.kv[e0 + k];
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) euu[k] = a.uin[eidx[k]];
  }
  auto row_end = [&]() -> int { return !valid ? e0 : endv; };
  const size_t Lp = (size_t)a.Lp;

  V ssum = 0;                       // scaled: capacity column sum (lane partial)
  V lm = ninf<V>(), ls = 0;         // log: running LSE of the column sum
  double st[kNSt] = {0, 0, 0, 0, 0, 0, 0, 0};
  double occ_row = 0.0;             // sink / output: occupancy of this row
  // commodity capacities: w_t, projected before u_t with the u_t of the last sweep
  constexpr bool comm = CM;
  // (the update-free pass reads u only where it outputs per-commodity terms, below:
  // a load here would be waited for with everything issued before it)
  V ucur = LOG ? V(0) : V(1);
  if (FWD && a.epi == 1 && comm) ucur = a.uout[rowc];

  // (the same trip count for every wave of the block: the calibration steps hold barriers)
  const int nit = (a.nchunk + (1 << lw) - 1) >> lw;
  for (int it = 0; it < nit; ++it) {
    const int ch = (it << lw) + sub;
    const int col = (ch * G + gl) * NV;
    const bool cv = valid && col < a.Lp;
    V o[NV];
    // operands of the epilogue that do not depend on the product (unconditional
    // loads at clamped addresses).  The backward panel row W is read from HBM:
    // it is requested after the first batch's gathers, so that it is in flight
    // with them while the waits for the (cached) operator entries and for the
    // gathered rows, which count loads in issue order, do not include it
    V w[NV], g[NV], f[NV];
    const bool capepi = FWD && a.epi == 1 && cv;
    const int colc = cv ? col : 0;
    // (branch-free: the sink step, which has no W, re-reads the factor row instead)
    auto epi_loads = [&]() {
      if (FWD) {
        vld(a.epi == 1 ? a.wpan + rowc * Lp + colc : a.fac + colc, w);
        vld(a.epi == 1 ? a.wgt + colc : a.fac + colc, g);
      }
    };
    vld(a.fac + colc, f);
    // ---------------- product ----------------
    // neighbours in batches of KB: all indices, then all u values and rows are
    // requested before any of them is used, so one batch costs two memory
    // latencies (entries, then rows and u), an ELL chunk one (its entries are
    // already loaded).  All loads of a batch are unconditional, so the wave keeps
    // them all in flight: CSR entries past the row end re-read the batch's first
    // entry, and their coefficient is masked.  u at the input time is always
    // given (a vector of ones, or zeros in the log domain, where the input has none).
    struct Batch {
      int idx[KB];
      V cf[KB], uu[KB];
      V x[KB][NV];
      int cnt;
    };
    auto load_csr = [&](Batch& b, int e, auto first) {
      b.cnt = min(KB, row_end() - e);
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const int ek = (k < b.cnt) ? e + k : e;
        b.idx[k] = a.ci[ek];
        b.cf[k] = a.kv[ek];
      }
#pragma unroll
      for (int k = 0; k < KB; ++k) b.uu[k] = a.uin[b.idx[k]];
#pragma unroll
      for (int k = 0; k < KB; ++k) vld(a.xin + b.idx[k] * Lp + col, b.x[k]);
      if constexpr (decltype(first)::value) epi_loads();
    };
    auto load_ell = [&](Batch& b) {
      b.cnt = KB;
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        b.idx[k] = eidx[k];
        b.cf[k] = ecf[k];
        b.uu[k] = euu[k];
      }
      // rows of 16: padding entries (zero coefficient, -inf in the log domain)
      // gather nothing, their term being exactly zero (for whole-wave rows the
      // test is uniform and the wave issues no request).  Measured: the RGG steps
      // pad 9.2 neighbours on average to 16, and skipping took the forward step
      // from 5.24 to 4.94 us; on the road grid's rows of 5, which pad only at the
      // border, the tests cost more than they save (forward 64.0 -> 65.6 us).
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        if (KB < 16 || b.cf[k] != (LOG ? ninf<V>() : V(0))) {
          vld(a.xin + b.idx[k] * Lp + col, b.x[k]);
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) b.x[k][v] = V(0);
        }
      }
      epi_loads();
    };
    const bool nonempty = cv && (ell || row_end() > e0);
    if (!LOG) {
      V acc[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] = 0;
      auto fold = [&](const Batch& b) {
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          const V c = ((ell || k < b.cnt) ? b.cf[k] : V(0)) * b.uu[k];
#pragma unroll
          for (int v = 0; v < NV; ++v) acc[v] = fma(c, b.x[k][v], acc[v]);
        }
      };
      Batch b;
      if (nonempty) {
        if (ELL) {
          load_ell(b);
          fold(b);
        } else {
          int e = e0;
          load_csr(b, e, std::true_type{});
          fold(b);
          while (e + KB < row_end()) {
            e += KB;
            load_csr(b, e, std::false_type{});
            fold(b);
          }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) o[v] = acc[v] * f[v];
      } else {
        epi_loads();
#pragma unroll
        for (int v = 0; v < NV; ++v) o[v] = 0;
      }
    } else {
      V m[NV], sm[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) { m[v] = ninf<V>(); sm[v] = 0; }
      int batch = 0;
      auto fold = [&](Batch& b) {
#pragma unroll
        for (int k = 0; k < KB; ++k) b.cf[k] = ((ell || k < b.cnt) ? b.cf[k] : ninf<V>()) + b.uu[k];
        // (the ELL padding and masked CSR entries have coefficient -inf: their terms
        // are exactly 0; the rescaled running sum of a row's first batch is empty
        // and is not evaluated)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          // (the maximum and the sum start from the first term: the compiler keeps
          // a -inf or 0 start, which IEEE semantics do not let it drop)
          V y[KB];
#pragma unroll
          for (int k = 0; k < KB; ++k) y[k] = b.cf[k] + b.x[k][v];
          V bm = y[0];
#pragma unroll
          for (int k = 1; k < KB; ++k) bm = fmax(bm, y[k]);
          const V nm = (batch > 0) ? fmax(m[v], bm) : bm;
          const V bb = (nm == ninf<V>()) ? V(0) : nm;
          V acc = lexp2(y[0] - bb);
          if (batch > 0) acc = sm[v] * lexp2(m[v] - bb) + acc;
#pragma unroll
          for (int k = 1; k < KB; ++k) acc += lexp2(y[k] - bb);
          sm[v] = acc;
          m[v] = nm;
        }
        ++batch;
      };
      Batch b;
      if (nonempty) {
        if (ELL) {
          load_ell(b);
          fold(b);
        } else {
          int e = e0;
          load_csr(b, e, std::true_type{});
          fold(b);
          while (e + KB < row_end()) {
            e += KB;
            load_csr(b, e, std::false_type{});
            fold(b);
          }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) o[v] = (sm[v] > V(0)) ? m[v] + llog2(sm[v]) + f[v] : ninf<V>();
      } else {
        epi_loads();
#pragma unroll
        for (int v = 0; v < NV; ++v) o[v] = ninf<V>();
      }
    }

    // ---------------- epilogue ----------------
    // commodity capacities (loaded here, not with the operands above, so that
    // solves without them keep the product loop's register budget)
    V cwv[NV], dcv[NV];
    if (comm) {
      vld(a.cw + rowc * Lp + colc, cwv);
      if (FWD && a.epi == 1) vld(a.dc + rowc * Lp + colc, dcv);
    }
    V z[NV];   // value stored into the output panel (and calibrated on)
    V plT[NV];  // log domain sink: plan level at time T (= R0T after the update)
#pragma unroll
    for (int v = 0; v < NV; ++v) plT[v] = ninf<V>();
    if (FWD && a.epi == 2) {
      // sink: U0T = R0T ./ hatPsi_T (Algorithm 2), zero off the support
      if (cv) {
        V r[NV], cur[NV];
        vld(a.rdst + row * Lp + col, r);
        if (!CHK && a.hatT) vst(a.hatT + row * Lp + col, o);
        if (LOG) {
#pragma unroll
          for (int v = 0; v < NV; ++v) plT[v] = r[v];
        }
        if (!CHK) {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            if (!LOG) {
              if (r[v] > V(0)) {
                if (!(o[v] > V(0))) atomicOr(a.flags, FLAG_INFEASIBLE);
                z[v] = r[v] / o[v];
              } else z[v] = 0;
            } else {
              if (r[v] != ninf<V>()) {
                if (o[v] == ninf<V>()) atomicOr(a.flags, FLAG_INFEASIBLE);
                z[v] = r[v] - o[v];
              } else z[v] = ninf<V>();
            }
          }
          vst(a.u0t + row * Lp + col, z);
        } else {
          vld(a.u0t + row * Lp + col, cur);
#pragma unroll
          for (int v = 0; v < NV; ++v) z[v] = cur[v];
        }
        if (CHK) {
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
            if (a.pcomm && (unsigned)(l - a.pc_lo) < (unsigned)a.pc_cnt) a.pcomm[(size_t)(l - a.pc_lo) * a.n + row] = P;
          }
        }
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) z[v] = LOG ? ninf<V>() : V(0);
      }
    } else {
      V cwn[NV];   // w_t multiplied into the stored output (the new one after an update)
#pragma unroll
      for (int v = 0; v < NV; ++v) cwn[v] = comm ? cwv[v] : (LOG ? V(0) : V(1));
      if (capepi) {
        if (comm && !CHK && a.update) {
          // w_t = min(D_t ./ (P_{0,t} without w_t, times u_t), 1), 0 where D_t = 0; in the
          // multiplicative form w_old D / (P_{0,t} u_t), P_{0,t} taken with w_old (which is
          // folded into the stored backward panel), then P_{0,t} re-weighted to the new w_t
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            if (!LOG) {
              const V q = o[v] * w[v] * g[v];
              const V qu = q * ucur, lim = cwv[v] * dcv[v];
              const V wn = (dcv[v] == V(0)) ? V(0) : ((qu <= lim) ? V(1) : lim / qu);
              ssum += (cwv[v] > V(0)) ? q * (wn / cwv[v]) : V(0);
              cwn[v] = wn;
            } else {
              const V q = o[v] + w[v] + g[v];
              const V wn = (dcv[v] == ninf<V>()) ? ninf<V>()
                           : ((q == ninf<V>()) ? V(0) : fmin(V(0), cwv[v] + dcv[v] - q - ucur));
              const V y = (cwv[v] == ninf<V>() || wn == ninf<V>()) ? ninf<V>() : q - cwv[v] + wn;
              const V nm = fmax(lm, y);
              const V b = (nm == ninf<V>()) ? V(0) : nm;
              ls = ls * lexp2(lm - b) + lexp2(y - b);
              lm = nm;
              cwn[v] = wn;
            }
          }
        } else if (!LOG) {
#pragma unroll
          for (int v = 0; v < NV; ++v) ssum = fma(o[v] * w[v], g[v], ssum);
        } else {
          // the lane's NV terms against their common maximum, then one rescale of
          // the running sum (NV + 1 exponentials instead of 2 NV)
          V y[NV];
          V nm = lm;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            y[v] = o[v] + w[v] + g[v];
            nm = fmax(nm, y[v]);
          }
          const V b = (nm == ninf<V>()) ? V(0) : nm;
          V sum = ls * lexp2(lm - b);
#pragma unroll
          for (int v = 0; v < NV; ++v) sum += lexp2(y[v] - b);
          ls = sum;
          lm = nm;
        }
        if (CHK && (a.pcomm || a.kl || comm)) {
          // update-free pass: u is final, P_{0,t} = hatPsi (.) Psi (.) K_L w_t u_t (eq. proj_0t);
          // with state costs also accumulate <C_L, P_{0,t}> (cost tensor, eq. cost_multicommodity);
          // with commodity capacities their violation, dual term and gap term
          const V ur = comm ? ucur : a.uout[rowc];
          V k[NV];
          if (a.kl) vld(a.kl + row * Lp + col, k);
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const int l = col + v;
            if (l >= a.L) continue;
            double P = LOG ? ((o[v] == ninf<V>() || w[v] == ninf<V>()) ? 0.0
                                : exp2((double)o[v] + (double)w[v] + (double)g[v] + (double)ur))
                           : (double)o[v] * (double)w[v] * (double)g[v] * (double)ur;
            if (a.pcomm && (unsigned)(l - a.pc_lo) < (unsigned)a.pc_cnt) a.pcomm[(size_t)(l - a.pc_lo) * a.n + row] = P;
            if (a.kl && P > 0.0) {
              const double cl = LOG ? -(double)k[v] * a.eps * M_LN2 : -a.eps * log((double)k[v]);
              st[ST_SCOST] += P * cl;
            }
            if (comm) {
              const double D = LOG ? exp2((double)dcv[v]) : (double)dcv[v];
              if (isfinite(D) && D > 0.0) {
                const double lnw = LOG ? (double)cwv[v] * M_LN2 : log((double)cwv[v]);
                st[ST_CAP_VIOL] = fmax(st[ST_CAP_VIOL], fmax(P - D, 0.0) / D);
                st[ST_DUAL] += D * lnw;
                st[ST_GAP] += lnw * (P - D);
              }
            }
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
      if (comm) {
#pragma unroll
        for (int v = 0; v < NV; ++v) z[v] = LOG ? z[v] + cwn[v] : z[v] * cwn[v];
        if (FWD && !CHK && a.update && capepi && a.cwo) vst(a.cwo + row * Lp + col, cwn);
      }
      if (cv && a.out) vst(a.out + row * Lp + col, z);
      if (!cv) {
#pragma unroll
        for (int v = 0; v < NV; ++v) z[v] = LOG ? ninf<V>() : V(0);
      }
    }
    if (a.slots) calib_chunk<V, LOG>(z, G, it, lw, a.Lp, a.slots + (size_t)(bid % a.nslot) * a.nslot_stride);
    if (LOG && FWD && !CHK && a.epi == 1 && a.cslots_b) {
      // plan level at the output time: hatPsi + (Psi (.) K_L), up to per-column constants
      V pl[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) pl[v] = cv ? o[v] + w[v] : ninf<V>();
      const size_t cs = (size_t)(bid % a.ncslot) * a.cslot_stride;
      corr_chunk<V>(pl, w, G, it, lw, a.Lp, a.cslots_b + cs);
      corr_chunk<V>(pl, z, G, it, lw, a.Lp, a.cslots_f + cs);
    }
    if (LOG && FWD && !CHK && a.epi == 2 && a.cslots_f)
      corr_chunk<V>(plT, o, G, it, lw, a.Lp, a.cslots_f + (size_t)(bid % a.ncslot) * a.cslot_stride);
    if (FWD && a.slots_o) {
      if (!cv) {
#pragma unroll
        for (int v = 0; v < NV; ++v) o[v] = LOG ? ninf<V>() : V(0);
      }
      calib_chunk<V, LOG>(o, G, it, lw, a.Lp, a.slots_o + (size_t)(bid % a.nslot) * a.nslot_stride_o);
    }
  }

  // ---------------- capacity update (Corollary 1 + Proposition 1) ----------------
  if (FWD && a.epi == 1) {
    V sv;
    if (!LOG) sv = group_sum(ssum, G);
    else group_lse(lm, ls, G);
    if (lw) {
      // the row's waves combine their partial sums in wave order (deterministic)
      __shared__ V xm[kWaves], xs[kWaves];
      if (lane == 0) {
        if (!LOG) xs[wave] = sv;
        else { xm[wave] = lm; xs[wave] = ls; }
      }
      __syncthreads();
      if (sub == 0) {
        for (int k = 1; k < (1 << lw); ++k) {
          if (!LOG) sv += xs[wave + k];
          else {
            const V om = xm[wave + k], os = xs[wave + k];
            const V nm = fmax(lm, om);
            const V base = (nm == ninf<V>()) ? V(0) : nm;
            ls = ls * lexp2(lm - base) + os * lexp2(om - base);
            lm = nm;
          }
        }
      }
    }
    if (LOG) sv = (ls > V(0)) ? lm + llog2(ls) : ninf<V>();
    if (valid && gl == 0 && sub == 0) {
      const V d = a.cap[row];
      V u;
      if (!CHK) {
        if (!LOG) u = (sv <= d) ? V(1) : d / sv;
        else u = fmin(V(0), d - sv);
        a.uout[row] = u;
      } else {
        u = a.uout[row];
      }
      if (CHK) {
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
  if (CHK && a.epi == 2) {
    // gather the row's occupancy across the group lanes (and the row's waves) for the output
    double t = occ_row;
    for (int m = G >> 1; m > 0; m >>= 1) t += __shfl_xor(t, m, 64);
    if (lw) {
      __shared__ double xo[kWaves];
      if (lane == 0) xo[wave] = t;
      __syncthreads();
      if (sub == 0)
        for (int k = 1; k < (1 << lw); ++k) t += xo[wave + k];
    }
    if (valid && gl == 0 && sub == 0 && a.occ) a.occ[row] = t;
  }
  if (CHK && a.part) block_stats(st, a.part, bid);
}
// ---------------------------------------------------------------------------
// the steady-state ELL step
// ---------------------------------------------------------------------------
// Every step of a sweep on an ELL operator except the sink update: backward
// products and forward products with the capacity update (ell_fast), and as
// compile-time variants the steps of check passes (ell_check, ell_bcheck) and of
// FP32 calibration sweeps (ell_calib), without state costs or commodity
// capacities.  The
// arithmetic is step_body's, operation for operation (the results are bitwise
// the same); the difference is that nothing here is decided at run time, so
// a chunk's loads -- the neighbour rows, the factor row and (forward) the
// backward panel row and the weights -- are all issued before any is used, in
// straight-line code, and the kernel keeps no registers for the other epilogues.
template <typename V>
__host__ __device__ __forceinline__ bool ell_fast(const StepArgs<V>& a) {
  return a.ellD > 0 && !a.cw && !a.kl && !a.slots && !a.slots_o && !a.cslots_b && !a.cslots_f && a.epi != 2 &&
         (a.epi == 0 || a.update) && !a.part && !a.occ && !a.pcomm && a.out;
}
// the update-free forward step of a check pass in the same form: no u update, the
// occupancy and capacity statistics of each row into the block's partial (and the
// occupancy output), no per-commodity output
template <typename V>
__host__ __device__ __forceinline__ bool ell_check(const StepArgs<V>& a) {
  return a.ellD > 0 && !a.cw && !a.kl && !a.slots && !a.slots_o && !a.cslots_b && !a.cslots_f && a.epi == 1 &&
         !a.update && a.part && !a.pcomm && a.out;
}
// a step of a calibration sweep in the same form: the column levels of the stored
// panel (scaled domain) or the calibration keys of the forward step (log domain)
// recorded as step_body records them
template <typename V>
__host__ __device__ __forceinline__ bool ell_calib(const StepArgs<V>& a) {
  return a.ellD > 0 && !a.cw && !a.kl && !a.slots_o && a.epi != 2 && (a.epi == 0 || a.update) && !a.part &&
         !a.occ && !a.pcomm && a.out && (a.slots || a.cslots_b);
}
// a backward step of a fused check: the statistics of P_t from the fresh Psi_t and
// the kept hatPsi_t (wpan), weights wgt, u_t (uout) and d_t (cap)
template <typename V>
__host__ __device__ __forceinline__ bool ell_bcheck(const StepArgs<V>& a) {
  return a.ellD > 0 && !a.cw && !a.kl && !a.slots && !a.slots_o && !a.cslots_b && !a.cslots_f && a.epi == 0 &&
         a.part && !a.pcomm && !a.occ && a.out && a.wpan && a.wgt && a.uout && a.cap;
}
// every wave of the step has exactly one column chunk of its row
template <typename V>
__host__ __device__ __forceinline__ bool ell_one_chunk(const StepArgs<V>& a) {
  return ((a.nchunk + (1 << a.lwpr) - 1) >> a.lwpr) == 1;
}

// ONE: each wave has exactly one column chunk of its row (the launcher checks).
// Then the u values at the neighbours are requested after the chunk's gathers, so
// that the gathers go out as soon as the entries arrive; loaded ahead of the
// gathers (as rows of several chunks load them, once per row) they were waited
// for before any gather was issued, one more memory round trip per row (RGG
// workload, with the wait below: forward step 5.10 -> 4.61 us, backward 4.10 ->
// 3.69 us; on the road grid's rows of eight chunks the same order measured 3% slower).
// CHK: the check pass's update-free forward step (ell_check), the row-end
// statistics of step_body's check mode operation for operation; on a backward step
// (ell_bcheck) the same statistics with the roles of the panels exchanged: the
// product is Psi_t, the row read at its side the kept forward message hatPsi_t
// (K_L = 1), the weights 2^(sigma_hat_t + sigma_t) (a fused check).  CAL: a step of a
// calibration sweep (ell_calib), each chunk's levels or keys recorded after its store.
template <typename V, bool LOG, bool FWD, int KB, bool ONE, bool CHK = false, bool CAL = false>
__device__ __forceinline__ void ell_step_body(const StepArgs<V>& a, int bid, int nblk) {
  static_assert(!(CHK && CAL), "the check pass records no levels");
  constexpr int NV = VT<V>::N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int G = a.G;
  const int grp = lane / G, gl = lane & (G - 1);
  const int rpw = 64 / G;
  const int lb = xcd_block(bid, nblk);
  const int lw = a.lwpr;
  const int rslot = wave >> lw, sub = wave & ((1 << lw) - 1);
  const int row = ((lb * kWaves >> lw) + rslot) * rpw + grp;
  const bool valid = row < a.n;
  const int rowc = valid ? row : 0;
  const size_t Lp = (size_t)a.Lp;
  const V pad = LOG ? ninf<V>() : V(0);

  // the row's entries and (rows of several chunks) the u values at its neighbours, once per row
  int eidx[KB];
  V ecf[KB], euu[KB];
  const int e0 = rowc * a.ellD;
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    eidx[k] = a.ci[e0 + k];
    ecf[k] = a.kv[e0 + k];
  }
  if constexpr (!ONE) {
#pragma unroll
    for (int k = 0; k < KB; ++k) euu[k] = a.uin[eidx[k]];
  }
  // ONE: every entry is in before the first gather is issued.  Rows of 16 test
  // each entry before its gather (padding entries gather nothing), and left to
  // itself the compiler issued the gathers of the first eight entries as soon as
  // those were in, then waited for all outstanding loads, those gathers included,
  // before the other eight: one more memory round trip
  if constexpr (ONE && KB >= 16) __builtin_amdgcn_s_waitcnt(0);

  V ssum = 0;
  V lm = ninf<V>(), ls = 0;
  const int nit = ONE ? 1 : (a.nchunk + (1 << lw) - 1) >> lw;
  for (int it = 0; it < nit; ++it) {
    const int ch = (it << lw) + sub;
    const int col = (ch * G + gl) * NV;
    const bool cv = valid && col < a.Lp;
    const int colc = cv ? col : 0;
    // all loads of the chunk, at clamped addresses (a row of 16 skips its padding
    // entries: their term is exactly zero, and for whole-wave rows the test is uniform)
    V x[KB][NV];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      if (KB < 16 || ecf[k] != pad) {
        vld(a.xin + eidx[k] * Lp + colc, x[k]);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) x[k][v] = V(0);
      }
    }
    V f[NV], w[NV], g[NV];
    vld(a.fac + colc, f);
    if (FWD || CHK) {
      vld(a.wpan + rowc * Lp + colc, w);
      vld(a.wgt + colc, g);
    }
    if constexpr (ONE) {
#pragma unroll
      for (int k = 0; k < KB; ++k) euu[k] = a.uin[eidx[k]];
    }
    V o[NV];
    if (!LOG) {
      V acc[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] = 0;
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const V c = ecf[k] * euu[k];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = fma(c, x[k][v], acc[v]);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) o[v] = acc[v] * f[v];
    } else {
      V c[KB];
#pragma unroll
      for (int k = 0; k < KB; ++k) c[k] = ecf[k] + euu[k];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        V y[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) y[k] = c[k] + x[k][v];
        V bm = y[0];
#pragma unroll
        for (int k = 1; k < KB; ++k) bm = fmax(bm, y[k]);
        const V bb = (bm == ninf<V>()) ? V(0) : bm;
        V acc = lexp2(y[0] - bb);
#pragma unroll
        for (int k = 1; k < KB; ++k) acc += lexp2(y[k] - bb);
        o[v] = (acc > V(0)) ? bm + llog2(acc) + f[v] : ninf<V>();
      }
    }
    // (ONE: computed on every lane and kept where cv, so that the loads of w and g,
    // used on every path, are not sunk below the wait for the gathers)
    if ((FWD || CHK) && (ONE || cv)) {
      if (!LOG) {
        V t = ssum;
#pragma unroll
        for (int v = 0; v < NV; ++v) t = fma(o[v] * w[v], g[v], t);
        ssum = cv ? t : ssum;
      } else {
        V y[NV];
        V nm = lm;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          y[v] = o[v] + w[v] + g[v];
          nm = fmax(nm, y[v]);
        }
        const V b = (nm == ninf<V>()) ? V(0) : nm;
        V sum = ls * lexp2(lm - b);
#pragma unroll
        for (int v = 0; v < NV; ++v) sum += lexp2(y[v] - b);
        ls = cv ? sum : ls;
        lm = cv ? nm : lm;
      }
    }
    if (cv) vst(a.out + row * Lp + col, o);
    if constexpr (CAL) {
      // (every wave of the block runs the same chunks: the recordings hold barriers)
      V z[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) z[v] = cv ? o[v] : (LOG ? ninf<V>() : V(0));
      if (a.slots) calib_chunk<V, LOG>(z, G, it, lw, a.Lp, a.slots + (size_t)(bid % a.nslot) * a.nslot_stride);
      if constexpr (LOG && FWD) {
        if (a.cslots_b) {
          // plan level at the output time: hatPsi + (Psi (.) K_L), up to per-column constants
          V pl[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) pl[v] = cv ? o[v] + w[v] : ninf<V>();
          const size_t cs = (size_t)(bid % a.ncslot) * a.cslot_stride;
          corr_chunk<V>(pl, w, G, it, lw, a.Lp, a.cslots_b + cs);
          corr_chunk<V>(pl, z, G, it, lw, a.Lp, a.cslots_f + cs);
        }
      }
    }
  }

  if (FWD || CHK) {
    V sv;
    if (!LOG) sv = group_sum(ssum, G);
    else group_lse(lm, ls, G);
    if (lw) {
      __shared__ V xm[kWaves], xs[kWaves];
      if (lane == 0) {
        if (!LOG) xs[wave] = sv;
        else { xm[wave] = lm; xs[wave] = ls; }
      }
      __syncthreads();
      if (sub == 0) {
        for (int k = 1; k < (1 << lw); ++k) {
          if (!LOG) sv += xs[wave + k];
          else {
            const V om = xm[wave + k], os = xs[wave + k];
            const V nm = fmax(lm, om);
            const V base = (nm == ninf<V>()) ? V(0) : nm;
            ls = ls * lexp2(lm - base) + os * lexp2(om - base);
            lm = nm;
          }
        }
      }
    }
    if (LOG) sv = (ls > V(0)) ? lm + llog2(ls) : ninf<V>();
    if constexpr (!CHK) {
      if (valid && gl == 0 && sub == 0) {
        const V d = a.cap[row];
        a.uout[row] = !LOG ? ((sv <= d) ? V(1) : d / sv) : fmin(V(0), d - sv);
      }
    } else {
      // occupancy u_t s_t of the row and its capacity terms (Corollary 1)
      double st[kNSt] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (valid && gl == 0 && sub == 0) {
        const V d = a.cap[row];
        const V u = a.uout[row];
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
      block_stats(st, a.part, bid);
    }
  }
}
template <typename V, bool LOG, bool FWD, int KB, bool ONE, bool CHK, bool CAL = false>
__global__ __launch_bounds__(kBlock) void k_ell_step(StepArgs<V> a) {
  ell_step_body<V, LOG, FWD, KB, ONE, CHK, CAL>(a, blockIdx.x, gridDim.x);
}

// (at least two waves per SIMD: the wide CSR variants would otherwise take the
// whole register file for one)
template <typename V, bool LOG, bool FWD, bool CHK, bool ELL, int KB, bool CM>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_step(StepArgs<V> a) {
  step_body<V, LOG, FWD, CHK, ELL, KB, CM>(a, blockIdx.x, gridDim.x);
}


// ---------------------------------------------------------------------------
// source update: U01 = R01 ./ Psi_1 (Algorithm 2), stored scaled by fac
// ---------------------------------------------------------------------------
template <typename V, bool LOG>
__device__ __forceinline__ void source_body(const SourceArgs<V>& A, int bid, int nblk) {
  const int n = A.n, Lp = A.Lp, G = A.G, nchunk = A.nchunk, nslot = A.nslot;
  const V* __restrict__ psi0 = A.psi0;
  const V* __restrict__ rsrc = A.rsrc;
  V* __restrict__ u01 = A.u01;
  uint32_t* slots = A.slots;
  const size_t slot_stride = A.slot_stride;
  int* flags = A.flags;

  constexpr int NV = VT<V>::N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / G, gl = lane & (G - 1);
  const int lb = xcd_block(bid, nblk);
  const int row = (lb * kWaves + wave) * (64 / G) + grp;
  const bool valid = row < n;
  for (int ch = 0; ch < nchunk; ++ch) {
    const int col = (ch * G + gl) * NV;
    const bool cv = valid && col < Lp;
    V z[NV], pl[NV], xs[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) { pl[v] = ninf<V>(); xs[v] = ninf<V>(); }
    if (cv) {
      V x[NV], r[NV];
      vld(psi0 + (size_t)row * Lp + col, x);
      vld(rsrc + (size_t)row * Lp + col, r);
      if (LOG) {
#pragma unroll
        for (int v = 0; v < NV; ++v) { pl[v] = r[v]; xs[v] = x[v]; }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (!LOG) {
          if (r[v] > V(0)) {
            if (!(x[v] > V(0))) atomicOr(flags, FLAG_INFEASIBLE);
            z[v] = r[v] / x[v];
          } else z[v] = 0;
        } else {
          if (r[v] != ninf<V>()) {
            if (x[v] == ninf<V>()) atomicOr(flags, FLAG_INFEASIBLE);
            z[v] = r[v] - x[v];
          } else z[v] = ninf<V>();
        }
      }
      vst(u01 + (size_t)row * Lp + col, z);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) z[v] = LOG ? ninf<V>() : V(0);
    }
    if (slots) calib_chunk<V, LOG>(z, G, ch, 0, Lp, slots + (size_t)(bid % nslot) * slot_stride);
    // log domain calibration: Psi_1 at the plan peak (the plan at time 0 is R01)
    if (LOG && A.cslots)
      corr_chunk<V>(pl, xs, G, ch, 0, Lp, A.cslots + (size_t)(bid % A.ncslot) * A.cslot_stride);
  }
}
template <typename V, bool LOG>
__global__ __launch_bounds__(kBlock) void k_source(SourceArgs<V> A) {
  source_body<V, LOG>(A, blockIdx.x, gridDim.x);
}


// ---------------------------------------------------------------------------
// statistics at time 0: P_{0,1} = U01 (.) Psi_1 against R01 (check / output pass)
// ---------------------------------------------------------------------------
template <typename V, bool LOG>
__device__ __forceinline__ void check0_body(const Check0Args<V>& A, int bid, int nblk) {
  const int n = A.n, Lp = A.Lp, L = A.L, G = A.G, nchunk = A.nchunk;
  const V* __restrict__ psi0 = A.psi0;
  const V* __restrict__ u01 = A.u01;
  const V* __restrict__ rsrc = A.rsrc;
  const double* __restrict__ sigf0 = A.sigf0;
  const double* __restrict__ sigb0 = A.sigb0;
  double* part = A.part;
  double* occ = A.occ;
  double* pcomm = A.pcomm;

  constexpr int NV = VT<V>::N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / G, gl = lane & (G - 1);
  const int lb = xcd_block(bid, nblk);
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
      if (pcomm && (unsigned)(l - A.pc_lo) < (unsigned)A.pc_cnt) pcomm[(size_t)(l - A.pc_lo) * n + row] = P;
    }
  }
  if (occ) {
    double t = occ_row;
    for (int m = G >> 1; m > 0; m >>= 1) t += __shfl_xor(t, m, 64);
    if (valid && gl == 0) occ[row] = t;
  }
  if (part) block_stats(st, part, bid);
}
template <typename V, bool LOG>
__global__ __launch_bounds__(kBlock) void k_check0(Check0Args<V> A) {
  check0_body<V, LOG>(A, blockIdx.x, gridDim.x);
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
        if (F > 0.0) st[0] += cost[e] * F;   // a move closed at this step (+inf cost) carries nothing
      }
    }
  }
  if (part) block_stats(st, part, blockIdx.x);
}

// ---------------------------------------------------------------------------
// range-offset bookkeeping
// ---------------------------------------------------------------------------
// lev[t][l] = max over calibration slots (log2 column max of the panel stored
// at time t, -inf if nothing was recorded); slots cleared.  Thread per (t, l);
// all slot reads are issued before any clear.
__device__ __forceinline__ void levels_body(const LevelsArgs& A, int bid, int nblk) {
  uint32_t* slots = A.slots;
  float* lev = A.lev;
  const int T1 = A.T1, Lp = A.Lp, nslot = A.nslot;

  const int idx = bid * blockDim.x + threadIdx.x;
  if (idx >= T1 * Lp) return;
  const size_t stride = (size_t)T1 * Lp;
  uint32_t v[32];
#pragma unroll
  for (int p = 0; p < 32; ++p) v[p] = (p < nslot) ? slots[p * stride + idx] : 0u;
  float m = -INFINITY;
#pragma unroll
  for (int p = 0; p < 32; ++p) {
    if (v[p]) {
      m = fmaxf(m, dec_f32(v[p]));
      slots[p * stride + idx] = 0u;
    }
  }
  lev[idx] = m;
}
__global__ void k_levels(LevelsArgs A) { levels_body(A, blockIdx.x, gridDim.x); }

// Log domain: lev[t][l] = the value carried by the largest (plan level, value)
// key over the 64-bit slots; where none was recorded, the column maximum from
// the 32-bit slots (or -inf).  Both slot sets are cleared.
__device__ __forceinline__ void levels64_body(const Levels64Args& A, int bid, int nblk) {
  const int T1 = A.T1, Lp = A.Lp, ncslot = A.ncslot, nslot = A.nslot;
  const int idx = bid * blockDim.x + threadIdx.x;
  if (idx >= T1 * Lp) return;
  const size_t stride = (size_t)T1 * Lp;
  unsigned long long best = 0;
  for (int p = 0; p < ncslot; ++p) {
    const unsigned long long k = A.cslots[p * stride + idx];
    if (k) {
      best = k > best ? k : best;
      A.cslots[p * stride + idx] = 0ull;
    }
  }
  float m = -INFINITY;
  for (int p = 0; p < nslot; ++p) {
    const uint32_t e = A.slots[p * stride + idx];
    if (e) {
      m = fmaxf(m, dec_f32(e));
      A.slots[p * stride + idx] = 0u;
    }
  }
  A.lev[idx] = best ? dec_f32((uint32_t)(best & 0xffffffffull)) : m;
}
__global__ void k_levels64(Levels64Args A) { levels64_body(A, blockIdx.x, gridDim.x); }


// wave-level helpers for the one-wavefront-per-commodity prep kernels
__device__ __forceinline__ double wave_incl_scan(double x) {
  const int lane = threadIdx.x & 63;
  for (int d = 1; d < 64; d <<= 1) {
    const double y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}
// exact column level of a sweep's starting panel: lane p reads slot p (cleared);
// keeps the previous level when nothing was recorded
__device__ __forceinline__ double wave_take_level(uint32_t* slots, int nslot, int Lp, int l, double prev) {
  const int lane = threadIdx.x & 63;
  uint32_t e = 0;
  if (lane < nslot) {
    e = slots[(size_t)lane * Lp + l];
    if (e) slots[(size_t)lane * Lp + l] = 0u;
  }
  float m = e ? dec_f32(e) : -INFINITY;
  for (int d = 32; d > 0; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
  const bool any = __ballot(e != 0) != 0;
  if (!any) return prev;
  return (m > -INFINITY && isfinite(m)) ? (double)m : 0.0;
}

template <typename V, bool LOG>
__device__ __forceinline__ V to_fac(double c) {
  return LOG ? static_cast<V>(-c) : static_cast<V>(exp2(-c));
}
template <typename V, bool LOG>
__device__ __forceinline__ V to_wgt(double s) {
  return LOG ? static_cast<V>(s) : static_cast<V>(exp2(s));
}

// Growth update from a calibration sweep's column levels (thread per (t, l)):
// backward (dir 0): c[T-1] += lev[T-1], c[t] += lev[t] - lev[t+1];
// forward (dir 1):  c[1] += lev[1],     c[t] += lev[t] - lev[t-1] (t = 2..T).
__device__ __forceinline__ void growth_body(const GrowthArgs& A, int bid, int nblk) {
  double* c = A.c;
  const float* __restrict__ lev = A.lev;
  const int T = A.T, Lp = A.Lp, dir = A.dir;

  const int idx = bid * blockDim.x + threadIdx.x;
  if (idx >= (T + 1) * Lp) return;
  const int t = idx / Lp;
  const float a = lev[idx];
  if (!(a > -INFINITY)) return;
  if (dir == 0) {
    if (t > T - 1) return;
    if (t == T - 1) { c[idx] += (double)a; return; }
    const float b = lev[idx + Lp];
    if (b > -INFINITY) c[idx] += (double)a - (double)b;
  } else {
    if (t < 1) return;
    if (t == 1) { c[idx] += (double)a; return; }
    const float b = lev[idx - Lp];
    if (b > -INFINITY) c[idx] += (double)a - (double)b;
  }
}
__global__ void k_growth(GrowthArgs A) { growth_body(A, blockIdx.x, gridDim.x); }


// Backward sweep offsets, one wavefront per commodity l (lanes = times).
// Start level of the U0T panel from its slots; sigma_b[T] = gauge of U0T;
// sigma_b[t] = sigma_b[t+1] + c_b[t] (suffix scan), the first product also
// removing the start level.
template <typename V, bool LOG>
__device__ __forceinline__ void prep_bwd_body(const PrepBwdArgs<V>& A, int bid, int nblk) {
  const int T = A.T, Lp = A.Lp, nslot = A.nslot;
  const double* __restrict__ cb = A.cb;
  double* __restrict__ sigb = A.sigb;
  V* __restrict__ facb = A.facb;
  const double* __restrict__ gaugeT = A.gaugeT;
  double* __restrict__ lvlT = A.lvlT;
  uint32_t* slotsE = A.slotsE;

  const int lane = threadIdx.x & 63;
  const int l = bid * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (l >= Lp) return;
  const double lv = wave_take_level(slotsE, nslot, Lp, l, lvlT[l]);
  double carry = gaugeT[l];
  if (lane == 0) {
    lvlT[l] = lv;
    sigb[(size_t)T * Lp + l] = carry;
    facb[(size_t)T * Lp + l] = to_fac<V, LOG>(0.0);
  }
  for (int base = T - 1; base >= 0; base -= 64) {
    const int t = base - lane;
    const double c = (t >= 0) ? cb[(size_t)t * Lp + l] + ((t == T - 1) ? lv : 0.0) : 0.0;
    const double incl = wave_incl_scan(c);
    if (t >= 0) {
      sigb[(size_t)t * Lp + l] = carry + incl;
      facb[(size_t)t * Lp + l] = to_fac<V, LOG>(c);
    }
    carry += __shfl(incl, 63, 64);
  }
}
template <typename V, bool LOG>
__global__ void k_prep_bwd(PrepBwdArgs<V> A) { prep_bwd_body<V, LOG>(A, blockIdx.x, gridDim.x); }


// Forward sweep offsets, one wavefront per commodity.  mode 0 (Sinkhorn sweep,
// after the source update wrote U01 = R01 ./ Psi_1 unscaled):
// sigma_hat_0 = -sigma_b[0], start level from the source kernel's slots;
// mode 1 (check / output pass): U01 is kept, sigma_hat_0 = gauge0 and the stored
// start level.  sigma_hat_t = sigma_hat_{t-1} + c_f[t] (prefix scan); weights
// wgt[t] = 2^(sigma_hat_t + sigma_b[t]); mode 0 also sets the gauge of the U0T
// panel the sink update is about to write: -sigma_hat_T.
template <typename V, bool LOG>
__device__ __forceinline__ void prep_fwd_body(const PrepFwdArgs<V>& A, int bid, int nblk) {
  const int T = A.T, Lp = A.Lp, mode = A.mode, nslot = A.nslot;
  const double* __restrict__ cf = A.cf;
  double* __restrict__ sigf = A.sigf;
  const double* __restrict__ sigb = A.sigb;
  V* __restrict__ facf = A.facf;
  V* __restrict__ wgt = A.wgt;
  double* __restrict__ gauge0 = A.gauge0;
  double* __restrict__ gaugeT = A.gaugeT;
  double* __restrict__ lvl0 = A.lvl0;
  uint32_t* slotsS = A.slotsS;

  const int lane = threadIdx.x & 63;
  const int l = bid * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (l >= Lp) return;
  double s0, lv;
  if (mode == 0) {
    s0 = -sigb[l];
    lv = wave_take_level(slotsS, nslot, Lp, l, lvl0[l]);
  } else {
    s0 = gauge0[l];
    lv = lvl0[l];
  }
  if (lane == 0) {
    if (mode == 0) { gauge0[l] = s0; lvl0[l] = lv; }
    sigf[l] = s0;
    facf[l] = to_fac<V, LOG>(0.0);
    wgt[l] = to_wgt<V, LOG>(s0 + sigb[l]);
  }
  double carry = s0;
  for (int base = 1; base <= T; base += 64) {
    const int t = base + lane;
    const bool ok = t <= T;
    const double c = ok ? cf[(size_t)t * Lp + l] + ((t == 1) ? lv : 0.0) : 0.0;
    const double sb = ok ? sigb[(size_t)t * Lp + l] : 0.0;
    const double sg = carry + wave_incl_scan(c);
    if (ok) {
      sigf[(size_t)t * Lp + l] = sg;
      facf[(size_t)t * Lp + l] = to_fac<V, LOG>(c);
      wgt[(size_t)t * Lp + l] = to_wgt<V, LOG>(sg + sb);
      if (mode == 0 && t == T) gaugeT[l] = -sg;
    }
    carry = __shfl(sg, 63, 64);
  }
}
template <typename V, bool LOG>
__global__ void k_prep_fwd(PrepFwdArgs<V> A) { prep_fwd_body<V, LOG>(A, blockIdx.x, gridDim.x); }


// ---------------------------------------------------------------------------
// deterministic two-stage reduction of the stats partials
// ---------------------------------------------------------------------------
// stage 1: one block per time slot, sums its partials in block order
__device__ __forceinline__ void reduce1_body(const Reduce1Args& A, int bid, int nblk_grid) {
  const double* __restrict__ part = A.part;
  double* __restrict__ tpart = A.tpart;

  const int t = bid;
  const int nblk = (t == 0) ? A.nblk0 : A.nblk;
  const double* p = part + (size_t)t * A.stride * kNSt;
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
__global__ void k_reduce_stats1(Reduce1Args A) { reduce1_body(A, blockIdx.x, gridDim.x); }


// stage 2: combine the T+1 time slots into the stats record
//   out[0] dual_obj, [1] src_resid, [2] cap_viol, [3] mass_drift, [4] dual_gap, [5] mass, [6] nonfinite
__device__ __forceinline__ void reduce2_body(const Reduce2Args& A, int bid, int nblk) {
  const double* __restrict__ tpart = A.tpart;
  const int T1 = A.T1;
  const double eps = A.eps;
  double* __restrict__ out = A.out;

  if (threadIdx.x != 0 || bid != 0) return;
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
__global__ void k_reduce_stats2(Reduce2Args A) { reduce2_body(A, blockIdx.x, gridDim.x); }


// transport cost = move costs from the flow-kernel partials (tflow, T slots)
// + state costs from the update-free forward steps (tstate, slots 1..T-1)
__global__ void k_reduce_cost(const double* __restrict__ tflow, const double* __restrict__ tstate, int T,
                              double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0;
  for (int t = 0; t < T; ++t) s += tflow[(size_t)t * kNSt];
  for (int t = 1; t < T; ++t) s += tstate[(size_t)t * kNSt + ST_SCOST];
  out[0] = s;
}

// ---------------------------------------------------------------------------
// host-side launchers (explicit instantiations)
// ---------------------------------------------------------------------------
// fwd: 0 backward product, 1 forward Sinkhorn step, 2 forward update-free (check / output) step
// Time-T statistics of a fused check: P_{0,T} = U0T (.) hatPsi_T from the kept
// hatPsi_T of the last Sinkhorn sweep (the forward message the sink update divided
// R0T by), as the sink step's check mode computes them (mass, <R0T, log U0T>, gap);
// partials of nblk blocks (rows grid-stride), one per block.
template <typename V, bool LOG>
__global__ __launch_bounds__(kBlock) void k_sink_check(int n, int Lp, int L, int G, int nchunk,
                                                       const V* __restrict__ hat, const V* __restrict__ u0t,
                                                       const V* __restrict__ rdst, const double* __restrict__ sigT,
                                                       const double* __restrict__ sighT, double* part) {
  constexpr int NV = VT<V>::N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / G, gl = lane & (G - 1), rpw = 64 / G;
  double st[kNSt] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int r0 = (blockIdx.x * kWaves + wave) * rpw; r0 < n; r0 += gridDim.x * kWaves * rpw) {
    const int row = r0 + grp;
    if (row >= n) continue;
    for (int ch = 0; ch < nchunk; ++ch) {
      const int col = (ch * G + gl) * NV;
      if (col >= Lp) continue;
      V z[NV], o[NV], r[NV];
      vld(u0t + (size_t)row * Lp + col, z);
      vld(hat + (size_t)row * Lp + col, o);
      vld(rdst + (size_t)row * Lp + col, r);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int l = col + v;
        if (l >= L) continue;
        const double sg = sigT[l] + sighT[l];
        double P, lnU, R;
        if (!LOG) {
          P = (double)z[v] * (double)o[v] * exp2(sg);
          lnU = (z[v] > V(0)) ? (log2((double)z[v]) + sigT[l]) * M_LN2 : 0.0;
          R = (double)r[v];
        } else {
          P = (z[v] == ninf<V>() || o[v] == ninf<V>()) ? 0.0 : exp2((double)z[v] + (double)o[v] + sg);
          lnU = (z[v] != ninf<V>()) ? ((double)z[v] + sigT[l]) * M_LN2 : 0.0;
          R = (r[v] == ninf<V>()) ? 0.0 : exp2((double)r[v]);
        }
        st[ST_MASS] += P;
        st[ST_DUAL] += R * lnU;
        st[ST_GAP] += lnU * (P - R);
      }
    }
  }
  block_stats(st, part, blockIdx.x);
}
template <typename V, bool LOG>
void launch_sink_check(int n, int Lp, int L, int G, int nchunk, const V* hat, const V* u0t, const V* rdst,
                       const double* sigT, const double* sighT, double* part, int nblk, hipStream_t s) {
  hipLaunchKernelGGL((k_sink_check<V, LOG>), dim3(nblk), dim3(kBlock), 0, s, n, Lp, L, G, nchunk, hat, u0t, rdst,
                     sigT, sighT, part);
}

__global__ void k_or_flag(int* flags, int v) {
  if (threadIdx.x == 0) atomicOr(flags, v);
}
template <typename V, bool LOG>
void launch_step(const StepArgs<V>& a, int fwd, int nblk, hipStream_t s) {
  if (record_item(fwd == 0 ? IK_STEP_BWD : (fwd == 1 ? IK_STEP_FWD : IK_STEP_CHK), LOG, nblk, &a, sizeof(a))) return;
  // ELL rows padded to a multiple of 16 gather 16 neighbours per batch, to a
  // multiple of 8 (low-degree graphs such as road grids) 8; CSR batches are 16
  // commodity capacities run on CSR operators (the solver builds no ELL copy for them)
#define MMOT_STEP_LAUNCH(E, K, C)                                                                            \
  do {                                                                                                      \
    if (fwd == 1) hipLaunchKernelGGL((k_step<V, LOG, true, false, E, K, C>), dim3(nblk), dim3(kBlock), 0, s, a); \
    else if (fwd == 2) hipLaunchKernelGGL((k_step<V, LOG, true, true, E, K, C>), dim3(nblk), dim3(kBlock), 0, s, a); \
    else hipLaunchKernelGGL((k_step<V, LOG, false, false, E, K, C>), dim3(nblk), dim3(kBlock), 0, s, a);       \
  } while (0)
#define MMOT_ELL_LAUNCH1(K, O)                                                                                      \
  do {                                                                                                             \
    if (fwd == 2) hipLaunchKernelGGL((k_ell_step<V, LOG, true, K, O, true>), dim3(nblk), dim3(kBlock), 0, s, a);    \
    else if (fwd == 1) hipLaunchKernelGGL((k_ell_step<V, LOG, true, K, O, false>), dim3(nblk), dim3(kBlock), 0, s, a); \
    else if (a.part) hipLaunchKernelGGL((k_ell_step<V, LOG, false, K, O, true>), dim3(nblk), dim3(kBlock), 0, s, a); \
    else hipLaunchKernelGGL((k_ell_step<V, LOG, false, K, O, false>), dim3(nblk), dim3(kBlock), 0, s, a);          \
  } while (0)
#define MMOT_ELL_LAUNCH(K)                                                                                          \
  do {                                                                                                             \
    if (one) MMOT_ELL_LAUNCH1(K, true);                                                                            \
    else MMOT_ELL_LAUNCH1(K, false);                                                                               \
  } while (0)
  if (fwd == 0 && a.part && !ell_bcheck(a)) {
    // a backward step computes statistics only in that form (the caller checks):
    // anything else is a host error, reported through the flags, never run half-done
    hipLaunchKernelGGL(k_or_flag, dim3(1), dim3(64), 0, s, a.flags, (int)FLAG_BADINPUT);
    return;
  }
  if (fwd == 2 ? ell_check(a) : (a.part ? ell_bcheck(a) : ell_fast(a))) {
    const bool one = ell_one_chunk(a);
    if (a.ellD == 16) MMOT_ELL_LAUNCH(16);
    else if (a.ellD == 8) MMOT_ELL_LAUNCH(8);
    else if (a.ellD == 5) MMOT_ELL_LAUNCH(5);
    else MMOT_ELL_LAUNCH(4);
#undef MMOT_ELL_LAUNCH
#undef MMOT_ELL_LAUNCH1
    return;
  }
  if constexpr (std::is_same<V, float>::value) {
    // calibration sweeps (FP32 solves)
    if (fwd != 2 && ell_calib(a)) {
      const bool one = ell_one_chunk(a);
#define MMOT_CAL_LAUNCH1(K, O)                                                                                     \
  do {                                                                                                             \
    if (fwd == 1) hipLaunchKernelGGL((k_ell_step<V, LOG, true, K, O, false, true>), dim3(nblk), dim3(kBlock), 0, s, a); \
    else hipLaunchKernelGGL((k_ell_step<V, LOG, false, K, O, false, true>), dim3(nblk), dim3(kBlock), 0, s, a);    \
  } while (0)
#define MMOT_CAL_LAUNCH(K)                                                                                         \
  do {                                                                                                             \
    if (one) MMOT_CAL_LAUNCH1(K, true);                                                                            \
    else MMOT_CAL_LAUNCH1(K, false);                                                                               \
  } while (0)
      if (a.ellD == 16) MMOT_CAL_LAUNCH(16);
      else if (a.ellD == 8) MMOT_CAL_LAUNCH(8);
      else if (a.ellD == 5) MMOT_CAL_LAUNCH(5);
      else MMOT_CAL_LAUNCH(4);
#undef MMOT_CAL_LAUNCH
#undef MMOT_CAL_LAUNCH1
      return;
    }
  }
  if (a.cw) MMOT_STEP_LAUNCH(false, 16, true);
  else if (a.ellD == 16) MMOT_STEP_LAUNCH(true, 16, false);
  else if (a.ellD == 8) MMOT_STEP_LAUNCH(true, 8, false);
  else if (a.ellD == 5) MMOT_STEP_LAUNCH(true, 5, false);
  else if (a.ellD == 4) MMOT_STEP_LAUNCH(true, 4, false);
  else MMOT_STEP_LAUNCH(false, 16, false);
#undef MMOT_STEP_LAUNCH
}
template <typename V, bool LOG>
void launch_source(int n, int Lp, int G, int nchunk, const V* psi0, const V* rsrc, V* u01, uint32_t* slots,
                   int nslot, size_t slot_stride, int* flags, unsigned long long* cslots, int ncslot,
                   size_t cslot_stride, int nblk, hipStream_t s) {
  const SourceArgs<V> A{n, Lp, G, nchunk, nslot, psi0, rsrc, u01, slots, slot_stride, flags, cslots, ncslot,
                        cslot_stride};
  if (record_item(IK_SOURCE, LOG, nblk, &A, sizeof(A))) return;
  hipLaunchKernelGGL((k_source<V, LOG>), dim3(nblk), dim3(kBlock), 0, s, A);
}
template <typename V, bool LOG>
void launch_check0(int n, int Lp, int L, int G, int nchunk, const V* psi0, const V* u01, const V* rsrc,
                   const double* sigf0, const double* sigb0, double* part, double* occ, double* pcomm, int pc_lo,
                   int pc_cnt, int nblk, hipStream_t s) {
  const Check0Args<V> A{n, Lp, L, G, nchunk, psi0, u01, rsrc, sigf0, sigb0, part, occ, pcomm, pc_lo, pc_cnt};
  if (record_item(IK_CHECK0, LOG, nblk, &A, sizeof(A))) return;
  hipLaunchKernelGGL((k_check0<V, LOG>), dim3(nblk), dim3(kBlock), 0, s, A);
}
template <typename V, bool LOG>
void launch_flows(int n, int Lp, int L, int G, int nchunk, const int* rp, const int* ci, const V* kv,
                  const double* cost, const V* A, const V* ua, const V* B, const V* ub, const double* siga,
                  const double* sigb, double* flow, double* part, int nblk, hipStream_t s) {
  hipLaunchKernelGGL((k_flows<V, LOG>), dim3(nblk), dim3(kBlock), 0, s, n, Lp, L, G, nchunk, rp, ci, kv, cost, A,
                     ua, B, ub, siga, sigb, flow, part);
}
template <typename V, bool LOG>
void launch_prep_bwd(int T, int Lp, const double* cb, double* sigb, V* facb, const double* gaugeT, double* lvlT,
                     uint32_t* slotsE, int nslot, hipStream_t s) {
  const PrepBwdArgs<V> A{T, Lp, nslot, cb, sigb, facb, gaugeT, lvlT, slotsE};
  const int nb = (Lp + 3) / 4;
  if (record_item(IK_PREP_BWD, LOG, nb, &A, sizeof(A))) return;
  hipLaunchKernelGGL((k_prep_bwd<V, LOG>), dim3(nb), dim3(256), 0, s, A);
}
template <typename V, bool LOG>
void launch_prep_fwd(int T, int Lp, int mode, const double* cf, double* sigf, const double* sigb, V* facf, V* wgt,
                     double* gauge0, double* gaugeT, double* lvl0, uint32_t* slotsS, int nslot, hipStream_t s) {
  const PrepFwdArgs<V> A{T, Lp, mode, nslot, cf, sigf, sigb, facf, wgt, gauge0, gaugeT, lvl0, slotsS};
  const int nb = (Lp + 3) / 4;
  if (record_item(IK_PREP_FWD, LOG, nb, &A, sizeof(A))) return;
  hipLaunchKernelGGL((k_prep_fwd<V, LOG>), dim3(nb), dim3(256), 0, s, A);
}
void launch_growth(double* c, const float* lev, int T, int Lp, int dir, hipStream_t s) {
  const GrowthArgs A{c, lev, T, Lp, dir};
  const int nb = ((T + 1) * Lp + 255) / 256;
  if (record_item(IK_GROWTH, 0, nb, &A, sizeof(A))) return;
  hipLaunchKernelGGL(k_growth, dim3(nb), dim3(256), 0, s, A);
}
void launch_levels64(unsigned long long* cslots, uint32_t* slots, float* lev, int T1, int Lp, int ncslot, int nslot,
                     hipStream_t s) {
  const Levels64Args A{cslots, slots, lev, T1, Lp, ncslot, nslot};
  const int nb = (T1 * Lp + 255) / 256;
  if (record_item(IK_LEVELS64, 0, nb, &A, sizeof(A))) return;
  hipLaunchKernelGGL(k_levels64, dim3(nb), dim3(256), 0, s, A);
}
void launch_levels(uint32_t* slots, float* lev, int T1, int Lp, int nslot, hipStream_t s) {
  const LevelsArgs A{slots, lev, T1, Lp, nslot};
  const int nb = (T1 * Lp + 255) / 256;
  if (record_item(IK_LEVELS, 0, nb, &A, sizeof(A))) return;
  hipLaunchKernelGGL(k_levels, dim3(nb), dim3(256), 0, s, A);
}
void launch_reduce_stats(const double* part, int nblk0, int nblk, int stride, int T1, double* tpart, double eps,
                         double* out, hipStream_t s) {
  const Reduce1Args A{part, nblk0, nblk, stride, tpart};
  const Reduce2Args B{tpart, T1, eps, out};
  if (record_item(IK_REDUCE1, 0, T1, &A, sizeof(A))) {
    record_item(IK_REDUCE2, 0, 1, &B, sizeof(B));
    return;
  }
  hipLaunchKernelGGL(k_reduce_stats1, dim3(T1), dim3(kBlock), 0, s, A);
  hipLaunchKernelGGL(k_reduce_stats2, dim3(1), dim3(64), 0, s, B);
}
void launch_reduce_cost(const double* pflow, const double* pstate, int nblk_flow, int nblk_state, int stride, int T,
                        double* tflow, double* tstate, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_stats1, dim3(T), dim3(kBlock), 0, s,
                     Reduce1Args{pflow, nblk_flow, nblk_flow, stride, tflow});
  hipLaunchKernelGGL(k_reduce_stats1, dim3(T), dim3(kBlock), 0, s,
                     Reduce1Args{pstate, nblk_state, nblk_state, stride, tstate});
  hipLaunchKernelGGL(k_reduce_cost, dim3(1), dim3(64), 0, s, tflow, tstate, T, out);
}

// ---------------------------------------------------------------------------
// serving pool: one launch runs the next recorded item of every active solve
// (FP32 solves; items carry their own block counts, prefix[] the offsets)
// ---------------------------------------------------------------------------
static_assert(sizeof(StepArgs<float>) <= kItemArgBytes, "item argument area too small");

// LEAN: a tick whose items are all light (no check-pass step, no CSR or
// commodity-capacity step; pool_item_is_light decides on the host) runs a kernel
// without the heavy step variants, so it keeps more waves per SIMD.  A heavy step
// reaching a lean tick is a host error: it is reported through the request's
// flags, never run half-done.
template <bool LOG, bool LEAN>
__device__ __forceinline__ void run_item(const PoolItem& it, int bid) {
  const void* p = it.args;
  switch (it.kind) {
    case IK_STEP_BWD:
    case IK_STEP_FWD:
    case IK_STEP_CHK: {
      const StepArgs<float>& sa = *static_cast<const StepArgs<float>*>(p);
      // (a check-pass step is heavy: it reaches lean ticks only by a host error)
      const bool chk = it.kind == IK_STEP_CHK;
      if (chk ? (!LEAN && ell_check(sa)) : ell_fast(sa)) {
        const bool fw = it.kind == IK_STEP_FWD;
        const bool one = ell_one_chunk(sa);
#define MMOT_ELL_ITEM1(K, O)                                                          \
        do {                                                                          \
          if constexpr (!LEAN) {                                                      \
            if (chk) {                                                                \
              ell_step_body<float, LOG, true, K, O, true>(sa, bid, it.nblk);          \
              break;                                                                  \
            }                                                                         \
          }                                                                           \
          if (fw) ell_step_body<float, LOG, true, K, O>(sa, bid, it.nblk);            \
          else ell_step_body<float, LOG, false, K, O>(sa, bid, it.nblk);              \
        } while (0)
#define MMOT_ELL_ITEM(K)                                                              \
        do {                                                                          \
          if (one) MMOT_ELL_ITEM1(K, true);                                           \
          else MMOT_ELL_ITEM1(K, false);                                              \
        } while (0)
        if (sa.ellD == 16) MMOT_ELL_ITEM(16);
        else if (sa.ellD == 8) MMOT_ELL_ITEM(8);
        else if (sa.ellD == 5) MMOT_ELL_ITEM(5);
        else MMOT_ELL_ITEM(4);
#undef MMOT_ELL_ITEM
#undef MMOT_ELL_ITEM1
        break;
      }
      // 0: CSR, 1..4: ELL of width 8, 16, 5, 4, 5: CSR with commodity capacities
      const int e = sa.cw ? 5 : (sa.ellD == 8 ? 1 : sa.ellD == 16 ? 2 : sa.ellD == 5 ? 3 : sa.ellD == 4 ? 4 : 0);
      if constexpr (LEAN) {
        if (it.kind == IK_STEP_CHK || e == 5 || e == 0) {
          if (bid == 0 && threadIdx.x == 0) atomicOr(sa.flags, FLAG_NONFINITE);
          break;
        }
#define MMOT_STEP_ITEM(F, C)                                                                  \
        do {                                                                                  \
          if (e == 2) step_body<float, LOG, F, C, true, 16, false>(sa, bid, it.nblk);         \
          else if (e == 3) step_body<float, LOG, F, C, true, 5, false>(sa, bid, it.nblk);     \
          else if (e == 4) step_body<float, LOG, F, C, true, 4, false>(sa, bid, it.nblk);     \
          else step_body<float, LOG, F, C, true, 8, false>(sa, bid, it.nblk);                 \
        } while (0)
        if (it.kind == IK_STEP_BWD) MMOT_STEP_ITEM(false, false);
        else MMOT_STEP_ITEM(true, false);
#undef MMOT_STEP_ITEM
      } else {
#define MMOT_STEP_ITEM(F, C)                                                                  \
        do {                                                                                  \
          if (e == 5) step_body<float, LOG, F, C, false, 16, true>(sa, bid, it.nblk);         \
          else if (e == 2) step_body<float, LOG, F, C, true, 16, false>(sa, bid, it.nblk);    \
          else if (e == 1) step_body<float, LOG, F, C, true, 8, false>(sa, bid, it.nblk);     \
          else if (e == 3) step_body<float, LOG, F, C, true, 5, false>(sa, bid, it.nblk);     \
          else if (e == 4) step_body<float, LOG, F, C, true, 4, false>(sa, bid, it.nblk);     \
          else step_body<float, LOG, F, C, false, 16, false>(sa, bid, it.nblk);               \
        } while (0)
        if (it.kind == IK_STEP_BWD) MMOT_STEP_ITEM(false, false);
        else if (it.kind == IK_STEP_FWD) MMOT_STEP_ITEM(true, false);
        else MMOT_STEP_ITEM(true, true);
#undef MMOT_STEP_ITEM
      }
      break;
    }
    case IK_SOURCE: source_body<float, LOG>(*static_cast<const SourceArgs<float>*>(p), bid, it.nblk); break;
    case IK_CHECK0: check0_body<float, LOG>(*static_cast<const Check0Args<float>*>(p), bid, it.nblk); break;
    case IK_PREP_BWD: prep_bwd_body<float, LOG>(*static_cast<const PrepBwdArgs<float>*>(p), bid, it.nblk); break;
    case IK_PREP_FWD: prep_fwd_body<float, LOG>(*static_cast<const PrepFwdArgs<float>*>(p), bid, it.nblk); break;
    default: break;
  }
}

template <bool LEAN>
__global__ __launch_bounds__(kBlock) void k_pool_tick(const TickArgs ta) {
  int lo = 0, hi = ta.nslot - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ta.prefix[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const PoolItem& it = ta.prog[lo][ta.idx[lo]];
  const int bid = b - ta.prefix[lo];
  if (bid >= it.nblk) return;
  switch (it.kind) {
    case IK_LEVELS: levels_body(*reinterpret_cast<const LevelsArgs*>(it.args), bid, it.nblk); return;
    case IK_LEVELS64: levels64_body(*reinterpret_cast<const Levels64Args*>(it.args), bid, it.nblk); return;
    case IK_GROWTH: growth_body(*reinterpret_cast<const GrowthArgs*>(it.args), bid, it.nblk); return;
    case IK_REDUCE1: reduce1_body(*reinterpret_cast<const Reduce1Args*>(it.args), bid, it.nblk); return;
    case IK_REDUCE2: reduce2_body(*reinterpret_cast<const Reduce2Args*>(it.args), bid, it.nblk); return;
    default: break;
  }
  if (it.log_domain) run_item<true, LEAN>(it, bid);
  else run_item<false, LEAN>(it, bid);
}

void launch_pool_tick(const TickArgs& ta, bool lean, hipStream_t s) {
  if (ta.nslot > 0 && ta.prefix[ta.nslot] > 0) {
    if (lean) hipLaunchKernelGGL(k_pool_tick<true>, dim3(ta.prefix[ta.nslot]), dim3(kBlock), 0, s, ta);
    else hipLaunchKernelGGL(k_pool_tick<false>, dim3(ta.prefix[ta.nslot]), dim3(kBlock), 0, s, ta);
  }
}
// a recorded item that the lean tick runs (see run_item)
bool pool_item_is_light(const PoolItem& it) {
  if (it.kind != IK_STEP_BWD && it.kind != IK_STEP_FWD && it.kind != IK_STEP_CHK) return true;
  if (it.kind == IK_STEP_CHK) return false;
  const StepArgs<float>& sa = *reinterpret_cast<const StepArgs<float>*>(it.args);
  return !sa.cw && (sa.ellD == 16 || sa.ellD == 8 || sa.ellD == 5 || sa.ellD == 4);
}

#define MMOT_INST(V, LOG)                                                                                         \
  template void launch_step<V, LOG>(const StepArgs<V>&, int, int, hipStream_t);                                       \
  template void launch_sink_check<V, LOG>(int, int, int, int, int, const V*, const V*, const V*, const double*,    \
                                          const double*, double*, int, hipStream_t);                                 \
  template void launch_source<V, LOG>(int, int, int, int, const V*, const V*, V*, uint32_t*, int, size_t, int*,   \
                                      unsigned long long*, int, size_t, int, hipStream_t);                        \
  template void launch_check0<V, LOG>(int, int, int, int, int, const V*, const V*, const V*, const double*,      \
                                      const double*, double*, double*, double*, int, int, int, hipStream_t);     \
  template void launch_flows<V, LOG>(int, int, int, int, int, const int*, const int*, const V*, const double*,   \
                                     const V*, const V*, const V*, const V*, const double*, const double*,       \
                                     double*, double*, int, hipStream_t);                                        \
  template void launch_prep_bwd<V, LOG>(int, int, const double*, double*, V*, const double*, double*, uint32_t*,  \
                                        int, hipStream_t);                                                       \
  template void launch_prep_fwd<V, LOG>(int, int, int, const double*, double*, const double*, V*, V*, double*,    \
                                        double*, double*, uint32_t*, int, hipStream_t);
MMOT_INST(float, false)
MMOT_INST(float, true)
MMOT_INST(double, false)
MMOT_INST(double, true)

}  // namespace mmot
