// Dense-graph products of the graph-structured Sinkhorn scheme on MFMA.
//
// For a dense K (complete graph with finite costs) each message update of
// Theorem 5 is a GEMM over all commodities at once:
//   forward  hatPsi_{t+1}^T = K^T diag(u_t) (hatPsi_t (.) K_L)^T
//   backward Psi_{t-1}^T    = K   diag(u_t) (Psi_t (.) K_L)^T
// i.e. OUT[n x Lp] = A[n x n] * diag(u) * B[n x Lp] with A = K^T or K (row
// major, padded leading dimension lda) and B a state-major panel.  The
// dense-path cost is O(T L n^2) per sweep (remark after Corollary 1).
//
// Tiling for gfx950: 128 x 128 output tile per 512-thread workgroup (the
// 4096 x 1024 output of the benchmark is one tile per CU), two groups of four
// wavefronts, each group in a 2 x 2 arrangement of 64 x 64 = 2 x 2 MFMA 32x32
// tiles over half of the k-steps (two waves per SIMD).  Both
// operands reach LDS by direct 16-byte global->LDS copies through a 4-stage
// ring (k_gemm_lds): A = K or K^T as stored at setup, B = the next product's
// operand diag(u) B written by its producer (k_dense_operand / k_dense_operand32
// or the backward epilogue).  BF16: v_mfma_f32_32x32x16_bf16.  FP32:
// v_mfma_f32_32x32x2_f32 on operands whose 32-k blocks are stored interleaved so
// one 16-byte read holds a lane's values for four MFMAs.  Accumulation is FP32.
//
// Epilogue: per-column factor 2^-c (range offsets), K_L, store; for interior
// forward times the partial capacity column sums over the tile's commodities
// (sum_l out * Psi * 2^(sigma_hat + sigma)), written per column-tile and summed
// in a fixed order by k_dense_rows (deterministic); optional column levels.
#include "mmot_internal.h"
#include <hip/hip_bf16.h>
#include <math.h>
#include <type_traits>

namespace mmot {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int GBM = 128, GBN = 128, GBK = 64;
// position of k inside its 32-block in the FP32 operand layouts (the two k values
// of an MFMA k-pair sit 16 apart, so one 16-byte read holds four k-pairs)
__host__ __device__ __forceinline__ int ipos32(int k) { return (k & ~31) | ((k & 1) << 4) | ((k & 31) >> 1); }

// Epilogue of the product kernel: range factor, K_L, store, the next product's
// BF16 operand, capacity partial sums, column levels.  Two wave groups of four
// (2 x 2 over the tile) hold the whole sum; group g handles the 32-column half
// j = g of its wave's 64 x 64 quadrant.  smem: LDS that no wave reads any more
// (the operand ring), 2 * 256 + 2 * GBN floats.
constexpr int kWaveGroups = 2;
// CM: commodity-dependent capacities (see GemmArgs): 0 none, 1 w_t applied, 2 w_t
// projected (forward update) and applied
template <int CM>
__device__ __forceinline__ void gemm_epilogue(const GemmArgs& a, f32x16 (&acc)[2][2], int row0, int col0, int bn,
                                              int logical, float* smem) {
  // red[g][wm][wn][64]: capacity partial sums across the column waves (and groups)
  float (*red)[2][2][64] = reinterpret_cast<float (*)[2][2][64]>(smem);
  float (*cmx)[GBN] = reinterpret_cast<float (*)[GBN]>(smem + kWaveGroups * 2 * 2 * 64);   // column maxima
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int grp = wave >> 2, wq = wave & 3;
  const int wm = wq >> 1, wn = wq & 1;
  const int lr = lane & 31, lh = lane >> 5;
  (void)lane;
  float colmax[2] = {-INFINITY, -INFINITY};
  float rsum[2][16];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) rsum[i][r] = 0.f;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (j != grp) continue;
    const int gc = col0 + wn * 64 + j * 32 + lr;
    const bool cok = gc < a.Lp;
    const int gcc = cok ? gc : 0;
    const float f = cok ? a.fac[gcc] : 0.f;
    const bool capc = a.cap && gc < a.L;
    const float g = capc ? a.wgt[gcc] : 0.f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      // operands of the epilogue, loaded unconditionally (clamped) before use
      float klv[16], wv[16], uov[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int gr = row0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
        const int grc = gr < a.n ? gr : a.n - 1;
        const size_t off = (size_t)grc * a.Lp + gcc;
        klv[r] = a.kl ? a.kl[off] : 1.f;
        wv[r] = a.cap ? a.wpan[off] : 0.f;
        uov[r] = a.bout ? a.uo[grc] : 0.f;
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int gr = row0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
        const bool ok = cok && gr < a.n;
        const size_t off = (size_t)gr * a.Lp + gc;
        const float o = acc[i][j][r] * f;
        float z = a.kl ? o * klv[r] : o;
        if constexpr (CM) {
          // w_t multiplied into the stored output; at a forward update first projected
          // (before u_t, with the u_t of the last sweep): w = min(D / (P_{0,t} u_t), 1),
          // 0 where D = 0, in the multiplicative form w_old D / (P_{0,t} u_t) with
          // P_{0,t} taken with w_old (folded into the stored backward panel)
          const int grc = gr < a.n ? gr : a.n - 1;
          const size_t offc = (size_t)grc * a.Lp + gcc;
          const float cw = a.cw[offc];
          float wn = cw;
          if (CM == 2 && capc) {
            const float dc = a.dc[offc];
            const float q = o * wv[r] * g;
            const float qu = q * a.ucur[grc], lim = cw * dc;
            wn = (dc == 0.f) ? 0.f : ((qu <= lim) ? 1.f : lim / qu);
            if (ok) {
              a.cwo[off] = wn;
              rsum[i][r] += (cw > 0.f) ? q * (wn / cw) : 0.f;
            }
          } else if (ok && capc) {
            rsum[i][r] = fmaf(o * wv[r], g, rsum[i][r]);
          }
          z *= wn;
        } else {
          if (ok && capc) rsum[i][r] = fmaf(o * wv[r], g, rsum[i][r]);
        }
        if (ok) a.out[off] = z;
        if (ok && z > 0.f) colmax[j] = fmaxf(colmax[j], z);
        if (a.pcomm && ok && capc && (unsigned)(gc - a.pc_lo) < (unsigned)a.pc_cnt) {
          const double P = (double)o * (double)wv[r] * (double)g * (double)a.ucur[gr];
          a.pcomm[(size_t)(gc - a.pc_lo) * a.n + gr] = P;
        }
      }
      if (a.bout && cok) {
        // next product's operand: bf16(u (.) stored value), k-blocked; the four rows
        // r = 4q..4q+3 of this lane are consecutive within one block of 8
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int g0 = row0 + wm * 64 + i * 32 + 8 * q;          // multiple of 8
          if (g0 >= a.n) continue;
          bf16x4 p;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int r = 4 * q + e;
            const int gr = g0 + 4 * lh + e;
            const float o = acc[i][j][r] * f;
            float z = a.kl ? o * klv[r] : o;
            if constexpr (CM) {   // (backward products only: w_t as stored)
              const int grc = gr < a.n ? gr : a.n - 1;
              z *= a.cw[(size_t)grc * a.Lp + gc];
            }
            p[e] = (__bf16)(gr < a.n ? z * uov[r] : 0.f);
          }
          *reinterpret_cast<bf16x4*>(a.bout + ((size_t)(g0 >> 3) * a.Lp + gc) * 8 + 4 * lh) = p;
        }
      }
    }
  }
  if (a.cap) {
    // reduce over the 32 lanes that share rows (same lane half), then over the two column waves
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        float v = rsum[i][r];
        for (int m = 16; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
        rsum[i][r] = v;
      }
    if (lr == 0) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) red[grp][wm][wn][i * 32 + 8 * (r >> 2) + 4 * lh + (r & 3)] = rsum[i][r];
    }
    __syncthreads();
    if (tid < 128) {
      const int wmr = tid >> 6, rr = tid & 63;
      const int gr = row0 + wmr * 64 + rr;
      const float v = red[0][wmr][0][rr] + red[0][wmr][1][rr] + red[1][wmr][0][rr] + red[1][wmr][1][rr];
      if (gr < a.n) a.part_s[(size_t)bn * a.n + gr] = v;
    }
  }
  if (a.slots) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (j != grp) continue;
      float m = colmax[j];
      m = fmaxf(m, __shfl_xor(m, 32, 64));
      if (lh == 0) cmx[wm][wn * 64 + j * 32 + lr] = m;
    }
    __syncthreads();
    if (tid < GBN) {
      const float m = fmaxf(cmx[0][tid], cmx[1][tid]);
      const int gc = col0 + tid;
      if (gc < a.Lp && m > 0.f)
        atomicMax(a.slots + (size_t)(logical % a.nslot) * a.slot_stride + gc, enc_f32(log2f(m)));
    }
  }
}

// ---------------------------------------------------------------------------
// Products with both operands prepared (A = K or K^T, B = the pre-scaled
// operand): a four-stage ring of LDS buffers filled by direct global->LDS
// 16-byte loads (no registers in between), so three K-stages are in flight
// while one is on the matrix cores.  Tile 128 x 128, two groups of four waves
// 2 x 2, K-depth 64 (BF16) or 32 (FP32) per stage.  Rows of a stage are 8 chunks of 16
// bytes; chunk c of row r sits at slot 8r + (c ^ ((r >> 1) & 7)), which keeps
// the MFMA operand reads of 16 consecutive rows on distinct LDS banks.  The K
// extent is padded with zeros to a multiple of 64 in both operands (lda and
// the operand's row count), so every stage loads inside the buffers; rows and
// columns past the matrix read clamped addresses and only feed outputs that
// the epilogue discards.
// ---------------------------------------------------------------------------
constexpr int kStages = 4;
constexpr int kSlots = GBM * GBK / 8;   // 16-byte slots per operand per stage

__device__ __forceinline__ int swz_slot(int r, int c) { return r * 8 + (c ^ ((r >> 1) & 7)); }

// One direct global->LDS copy of 16 bytes per lane: lane l writes LDS bytes
// [lds_byte + 16 l, lds_byte + 16 l + 16).  Written as asm so that the compiler
// does not make every later LDS read wait for all copies in flight (it cannot
// tell the ring slots apart); the kernel orders them with explicit waits.  The
// instruction writes LDS only, no registers.
__device__ __forceinline__ void lds_copy16(const void* g, uint32_t lds_byte) {
  asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(g), "s"(lds_byte) : "memory", "m0");
}
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// s_waitcnt immediate: wait until at most n vector-memory operations are outstanding
template <int N>
__device__ __forceinline__ void wait_vm() {
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// The product kernel.  F32 = false: BF16 products (v_mfma_f32_32x32x16_bf16), a
// stage is 64 k (four steps of 16), the B operand Bb k-blocked by 8.  F32 = true:
// FP32 products (v_mfma_f32_32x32x2_f32), a stage is 32 k (four steps of four
// k-pairs); A (the FP32 K) and the B operand B32 hold each 32-k block interleaved
// (position (k%2)*16 + k/2), so the 16 bytes a lane reads are its values for four
// consecutive MFMAs, and each stage is summed into fresh accumulators that are
// added once per stage (blocked summation keeps the FP32 rounding of the long K
// sums small).  Either way a stage row is 128 bytes.
//
// Two groups of four waves per tile (eight waves, two per SIMD): each group
// computes the whole 128 x 128 tile 2 x 2 (64 x 64 per wave) over half of every
// stage's steps (group g: steps 2g and 2g+1), so while one wave of a SIMD waits
// for its LDS reads or at the stage barrier the other can issue MFMAs (one group
// of four waves took 53.2 us per BF16 product, two take 50.3 us).  At the end
// each group posts the 32-column half that the other group stores, adds the half
// it keeps, and the two groups share the epilogue.
template <bool F32, int CM>
__global__ __launch_bounds__(512) void k_gemm_lds(GemmArgs a) {
  constexpr int KS = F32 ? 32 : 64;          // k per stage
  constexpr int ES = F32 ? 4 : 2;            // element bytes
  __shared__ uint4 lds[kStages][2][kSlots];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int grp = wave >> 2, wq = wave & 3;
  const int wm = wq >> 1, wn = wq & 1;
  const int nbm = gridDim.x, nbn = gridDim.y;
  const int hw = blockIdx.y * nbm + blockIdx.x;
  const int tot = nbm * nbn;
  int logical = hw;
  if ((tot & 7) == 0) logical = (hw & 7) * (tot >> 3) + (hw >> 3);
  const int bn = logical % nbn, bm = logical / nbn;
  const int row0 = bm * GBM, col0 = bn * GBN;
  const char* A = static_cast<const char*>(a.A);
  const char* B = F32 ? reinterpret_cast<const char*>(a.B32) : reinterpret_cast<const char*>(a.Bb);

  // this lane's two slots per operand and stage (byte offsets at k0 = 0)
  size_t aoff[2], boff[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int slot = (wave * 2 + q) * 64 + lane;
    const int r = slot >> 3, c = (slot & 7) ^ ((r >> 1) & 7);
    const int gr = min(row0 + r, a.n - 1), gc = min(col0 + r, a.Lp - 1);
    aoff[q] = ((size_t)gr * a.lda) * ES + c * 16;
    boff[q] = F32 ? ((size_t)gc * 32) * 4 + c * 16              // + (k0/32) Lp 32 floats
                  : ((size_t)c * a.Lp + gc) * 16;               // + (k0/8) Lp 8 bf16
  }
  const size_t bstage = (size_t)a.Lp * (F32 ? 32 * 4 : 8 * 8 * 2);   // bytes per stage of B
  auto issue = [&](int st, int kt) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      lds_copy16(A + aoff[q] + (size_t)kt * KS * ES, lds_addr(&lds[st][0][(wave * 2 + q) * 64]));
      lds_copy16(B + boff[q] + (size_t)kt * bstage, lds_addr(&lds[st][1][(wave * 2 + q) * 64]));
    }
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int nk = (a.n + KS - 1) / KS;
  for (int st = 0; st < kStages - 1 && st < nk; ++st) issue(st, st);
  const int lr = lane & 31, lh = lane >> 5;
  for (int kt = 0; kt < nk; ++kt) {
    // stage kt has landed once at most the later stages' copies (4 per stage and
    // thread) are outstanding; the barrier extends that to the block and frees
    // the ring slot read in the previous stage
    const int later = min(kStages - 2, nk - 1 - kt);
    if (later >= 2) wait_vm<8>();
    else if (later == 1) wait_vm<4>();
    else wait_vm<0>();
    asm volatile("s_barrier" ::: "memory");
    if (kt + kStages - 1 < nk) issue((kt + kStages - 1) % kStages, kt + kStages - 1);
    const uint4* as = lds[kt % kStages][0];
    const uint4* bs = lds[kt % kStages][1];
    // both of this group's steps read at once; BF16: step ks covers 16 k (chunks
    // 2 ks + lh); FP32: step ks covers 4 k-pairs (chunk 4 lh + ks of the
    // interleaved row)
    uint4 af[2][2], bf[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int ks = grp * 2 + h;
      const int ch = F32 ? lh * 4 + ks : ks * 2 + lh;
#pragma unroll
      for (int i = 0; i < 2; ++i) af[h][i] = as[swz_slot(wm * 64 + i * 32 + lr, ch)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[h][j] = bs[swz_slot(wn * 64 + j * 32 + lr, ch)];
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (F32) {
      // the stage's products summed apart and added once (blocked summation)
      f32x16 sacc[2][2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) sacc[i][j][r] = 0.f;
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              const uint4 av = af[h][i], bv = bf[h][j];
              const uint32_t aq = q == 0 ? av.x : q == 1 ? av.y : q == 2 ? av.z : av.w;
              const uint32_t bq = q == 0 ? bv.x : q == 1 ? bv.y : q == 2 ? bv.z : bv.w;
              sacc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(aq), __uint_as_float(bq),
                                                                sacc[i][j], 0, 0, 0);
            }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] += sacc[i][j];
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, af[h][i]),
                                                                __builtin_bit_cast(bf16x8, bf[h][j]), acc[i][j], 0,
                                                                0, 0);
    }
  }
  // group g keeps column half j = g of its quadrant: it posts its half 1 - g (two
  // 32 x 32 tiles, 8 KB per wave) and adds the other group's half g
  __syncthreads();
  float4* rbuf = reinterpret_cast<float4*>(&lds[0][0][0]);
  auto post = [&](auto jc) {
    constexpr int J = decltype(jc)::value;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        rbuf[((wave * 2 + i) * 4 + r) * 64 + lane] =
            make_float4(acc[i][J][4 * r], acc[i][J][4 * r + 1], acc[i][J][4 * r + 2], acc[i][J][4 * r + 3]);
  };
  auto take = [&](auto jc) {
    constexpr int J = decltype(jc)::value;
    const int src = (1 - grp) * 4 + wq;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float4 v = rbuf[((src * 2 + i) * 4 + r) * 64 + lane];
        acc[i][J][4 * r] += v.x;
        acc[i][J][4 * r + 1] += v.y;
        acc[i][J][4 * r + 2] += v.z;
        acc[i][J][4 * r + 3] += v.w;
      }
  };
  if (grp == 0) post(std::integral_constant<int, 1>{});
  else post(std::integral_constant<int, 0>{});
  __syncthreads();
  if (grp == 0) take(std::integral_constant<int, 0>{});
  else take(std::integral_constant<int, 1>{});
  __syncthreads();
  gemm_epilogue<CM>(a, acc, row0, col0, bn, logical, reinterpret_cast<float*>(&lds[0][0][0]));
}

// ---------------------------------------------------------------------------
// row kernels of the dense path
// ---------------------------------------------------------------------------
// The block's statistics partial: each of the kNSt values summed (the capacity
// violation maximised) over the 256 threads, within each wave by shuffles, then
// over the four waves in order; thread k writes part[block][k].
__device__ __forceinline__ void block_partials(const double (&st)[kNSt], double* part) {
  __shared__ double red[4][kNSt];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kNSt; ++k) {
    double v = st[k];
    for (int m = 32; m > 0; m >>= 1) {
      const double o = __shfl_xor(v, m, 64);
      v = (k == ST_CAP_VIOL) ? fmax(v, o) : v + o;
    }
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < kNSt) {
    const int k = threadIdx.x;
    double v = red[0][k];
    for (int w = 1; w < 4; ++w) v = (k == ST_CAP_VIOL) ? fmax(v, red[w][k]) : v + red[w][k];
    part[(size_t)blockIdx.x * kNSt + k] = v;
  }
}
// capacity update (Corollary 1 + Proposition 1) from the column-tile partial
// sums: s_j = sum_p part_s[p][j]; update: u_j = 1 if s_j <= d_j else d_j / s_j;
// check: occupancy u_j s_j and the capacity / dual / gap statistics.
__global__ void k_dense_rows(int n, int ntn, const float* __restrict__ part_s, const float* __restrict__ cap,
                             float* __restrict__ u, int update, double* part, double* occ,
                             const double* __restrict__ cc, int ncc) {
  double st[kNSt] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (cc && blockIdx.x == 0) {
    // the commodity-capacity terms of the product's blocks (check pass), folded into block 0
    for (int b = threadIdx.x; b < ncc; b += blockDim.x) {
      st[ST_CAP_VIOL] = fmax(st[ST_CAP_VIOL], cc[(size_t)b * kNSt + ST_CAP_VIOL]);
      st[ST_DUAL] += cc[(size_t)b * kNSt + ST_DUAL];
      st[ST_GAP] += cc[(size_t)b * kNSt + ST_GAP];
    }
  }
  const int per = (n + gridDim.x - 1) / gridDim.x;
  const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
  for (int j = r0 + threadIdx.x; j < r1; j += blockDim.x) {
    float s = 0.f;
    for (int p = 0; p < ntn; ++p) s += part_s[(size_t)p * n + j];
    const float d = cap[j];
    if (update) {
      u[j] = (s <= d) ? 1.f : d / s;
    } else {
      const double uu = (double)u[j], occv = uu * (double)s, dd = (double)d, lnu = log(uu);
      st[ST_MASS] += occv;
      if (isfinite(dd)) {
        st[ST_CAP_VIOL] = fmax(st[ST_CAP_VIOL], fmax(occv - dd, 0.0) / dd);
        st[ST_DUAL] += dd * lnu;
        st[ST_GAP] += lnu * (occv - dd);
      }
      if (!isfinite(occv)) st[ST_NONFINITE] += 1.0;
      if (occ) occ[j] = occv;
    }
  }
  if (part) block_partials(st, part);
}

// The capacity update of the R rows r0.. (as in k_dense_rows, same order of the
// partial sums, so the same u) computed inside an operand kernel: into LDS for
// the block, and into u by the blocks of the first column range.  Every thread
// of the block reaches the barrier.
template <int R>
__device__ __forceinline__ void rows_update(int n, int ntn, const float* __restrict__ part_s,
                                            const float* __restrict__ cap, float* __restrict__ u, int r0,
                                            float* us) {
  if ((int)threadIdx.x < R) {
    const int j = r0 + threadIdx.x;
    float uj = 0.f;
    if (j < n) {
      float s = 0.f;
      for (int p = 0; p < ntn; ++p) s += part_s[(size_t)p * n + j];
      const float d = cap[j];
      uj = (s <= d) ? 1.f : d / s;
      if (blockIdx.y == 0) u[j] = uj;
    }
    us[threadIdx.x] = uj;
  }
  __syncthreads();
}

// BF16 operand of the next product, bf16(u_j x_j) k-blocked (element (j, c) at
// ((j/8) Lp + c) 8 + j%8), one 16-byte store per k-block and column; rows past n
// (the zero padding of the last k-block) store 0.  u == nullptr: no scaling (the
// first product of a sweep, which reads U0T or U01).  part_s != nullptr: the
// capacity update of the block's rows is done here first (u written, then used).
__global__ void k_dense_operand(int n, int Lp, const float* __restrict__ x, const float* __restrict__ u,
                                uint16_t* __restrict__ bout, int ntn, const float* __restrict__ part_s,
                                const float* __restrict__ cap, float* __restrict__ uw) {
  const int kb = blockIdx.x, c = blockIdx.y * blockDim.x + threadIdx.x;
  __shared__ float us[8];
  // the panel values are requested before the update's partial sums, so both are in flight together
  const int cc = c < Lp ? c : Lp - 1;
  float xv[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int j = kb * 8 + e;
    xv[e] = x[(size_t)(j < n ? j : n - 1) * Lp + cc];
  }
  if (part_s) rows_update<8>(n, ntn, part_s, cap, uw, kb * 8, us);
  if (c >= Lp) return;
  bf16x8 p;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int j = kb * 8 + e;
    const int jc = j < n ? j : n - 1;
    const float sc = part_s ? us[e] : (u ? u[jc] : 1.f);
    p[e] = (j < n) ? (__bf16)(xv[e] * sc) : (__bf16)0.f;
  }
  *reinterpret_cast<bf16x8*>(bout + ((size_t)kb * Lp + c) * 8) = p;
}

// sink update U0T = R0T ./ hatPsi_T (Algorithm 2) from the stored product
// (update), or the sink statistics P_{0,T} = U0T (.) hatPsi_T (check).  Row
// blocks as k_dense_rows; each thread owns commodity columns and walks the
// block's rows, so the column levels of the new U0T (slotsE) and of hatPsi_T
// (slots_o, calibration) cost one atomic per block and column.
__global__ void k_dense_sink(int n, int Lp, int L, const float* __restrict__ hat, const float* __restrict__ rdst,
                             float* __restrict__ u0t, int update, const double* __restrict__ sigT,
                             const double* __restrict__ sighT, uint32_t* slotsE, int nslot, uint32_t* slots_o,
                             size_t stride_o, int* flags, double* part, double* occ, double* pcomm, int pc_lo,
                             int pc_cnt) {
  double st[kNSt] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int per = (n + gridDim.x - 1) / gridDim.x;
  const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
  for (int l = threadIdx.x; l < Lp; l += blockDim.x) {
    float cz = -INFINITY, co = -INFINITY;
    const double sg = (l < L) ? sigT[l] + sighT[l] : 0.0;
    for (int j = r0; j < r1; ++j) {
      const size_t off = (size_t)j * Lp + l;
      const float o = hat[off], r = rdst[off];
      if (update) {
        float z = 0.f;
        if (r > 0.f) {
          if (!(o > 0.f)) atomicOr(flags, FLAG_INFEASIBLE);
          z = r / o;
        }
        u0t[off] = z;
        if (z > 0.f) cz = fmaxf(cz, log2f(z));
        if (o > 0.f) co = fmaxf(co, log2f(o));
      } else if (l < L) {
        const float z = u0t[off];
        const double P = (double)z * (double)o * exp2(sg);
        const double lnU = (z > 0.f) ? (log2((double)z) + sigT[l]) * M_LN2 : 0.0;
        st[ST_MASS] += P;
        st[ST_DUAL] += (double)r * lnU;
        st[ST_GAP] += lnU * (P - (double)r);
        if (pcomm && (unsigned)(l - pc_lo) < (unsigned)pc_cnt) pcomm[(size_t)(l - pc_lo) * n + j] = P;
      }
    }
    if (update && r1 > r0) {
      if (cz > -INFINITY) atomicMax(slotsE + (size_t)(blockIdx.x % nslot) * Lp + l, enc_f32(cz));
      if (slots_o && co > -INFINITY) atomicMax(slots_o + (size_t)(blockIdx.x % nslot) * stride_o + l, enc_f32(co));
    }
  }
  if (!update && occ) {
    // one wavefront per row, lanes over commodities (fixed order)
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int j = r0 + w; j < r1; j += nw) {
      double s = 0;
      for (int l = lane; l < L; l += 64)
        s += (double)u0t[(size_t)j * Lp + l] * (double)hat[(size_t)j * Lp + l] * exp2(sigT[l] + sighT[l]);
      for (int m = 32; m > 0; m >>= 1) s += __shfl_xor(s, m, 64);
      if (lane == 0) occ[j] = s;
    }
  }
  if (part) block_partials(st, part);
}

// ---------------------------------------------------------------------------
// setup: dense K = exp(-C/eps) (+inf -> 0), its transpose, BF16 copies
// ---------------------------------------------------------------------------
__global__ void k_dense_gibbs(const double* __restrict__ C, int n, int lda, double eps, float* __restrict__ K,
                              float* __restrict__ Kt, __bf16* __restrict__ Kb, __bf16* __restrict__ Ktb) {
  __shared__ float tile[32][33];
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + r, j = j0 + tx;
    float v = 0.f;
    if (i < n && j < n) {
      const double c = C[(size_t)i * n + j];
      v = isinf(c) ? 0.f : (float)exp(-c / eps);
    }
    tile[r][tx] = v;
    if (i < n && j < lda) {
      K[(size_t)i * lda + ipos32(j)] = v;
      if (Kb) Kb[(size_t)i * lda + j] = (__bf16)v;
    }
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int j = j0 + r, i = i0 + tx;   // Kt[j][i] = K[i][j]
    if (j < n && i < lda) {
      const float v = (i < n) ? tile[tx][r] : 0.f;
      Kt[(size_t)j * lda + ipos32(i)] = v;
      if (Ktb) Ktb[(size_t)j * lda + i] = (__bf16)v;
    }
  }
}

__global__ void k_dense_rowsum_max(const float* __restrict__ K, int n, int lda, uint32_t* out) {
  const int i = blockIdx.x;
  __shared__ double red[256];
  double s = 0;
  for (int j = threadIdx.x; j < lda; j += blockDim.x) s += (double)K[(size_t)i * lda + j];   // (zero padding)
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] > 0) atomicMax(out, enc_f32((float)log2(red[0])));
}

// launchers
void launch_dense_operand(int n, int Lp, const float* x, const float* u, uint16_t* bout, hipStream_t s);
void launch_dense_operand32(int n, int n8, int Lp, const float* x, const float* u, float* bout, hipStream_t s);
void launch_gemm(const GemmArgs& a, bool bf16, hipStream_t s) {
  dim3 grid((a.n + GBM - 1) / GBM, (a.Lp + GBN - 1) / GBN);
  // (one variant per commodity-capacity mode: the projection's loads and division
  // in the one kernel that needs them keep the others' registers)
  if (a.cw && a.cc_update) {
    if (bf16) hipLaunchKernelGGL((k_gemm_lds<false, 2>), grid, dim3(512), 0, s, a);
    else hipLaunchKernelGGL((k_gemm_lds<true, 2>), grid, dim3(512), 0, s, a);
  } else if (a.cw) {
    if (bf16) hipLaunchKernelGGL((k_gemm_lds<false, 1>), grid, dim3(512), 0, s, a);
    else hipLaunchKernelGGL((k_gemm_lds<true, 1>), grid, dim3(512), 0, s, a);
  } else {
    if (bf16) hipLaunchKernelGGL((k_gemm_lds<false, 0>), grid, dim3(512), 0, s, a);
    else hipLaunchKernelGGL((k_gemm_lds<true, 0>), grid, dim3(512), 0, s, a);
  }
}
int gemm_col_tiles(int Lp) { return (Lp + GBN - 1) / GBN; }
__global__ void k_dense_operand32(int n, int Lp, const float* __restrict__ x, const float* __restrict__ u,
                                  float* __restrict__ bout, int ntn, const float* __restrict__ part_s,
                                  const float* __restrict__ cap, float* __restrict__ uw);
void launch_dense_rows(int n, int ntn, const float* part_s, const float* cap, float* u, int update, double* part,
                       double* occ, const float* x, uint16_t* bout, float* bout32, int n8, int Lp, int nblk,
                       const double* cc, int ncc, hipStream_t s) {
  // an update that feeds a next product is done by the operand kernel itself (one
  // launch); statistics come as one partial per block of the check pass's fixed
  // grid, and an update alone needs one thread per state
  if (update && !part && (bout || bout32)) {
    if (bout)
      hipLaunchKernelGGL(k_dense_operand, dim3((n + 7) / 8, (Lp + 255) / 256), dim3(256), 0, s, n, Lp, x, u, bout,
                         ntn, part_s, cap, u);
    else
      hipLaunchKernelGGL(k_dense_operand32, dim3(n8 / 32, (Lp + 255) / 256), dim3(256), 0, s, n, Lp, x, u, bout32,
                         ntn, part_s, cap, u);
    return;
  }
  const int g = part ? nblk : (n + 255) / 256;
  hipLaunchKernelGGL(k_dense_rows, dim3(g), dim3(256), 0, s, n, ntn, part_s, cap, u, update, part, occ, cc, ncc);
  // the next product's operand, u_j x_j in BF16 or FP32, once u is final
  if (bout) launch_dense_operand(n, Lp, x, u, bout, s);
  if (bout32) launch_dense_operand32(n, n8, Lp, x, u, bout32, s);
}
// FP32 operand of the next product, u_j x_j in 32-row blocks per column with the
// rows of a block interleaved (element (j, c) at ((j/32) Lp + c) 32 + ipos32(j%32));
// rows past n store 0.  One thread per (block, column): 32 loads down the column,
// eight 16-byte stores.
__global__ void k_dense_operand32(int n, int Lp, const float* __restrict__ x, const float* __restrict__ u,
                                  float* __restrict__ bout, int ntn, const float* __restrict__ part_s,
                                  const float* __restrict__ cap, float* __restrict__ uw) {
  const int kb = blockIdx.x, c = blockIdx.y * blockDim.x + threadIdx.x;
  __shared__ float us[32];
  // the panel values are requested before the update's partial sums, so both are in flight together
  const int cc = c < Lp ? c : Lp - 1;
  float xv[32];
#pragma unroll
  for (int e = 0; e < 32; ++e) {
    const int j = kb * 32 + e;
    xv[e] = x[(size_t)(j < n ? j : n - 1) * Lp + cc];
  }
  if (part_s) rows_update<32>(n, ntn, part_s, cap, uw, kb * 32, us);
  if (c >= Lp) return;
  float v[32];
#pragma unroll
  for (int e = 0; e < 32; ++e) {
    const int j = kb * 32 + e;
    const int jc = j < n ? j : n - 1;
    const float y = xv[e] * (part_s ? us[e] : (u ? u[jc] : 1.f));
    v[ipos32(e)] = (j < n) ? y : 0.f;
  }
  float4* o = reinterpret_cast<float4*>(bout + ((size_t)kb * Lp + c) * 32);
#pragma unroll
  for (int q = 0; q < 8; ++q) o[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
}
void launch_dense_operand32(int n, int n8, int Lp, const float* x, const float* u, float* bout, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_operand32, dim3(n8 / 32, (Lp + 255) / 256), dim3(256), 0, s, n, Lp, x, u, bout, 0,
                     nullptr, nullptr, nullptr);
}
void launch_dense_operand(int n, int Lp, const float* x, const float* u, uint16_t* bout, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_operand, dim3((n + 7) / 8, (Lp + 255) / 256), dim3(256), 0, s, n, Lp, x, u, bout, 0,
                     nullptr, nullptr, nullptr);
}
void launch_dense_sink(int n, int Lp, int L, const float* hat, const float* rdst, float* u0t, int update,
                       const double* sigT, const double* sighT, uint32_t* slotsE, int nslot, uint32_t* slots_o,
                       size_t stride_o, int* flags, double* part, double* occ, double* pcomm, int pc_lo,
                       int pc_cnt, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_sink, dim3(nblk), dim3(256), 0, s, n, Lp, L, hat, rdst, u0t, update, sigT, sighT,
                     slotsE, nslot, slots_o, stride_o, flags, part, occ, pcomm, pc_lo, pc_cnt);
}
void launch_dense_gibbs(const double* C, int n, int lda, double eps, float* K, float* Kt, void* Kb, void* Ktb,
                        hipStream_t s) {
  // both grid dimensions cover lda, so the zero padding columns of K^T are written too
  dim3 grid((lda + 31) / 32, (lda + 31) / 32);
  hipLaunchKernelGGL(k_dense_gibbs, grid, dim3(256), 0, s, C, n, lda, eps, K, Kt, static_cast<__bf16*>(Kb),
                     static_cast<__bf16*>(Ktb));
}
void launch_dense_rowsum_max(const float* K, int n, int lda, uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_rowsum_max, dim3(n), dim3(256), 0, s, K, n, lda, out);
}

// ---------------------------------------------------------------------------
// outputs of a dense network: edge flows and transport cost
// ---------------------------------------------------------------------------
// Commodity factors of the flows at one time: the offsets of the two panels
// (sa of A_t, sb of B_{t+1}, log2 units, FP64) split into two powers of two,
// one per operand, so that neither factor leaves the FP32 range alone; zero for
// the padding commodities l >= L.
__global__ void k_flow_factors(const double* __restrict__ sa, const double* __restrict__ sb, int L, int Lp,
                               float* __restrict__ fa, float* __restrict__ fb) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= Lp) return;
  if (l >= L) { fa[l] = 0.f; fb[l] = 0.f; return; }
  const double sg = sa[l] + sb[l];
  const double ha = floor(0.5 * sg);
  fa[l] = (float)exp2(ha);
  fb[l] = (float)exp2(sg - ha);
}

// Edge flows of one time step (Theorem 5, eq. proj_discrete_bi) on a dense
// network: F[i][j] = K_ij ua[i] ub[j] sum_l A[i][l] B[j][l] fa[l] fb[l], the
// sum over commodities on MFMA (v_mfma_f32_32x32x2f32).  Both panels are
// state-major ([n][Lp], commodities contiguous), so the product is A B^T with
// the commodity as the contraction index; the two halves of a wave take the
// first and the second four of every eight commodities (the order of the sum is
// free), so each 16-byte load feeds four MFMA steps.  A block of four waves
// owns 128 x 128 tiles of F (a wave 64 x 64: 2 x 2 MFMA tiles), taking tiles
// b, b + nblk, ...; it writes F as doubles (row-major n x n, zero where K_ij = 0)
// and its share of the move costs sum_ij C_ij F_ij (C_ij = -eps ln K_ij) into
// field 0 of its stats partial.
__global__ __launch_bounds__(256) void k_dense_flows(int n, int Lp, int lda, const float* __restrict__ A,
                                                      const float* __restrict__ ua, const float* __restrict__ B,
                                                      const float* __restrict__ ub, const float* __restrict__ fa,
                                                      const float* __restrict__ fb, const float* __restrict__ K,
                                                      double eps, double* __restrict__ flow, double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1, lr = lane & 31, lh = lane >> 5;
  const int nt = (n + 127) >> 7;
  double cost = 0.0;
  for (int tile = blockIdx.x; tile < nt * nt; tile += gridDim.x) {
    const int i0 = (tile / nt) * 128 + wm * 64, j0 = (tile % nt) * 128 + wn * 64;
    int ra[2], rb[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      ra[q] = min(i0 + q * 32 + lr, n - 1);
      rb[q] = min(j0 + q * 32 + lr, n - 1);
    }
    f32x16 acc[2][2];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[q][p][r] = 0.f;
    for (int l0 = 0; l0 < Lp; l0 += 8) {
      const int lc = l0 + 4 * lh;
      const bool lok = lc < Lp;           // Lp is a multiple of 4, not always of 8
      const int lcc = lok ? lc : 0;
      const float4 f4a = *reinterpret_cast<const float4*>(fa + lcc);
      const float4 f4b = *reinterpret_cast<const float4*>(fb + lcc);
      float4 av[2], bv[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        av[q] = *reinterpret_cast<const float4*>(A + (size_t)ra[q] * Lp + lcc);
        bv[q] = *reinterpret_cast<const float4*>(B + (size_t)rb[q] * Lp + lcc);
      }
      const float m = lok ? 1.f : 0.f;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        av[q].x *= f4a.x * m; av[q].y *= f4a.y * m; av[q].z *= f4a.z * m; av[q].w *= f4a.w * m;
        bv[q].x *= f4b.x; bv[q].y *= f4b.y; bv[q].z *= f4b.z; bv[q].w *= f4b.w;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            const float x = s == 0 ? av[q].x : s == 1 ? av[q].y : s == 2 ? av[q].z : av[q].w;
            const float y = s == 0 ? bv[p].x : s == 1 ? bv[p].y : s == 2 ? bv[p].z : bv[p].w;
            acc[q][p] = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, acc[q][p], 0, 0, 0);
          }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int j = j0 + p * 32 + lr;
        const bool jok = j < n;
        const double ubj = jok ? (double)ub[j] : 0.0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = i0 + q * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
          if (!jok || i >= n) continue;
          const float kij = K[(size_t)i * lda + ipos32(j)];
          const double F = (double)kij * (double)ua[i] * ubj * (double)acc[q][p][r];
          flow[(size_t)i * n + j] = F;
          if (F > 0.0) cost += -eps * log((double)kij) * F;
        }
      }
  }
  // block partial of the move costs (waves in order)
  __shared__ double red[4];
  for (int m = 32; m > 0; m >>= 1) cost += __shfl_xor(cost, m, 64);
  if (lane == 0) red[wave] = cost;
  __syncthreads();
  if (threadIdx.x == 0) {
    part[(size_t)blockIdx.x * kNSt] = ((red[0] + red[1]) + red[2]) + red[3];
    part[(size_t)blockIdx.x * kNSt + ST_SCOST] = 0.0;   // (the state-cost kernel, where it runs, follows)
  }
}

// State costs of one interior time on a dense network: sum_{i,l} C_L[i][l]
// P_{0,t}[l][i], P_{0,t} = hatPsi_t (.) Psi_t (.) K_L (.) w_t (.) u_t (eq. proj_0t) with
// zh = hatPsi_t (.) K_L (.) w_t and psi = Psi_t (.) K_L (.) w_t as stored (w_t the
// commodity-capacity scaling, cw == nullptr: none) and C_L = -eps ln K_L, into field
// ST_SCOST of the block partials (nblk blocks, grid-stride, fixed order).
__global__ __launch_bounds__(256) void k_dense_state_cost(int n, int L, int Lp, const float* __restrict__ zh,
                                                           const float* __restrict__ psi, const float* __restrict__ kl,
                                                           const float* __restrict__ cw,
                                                           const float* __restrict__ u, const double* __restrict__ sa,
                                                           const double* __restrict__ sb, double eps,
                                                           double* __restrict__ part) {
  double c = 0.0;
  const size_t total = (size_t)n * Lp;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / Lp), l = (int)(e % Lp);
    if (l >= L) continue;
    const double k = (double)kl[e], w = cw ? (double)cw[e] : 1.0;
    if (!(k > 0.0) || !(w > 0.0)) continue;
    const double P = (double)zh[e] * (double)psi[e] / (k * w) * (double)u[i] * exp2(sa[l] + sb[l]);
    if (P > 0.0) c += -eps * log(k) * P;
  }
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int m = 32; m > 0; m >>= 1) c += __shfl_xor(c, m, 64);
  if (lane == 0) red[wave] = c;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)blockIdx.x * kNSt + ST_SCOST] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Commodity-capacity statistics of one interior time on a dense network (check
// pass): P_{0,t} = hatPsi_t (.) Psi_t (.) K_L (.) w_t (.) u_t (eq. proj_0t) from the
// stored panels zh = hatPsi_t (.) K_L (.) w_t and psi = Psi_t (.) K_L (.) w_t (kl ==
// nullptr: K_L = 1), and over the bounds D_t[l][i] that are finite and positive the
// relative violation max(P - D, 0) / D (maximised), the dual term D ln w_t and the
// gap term ln w_t (P - D) (summed), into fields ST_CAP_VIOL, ST_DUAL and ST_GAP of
// part[block] (nblk blocks, grid-stride, fixed order; the row kernel of the same
// time folds them into its statistics).
__global__ __launch_bounds__(256) void k_dense_comm_stats(int n, int L, int Lp, const float* __restrict__ zh,
                                                           const float* __restrict__ psi, const float* __restrict__ kl,
                                                           const float* __restrict__ cw, const float* __restrict__ dc,
                                                           const float* __restrict__ u, const double* __restrict__ sa,
                                                           const double* __restrict__ sb, double* __restrict__ part) {
  double v = 0.0, du = 0.0, ga = 0.0;
  const size_t total = (size_t)n * Lp;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / Lp), l = (int)(e % Lp);
    if (l >= L) continue;
    const double D = (double)dc[e];
    if (!(D > 0.0) || !isfinite(D)) continue;
    const double w = (double)cw[e], k = kl ? (double)kl[e] : 1.0;
    const double P = (w > 0.0 && k > 0.0) ? (double)zh[e] * (double)psi[e] / (k * w) * (double)u[i] * exp2(sa[l] + sb[l])
                                          : 0.0;
    const double lnw = log(w);
    v = fmax(v, fmax(P - D, 0.0) / D);
    du += D * lnw;
    ga += lnw * (P - D);
  }
  __shared__ double red[4][3];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int m = 32; m > 0; m >>= 1) {
    v = fmax(v, __shfl_xor(v, m, 64));
    du += __shfl_xor(du, m, 64);
    ga += __shfl_xor(ga, m, 64);
  }
  if (lane == 0) { red[wave][0] = v; red[wave][1] = du; red[wave][2] = ga; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = part + (size_t)blockIdx.x * kNSt;
    o[ST_CAP_VIOL] = fmax(fmax(red[0][0], red[1][0]), fmax(red[2][0], red[3][0]));
    o[ST_DUAL] = ((red[0][1] + red[1][1]) + red[2][1]) + red[3][1];
    o[ST_GAP] = ((red[0][2] + red[1][2]) + red[2][2]) + red[3][2];
  }
}

void launch_dense_comm_stats(int n, int L, int Lp, const float* zh, const float* psi, const float* kl, const float* cw,
                             const float* dc, const float* u, const double* sa, const double* sb, double* part,
                             int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_comm_stats, dim3(nblk), dim3(256), 0, s, n, L, Lp, zh, psi, kl, cw, dc, u, sa, sb, part);
}
void launch_dense_flows(int n, int L, int Lp, int lda, const float* A, const float* ua, const float* B,
                        const float* ub, const double* sa, const double* sb, float* fab, const float* K, double eps,
                        double* flow, double* part, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_flow_factors, dim3((Lp + 255) / 256), dim3(256), 0, s, sa, sb, L, Lp, fab, fab + Lp);
  hipLaunchKernelGGL(k_dense_flows, dim3(nblk), dim3(256), 0, s, n, Lp, lda, A, ua, B, ub, fab, fab + Lp, K, eps,
                     flow, part);
}
void launch_dense_state_cost(int n, int L, int Lp, const float* zh, const float* psi, const float* kl, const float* cw,
                             const float* u, const double* sa, const double* sb, double eps, double* part, int nblk,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_dense_state_cost, dim3(nblk), dim3(256), 0, s, n, L, Lp, zh, psi, kl, cw, u, sa, sb, eps, part);
}

}  // namespace mmot
