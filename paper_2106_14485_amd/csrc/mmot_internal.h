// Internal declarations of the MI355X graph-structured Sinkhorn library.
//
// Layout (HBM): every L x n quantity of the paper (messages Psi_t, hatPsi_t,
// scalings U^(0,1), U^(0,TT), marginals R, state-cost kernel K_L) is stored
// state-major as a "panel" [n][Lp]: row i holds the Lp >= L commodity values
// of state i contiguously (Lp padded to 16 bytes), so a sparse product gathers
// whole contiguous rows and the capacity reduction over commodities is a
// wavefront reduction inside one row.
//
// Range control.  Scaled domain: panel value x represents x * 2^sigma[l] with
// a per-commodity FP64 offset sigma (one per time and sweep direction).  Log
// domain: panel value y represents 2^(y + sigma[l]).  Each product step
// multiplies its output by 2^-c[t][l] (adds -c in the log domain), where c is
// the step's growth (log2 column-max of the output minus that of the input,
// measured on calibration sweeps, so it does not depend on how the input was
// scaled).  The first product of each sweep also removes the exact column
// level of the sweep's starting panel (U0T or U01), recorded by the kernel
// that wrote that panel every iteration.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/mmot.h"

namespace mmot {

constexpr int kBlock = 256;            // threads per block (4 wavefronts)
constexpr int kWaves = kBlock / 64;
constexpr int kNSt = 8;                // doubles per stats partial
// stats partial fields
enum { ST_SRC_ABS = 0, ST_SRC_MASS = 1, ST_CAP_VIOL = 2, ST_DUAL = 3, ST_GAP = 4, ST_MASS = 5, ST_NONFINITE = 6,
       ST_SCOST = 7 };
// device flag bits
enum { FLAG_INFEASIBLE = 1, FLAG_NONFINITE = 2, FLAG_BADINPUT = 4, FLAG_BADCSR = 8, FLAG_MASS = 16 };

// Arguments of one sparse sweep step: out = (in (.) u_in) * K-operator, scaled
// per column by fac, followed by an epilogue that depends on the output time.
template <typename V>
struct StepArgs {
  int n, Lp, L, G, nchunk;
  int lwpr;             // log2 of the waves sharing one whole-wave row (0, 1 or 2; 0 when G < 64)
  double eps;
  const int* rp;        // operator CSR (rows = output states); unused when ellD > 0
  const int* ci;        // CSR column indices, or ELL [n][ellD] (padding: index = row)
  const V* kv;          // K values (scaled) or log2 K (log); ELL padding 0 / -inf
  int ellD;             // > 0: ELL layout, rows of exactly this many entries (4, 5, 8 or 16: one gather batch)
  const V* xin;         // input panel (already multiplied by K_L at its time)
  const V* uin;         // [n] u at the input time (a vector of ones -- zeros in the log domain -- where none)
  const V* fac;         // [Lp] per-column output factor 2^-c (scaled) or -c (log)
  V* out;               // output panel (nullptr = do not store)
  const V* kl;          // [n][Lp] K_L multiplied into the stored output (interior times), nullptr = none
  // commodity-dependent capacities P_{0,t} <= D_t (interior output times), nullptr = none:
  // cw = w_t [n][Lp] multiplied into the stored output with K_L; a forward update
  // projects w_t first (with the current u_t), writes it to cwo (nullptr = do not
  // store) and multiplies the new value in; dc = D_t [n][Lp] (log2 in the log domain)
  const V* cw;
  V* cwo;
  const V* dc;
  // forward epilogue: capacity update at an interior output time
  int epi;              // 0 plain store, 1 capacity (u-update / check), 2 sink (E update / check)
  int update;           // 1: Sinkhorn update, 0: update-free (check / output pass)
  const V* wpan;        // backward stored panel W at the output time
  const V* wgt;         // [Lp] 2^(sigma_hat + sigma) (scaled) or sigma_hat + sigma (log)
  const V* cap;         // [n] capacity (log2 in the log domain) at the output time
  V* uout;              // [n] u at the output time
  const V* rdst;        // sink: R0T panel (log2 in the log domain)
  V* u0t;               // sink: U0T panel (written when update)
  V* hatT;              // sink update: hatPsi_T stored here as well (kept forward messages), nullptr = not
  const double* sigT;   // sink/check: [Lp] sigma of U0T (log2 units), sigma_hat of hatPsi_T
  const double* sighT;
  // column-level recording (log2 column maxima, encoded, slot p at base + p*nslot_stride)
  uint32_t* slots;      // levels of the stored output panel (sink: of the new U0T panel), nullptr = off
  uint32_t* slots_o;    // sink only: levels of hatPsi_T itself, nullptr = off
  int nslot;
  size_t nslot_stride;
  size_t nslot_stride_o;
  // log domain, forward calibration sweeps: per column, the stored values of the
  // backward panel (cslots_b) and of the forward output (cslots_f) at the state
  // where the plan Psi_hat (.) Psi peaks, as 64-bit keys (plan level, value)
  unsigned long long* cslots_b;
  unsigned long long* cslots_f;
  int ncslot;
  size_t cslot_stride;
  int* flags;
  // check pass
  double* part;         // [nblk][kNSt] stats partials of this time (nullptr = no stats)
  int tout;             // output time (for per-commodity output)
  double* occ;          // [n] occupancy at the output time (output pass), nullptr = none
  double* pcomm;        // [pc_cnt][n] per-commodity marginal at the output time, nullptr = none
  int pc_lo, pc_cnt;    // commodities pc_lo .. pc_lo + pc_cnt - 1 go to pcomm (row l - pc_lo)
};

// source update U01 = R01 ./ Psi_1 (row kernel)
template <typename V>
struct SourceArgs {
  int n, Lp, G, nchunk, nslot;
  const V* psi0;
  const V* rsrc;
  V* u01;
  uint32_t* slots;
  size_t slot_stride;
  int* flags;
  unsigned long long* cslots;   // log domain calibration: Psi_1 at the plan peak (time 0)
  int ncslot;
  size_t cslot_stride;
};
// statistics at time 0 (row kernel)
template <typename V>
struct Check0Args {
  int n, Lp, L, G, nchunk;
  const V* psi0;
  const V* u01;
  const V* rsrc;
  const double* sigf0;
  const double* sigb0;
  double* part;
  double* occ;
  double* pcomm;        // [pc_cnt][n], commodities pc_lo .. pc_lo + pc_cnt - 1
  int pc_lo, pc_cnt;
};
template <typename V>
struct PrepBwdArgs {
  int T, Lp, nslot;
  const double* cb;
  double* sigb;
  V* facb;
  const double* gaugeT;
  double* lvlT;
  uint32_t* slotsE;
};
template <typename V>
struct PrepFwdArgs {
  int T, Lp, mode, nslot;
  const double* cf;
  double* sigf;
  const double* sigb;
  V* facf;
  V* wgt;
  double* gauge0;
  double* gaugeT;
  double* lvl0;
  uint32_t* slotsS;
};
struct LevelsArgs {
  uint32_t* slots;
  float* lev;
  int T1, Lp, nslot;
};
// lev[t][l] = stored value carried by the largest 64-bit key over the slots
// (-inf if none; falls back to the 32-bit column-max slots); slots cleared
struct Levels64Args {
  unsigned long long* cslots;
  uint32_t* slots;
  float* lev;
  int T1, Lp, ncslot, nslot;
};
struct GrowthArgs {
  double* c;
  const float* lev;
  int T, Lp, dir;
};
struct Reduce1Args {
  const double* part;   // [slot][stride][kNSt]
  int nblk0, nblk;      // partials of slot 0 (the time-0 row kernel) and of the other slots
  int stride;
  double* tpart;
};
struct Reduce2Args {
  const double* tpart;
  int T1;
  double eps;
  double* out;
};

// Dense product OUT[n x Lp] = A[n x n] diag(u) B[n x Lp] on MFMA (see dense_mfma.hip).
struct GemmArgs {
  int n, Lp, L, lda;
  const void* A;        // [n][lda] (bf16 or f32), lda a multiple of 64, zero beyond n
  // BF16 operand already scaled by u, k-blocked: element (k, c) at ((k/8)*Lp + c)*8 + k%8,
  // rows padded to a multiple of 64 with zeros
  const uint16_t* Bb;
  int n8;               // rows of Bb (n rounded up to 64, zero padding)
  // FP32 operand already scaled by u, in 32-row blocks per column with the k
  // values of a block interleaved: element (k, c) at ((k/32)*Lp + c)*32 + ipos(k%32),
  // ipos(k) = (k%2)*16 + k/2 (rows padded to n8 with zeros).  The FP32 K of these
  // products is stored with the same interleave inside each 32-column block.
  const float* B32;
  const float* fac;     // [Lp] output column factor
  float* out;           // [n][Lp]
  const float* kl;      // [n][Lp] K_L multiplied into the stored output, nullptr = none
  // epilogue: also store bf16(uo[row] * stored value) k-blocked into bout (the
  // next product's operand); nullptr = off
  uint16_t* bout;
  const float* uo;
  int cap;              // 1: capacity partial sums (interior forward time)
  const float* wpan;    // Psi_{t} panel at the output time
  const float* wgt;     // [Lp]
  float* part_s;        // [nTN][n] partial column sums
  const float* ucur;    // check pass: u at the output time (per-commodity output)
  double* pcomm;        // check pass: [pc_cnt][n] per-commodity marginal, nullptr = none
  int pc_lo, pc_cnt;    // (commodities pc_lo .. pc_lo + pc_cnt - 1)
  uint32_t* slots;      // column levels of the stored output, nullptr = off
  int nslot;
  size_t slot_stride;
  // commodity-dependent capacities (kernel variant CM, nullptr = none): cw = w_t
  // [n][Lp] multiplied into the stored output; forward update (cc_update): w_t
  // projected before u_t with ucur (the u_t of the last sweep) against dc = D_t,
  // written to cwo
  const float* cw;
  float* cwo;
  const float* dc;
  int cc_update;
};

// Work items of the serving pool: one recorded kernel launch of one solve.
// A pool tick runs the next item of every active solve in one launch.
enum ItemKind {
  IK_STEP_BWD = 0, IK_STEP_FWD, IK_STEP_CHK, IK_SOURCE, IK_CHECK0, IK_PREP_BWD, IK_PREP_FWD, IK_LEVELS,
  IK_GROWTH, IK_REDUCE1, IK_REDUCE2, IK_LEVELS64, IK_COUNT
};
constexpr int kItemArgBytes = 352;
struct alignas(16) PoolItem {
  int kind;
  int log_domain;
  int nblk;
  int pad;
  unsigned char args[kItemArgBytes];
};
// One pool tick, passed by value: slot r runs item idx[r] of its
// device-resident program prog[r] with blocks prefix[r] .. prefix[r+1]-1 of
// the launch (blocks past the item's own count return at once).
constexpr int kTickSlots = 64;
struct TickArgs {
  int nslot;
  int prefix[kTickSlots + 1];
  int idx[kTickSlots];
  const PoolItem* prog[kTickSlots];
};
// Set while a solve's program is being recorded: launchers append items
// instead of launching (host only).
struct Recorder;
extern thread_local Recorder* tl_recorder;
bool record_item(int kind, int log_domain, int nblk, const void* args, size_t bytes);

// order-preserving float encoding for atomicMax on signed values (0 = empty)
__device__ __forceinline__ uint32_t enc_f32(float f) {
  uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ __forceinline__ float dec_f32(uint32_t e) {
  uint32_t b = (e & 0x80000000u) ? (e & 0x7fffffffu) : ~e;
  union { uint32_t u; float f; } c; c.u = b; return c.f;
}

// XCD-aware block order: hardware dispatches block b to XCD b % 8; give each
// XCD a contiguous range of logical blocks so neighbouring states (which share
// gathered rows) meet in the same L2.  nblk must be a multiple of 8.
__device__ __forceinline__ int xcd_block(int b, int nblk) {
  const int per = nblk >> 3;
  return (b & 7) * per + (b >> 3);
}

}  // namespace mmot
