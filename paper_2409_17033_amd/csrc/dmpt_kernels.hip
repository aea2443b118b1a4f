// gfx950 (CDNA4) kernels for the SP2 recursion and its susceptibility sweep
// (arXiv 2409.17033, Eq. DM0, DM2, DM3, DMSuscept, doubleHalf, MixPrecMult).
//
// Data layout (device workspace)
//   X_n, Y_n   n_pad x n_pad FP32 masters, row-major, full symmetric storage,
//              plus (all formats but FP32) an operand copy in a tiled layout:
//              chunks of 128 rows x one K-stage, each chunk contiguous, each
//              row's 16-byte slots holding one split term of 8 consecutive
//              columns and XOR-swizzled the way the LDS ring expects them
//              (Eq. doubleHalf with BF16 terms: hi = RNE(x), lo = RNE(x - hi),
//              and a middle term for the three-term split).
//   Padding rows/columns (n <= i < n_pad) are zero in X- and Y-space: 0 is a
//   fixed point of x^2 and 2x - x^2 and contributes nothing to any trace.
//
// Step kernel (one launch per SP2 step n)
//   A job is one 256 x 128 output tile (I, J >= 2I) of
//     P = X_n X_n                    (kind P; symmetric, so X_n rows serve as
//                                      both operands: P_IJ = X_I X_J^T)
//     Z = Y_n X_n + X_n Y_n          (kind Z; = Y_I X_J^T + X_I Y_J^T, the two
//                                      products K-concatenated)
//   When the residual correction follows, most Z-jobs are 256 x 256 tiles
//   (one accumulation level; fewer DMA bytes per flop), and each list ends
//   with K-split tiles: two jobs that each run half of a tile's stages and
//   store a partial sum, added by a combine launch that runs the tile's
//   epilogue before the next step launch.
//   The grid is persistent (one workgroup per CU): workgroups take jobs from
//   per-XCD queues with atomic tickets and steal from the other queues when
//   their own runs dry.
//   Operands stream HBM -> LDS with global_load_lds_dwordx4 (no VGPR staging)
//   through a ring of four stages, three in flight; the next stage's
//   operands are read into a second register set while the current stage's
//   MFMAs run, in a fixed interleaving of LDS reads and MFMAs.  Products run
//   on v_mfma_f32_32x32x16_f16 (FP16 split), v_mfma_f32_32x32x16_bf16 (BF16
//   splits / plain BF16) or v_mfma_f32_32x32x2f32 (FP32) with two-level FP32
//   accumulation.
//   Epilogue: X_{n+1} = P (sigma=+1) or 2 X_n - P (sigma=-1), likewise Y;
//   the tile and its mirror are stored (exact symmetry), the operand copy is
//   re-split, and P-jobs emit FP64 partials of Tr X_{n+1}, ||X_{n+1}||_F^2
//   and ||X_n - X_n^2||_F^2.  sigma_n and the stopping test are evaluated at
//   kernel start by every workgroup from the previous launch's partials
//   (fixed reduction order, so every workgroup reaches the same decision);
//   workgroup 0 records it in the control block.  No host round trip per step.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dmpt_internal.h"
#include "sp2_rule.h"

namespace dmpt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

#define LDS_AS __attribute__((address_space(3)))
#define GLB_AS __attribute__((address_space(1)))

// Bytes per LDS row per pipeline stage: 16 k values of FP32 / packed split-2
// (BF16 or FP16; 64 B = 4 slots of 16 B), 32 k values of plain BF16 (64 B),
// 16 k values of packed split-3 (96 B = 6 slots).
template <int PREC> struct Fmt {
  static constexpr int RB = PREC == kSplit3 ? 96 : 64;
  static constexpr int S = RB / 16;
  static constexpr int K = PREC == kBF16 ? 32 : 16;
};
// Format of the operand copy in HBM (the same as the staged one).
template <int PREC> struct Store { static constexpr int F = PREC; };

int stage_k(int prec) { return prec == kBF16 ? 32 : 16; }

// Step-kernel geometry: output tiles of TM x TN = 256 x 128 computed by
// eight waves (two per SIMD, 4 x 2), each owning a 64 x 64 region = 2 x 2
// MFMA blocks of 32 x 32.  Operands stream through a ring of RING LDS slots,
// each holding one stage (16 or 32 k values) of the 256-row A panel and the
// 128-row B panel.
constexpr int TM = 256, TN = 128, NW = 8, NT = 512, RING = 4;
constexpr int BR = 2, BC = 2;
constexpr int RBLK = 128;   // rows per chunk of the tiled operand layout
// Epilogue staging of one wave's 64 x 64 output region: row stride 65 floats,
// so both a row walk and a column walk over 64 lanes hit 64 distinct banks.
constexpr int kLS = 65;
constexpr int kStageBytes = 64 * kLS * 4;

// Tiled operand layout (all formats except FP32, which stays row-major): the
// copy of an n_pad x n_pad matrix is cut into chunks of 128 rows x one stage
// of K.  Chunk (rb, st) sits at byte ((rb * nst + st) * CHUNK) and holds its
// rows back to back, RB bytes each, with the same XOR slot swizzle the LDS
// ring uses, so a stage is DMA'd with contiguous 1 KB copies and lands in LDS
// already swizzled.
template <int PREC> struct Pipe {
  static constexpr int RB = Fmt<PREC>::RB;             // bytes per panel row per stage
  static constexpr int S = Fmt<PREC>::S;               // 16-byte slots per row
  static constexpr int A_BYTES = TM * RB, B_BYTES = TN * RB;
  static constexpr int SLOT = A_BYTES + B_BYTES;       // bytes per ring slot
  static constexpr int CHUNK = RBLK * Fmt<Store<PREC>::F>::RB;   // bytes per 128-row stage chunk in HBM
  static constexpr int NI = SLOT / 1024;               // 1 KB DMA instructions per stage
  static constexpr int L = (NI + NW - 1) / NW;         // per wave (padded with dummies)
  static constexpr bool TILED = PREC != kFP32;
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ unsigned short bf16_bits(float x) {
  return __builtin_bit_cast(unsigned short, (__bf16)x);   // round to nearest even
}
__device__ __forceinline__ float bf16_val(unsigned short b) {
  return __builtin_bit_cast(float, ((unsigned int)b) << 16);
}
__device__ __forceinline__ unsigned short f16_bits(float x) {
  return __builtin_bit_cast(unsigned short, (_Float16)x);   // round to nearest even, subnormals kept
}
__device__ __forceinline__ float f16_val(unsigned short b) { return (float)__builtin_bit_cast(_Float16, b); }
// Eq. doubleHalf with BF16 terms: part_0 = RNE(x), part_t = RNE(x - sum_{s<t} part_s).
template <int T>
__device__ __forceinline__ void split_terms(float x, unsigned short (&p)[T]) {
  float r = x;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    p[t] = bf16_bits(r);
    r = r - bf16_val(p[t]);
  }
}
// Eq. doubleHalf with FP16 terms on the scaled value: hi = RNE(x sc),
// lo = RNE(x sc - hi); sc is a power of two, x sc - hi is exact in FP32.
__device__ __forceinline__ void split_terms_h(float x, float sc, unsigned short (&p)[2]) {
  const float xs = x * sc;
  p[0] = f16_bits(xs);
  p[1] = f16_bits(xs - f16_val(p[0]));
}
template <int PREC> struct Terms {
  static constexpr int T = PREC == kSplit3 ? 3 : (PREC == kSplit2 || PREC == kSplitH) ? 2 : 1;
};
// The split terms of one element in the operand format F (sc: kSplitH scale).
template <int F>
__device__ __forceinline__ void split_for(float v, float sc, unsigned short (&p)[Terms<F>::T]) {
  if constexpr (F == kSplitH) split_terms_h(v, sc, p);
  else split_terms<Terms<F>::T>(v, p);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// kSplitH: exponent s of the scale 2^s of a Y copy whose entries are bounded
// by bound * nrm (nrm a Frobenius norm): the largest s with bound * nrm * 2^s
// <= kYTarget, clamped to [-100, 100]; 0 for a zero or non-finite norm.
__device__ __forceinline__ int yscale_exp(double nrm, double bound) {
  const double b = bound * nrm;
  if (!(b > 0.0) || !(b < 1e300)) return 0;
  const int e = (int)floor(log2(kYTarget / b));
  return e < -100 ? -100 : e > 100 ? 100 : e;
}

// Frobenius norm of a matrix from its producer's partials (count of them in
// meta->nrm, at most cap = the allocated number), summed in a fixed order by
// wave 0 of the block (every block gets the same value); the result is
// broadcast through *s_out.
__device__ __forceinline__ double meta_norm(const MatMeta* m, int cap, double* s_out) {
  if (threadIdx.x < 64) {
    const int cnt = m->count < cap ? m->count : cap;
    double t = 0.0;
    for (int i = threadIdx.x; i < cnt; i += 64) t += m->nrm[i];
    t = wave_sum(t);
    if (threadIdx.x == 0) *s_out = sqrt(t);
  }
  __syncthreads();
  return *s_out;
}

// Physical 16-byte slot of logical slot ls in LDS row r.  4 slots/row:
// XOR with (r/4)&3; 6 slots/row: XOR with (r/8)&1.  Either way 16 lanes that
// read one logical slot of 16 consecutive rows hit 16 distinct 4-bank groups.
template <int S>
__device__ __forceinline__ int phys_slot(int r, int ls) {
  if constexpr (S == 4) return ls ^ ((r >> 2) & 3);
  else return ls ^ ((r >> 3) & 1);
}
template <int S>
__device__ __forceinline__ int swz(int r, int ls) { return r * (S * 16) + 16 * phys_slot<S>(r, ls); }

__device__ __forceinline__ u32x4 lds16(const LDS_AS char* p) { return *(const LDS_AS u32x4*)p; }

// s_waitcnt with vmcnt = V and lgkmcnt = 0 (LGKM0) or untouched.  The builtin
// (not inline asm) lets the compiler's wait-count pass see the wait.
template <int V, bool LGKM0>
__device__ __forceinline__ void wait_vm() {
  static_assert(V >= 0 && V < 64, "vmcnt range");
  constexpr int enc = (V & 15) | ((V >> 4) << 14) | (7 << 4) | ((LGKM0 ? 0 : 15) << 8);
  __builtin_amdgcn_s_waitcnt(enc);
}

// Workgroup barrier without the implicit memory fence of __syncthreads (which
// would drain every in-flight prefetch); the empty asm statements stop the
// compiler from moving LDS accesses across it.
__device__ __forceinline__ void barrier_nofence() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// DMA of one stage into a ring slot, row-major operands (FP32): rows [0, TM)
// of the A panel and [0, TN) of the B panel, `a` / `b` pointing at row 0 at
// the stage's byte offset.  The panel is (rows x S) 16-byte slots;
// instruction j covers slots [64 j, 64 j + 64): lane i takes slot
// q = 64 j + i = (row q / S, physical slot q % S) and fetches the logical
// slot the swizzle maps there (the XOR swizzle is its own inverse).
template <int PREC>
__device__ __forceinline__ void dma_stage_rows(LDS_AS char* slot, const char* a, const char* b, uint32_t ldb,
                                               int wave, int lane) {
  using P = Pipe<PREC>;
  constexpr int NA = TM * P::S / 64;   // A instructions
#pragma unroll
  for (int jj = 0; jj < P::L; ++jj) {
    const int j = wave + jj * NW;
    const bool isA = j < NA;
    const int q = 64 * (isA ? j : j - NA) + lane;
    const int r = q / P::S;
    const uint32_t off = (uint32_t)r * ldb + 16u * (uint32_t)phys_slot<P::S>(r, q % P::S);
    __builtin_amdgcn_global_load_lds((const GLB_AS void*)((isA ? a : b) + off), (LDS_AS void*)(slot + j * 1024),
                                     16, 0, 0);
  }
}

// DMA of one stage, tiled operands: the stage is three contiguous chunks (A
// rows 0-127, A rows 128-255, B rows 0-127) copied 1 KB per instruction.
// When NI is not a multiple of NW the last round has more instructions than
// kilobytes; the surplus ones repeat an earlier copy (same source, same
// destination, same bytes), so every wave issues L and the control flow stays
// branch-free.
template <int PREC>
__device__ __forceinline__ void dma_stage_tiled(LDS_AS char* slot, const char* a0, const char* a1, const char* b,
                                                int wave, int lane) {
  using P = Pipe<PREC>;
  constexpr int NC = P::CHUNK / 1024;   // instructions per chunk
  if constexpr (P::NI == 3 * NW && NC == NW) {
    // one instruction per wave in each of the three chunks: instruction
    // j = wave + jj NW copies kilobyte `wave` of chunk jj
    const size_t off = (size_t)wave * 1024 + (size_t)lane * 16;
    __builtin_amdgcn_global_load_lds((const GLB_AS void*)(a0 + off), (LDS_AS void*)(slot + wave * 1024), 16, 0, 0);
    __builtin_amdgcn_global_load_lds((const GLB_AS void*)(a1 + off), (LDS_AS void*)(slot + (wave + NW) * 1024), 16, 0, 0);
    __builtin_amdgcn_global_load_lds((const GLB_AS void*)(b + off), (LDS_AS void*)(slot + (wave + 2 * NW) * 1024), 16, 0, 0);
    return;
  }
#pragma unroll
  for (int jj = 0; jj < P::L; ++jj) {
    const int jv = wave + jj * NW;
    const int j = (P::NI % NW != 0 && jv >= P::NI) ? jv - P::NI : jv;
    const int region = j / NC;
    const char* src = (region == 0 ? a0 : region == 1 ? a1 : b) + (j - region * NC) * 1024 + lane * 16;
    __builtin_amdgcn_global_load_lds((const GLB_AS void*)src, (LDS_AS void*)(slot + j * 1024), 16, 0, 0);
  }
}

// Byte offset of element (r, c), split term `part`, in the tiled operand copy.
template <int PREC>
__device__ __forceinline__ size_t op_off(int r, int c, int part, int nst) {
  constexpr int RB = Fmt<PREC>::RB, S = Fmt<PREC>::S, K = Fmt<PREC>::K, T = Terms<PREC>::T;
  const int rr = r & (RBLK - 1);
  const int st = c / K, kk = c % K;
  const int ls = PREC == kBF16 ? (kk >> 3) : T * (kk >> 3) + part;
  return ((size_t)(r / RBLK) * nst + st) * (size_t)(RBLK * RB) + (size_t)rr * RB + 16 * phys_slot<S>(rr, ls) +
         (kk & 7) * 2;
}

// Operand registers of one stage for one wave.
template <int PREC> struct Ops;
template <> struct Ops<kSplit3> { bf16x8 a[BR][3], b[BC][3]; };
template <> struct Ops<kSplit2> { bf16x8 a[BR][2], b[BC][2]; };
template <> struct Ops<kSplitH> { f16x8 a[BR][2], b[BC][2]; };
template <> struct Ops<kBF16> { bf16x8 a[BR][2], b[BC][2]; };     // [t]: k16 step
template <> struct Ops<kFP32> { f32x4 a[BR][2], b[BC][2]; };       // [q]: slot h + 2q

// Read one stage's operands from a ring slot.
//   split: logical slot T*h + p = k-group h (8 values), part p
//   BF16:  32-k stage, k16 step t uses slot 2t + h
//   FP32:  lane half h holds k in {4h..4h+3} (slot h) and {8+4h..} (slot h+2);
//          the same k-permutation on A and B leaves the contraction unchanged.
template <int PREC>
__device__ __forceinline__ void read_ops(const LDS_AS char* slot, Ops<PREC>& o, int rowA, int rowB, int h) {
  constexpr int S = Pipe<PREC>::S;
  const LDS_AS char* pA = slot;
  const LDS_AS char* pB = slot + Pipe<PREC>::A_BYTES;
  if constexpr (PREC == kSplit3 || PREC == kSplit2 || PREC == kSplitH) {
    constexpr int T = Terms<PREC>::T;
    using E = typename std::remove_reference<decltype(o.a[0][0])>::type;
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
      for (int p = 0; p < T; ++p) o.a[i][p] = __builtin_bit_cast(E, lds16(pA + swz<S>(rowA + 32 * i, T * h + p)));
#pragma unroll
    for (int j = 0; j < BC; ++j)
#pragma unroll
      for (int p = 0; p < T; ++p) o.b[j][p] = __builtin_bit_cast(E, lds16(pB + swz<S>(rowB + 32 * j, T * h + p)));
  } else if constexpr (PREC == kBF16) {
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
      for (int t = 0; t < 2; ++t) o.a[i][t] = __builtin_bit_cast(bf16x8, lds16(pA + swz<S>(rowA + 32 * i, 2 * t + h)));
#pragma unroll
    for (int j = 0; j < BC; ++j)
#pragma unroll
      for (int t = 0; t < 2; ++t) o.b[j][t] = __builtin_bit_cast(bf16x8, lds16(pB + swz<S>(rowB + 32 * j, 2 * t + h)));
  } else {
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
      for (int q = 0; q < 2; ++q) o.a[i][q] = __builtin_bit_cast(f32x4, lds16(pA + swz<S>(rowA + 32 * i, h + 2 * q)));
#pragma unroll
    for (int j = 0; j < BC; ++j)
#pragma unroll
      for (int q = 0; q < 2; ++q) o.b[j][q] = __builtin_bit_cast(f32x4, lds16(pB + swz<S>(rowB + 32 * j, h + 2 * q)));
  }
}

// acc[i][j] += A_i B_j^T for one stage.
//   split-3: products of order >= 2^-16 (hh, hm, mh, hl, lh, mm), smallest first
//   split-2: hh + hl + lh (lo*lo dropped, Eq. MixPrecMult), BF16 or FP16 terms
template <int PREC>
__device__ __forceinline__ void mma_ops(const Ops<PREC>& o, f32x16 (&acc)[BR][BC]) {
#pragma unroll
  for (int i = 0; i < BR; ++i)
#pragma unroll
    for (int j = 0; j < BC; ++j) {
      f32x16 c = acc[i][j];
      if constexpr (PREC == kSplit3) {
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.a[i][1], o.b[j][1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.a[i][0], o.b[j][2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.a[i][2], o.b[j][0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.a[i][0], o.b[j][1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.a[i][1], o.b[j][0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.a[i][0], o.b[j][0], c, 0, 0, 0);
      } else if constexpr (PREC == kSplit2) {
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.a[i][0], o.b[j][1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.a[i][1], o.b[j][0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.a[i][0], o.b[j][0], c, 0, 0, 0);
      } else if constexpr (PREC == kSplitH) {
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(o.a[i][0], o.b[j][1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(o.a[i][1], o.b[j][0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(o.a[i][0], o.b[j][0], c, 0, 0, 0);
      } else if constexpr (PREC == kBF16) {
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.a[i][0], o.b[j][0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.a[i][1], o.b[j][1], c, 0, 0, 0);
      } else {
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            c = __builtin_amdgcn_mfma_f32_32x32x2f32(o.a[i][q][e], o.b[j][q][e], c, 0, 0, 0);
      }
      acc[i][j] = c;
    }
}

// FP32 stage products with the accumulator blocks taken in the order
// F, F + 1, F + 2, F + 3 (block b = (b / 2, b % 2)).
template <int F>
__device__ __forceinline__ void mma_fp32_from(const Ops<kFP32>& o, f32x16 (&acc)[BR][BC]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int b = (F + t) & 3, i = b >> 1, j = b & 1;
    f32x16 c = acc[i][j];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) c = __builtin_amdgcn_mfma_f32_32x32x2f32(o.a[i][q][e], o.b[j][q][e], c, 0, 0, 0);
    acc[i][j] = c;
  }
}

// Issue order inside one pipeline stage: the R LDS reads of the next stage
// are spread among the M MFMAs of this one (a read, then M / R MFMAs; when R
// does not divide M, a read per MFMA and the remaining MFMAs last; the
// three-term split takes its 12 reads in pairs, each pair followed by four
// MFMAs, which measured 1.4 % faster than one read per two).  Left to itself
// the scheduler puts some reads at the end of the stage, where their
// latency, queued behind every wave's reads, stalls the stage's barrier.
template <int PREC> struct StageMix {
  static constexpr int R = (BR + BC) * (PREC == kSplit3 ? 3 : 2);   // ds_read_b128 per stage
  static constexpr int M = BR * BC * (PREC == kSplit3 ? 6 : (PREC == kSplit2 || PREC == kSplitH) ? 3 :
                                      PREC == kBF16 ? 2 : 8);           // MFMAs per stage
};
template <int PREC>
__device__ __forceinline__ void stage_order() {
  constexpr int R = StageMix<PREC>::R, M = StageMix<PREC>::M;
  if constexpr (PREC == kSplit3) {
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 2 * M / R, 0);
    }
  } else if constexpr (M % R == 0) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);       // DS read
      __builtin_amdgcn_sched_group_barrier(0x008, M / R, 0);   // MFMA
    }
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, M - R, 0);
  }
}

// ---------------------------------------------------------------- step kernel

// Launch k of the step kernel: wave 0 reduces the partials the previous
// launch (or X_1's initialisation) wrote, in a fixed order, giving
// Tr X_k, ||X_k||_F^2 and eps_{k-1} = ||X_{k-1} - X_{k-1}^2||_F^2.  Then, in
// order: stop at X_{k-1} (its stopping test), give up at X_{k-1} (step limit),
// bounds check of X_k, else sigma_k.  Every workgroup evaluates the same FP64
// numbers in the same order and reaches the same decision; workgroup 0
// records it.  Returns sigma_k (+1 / -1) or a stop code.
__device__ __forceinline__ int step_controller(const StepArgs& a, int* s_code, int* s_zskip) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    double tr = 0.0, sq = 0.0, eps = 0.0;
    for (int t = lane; t < a.nparts; t += 64) {
      const Part p = a.part_in[t];
      tr += p.tr;
      sq += p.sq;
      eps += p.eps;
    }
    tr = wave_sum(tr);
    sq = wave_sum(sq);
    eps = wave_sum(eps);
    if (lane == 0) {
      Ctl* c = a.ctl;
      const int k = a.step;
      int code = 1, m = -1;   // m >= 0: the recursion ends with X_{m+1}
      if (c->nonfinite) {
        code = kDecideNonfinite;
        m = k - 1;
      } else {
        if (k >= 2) {
          // eps of X_{k-1} is this launch's; X_j's was recorded at rec[j]
          const double e1 = k >= 3 ? c->rec[k - 2].eps : 0.0;
          const double e2 = k >= 4 ? c->rec[k - 3].eps : 0.0;
          const double e3 = k >= 5 ? c->rec[k - 4].eps : 0.0;
          if (sp2_should_stop(eps, e1, e2, e3, k - 2, a.n, a.min_iter, a.idem_tol, a.unit)) {
            code = kDecideStop;
            m = k - 2;
          } else if (k - 2 >= a.max_iter) {
            code = kDecideNotConverged;
            m = k - 2;
          }
        }
        if (m < 0) {
          if (!sp2_bounds_ok(tr, sq, a.n)) {
            code = kDecideBounds;
            m = k - 1;
          } else {
            code = sp2_sigma(tr, sq, a.nocc);
          }
        }
      }
      // Sweep stop (ytol2 > 0): the Z-jobs of this launch would form Y_{k+1}
      // from X_k; once X_{k-1} (the operand of Y_k) is within the tolerance
      // they are skipped here and in every later launch, and Y_k is the
      // result.  Every workgroup evaluates the same test on the same eps;
      // workgroup 0 records k.
      int zs = 0;
      if (a.ytol2 > 0.0 && k >= 2 && m < 0) {
        zs = (c->ystop != 0 || eps <= a.ytol2) ? 1 : 0;
        if (zs && blockIdx.x == 0 && c->ystop == 0) c->ystop = k;
      }
      *s_zskip = zs;
      if (blockIdx.x == 0) {
        c->rec[k].tr = tr;
        c->rec[k].sq = sq;
        if (k >= 2) c->rec[k - 1].eps = eps;
        c->rec[k].sigma = m < 0 ? code : 0;
        if (m >= 0) {
          c->m = m;
          c->code = code;
          __threadfence();
          c->done = 1;
        }
      }
      *s_code = m < 0 ? code : (code == kDecideStop ? 2 : code);
    }
  }
  __syncthreads();
  return *s_code;
}

template <int PREC>
__device__ __forceinline__ void store_split1(char* oop, int nst, int r, int c, float v, float sc) {
  constexpr int T = Terms<PREC>::T;
  unsigned short part[T];
  split_for<PREC>(v, sc, part);
#pragma unroll
  for (int t = 0; t < T; ++t) *(unsigned short*)(oop + op_off<PREC>(r, c, t, nst)) = part[t];
}

// Operand copy of 8 consecutive columns c0..c0+7 (c0 % 8 == 0) of row r, in
// the tiled layout: each split term of the group is one 16-byte slot.
template <int PREC>
__device__ __forceinline__ void store_group8_t(char* op, int nst, int r, int c0, const float (&v)[8], float sc) {
  constexpr int T = Terms<PREC>::T;
  unsigned short part[8][T];
#pragma unroll
  for (int e = 0; e < 8; ++e) split_for<PREC>(v[e], sc, part[e]);
#pragma unroll
  for (int t = 0; t < T; ++t) {
    u32x4 w;
#pragma unroll
    for (int e = 0; e < 4; ++e) w[e] = part[2 * e][t] | ((unsigned)part[2 * e + 1][t] << 16);
    *(u32x4*)(op + op_off<PREC>(r, c0, t, nst)) = w;
  }
}

// s_getreg operand for the 32-bit HW_REG_XCC_ID register (id 20): the XCD a
// wave runs on in its low bits.
constexpr int kHwRegXccId = (31 << 11) | 20;

// Index of step tile (I, J) among the tiles that cover the upper triangle:
// row block I (256 rows), column block J >= 2I (128 columns), tcols = n_pad/128.
__device__ __forceinline__ int tile_index(int ti, int tj, int tcols) {
  return ti * tcols - ti * (ti - 1) + (tj - 2 * ti);
}

// Epilogue of one regular tile (256 x 128) of P = X_n^2 or Z = Y_n X_n + X_n Y_n
// from the tile sums `tot` (MFMA accumulator layout): sigma-update, direct and
// mirror stores, operand copies, and for P-jobs the FP64 partials of
// Tr X_{n+1}, ||X_{n+1}||_F^2 and ||X_n - X_n^2||_F^2.  R0..R3: LDS areas of at
// least two 64 x 65 FP32 staging blocks each (wave w stages in R[w / 2]);
// sc_out / s_out: the scale of the FP16 copy (kSplitH).  The workgroup's
// waves are waves wave_base .. wave_base + nwaves - 1 of the tile's eight
// (the step kernel: all of them); P-jobs write the FP64 partials of those
// waves to part_out[part_idx].
template <int PREC, bool MIX>
__device__ __forceinline__ void step_epilogue(const StepArgs& a, const uint32_t job, const int sigma,
                                              f32x16 (&tot)[BR][BC], LDS_AS char* R0, LDS_AS char* R1,
                                              LDS_AS char* R2, LDS_AS char* R3, double* s_red, const float sc_out,
                                              const int s_out, const int wave_base, const int nwaves,
                                              const int part_idx) {
  const int kind = job & 1;
  const int obs = (job >> 1) & 63;
  const int ti = (job >> 8) & 4095;    // 256-row block
  const int tj = (job >> 20) & 2047;   // 128-column block
  unsigned int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & 63;
  const int wave = wave_base + __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;   // 4 x 2 waves of 64 x 64
  const int h = lane >> 5, l32 = lane & 31;
  (void)s_out;
  const size_t np = a.n_pad;
  // field-wise selects (a selected reference would keep the argument block in
  // private memory)
  const bool zk = kind == kJobZ;
  const float* cur = zk ? a.y_in.f32 + obs * a.y_in.stride_f32 : a.x_in.f32;
  float* o32 = zk ? a.y_out.f32 + obs * a.y_out.stride_f32 : a.x_out.f32;
  char* oop = zk ? (char*)a.y_out.op + obs * a.y_out.stride_op : (char*)a.x_out.op;
  // kSplit3 matrices of the three-term-X^2 option also get their two-term copy
  char* oop2 = nullptr;
  if constexpr (MIX) {
    char* o2 = (char*)(zk ? a.y_out.op2 : a.x_out.op2);
    oop2 = o2 ? o2 + (zk ? obs * a.y_out.stride_op : 0) : nullptr;
  }
  const int nstp = a.n_pad / Fmt<PREC>::K;   // stages per row (tiled layout)
  // P-jobs of a run with the residual correction keep every X_{n+1} as plain BF16
  char* hop = kind == kJobP && a.hist ? a.hist + (size_t)(a.step + 1) * a.hist_stride : nullptr;
  const int nsth = a.n_pad / Fmt<kBF16>::K;
  const bool wsplit = a.write_split && PREC != kFP32;
  const bool onDiag = tj <= 2 * ti + 1;   // tile straddles the diagonal
  double tr = 0.0, sq = 0.0, ep = 0.0;
  double yq = 0.0;   // kSplitH Z-jobs: ||Y_{n+1}||_F^2 over this tile (and its mirror)
  const bool need_cur = kind == kJobP || sigma < 0;
  if (!onDiag) {
    // Off-diagonal tile: every element is stored twice (direct and mirror).
    // Each wave stages its 64 x 64 region in LDS (private area, no cross-wave
    // traffic) and writes rows of 16-byte vectors: direct rows, mirror rows,
    // and 16-byte split-term slots of 8 consecutive columns in both
    // orientations.  The barrier makes sure every wave is past its last ring
    // read and every ring DMA has landed.
    barrier_nofence();
    LDS_AS char* rb = (wave >> 1) == 0 ? R0 : (wave >> 1) == 1 ? R1 : (wave >> 1) == 2 ? R2 : R3;
    LDS_AS float* T = (LDS_AS float*)(rb + (wave & 1) * kStageBytes);
    // 32x32 MFMA output layout: lane l, register 4g+e holds row 8g + 4(l/32) + e, column l%32.
#pragma unroll
    for (int bi = 0; bi < BR; ++bi)
#pragma unroll
      for (int bj = 0; bj < BC; ++bj)
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
          for (int e = 0; e < 4; ++e) T[(bi * 32 + 8 * g + 4 * h + e) * kLS + bj * 32 + l32] = tot[bi][bj][4 * g + e];
    wait_vm<63, true>();
    const int gr0 = ti * TM + wr * 64, gc0 = tj * TN + wc * 64;   // global origin of the region
    // direct rows: 4 rows x 64 columns per round, 4 columns per lane
#pragma unroll 4
    for (int rd = 0; rd < 16; ++rd) {
      const int r = 4 * rd + (lane >> 4), c = 4 * (lane & 15);
      f32x4 v = f32x4{T[r * kLS + c], T[r * kLS + c + 1], T[r * kLS + c + 2], T[r * kLS + c + 3]};
      if (need_cur) {
        const f32x4 x = *(const f32x4*)(cur + (size_t)(gr0 + r) * np + gc0 + c);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float p = v[k];
          v[k] = sigma > 0 ? p : 2.0f * x[k] - p;
          if (kind == kJobP) {
            const double d = x[k] - p;                // X_n - X_n^2
            sq += 2.0 * (double)v[k] * (double)v[k];
            ep += 2.0 * d * d;
          }
        }
        if (sigma < 0) {
#pragma unroll
          for (int k = 0; k < 4; ++k) T[r * kLS + c + k] = v[k];
        }
      }
      if constexpr (PREC == kSplitH) {
        if (kind == kJobZ)
#pragma unroll
          for (int k = 0; k < 4; ++k) yq += 2.0 * (double)v[k] * (double)v[k];
      }
      *(f32x4*)(o32 + (size_t)(gr0 + r) * np + gc0 + c) = v;
    }
    wait_vm<63, true>();
    // mirror rows: 4 mirror rows x 64 columns per round
#pragma unroll 4
    for (int rd = 0; rd < 16; ++rd) {
      const int c = 4 * rd + (lane >> 4), q = 4 * (lane & 15);
      *(f32x4*)(o32 + (size_t)(gc0 + c) * np + gr0 + q) =
          f32x4{T[q * kLS + c], T[(q + 1) * kLS + c], T[(q + 2) * kLS + c], T[(q + 3) * kLS + c]};
    }
    if constexpr (PREC != kFP32) {
      if (wsplit) {
        // split-term slots: 8 rows x 8 groups of 8 columns per round, both orientations
#pragma unroll 2
        for (int rd = 0; rd < 8; ++rd) {
          const int r = 8 * rd + (lane >> 3), c = 8 * (lane & 7);
          float v[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) v[k] = T[r * kLS + c + k];
          store_group8_t<Store<PREC>::F>(oop, nstp, gr0 + r, gc0 + c, v, sc_out);
          if constexpr (MIX) {
            if (oop2) store_group8_t<kSplit2>(oop2, nstp, gr0 + r, gc0 + c, v, 1.0f);
          }
        }
#pragma unroll 2
        for (int rd = 0; rd < 8; ++rd) {
          const int c = 8 * rd + (lane >> 3), q = 8 * (lane & 7);
          float v[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) v[k] = T[(q + k) * kLS + c];
          store_group8_t<Store<PREC>::F>(oop, nstp, gc0 + c, gr0 + q, v, sc_out);
          if constexpr (MIX) {
            if (oop2) store_group8_t<kSplit2>(oop2, nstp, gc0 + c, gr0 + q, v, 1.0f);
          }
        }
      }
    }
    if (hop) {
      // plain BF16 copy of X_{n+1}, both orientations
#pragma unroll 2
      for (int rd = 0; rd < 8; ++rd) {
        const int r = 8 * rd + (lane >> 3), c = 8 * (lane & 7);
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = T[r * kLS + c + k];
        store_group8_t<kBF16>(hop, nsth, gr0 + r, gc0 + c, v, 1.0f);
      }
#pragma unroll 2
      for (int rd = 0; rd < 8; ++rd) {
        const int c = 8 * rd + (lane >> 3), q = 8 * (lane & 7);
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = T[(q + k) * kLS + c];
        store_group8_t<kBF16>(hop, nsth, gc0 + c, gr0 + q, v, 1.0f);
      }
    }
  } else {
    // Diagonal tile: keep the upper triangle (row <= col) and mirror it.
    // 32x32 MFMA output layout: lane l, register 4g+e holds row 8g + 4(l/32) + e, column l%32.
#pragma unroll
    for (int bi = 0; bi < BR; ++bi)
#pragma unroll
      for (int bj = 0; bj < BC; ++bj) {
        const int col = tj * TN + wc * 64 + bj * 32 + l32;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int row0 = ti * TM + wr * 64 + bi * 32 + 8 * g + 4 * h;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int r = row0 + e;
            if (r > col) continue;
            const float p = tot[bi][bj][4 * g + e];
            float v = p, dd = 0.0f;
            if (need_cur) {
              const float c0 = cur[(size_t)r * np + col];
              v = sigma > 0 ? p : 2.0f * c0 - p;
              dd = c0 - p;                               // X_n - X_n^2 (P-jobs)
            }
            o32[(size_t)r * np + col] = v;
            o32[(size_t)col * np + r] = v;
            if (wsplit) {
              store_split1<Store<PREC>::F>(oop, nstp, r, col, v, sc_out);
              if (r != col) store_split1<Store<PREC>::F>(oop, nstp, col, r, v, sc_out);
              if constexpr (MIX) {
                if (oop2) {
                  store_split1<kSplit2>(oop2, nstp, r, col, v, 1.0f);
                  if (r != col) store_split1<kSplit2>(oop2, nstp, col, r, v, 1.0f);
                }
              }
            }
            if (hop) {
              store_split1<kBF16>(hop, nsth, r, col, v, 1.0f);
              if (r != col) store_split1<kBF16>(hop, nsth, col, r, v, 1.0f);
            }
            if constexpr (PREC == kSplitH) {
              if (kind == kJobZ) yq += (r == col ? 1.0 : 2.0) * (double)v * (double)v;
            }
            if (kind == kJobP) {
              const double w = r == col ? 1.0 : 2.0;
              if (r == col) tr += v;
              sq += w * (double)v * (double)v;
              ep += w * (double)dd * (double)dd;
            }
          }
        }
      }
  }

  if (kind == kJobP) {
    tr = wave_sum(tr);
    sq = wave_sum(sq);
    ep = wave_sum(ep);
    if (lane == 0) {
      s_red[3 * (wave - wave_base)] = tr;
      s_red[3 * (wave - wave_base) + 1] = sq;
      s_red[3 * (wave - wave_base) + 2] = ep;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      Part p = {0.0, 0.0, 0.0, 0.0};
      for (int w = 0; w < nwaves; ++w) {
        p.tr += s_red[3 * w];
        p.sq += s_red[3 * w + 1];
        p.eps += s_red[3 * w + 2];
      }
      a.part_out[part_idx] = p;
    }
  }
  if constexpr (PREC == kSplitH) {
    if (kind == kJobZ) {
      yq = wave_sum(yq);
      if (lane == 0) s_red[wave - wave_base] = yq;
      __syncthreads();
      if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < nwaves; ++w) t += s_red[w];
        MatMeta* mo = (MatMeta*)(a.y_out.meta + obs * a.y_out.stride_op);
        const int idx = tile_index(ti, tj, a.ntile);
        mo->nrm[idx] = t;
        if (idx == 0) {
          const int tr_ = a.n_pad / TM;
          mo->scale = s_out;
          mo->count = tr_ * (tr_ + 1);
        }
      }
    }
  }
}

// One job of the step kernel (one output tile of P = X_n^2 or of
// Z = Y_n X_n + X_n Y_n) in operand format PREC: DMA + MFMA main loop and the
// fused epilogue.  R0..R3: the LDS ring (each slot also holds two waves'
// epilogue staging); s_red, s_nrm: workgroup scratch.
// MIX: a job of the mixed launch of the three-term-X^2 option: its P-jobs
// (kSplit3) also write the two-term copy of their output, its Z-jobs
// (kSplit2) read X's two-term copy and take their own flush interval.
// jpos: the job's list position (the scratch slot of a K-split job).
template <int PREC, bool MIX = false>
__device__ __forceinline__ void step_job(const StepArgs& a, const uint32_t job, const int jpos, const int sigma,
                                         LDS_AS char* R0, LDS_AS char* R1, LDS_AS char* R2, LDS_AS char* R3,
                                         double* s_red, double* s_nrm) {
  using P = Pipe<PREC>;
  const int kind = job & 1;
  const int obs = (job >> 1) & 63;
  const int ti = (job >> 8) & 4095;    // 256-row block
  const int tj = (job >> 20) & 2047;   // 128-column block
  constexpr int opb = operand_bytes(PREC);
  const size_t ldb = (size_t)a.n_pad * opb;
  const int spass = a.n_pad / Fmt<PREC>::K;           // stages per product
  const int nst = kind == kJobZ ? 2 * spass : spass;  // Z-job: Y_I X_J^T, then X_I Y_J^T
  // K-split job (two-term / three-term BF16 and plain BF16 formats): stages
  // [sb, se) of the tile's stream, half of it (nst is a multiple of 8)
  constexpr bool kCanSplit = PREC == kSplit2 || PREC == kSplit3 || PREC == kBF16;
  const bool split = kCanSplit && (job & kJobSplit) != 0;
  const int half = split && (job & kJobHalf1) ? 1 : 0;
  const int sb = split && half ? nst / 2 : 0;
  const int se = split && !half ? nst / 2 : nst;

  // X operand: the two-term copy for the Z-jobs of the mixed launch (op2),
  // the copy in this job's format otherwise
  const char* xop = (const char*)(MIX && kind == kJobZ ? a.x_in.op2 : a.x_in.op);
  const char* yop = (const char*)a.y_in.op + obs * a.y_in.stride_op;
  // row block I / J starts at the same byte offset in both layouts:
  // row-major rows * ldb, tiled (row block * nst) chunks of 128 rows
  const size_t rowI = (size_t)ti * TM * ldb, rowJ = (size_t)tj * TN * ldb;
  const char* a0 = (kind == kJobZ ? yop : xop) + rowI;
  const char* b0 = xop + rowJ;
  const char* a1 = xop + rowI;
  const char* b1 = (kind == kJobZ ? yop : xop) + rowJ;

  // kSplitH: the products come out scaled by 2^(s_a + s_b) (usc undoes it);
  // the copy this job writes is scaled by sc_out = 2^s_out.  P-jobs: both
  // operands X_n at 2^14.  Z-jobs: Y_n at its own 2^s_in; Y_{n+1} gets the
  // exponent bounded from ||Y_n||_F.
  float usc = 1.0f, sc_out = 1.0f;
  int s_out = 0;
  if constexpr (PREC == kSplitH) {
    if (kind == kJobZ) {
      const MatMeta* mi = (const MatMeta*)(a.y_in.meta + obs * a.y_in.stride_op);
      usc = ldexpf(1.0f, -(kXScaleExp + mi->scale));
      const int nb = a.n_pad / 64;   // metadata holds (n_pad / 64)^2 partials
      s_out = yscale_exp(meta_norm(mi, nb * nb, s_nrm), kYBound);
    } else {
      usc = ldexpf(1.0f, -2 * kXScaleExp);
      s_out = kXScaleExp;
    }
    sc_out = ldexpf(1.0f, s_out);
  }

  // The thread index is made opaque per job so that the compiler keeps the
  // lane-dependent address arithmetic inside the job (hoisted out of the
  // job loop it would stay live through the main loop and spill).
  unsigned int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;   // 4 x 2 waves of 64 x 64
  const int h = lane >> 5, l32 = lane & 31;
  const int rowA = wr * 64 + l32, rowB = wc * 64 + l32;

  f32x16 acc[BR][BC], tot[BR][BC];
#pragma unroll
  for (int i = 0; i < BR; ++i)
#pragma unroll
    for (int j = 0; j < BC; ++j) acc[i][j] = f32x16{0};

  // The stages of the job's K stream are fetched in order, each call of dma
  // the next one: cA / cB address stage cs of the A / B panel (tiled: its
  // chunk, which advances by one chunk per stage; row-major: its column
  // offset).  A Z-job's stream switches to the second product at stage
  // spass; stages past the end re-fetch stage 0 into a slot that is never
  // read again, which keeps the vmcnt bookkeeping uniform.
  const uint32_t ldb32 = (uint32_t)ldb;
  const size_t chunkb = (size_t)P::CHUNK;
  const size_t step_b = P::TILED ? chunkb : (size_t)P::RB;   // bytes from one stage to the next
  const size_t a_hi = (size_t)spass * chunkb;                // tiled: A rows 128-255 (next row block)
  const char* cA = sb < spass ? a0 + (size_t)sb * step_b : a1 + (size_t)(sb - spass) * step_b;
  const char* cB = sb < spass ? b0 + (size_t)sb * step_b : b1 + (size_t)(sb - spass) * step_b;
  int cs = sb;
  auto dma = [&](LDS_AS char* slot) {
    if constexpr (P::TILED) dma_stage_tiled<PREC>(slot, cA, cA + a_hi, cB, wave, lane);
    else dma_stage_rows<PREC>(slot, cA, cB, ldb32, wave, lane);
    ++cs;   // selects, not branches: the stage body stays one basic block
    const bool wrap = cs >= se, second = cs == spass;
    cA = wrap ? a0 : second ? a1 : cA + step_b;
    cB = wrap ? b0 : second ? b1 : cB + step_b;
  };

  if constexpr (PREC == kFP32) {
    // FP32 products: the MFMA accumulator is added into an FP64 tile sum
    // every `flush` stages (exact outer sum: the only FP32 rounding chain
    // left is the accumulator's own, `flush` stages long).  One operand
    // register set: with 32 MFMAs of 64 cycles per stage the other wave of
    // the SIMD covers this wave's LDS reads.
    double td[BR][BC][16];
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
      for (int j = 0; j < BC; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) td[i][j][e] = 0.0;
    Ops<PREC> o;
    dma(R0);
    dma(R1);
    dma(R2);
    // Block b = (bi, bj) of the accumulator is added into the FP64 sum
    // every `flush` = 4g stages, the four blocks one stage apart (block b at
    // stages 4g q + b).  In the stage that flushes block b its MFMAs are
    // issued first; the conversions follow the stage's last MFMA, when the
    // operand registers are free and block b's chain has long completed.
    const int grp = a.flush >= 4 ? a.flush / 4 : 0;   // 0: single level
    int gq = 0;   // group of 4 stages, modulo grp
#define DMPT_ITER1(CUR, REFILL, K)                                    \
    {                                                                 \
      wait_vm<2 * P::L, true>();                                      \
      barrier_nofence();                                              \
      dma(REFILL);                                                    \
      __builtin_amdgcn_sched_barrier(0);                              \
      read_ops<PREC>(CUR, o, rowA, rowB, h);                          \
      mma_fp32_from<K>(o, acc);                                       \
      if (grp && gq == 0) {                                           \
        _Pragma("unroll") for (int e = 0; e < 16; ++e)                \
          td[(K) >> 1][(K) & 1][e] += (double)acc[(K) >> 1][(K) & 1][e]; \
        acc[(K) >> 1][(K) & 1] = f32x16{0};                           \
      }                                                               \
    }
    for (int s = 0; s < nst; s += 4) {
      DMPT_ITER1(R0, R3, 0)
      DMPT_ITER1(R1, R0, 1)
      DMPT_ITER1(R2, R1, 2)
      DMPT_ITER1(R3, R2, 3)
      if (++gq == grp) gq = 0;
    }
#undef DMPT_ITER1
    wait_vm<0, true>();
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
      for (int j = 0; j < BC; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) tot[i][j][e] = (float)(td[i][j][e] + (double)acc[i][j][e]);
  } else {
#pragma unroll
  for (int i = 0; i < BR; ++i)
#pragma unroll
    for (int j = 0; j < BC; ++j) tot[i][j] = f32x16{0};
  Ops<PREC> o0, o1;
  dma(R0);
  dma(R1);
  dma(R2);
  wait_vm<2 * P::L, false>();   // stage 0 landed (1 and 2 may be in flight)
  barrier_nofence();
  dma(R3);
  __builtin_amdgcn_sched_barrier(0);
  read_ops<PREC>(R0, o0, rowA, rowB, h);

  // Iteration s: the operands of stage s are in registers (OC).  Wait until
  // this wave's DMA of stage s+1 landed (s+2 and s+3 may be in flight) and its
  // LDS reads of stage s are done, barrier (so has every wave), refill the
  // slot of stage s with stage s+4, read stage s+1 into the other register
  // set and multiply stage s: the LDS reads of one stage overlap the MFMAs
  // of the previous one.
#define DMPT_ITER(S_, NEXT, REFILL, OC, ON)                \
  {                                                       \
    wait_vm<2 * P::L, true>();                            \
    barrier_nofence();                                    \
    dma(REFILL);   /* stage (S_) + 4 */                   \
    __builtin_amdgcn_sched_barrier(0);                    \
    read_ops<PREC>(NEXT, ON, rowA, rowB, h);              \
    mma_ops<PREC>(OC, acc);                               \
    stage_order<PREC>();                                  \
  }
  const int flj = MIX && kind == kJobZ && a.flush_z > 0 ? a.flush_z : a.flush;
  const int fl4 = flj > 0 ? flj : 1 << 30;   // flush every fl4 groups of 4 stages
  int since = 0;
  for (int s = sb; s < se; s += 4) {
    DMPT_ITER(s + 0, R1, R0, o0, o1)
    DMPT_ITER(s + 1, R2, R1, o1, o0)
    DMPT_ITER(s + 2, R3, R2, o0, o1)
    DMPT_ITER(s + 3, R0, R3, o1, o0)
    if (++since == fl4) {
      since = 0;
#pragma unroll
      for (int i = 0; i < BR; ++i)
#pragma unroll
        for (int j = 0; j < BC; ++j) {
          tot[i][j] += acc[i][j];
          acc[i][j] = f32x16{0};
        }
    }
  }
#undef DMPT_ITER
  wait_vm<0, true>();
#pragma unroll
  for (int i = 0; i < BR; ++i)
#pragma unroll
    for (int j = 0; j < BC; ++j) tot[i][j] += acc[i][j];
  }
  if constexpr (PREC == kSplitH) {
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
      for (int j = 0; j < BC; ++j) tot[i][j] *= usc;   // a power of two: exact
  }
  if (split) {
    // K-split half: the partial tile sum goes to its scratch slot (coalesced:
    // 16 stores of 1 KB per wave); the combine launch finishes the tile
    float* sb_out = a.split_buf + ((size_t)a.split_slot[jpos] * 2 + half) * kSplitTileFloats;
#pragma unroll
    for (int q = 0; q < BR * BC; ++q)
#pragma unroll
      for (int e4 = 0; e4 < 4; ++e4) {
        const f32x16& t = tot[q / BC][q % BC];
        *(f32x4*)(sb_out + ((size_t)((q * 4 + e4) * NW + wave) * 64 + lane) * 4) =
            f32x4{t[4 * e4], t[4 * e4 + 1], t[4 * e4 + 2], t[4 * e4 + 3]};
      }
    return;
  }
  if (a.oscale != 0.0f && a.oscale != 1.0f) {
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
      for (int j = 0; j < BC; ++j) tot[i][j] *= a.oscale;
  }
  step_epilogue<PREC, MIX>(a, job, sigma, tot, R0, R1, R2, R3, s_red, sc_out, s_out, 0, NW,
                           tile_index(ti, tj, a.ntile));
}

// ---------------------------------------------------------------- wide sweep jobs

// Z-jobs on 256 x 256 output tiles (I, J >= I): twice the columns of a
// regular tile for the same A panel, so a stage brings 21 bytes per MFMA
// cycle instead of 32 (two-term split) and the DMA-bound loop gets closer to
// the MFMA rate.  Eight waves as 2 x 4, each a 128 x 64 region (4 x 2 blocks
// of 32 x 32): 128 accumulator registers, so one accumulation level only —
// these jobs run only when the residual correction of chi follows, which
// removes the sweep's accumulation error.  Formats: the two-term BF16 split
// and plain BF16 (stages of 64 bytes per row, 8 KB per 128-row chunk).
constexpr int WTN = 256, WBR = 4, WBC = 2, WL = 4;
template <int PREC> struct WPipe {
  static_assert(PREC == kSplit2 || PREC == kBF16, "wide sweep jobs: two-term BF16 split or plain BF16");
  static constexpr int RB = Fmt<PREC>::RB;
  static constexpr int A_BYTES = TM * RB, B_BYTES = WTN * RB;
  static constexpr int SLOT = A_BYTES + B_BYTES;     // 32 KB: 32 one-KB DMA copies, WL per wave
  static constexpr int CHUNK = RBLK * RB;            // 8 KB: one 128-row stage chunk in HBM
  static constexpr int R = (WBR + WBC) * 2;          // ds_read_b128 per stage
  static constexpr int M = WBR * WBC * (PREC == kSplit2 ? 3 : 2);   // MFMAs per stage
};
struct WOps { bf16x8 a[WBR][2], b[WBC][2]; };        // [p]: split term (kSplit2) or k16 step (kBF16)
template <int PREC> struct WSlot { static constexpr int V = TM * Fmt<PREC>::RB + WTN * Fmt<PREC>::RB; };

// One stage into a ring slot: A rows 0-127, A rows 128-255, B rows 0-127,
// B rows 128-255, each a contiguous 8 KB chunk; wave w copies kilobyte w of each.
__device__ __forceinline__ void wdma(LDS_AS char* slot, const char* a0, const char* a1, const char* b0,
                                     const char* b1, int wave, int lane) {
  const size_t off = (size_t)wave * 1024 + (size_t)lane * 16;
  __builtin_amdgcn_global_load_lds((const GLB_AS void*)(a0 + off), (LDS_AS void*)(slot + wave * 1024), 16, 0, 0);
  __builtin_amdgcn_global_load_lds((const GLB_AS void*)(a1 + off), (LDS_AS void*)(slot + (wave + NW) * 1024), 16, 0, 0);
  __builtin_amdgcn_global_load_lds((const GLB_AS void*)(b0 + off), (LDS_AS void*)(slot + (wave + 2 * NW) * 1024), 16, 0, 0);
  __builtin_amdgcn_global_load_lds((const GLB_AS void*)(b1 + off), (LDS_AS void*)(slot + (wave + 3 * NW) * 1024), 16, 0, 0);
}

template <int PREC>
__device__ __forceinline__ void wread(const LDS_AS char* slot, WOps& o, int rowA, int rowB, int h) {
  const LDS_AS char* pA = slot;
  const LDS_AS char* pB = slot + WPipe<PREC>::A_BYTES;
#pragma unroll
  for (int i = 0; i < WBR; ++i)
#pragma unroll
    for (int p = 0; p < 2; ++p)
      o.a[i][p] = __builtin_bit_cast(bf16x8, lds16(pA + swz<4>(rowA + 32 * i, PREC == kSplit2 ? 2 * h + p : 2 * p + h)));
#pragma unroll
  for (int j = 0; j < WBC; ++j)
#pragma unroll
    for (int p = 0; p < 2; ++p)
      o.b[j][p] = __builtin_bit_cast(bf16x8, lds16(pB + swz<4>(rowB + 32 * j, PREC == kSplit2 ? 2 * h + p : 2 * p + h)));
}

// acc[i][j] += A_i B_j^T for one stage, product-major so that eight
// independent accumulator chains separate dependent MFMAs.
template <int PREC>
__device__ __forceinline__ void wmma(const WOps& o, f32x16 (&acc)[WBR][WBC]) {
  if constexpr (PREC == kSplit2) {
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int i = 0; i < WBR; ++i)
#pragma unroll
        for (int j = 0; j < WBC; ++j) {
          const int pa = q == 1 ? 1 : 0, pb = q == 0 ? 1 : 0;   // hl, lh, hh
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.a[i][pa], o.b[j][pb], acc[i][j], 0, 0, 0);
        }
  } else {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int i = 0; i < WBR; ++i)
#pragma unroll
        for (int j = 0; j < WBC; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.a[i][t], o.b[j][t], acc[i][j], 0, 0, 0);
  }
}

// The next stage's LDS reads spread among this stage's MFMAs.
template <int R, int M>
__device__ __forceinline__ void stage_order_rm() {
  if constexpr (M % R == 0) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, M / R, 0);
    }
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, M - R, 0);
  }
}

// One wide Z-job: Z_IJ = Y_I X_J^T + X_I Y_J^T (256 x 256), then the
// sigma-update, the direct and mirror stores and the operand copy of Y_{n+1}.
// MIX: X's two-term copy is op2 (three-term-X^2 option).
template <int PREC, bool MIX>
__device__ __forceinline__ void step_job_wide(const StepArgs& a, const uint32_t job, const int sigma, LDS_AS char* R0,
                                              LDS_AS char* R1, LDS_AS char* R2, LDS_AS char* R3) {
  using P = WPipe<PREC>;
  const int obs = (job >> 1) & 63;
  const int ti = (job >> 8) & 4095;    // 256-row block
  const int tj = (job >> 20) & 2047;   // 256-column block, tj >= ti
  const size_t ldb = (size_t)a.n_pad * operand_bytes(PREC);
  const int spass = a.n_pad / Fmt<PREC>::K;
  const int nst = 2 * spass;
  const char* xop = (const char*)(MIX ? a.x_in.op2 : a.x_in.op);
  const char* yop = (const char*)a.y_in.op + obs * a.y_in.stride_op;
  const size_t rowI = (size_t)ti * TM * ldb, rowJ = (size_t)tj * WTN * ldb;
  const char* a0 = yop + rowI;   // Y_I, then X_I
  const char* b0 = xop + rowJ;   // X_J, then Y_J
  const char* a1 = xop + rowI;
  const char* b1 = yop + rowJ;

  unsigned int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 2, wc = wave & 3;   // 2 x 4 waves of 128 x 64
  const int h = lane >> 5, l32 = lane & 31;
  const int rowA = wr * 128 + l32, rowB = wc * 64 + l32;

  f32x16 acc[WBR][WBC];
#pragma unroll
  for (int i = 0; i < WBR; ++i)
#pragma unroll
    for (int j = 0; j < WBC; ++j) acc[i][j] = f32x16{0};

  const size_t chunkb = (size_t)P::CHUNK;
  const size_t hi = (size_t)spass * chunkb;   // rows 128-255 of a 256-row panel: the next row block
  const char* cA = a0;
  const char* cB = b0;
  int cs = 0;
  auto dma = [&](LDS_AS char* slot) {
    wdma(slot, cA, cA + hi, cB, cB + hi, wave, lane);
    ++cs;
    const bool wrap = cs >= nst, second = cs == spass;
    cA = wrap ? a0 : second ? a1 : cA + chunkb;
    cB = wrap ? b0 : second ? b1 : cB + chunkb;
  };
  WOps o0, o1;
  dma(R0);
  dma(R1);
  dma(R2);
  wait_vm<2 * WL, false>();
  barrier_nofence();
  dma(R3);
  __builtin_amdgcn_sched_barrier(0);
  wread<PREC>(R0, o0, rowA, rowB, h);
#define DMPT_WITER(NEXT, REFILL, OC, ON)          \
  {                                               \
    wait_vm<2 * WL, true>();                      \
    barrier_nofence();                            \
    dma(REFILL);                                  \
    __builtin_amdgcn_sched_barrier(0);            \
    wread<PREC>(NEXT, ON, rowA, rowB, h);         \
    wmma<PREC>(OC, acc);                          \
    stage_order_rm<P::R, P::M>();                 \
  }
  for (int s = 0; s < nst; s += 4) {
    DMPT_WITER(R1, R0, o0, o1)
    DMPT_WITER(R2, R1, o1, o0)
    DMPT_WITER(R3, R2, o0, o1)
    DMPT_WITER(R0, R3, o1, o0)
  }
#undef DMPT_WITER
  wait_vm<0, true>();
  if (a.oscale != 0.0f && a.oscale != 1.0f) {
#pragma unroll
    for (int i = 0; i < WBR; ++i)
#pragma unroll
      for (int j = 0; j < WBC; ++j) acc[i][j] *= a.oscale;
  }

  // ---------------------------------------------------------- epilogue
  const size_t np = a.n_pad;
  const float* cur = a.y_in.f32 + obs * a.y_in.stride_f32;
  float* o32 = a.y_out.f32 + obs * a.y_out.stride_f32;
  char* oop = (char*)a.y_out.op + obs * a.y_out.stride_op;
  const int nstp = a.n_pad / Fmt<PREC>::K;
  const bool wsplit = a.write_split != 0;
  const bool need_cur = sigma < 0;
  const int gr_base = ti * TM + wr * 128, gc0 = tj * WTN + wc * 64;
  if (ti != tj) {
    // Off-diagonal tile: the wave's 128 x 64 region in two 64 x 64 halves,
    // each staged in the wave's private LDS area (the ring, free after the
    // barrier) and stored as rows of 16-byte vectors, direct and mirrored.
    barrier_nofence();
    LDS_AS char* rb = (wave >> 1) == 0 ? R0 : (wave >> 1) == 1 ? R1 : (wave >> 1) == 2 ? R2 : R3;
    LDS_AS float* T = (LDS_AS float*)(rb + (wave & 1) * kStageBytes);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int gr0 = gr_base + half * 64;
      if (half) wait_vm<63, true>();   // this wave's reads of the first half are done
      // 32x32 MFMA output layout: lane l, register 4g+e holds row 8g + 4(l/32) + e, column l%32.
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < WBC; ++bj)
#pragma unroll
          for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int e = 0; e < 4; ++e)
              T[(bi * 32 + 8 * g + 4 * h + e) * kLS + bj * 32 + l32] = acc[2 * half + bi][bj][4 * g + e];
      wait_vm<63, true>();
#pragma unroll 4
      for (int rd = 0; rd < 16; ++rd) {
        const int r = 4 * rd + (lane >> 4), c = 4 * (lane & 15);
        f32x4 v = f32x4{T[r * kLS + c], T[r * kLS + c + 1], T[r * kLS + c + 2], T[r * kLS + c + 3]};
        if (need_cur) {
          const f32x4 x = *(const f32x4*)(cur + (size_t)(gr0 + r) * np + gc0 + c);
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            v[k] = 2.0f * x[k] - v[k];
            T[r * kLS + c + k] = v[k];
          }
        }
        *(f32x4*)(o32 + (size_t)(gr0 + r) * np + gc0 + c) = v;
      }
      wait_vm<63, true>();
#pragma unroll 4
      for (int rd = 0; rd < 16; ++rd) {
        const int c = 4 * rd + (lane >> 4), q = 4 * (lane & 15);
        *(f32x4*)(o32 + (size_t)(gc0 + c) * np + gr0 + q) =
            f32x4{T[q * kLS + c], T[(q + 1) * kLS + c], T[(q + 2) * kLS + c], T[(q + 3) * kLS + c]};
      }
      if (wsplit) {
#pragma unroll 2
        for (int rd = 0; rd < 8; ++rd) {
          const int r = 8 * rd + (lane >> 3), c = 8 * (lane & 7);
          float v[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) v[k] = T[r * kLS + c + k];
          store_group8_t<PREC>(oop, nstp, gr0 + r, gc0 + c, v, 1.0f);
        }
#pragma unroll 2
        for (int rd = 0; rd < 8; ++rd) {
          const int c = 8 * rd + (lane >> 3), q = 8 * (lane & 7);
          float v[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) v[k] = T[(q + k) * kLS + c];
          store_group8_t<PREC>(oop, nstp, gc0 + c, gr0 + q, v, 1.0f);
        }
      }
    }
  } else {
    // Diagonal tile: keep the upper triangle (row <= col) and mirror it.
#pragma unroll
    for (int bi = 0; bi < WBR; ++bi)
#pragma unroll
      for (int bj = 0; bj < WBC; ++bj) {
        const int col = gc0 + bj * 32 + l32;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int row0 = gr_base + bi * 32 + 8 * g + 4 * h;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int r = row0 + e;
            if (r > col) continue;
            float v = acc[bi][bj][4 * g + e];
            if (need_cur) v = 2.0f * cur[(size_t)r * np + col] - v;
            o32[(size_t)r * np + col] = v;
            o32[(size_t)col * np + r] = v;
            if (wsplit) {
              store_split1<PREC>(oop, nstp, r, col, v, 1.0f);
              if (r != col) store_split1<PREC>(oop, nstp, col, r, v, 1.0f);
            }
          }
        }
      }
  }
}

// The step kernel: a persistent grid over the job list.  PP is the operand
// format of the P-jobs, PZ of the Z-jobs (equal except for the three-term-X^2
// option, whose sweep products read two-term copies).
template <int PP, int PZ, bool ZW>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_step(StepArgs a) {
  // Ring slots; after the main loop each holds the 64 x 65 FP32 staging
  // areas of two waves for the epilogue.  ZW: the Z-jobs are wide (256 x 256).
  constexpr int SLOTP = Pipe<PP>::SLOT;
  constexpr int SLOTZ = ZW ? WSlot<PZ>::V : Pipe<PZ>::SLOT;
  constexpr int SLOTM = SLOTP > SLOTZ ? SLOTP : SLOTZ;
  constexpr int RSZ = SLOTM > 2 * kStageBytes ? SLOTM : 2 * kStageBytes;
  __shared__ __attribute__((aligned(1024))) char ring0[RSZ];
  __shared__ __attribute__((aligned(1024))) char ring1[RSZ];
  __shared__ __attribute__((aligned(1024))) char ring2[RSZ];
  __shared__ __attribute__((aligned(1024))) char ring3[RSZ];
  __shared__ int s_code;
  __shared__ int s_zskip;
  __shared__ int s_job;
  __shared__ double s_red[3 * NW];
  __shared__ double s_nrm;

  if (blockIdx.x == 0 && threadIdx.x < kXcdQueues) a.qclear[threadIdx.x * kQStride] = 0u;
  if (a.decide && a.ctl->done) return;
  int sigma;
  bool zskip = false;
  if (a.decide) {
    const int code = step_controller(a, &s_code, &s_zskip);
    if (!(code == 1 || code == -1)) return;
    sigma = code;
    zskip = s_zskip != 0;
  } else {
    sigma = a.sigma_src ? a.sigma_src[a.step].sigma : a.fixed_sigma;
  }

  // Persistent loop: thread 0 takes the next ticket of this XCD's queue, and
  // once that queue is used up, of the others in turn; a ticket past a
  // queue's end marks that queue used up for this workgroup, so every
  // workgroup leaves after at most njobs + 8 tickets.
  const int home = (int)(__builtin_amdgcn_s_getreg(kHwRegXccId) & (kXcdQueues - 1));
  unsigned int used_up = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      int pos = -1;
      for (int k = 0; k < kXcdQueues && pos < 0; ++k) {
        const int q = (home + k) & (kXcdQueues - 1);
        if (used_up & (1u << q)) continue;
        const unsigned t = atomicAdd(&a.qhead[q * kQStride], 1u);
        const size_t p = (size_t)t * kXcdQueues + q;
        if (p < (size_t)a.njobs) pos = (int)p;
        else used_up |= 1u << q;
      }
      s_job = pos;
    }
    // every wave is past the previous job's epilogue (LDS staging, s_red)
    // before the next job's DMA refills the ring
    wait_vm<63, true>();
    barrier_nofence();
    const int jpos = s_job;
    if (jpos < 0) break;
    const uint32_t job = a.jobs[jpos];
    if (zskip && (job & 1) == kJobZ) {   // the sweep has stopped (ytol2)
      __syncthreads();   // every thread has read s_job before thread 0 takes the next ticket
      continue;
    }
    LDS_AS char* R0 = (LDS_AS char*)ring0;
    LDS_AS char* R1 = (LDS_AS char*)ring1;
    LDS_AS char* R2 = (LDS_AS char*)ring2;
    LDS_AS char* R3 = (LDS_AS char*)ring3;
    constexpr bool MIX = PP != PZ;
    if constexpr (ZW) {
      if ((job & (kJobSplit | kJobWide)) == kJobWide) step_job_wide<PZ, MIX>(a, job, sigma, R0, R1, R2, R3);
      else if (MIX && (job & 1) == kJobZ) step_job<PZ, true>(a, job, jpos, sigma, R0, R1, R2, R3, s_red, &s_nrm);
      else step_job<PP, MIX>(a, job, jpos, sigma, R0, R1, R2, R3, s_red, &s_nrm);
    } else if constexpr (!MIX) {
      step_job<PP>(a, job, jpos, sigma, R0, R1, R2, R3, s_red, &s_nrm);
    } else {
      if ((job & 1) == kJobZ) step_job<PZ, true>(a, job, jpos, sigma, R0, R1, R2, R3, s_red, &s_nrm);
      else step_job<PP, true>(a, job, jpos, sigma, R0, R1, R2, R3, s_red, &s_nrm);
    }
  }
}

// Workgroups of a persistent step launch: one per CU (the step kernel's LDS
// use allows no second workgroup on a CU), never more than the jobs.
int persistent_grid(int njobs) {
  constexpr int kMaxDevices = 64;
  static int cus[kMaxDevices] = {};   // per device; concurrent first calls store the same value
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
  if (cus[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cus[dev] = n;
  }
  return njobs < cus[dev] ? njobs : cus[dev];
}

hipError_t launch_step(int prec, StepArgs args, int njobs, hipStream_t s, bool wide) {
  if (njobs <= 0) return hipSuccess;
  args.njobs = njobs;
  const dim3 grid(persistent_grid(njobs));
  if (wide) {
    switch (prec) {
      case kSplit2: hipLaunchKernelGGL((k_step<kSplit2, kSplit2, true>), grid, dim3(NT), 0, s, args); break;
      case kSplit32: hipLaunchKernelGGL((k_step<kSplit3, kSplit2, true>), grid, dim3(NT), 0, s, args); break;
      case kBF16: hipLaunchKernelGGL((k_step<kBF16, kBF16, true>), grid, dim3(NT), 0, s, args); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (prec) {
    case kFP32: hipLaunchKernelGGL((k_step<kFP32, kFP32, false>), grid, dim3(NT), 0, s, args); break;
    case kSplit2: hipLaunchKernelGGL((k_step<kSplit2, kSplit2, false>), grid, dim3(NT), 0, s, args); break;
    case kSplit3: hipLaunchKernelGGL((k_step<kSplit3, kSplit3, false>), grid, dim3(NT), 0, s, args); break;
    case kSplit32: hipLaunchKernelGGL((k_step<kSplit3, kSplit2, false>), grid, dim3(NT), 0, s, args); break;
    case kBF16: hipLaunchKernelGGL((k_step<kBF16, kBF16, false>), grid, dim3(NT), 0, s, args); break;
    case kSplitH: hipLaunchKernelGGL((k_step<kSplitH, kSplitH, false>), grid, dim3(NT), 0, s, args); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Combine launch of K-split tiles (see kJobSplit): four workgroups of two
// waves per split tile q (the slot), workgroup 4q + s taking the tile's row
// stripe s (waves 2s, 2s + 1 of the step kernel's eight), add the two partial
// sums and run those waves' part of the tile's epilogue with the sigma of the
// step launch it follows.  The X^2 partials of stripe 0 go to the tile's own
// entry, those of stripes 1-3 to entries 3q + s - 1 after the step tiles'
// (the next launch's controller sums nparts = tiles + 3 x split tiles).
constexpr int kCombWaves = 2, kCombStripes = NW / kCombWaves;
template <int PP, int PZ>
__global__ __launch_bounds__(kCombWaves * 64) void k_step_combine(StepArgs a, const uint32_t* cjobs) {
  __shared__ __attribute__((aligned(1024))) char stage[kCombWaves * kStageBytes];
  __shared__ double s_red[3 * kCombWaves];
  const int q = blockIdx.x / kCombStripes, stripe = blockIdx.x % kCombStripes;
  const uint32_t job = cjobs[q];
  const int kind = job & 1;
  const int tiles = (a.n_pad / TM) * (a.n_pad / TM + 1);
  // A Z tile has no X^2 partials, but the next launch's controller sums the
  // three extra entries of every split slot: they are zeroed (before any
  // early return; only step launches with the controller read partials)
  if (a.decide && kind == kJobZ && stripe > 0 && threadIdx.x == 0)
    a.part_out[tiles + 3 * q + stripe - 1] = Part{0.0, 0.0, 0.0, 0.0};
  int sigma;
  if (a.decide) {
    // the step launch recorded sigma_n, or 0 when it stopped (or never ran
    // after the stop); its Z-jobs were skipped once the sweep had stopped
    sigma = a.ctl->rec[a.step].sigma;
    if (!(sigma == 1 || sigma == -1)) return;
    if (kind == kJobZ && a.ytol2 > 0.0 && a.ctl->ystop != 0 && a.step >= a.ctl->ystop) return;
  } else {
    sigma = a.sigma_src ? a.sigma_src[a.step].sigma : a.fixed_sigma;
  }
  const int lane = threadIdx.x & 63;
  const int wave_base = stripe * kCombWaves;
  const int wave = wave_base + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const float* h0 = a.split_buf + (size_t)q * 2 * kSplitTileFloats;
  const float* h1 = h0 + kSplitTileFloats;
  f32x16 tot[BR][BC];
#pragma unroll
  for (int qq = 0; qq < BR * BC; ++qq)
#pragma unroll
    for (int e4 = 0; e4 < 4; ++e4) {
      const size_t off = ((size_t)((qq * 4 + e4) * NW + wave) * 64 + lane) * 4;
      const f32x4 u = *(const f32x4*)(h0 + off), v = *(const f32x4*)(h1 + off);
#pragma unroll
      for (int e = 0; e < 4; ++e) tot[qq / BC][qq % BC][4 * e4 + e] = u[e] + v[e];
    }
  if (a.oscale != 0.0f && a.oscale != 1.0f) {
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
      for (int j = 0; j < BC; ++j) tot[i][j] *= a.oscale;
  }
  // wave w stages in R[w / 2] + (w % 2) blocks: this workgroup's two waves
  // (2 stripe, 2 stripe + 1) both map to the one staging area
  LDS_AS char* R = (LDS_AS char*)stage;
  const int ti = (job >> 8) & 4095, tj = (job >> 20) & 2047;
  const int part_idx = stripe == 0 ? tile_index(ti, tj, a.ntile) : tiles + 3 * q + stripe - 1;
  constexpr bool MIX = PP != PZ;
  if (MIX && kind == kJobZ)
    step_epilogue<PZ, true>(a, job, sigma, tot, R, R, R, R, s_red, 1.0f, 0, wave_base, kCombWaves, part_idx);
  else
    step_epilogue<PP, MIX>(a, job, sigma, tot, R, R, R, R, s_red, 1.0f, 0, wave_base, kCombWaves, part_idx);
}

hipError_t launch_step_combine(int prec, StepArgs args, const uint32_t* cjobs, int ncomb, hipStream_t s) {
  if (ncomb <= 0) return hipSuccess;
  const dim3 grid(ncomb * kCombStripes), block(kCombWaves * 64);
  switch (prec) {
    case kSplit2: hipLaunchKernelGGL((k_step_combine<kSplit2, kSplit2>), grid, block, 0, s, args, cjobs); break;
    case kSplit32: hipLaunchKernelGGL((k_step_combine<kSplit3, kSplit2>), grid, block, 0, s, args, cjobs); break;
    case kBF16: hipLaunchKernelGGL((k_step_combine<kBF16, kBF16>), grid, block, 0, s, args, cjobs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ void k_queue_reset(Ctl* c) {
  unsigned int* q = &c->qhead[0][0];
  for (int i = threadIdx.x; i < kQSets * kXcdQueues * kQStride; i += blockDim.x) q[i] = 0u;
}

hipError_t launch_queue_reset(Ctl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(256), 0, s, ctl);
  return hipGetLastError();
}

// ---------------------------------------------------------------- general products

// C = alpha A B^T over all 256 x 128 tiles of an n_pad x n_pad result (or,
// with sym, only the tiles (I, J >= 2I) that cover the upper triangle, for a
// product known to be symmetric); C is n_pad x n_pad row-major FP32 (zero
// padded).  The operands are FP32 row-major (PREC = kFP32) or tiled FP16
// split copies (PREC = kSplitH; alpha then carries the 2^-(s_a + s_b) that
// undoes their scales).  Used for the congruences of the non-orthonormal
// basis (Sec. V.A: Z^T H Z, Z^T A Z, Z D Z^T, two NT products each) and the
// products of the finite-temperature recursion (Sec. V.B).  Same operand
// pipeline as the step kernel (DMA into the four-slot LDS ring, MFMA,
// two-level accumulation every `flush` groups of 4 stages); the epilogue
// stores the tile as is.
template <int PREC>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gemm_nt(
    const void* A, const void* B, float* C, int n_pad, float alpha, int flush, int sym) {
  using P = Pipe<PREC>;
  __shared__ __attribute__((aligned(1024))) char ring0[P::SLOT];
  __shared__ __attribute__((aligned(1024))) char ring1[P::SLOT];
  __shared__ __attribute__((aligned(1024))) char ring2[P::SLOT];
  __shared__ __attribute__((aligned(1024))) char ring3[P::SLOT];
  const int tcols = n_pad / TN;
  int ti, tj;
  if (sym) {   // row-major order over the triangle tiles
    int b = blockIdx.x;
    ti = 0;
    while (b >= tcols - 2 * ti) {
      b -= tcols - 2 * ti;
      ++ti;
    }
    tj = 2 * ti + b;
  } else {
    ti = blockIdx.x / tcols;
    tj = blockIdx.x % tcols;
  }
  // row block I / J starts at the same byte offset in the row-major and the
  // tiled layouts (rows * ldb, or row blocks * nst chunks of 128 rows)
  const size_t ldb = (size_t)n_pad * operand_bytes(PREC);
  const uint32_t ldb32 = (uint32_t)ldb;
  const int nst = n_pad / Fmt<PREC>::K;
  const char* a0 = (const char*)A + (size_t)ti * TM * ldb;
  const char* b0 = (const char*)B + (size_t)tj * TN * ldb;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int h = lane >> 5, l32 = lane & 31;
  const int rowA = wr * 64 + l32, rowB = wc * 64 + l32;
  f32x16 acc[BR][BC], tot[BR][BC];
#pragma unroll
  for (int i = 0; i < BR; ++i)
#pragma unroll
    for (int j = 0; j < BC; ++j) {
      acc[i][j] = f32x16{0};
      tot[i][j] = f32x16{0};
    }
  // stages past the end re-fetch stage 0 into a slot that is never read again
  auto dma = [&](LDS_AS char* slot, int s) {
    const int st = s < nst ? s : 0;
    if constexpr (P::TILED) {
      const char* ca = a0 + (size_t)st * P::CHUNK;
      dma_stage_tiled<PREC>(slot, ca, ca + (size_t)nst * P::CHUNK, b0 + (size_t)st * P::CHUNK, wave, lane);
    } else {
      const size_t kb = (size_t)st * P::RB;
      dma_stage_rows<PREC>(slot, a0 + kb, b0 + kb, ldb32, wave, lane);
    }
  };
  LDS_AS char* R0 = (LDS_AS char*)ring0;
  LDS_AS char* R1 = (LDS_AS char*)ring1;
  LDS_AS char* R2 = (LDS_AS char*)ring2;
  LDS_AS char* R3 = (LDS_AS char*)ring3;
  Ops<PREC> o0, o1;
  dma(R0, 0);
  dma(R1, 1);
  dma(R2, 2);
  wait_vm<2 * P::L, false>();
  barrier_nofence();
  dma(R3, 3);
  __builtin_amdgcn_sched_barrier(0);
  read_ops<PREC>(R0, o0, rowA, rowB, h);
#define DMPT_GITER(S_, NEXT, REFILL, OC, ON)              \
  {                                                       \
    wait_vm<2 * P::L, true>();                            \
    barrier_nofence();                                    \
    dma(REFILL, (S_) + 4);                                \
    __builtin_amdgcn_sched_barrier(0);                    \
    read_ops<PREC>(NEXT, ON, rowA, rowB, h);              \
    mma_ops<PREC>(OC, acc);                               \
    stage_order<PREC>();                                  \
  }
  const int fl4 = flush > 0 ? flush : 1 << 30;
  int since = 0;
  for (int s = 0; s < nst; s += 4) {
    DMPT_GITER(s + 0, R1, R0, o0, o1)
    DMPT_GITER(s + 1, R2, R1, o1, o0)
    DMPT_GITER(s + 2, R3, R2, o0, o1)
    DMPT_GITER(s + 3, R0, R3, o1, o0)
    if (++since == fl4) {
      since = 0;
#pragma unroll
      for (int i = 0; i < BR; ++i)
#pragma unroll
        for (int j = 0; j < BC; ++j) {
          tot[i][j] += acc[i][j];
          acc[i][j] = f32x16{0};
        }
    }
  }
#undef DMPT_GITER
  wait_vm<0, true>();
  // 32x32 MFMA output layout: lane l, register 4g+e holds row 8g + 4(l/32) + e, column l%32.
#pragma unroll
  for (int bi = 0; bi < BR; ++bi)
#pragma unroll
    for (int bj = 0; bj < BC; ++bj) {
      const f32x16 v = tot[bi][bj] + acc[bi][bj];
      const int col = tj * TN + wc * 64 + bj * 32 + l32;
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = ti * TM + wr * 64 + bi * 32 + 8 * g + 4 * h + e;
          C[(size_t)r * n_pad + col] = alpha * v[4 * g + e];
        }
    }
}

hipError_t launch_gemm_nt(const float* A, const float* B, float* C, int n_pad, float alpha, int flush,
                          hipStream_t s) {
  if (n_pad <= 0 || n_pad % TM != 0) return hipErrorInvalidValue;
  const int tiles = (n_pad / TM) * (n_pad / TN);
  hipLaunchKernelGGL(k_gemm_nt<kFP32>, dim3(tiles), dim3(NT), 0, s, A, B, C, n_pad, alpha, flush, 0);
  return hipGetLastError();
}

// Strictly lower triangle of C := transpose of the upper one (64 x 64 blocks
// through LDS; blocks above the diagonal are read, never written).
__global__ __launch_bounds__(256) void k_mirror_lower(float* C, int n_pad) {
  __shared__ float t[64][65];
  const int bi = blockIdx.y, bj = blockIdx.x;   // destination block (bi >= bj)
  if (bi < bj) return;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    t[r][c] = C[(size_t)(bj * 64 + r) * n_pad + bi * 64 + c];   // source block (bj, bi)
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    if (bi == bj && r <= c) continue;
    C[(size_t)(bi * 64 + r) * n_pad + bj * 64 + c] = t[c][r];
  }
}

hipError_t launch_gemm_nt_sym(const float* A, const float* B, float* C, int n_pad, float alpha, int flush,
                              hipStream_t s) {
  return launch_gemm_op(kFP32, A, B, C, n_pad, alpha, flush, 1, s);
}

hipError_t launch_gemm_op(int prec, const void* A, const void* B, float* C, int n_pad, float alpha, int flush,
                          int sym, hipStream_t s) {
  if (n_pad <= 0 || n_pad % TM != 0) return hipErrorInvalidValue;
  const int tr = n_pad / TM;
  const int tiles = sym ? tr * (tr + 1) : (n_pad / TM) * (n_pad / TN);
  switch (prec) {
    case kFP32: hipLaunchKernelGGL(k_gemm_nt<kFP32>, dim3(tiles), dim3(NT), 0, s, A, B, C, n_pad, alpha, flush, sym); break;
    case kSplitH: hipLaunchKernelGGL(k_gemm_nt<kSplitH>, dim3(tiles), dim3(NT), 0, s, A, B, C, n_pad, alpha, flush, sym); break;
    case kSplit3: hipLaunchKernelGGL(k_gemm_nt<kSplit3>, dim3(tiles), dim3(NT), 0, s, A, B, C, n_pad, alpha, flush, sym); break;
    case kSplit2: hipLaunchKernelGGL(k_gemm_nt<kSplit2>, dim3(tiles), dim3(NT), 0, s, A, B, C, n_pad, alpha, flush, sym); break;
    default: return hipErrorInvalidValue;
  }
  if (sym) {
    const int nb = n_pad / 64;
    hipLaunchKernelGGL(k_mirror_lower, dim3(nb, nb), dim3(256), 0, s, C, n_pad);
  }
  return hipGetLastError();
}

// dst (n_pad x n_pad, zero padded) = src (n x n, row-major, ld n), or its
// transpose; one 64 x 64 block per workgroup, transposed through LDS.
__global__ __launch_bounds__(256) void k_pad(const float* src, int n, int n_pad, float* dst, int transpose) {
  __shared__ float tile[64][65];
  const int bi = blockIdx.y, bj = blockIdx.x;          // output block
  const int si = transpose ? bj : bi, sj = transpose ? bi : bj;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    const int gi = si * 64 + r, gj = sj * 64 + c;
    tile[r][c] = (gi < n && gj < n) ? src[(size_t)gi * n + gj] : 0.0f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    dst[(size_t)(bi * 64 + r) * n_pad + bj * 64 + c] = transpose ? tile[c][r] : tile[r][c];
  }
}

hipError_t launch_pad(const float* src, int n, int n_pad, float* dst, int transpose, hipStream_t s) {
  const int nb = n_pad / 64;
  hipLaunchKernelGGL(k_pad, dim3(nb, nb), dim3(256), 0, s, src, n, n_pad, dst, transpose);
  return hipGetLastError();
}

// ---------------------------------------------------------------- control

__global__ void k_ctl_reset(Ctl* c) {
  char* p = (char*)c;
  for (size_t i = threadIdx.x; i < sizeof(Ctl); i += blockDim.x) p[i] = 0;
}

hipError_t launch_ctl_reset(Ctl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(256), 0, s, ctl);
  return hipGetLastError();
}

__device__ void set_coeffs(Ctl* c, double emin, double emax) {
  c->emin = emin;
  c->emax = emax;
  const double w = emax - emin;
  c->alpha = emax / w;   // Eq. DM0: X_1 = alpha I + beta H maps [emin, emax] onto [1, 0]
  c->beta = -1.0 / w;
}

__global__ void k_set_bounds(Ctl* c, double emin, double emax) {
  if (threadIdx.x == 0) set_coeffs(c, emin, emax);
}

hipError_t launch_set_bounds(Ctl* ctl, double emin, double emax, hipStream_t s) {
  hipLaunchKernelGGL(k_set_bounds, dim3(1), dim3(64), 0, s, ctl, emin, emax);
  return hipGetLastError();
}

// ---------------------------------------------------------------- Gershgorin

// One wave per row: c_i = H_ii, r_i = sum_{j != i} |H_ij| (FP64).  Each block
// reduces its rows to (min c - r, max c + r); block partials go to scratch.
constexpr int kGershRowsPerBlock = 16;   // 4 waves x 4 rows

int gershgorin_blocks(int n) { return (n + kGershRowsPerBlock - 1) / kGershRowsPerBlock; }

__global__ __launch_bounds__(256) void k_gersh_rows(const float* h, int n, double2* part, Ctl* ctl) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ double s_lo[4], s_hi[4];
  double lo = INFINITY, hi = -INFINITY;
  int bad = 0;
  for (int k = 0; k < 4; ++k) {
    const int i = blockIdx.x * kGershRowsPerBlock + wave * 4 + k;
    if (i >= n) break;
    const float* row = h + (size_t)i * n;
    double rs = 0.0;
    if ((n & 3) == 0 && ((uintptr_t)h & 15) == 0) {   // 16-byte loads, 4 consecutive columns per lane
      const f32x4* row4 = (const f32x4*)row;
      for (int q = lane; q < (n >> 2); q += 64) {
        const f32x4 x = row4[q];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (!isfinite(x[e])) bad = 1;
          if (4 * q + e != i) rs += fabs((double)x[e]);
        }
      }
    } else {
      for (int j = lane; j < n; j += 64) {
        const float x = row[j];
        if (!isfinite(x)) bad = 1;
        if (j != i) rs += fabs((double)x);
      }
    }
    rs = wave_sum(rs);
    const double c = row[i];
    lo = fmin(lo, c - rs);
    hi = fmax(hi, c + rs);
  }
  if (bad) ctl->nonfinite = 1;
  if (lane == 0) {
    s_lo[wave] = lo;
    s_hi[wave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      s_lo[0] = fmin(s_lo[0], s_lo[w]);
      s_hi[0] = fmax(s_hi[0], s_hi[w]);
    }
    part[blockIdx.x] = double2{s_lo[0], s_hi[0]};
  }
}

__global__ __launch_bounds__(256) void k_gersh_final(const double2* part, int nblk, Ctl* ctl, int set) {
  __shared__ double s_lo[256], s_hi[256];
  double lo = INFINITY, hi = -INFINITY;
  for (int b = threadIdx.x; b < nblk; b += 256) {
    lo = fmin(lo, part[b].x);
    hi = fmax(hi, part[b].y);
  }
  s_lo[threadIdx.x] = lo;
  s_hi[threadIdx.x] = hi;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      s_lo[threadIdx.x] = fmin(s_lo[threadIdx.x], s_lo[threadIdx.x + st]);
      s_hi[threadIdx.x] = fmax(s_hi[threadIdx.x], s_hi[threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double g0 = s_lo[0], g1 = s_hi[0];
    if (!(g1 > g0)) {   // scalar spectrum (e.g. H = c I or n = 1): widen symmetrically
      const double d = fmax(1.0, fabs(g0)) * 1e-3;
      g0 -= d;
      g1 += d;
    }
    ctl->gmin = g0;
    ctl->gmax = g1;
    if (set) set_coeffs(ctl, g0, g1);
  }
}

hipError_t launch_gershgorin(const float* h, int n, double2* scratch, int nblk, Ctl* ctl,
                             int set_coeffs, hipStream_t s) {
  hipLaunchKernelGGL(k_gersh_rows, dim3(nblk), dim3(256), 0, s, h, n, scratch, ctl);
  hipLaunchKernelGGL(k_gersh_final, dim3(1), dim3(256), 0, s, scratch, nblk, ctl, set_coeffs);
  return hipGetLastError();
}

// ---------------------------------------------------------------- Lanczos

// v_1: deterministic pseudo-random start (splitmix64 of the index), normalised.
__device__ __forceinline__ double hash_unit(unsigned long long i) {
  unsigned long long z = i + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

__global__ __launch_bounds__(1024) void k_lanczos_start(double* v, double* vprev, int n) {
  __shared__ double s[16];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    const double x = hash_unit(i);
    v[i] = x;
    vprev[i] = 0.0;
    acc += x * x;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  double tot = 0.0;
  for (int w = 0; w < 16; ++w) tot += s[w];
  const double inv = 1.0 / sqrt(tot);
  for (int i = threadIdx.x; i < n; i += 1024) v[i] *= inv;
}

// w = H v, one wave per row, FP64 accumulation.
// One wave per row.  When rows are 16-byte aligned (n % 4 == 0, aligned H) each lane
// takes 4 consecutive columns per load, two loads in flight on separate
// accumulators; otherwise one column per lane.  The summation order is fixed.
__global__ __launch_bounds__(256) void k_gemv(const float* h, const double* v, double* w, int n) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const float* row = h + (size_t)i * n;
  double acc0 = 0.0, acc1 = 0.0;
  if ((n & 3) == 0 && ((uintptr_t)h & 15) == 0) {
    const int n4 = n >> 2;
    const f32x4* row4 = (const f32x4*)row;
    int q = lane;
    for (; q + 64 < n4; q += 128) {
      const f32x4 x0 = row4[q], x1 = row4[q + 64];
      const double* v0 = v + 4 * (size_t)q;
      const double* v1 = v0 + 256;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc0 += (double)x0[e] * v0[e];
        acc1 += (double)x1[e] * v1[e];
      }
    }
    if (q < n4) {
      const f32x4 x0 = row4[q];
#pragma unroll
      for (int e = 0; e < 4; ++e) acc0 += (double)x0[e] * v[4 * (size_t)q + e];
    }
  } else {
    for (int j = lane; j < n; j += 64) acc0 += (double)row[j] * v[j];
  }
  const double acc = wave_sum(acc0 + acc1);
  if (lane == 0) w[i] = acc;
}

// alpha_j = v.w ; w -= alpha_j v + beta_{j-1} vprev ; beta_j = |w| ; vprev = v ; v = w / beta_j
__global__ __launch_bounds__(1024) void k_lanczos_update(double* v, double* vprev, double* w,
                                                         double* ab, int j, int n) {
  __shared__ double s[16];
  __shared__ double s_alpha;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) acc += v[i] * w[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < 16; ++q) t += s[q];
    s_alpha = t;
  }
  __syncthreads();
  const double alpha = s_alpha;
  const double bprev = j > 0 ? ab[2 * j - 1] : 0.0;
  acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    const double x = w[i] - alpha * v[i] - bprev * vprev[i];
    w[i] = x;
    acc += x * x;
  }
  acc = wave_sum(acc);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  double nrm2 = 0.0;
  for (int q = 0; q < 16; ++q) nrm2 += s[q];
  const double beta = sqrt(nrm2);
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    vprev[i] = v[i];
    v[i] = w[i] * inv;
  }
  if (threadIdx.x == 0) {
    ab[2 * j] = alpha;
    ab[2 * j + 1] = beta;
  }
}

hipError_t launch_lanczos_start(double* v, double* vprev, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_lanczos_start, dim3(1), dim3(1024), 0, s, v, vprev, n);
  return hipGetLastError();
}

hipError_t launch_lanczos_step(const float* h, int n, double* v, double* vprev, double* w,
                               double* ab, int j, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv, dim3((n + 3) / 4), dim3(256), 0, s, h, v, w, n);
  hipLaunchKernelGGL(k_lanczos_update, dim3(1), dim3(1024), 0, s, v, vprev, w, ab, j, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- operand copies

__device__ __forceinline__ void store_group8(int prec, char* op, int n_pad, int r, int c0, const float (&v)[8],
                                             float sc) {
  if (prec == kSplit2) store_group8_t<kSplit2>(op, n_pad / Fmt<kSplit2>::K, r, c0, v, sc);
  else if (prec == kSplit3) store_group8_t<kSplit3>(op, n_pad / Fmt<kSplit3>::K, r, c0, v, sc);
  else if (prec == kBF16) store_group8_t<kBF16>(op, n_pad / Fmt<kBF16>::K, r, c0, v, sc);
  else if (prec == kSplitH) store_group8_t<kSplitH>(op, n_pad / Fmt<kSplitH>::K, r, c0, v, sc);
}

// Rebuild the operand copy of nmat matrices from their FP32 masters.  For
// kSplitH (used for the Y matrices written by k_init) the scale comes from
// the matrix's own norm partials: |M_ij| <= ||M||_F, and block (0, z) records
// the exponent in the matrix's metadata.
__global__ __launch_bounds__(256) void k_resplit(int prec, MatRef m, int n_pad) {
  __shared__ double s_nrm;
  const int z = blockIdx.y;
  const float* src = m.f32 + (size_t)z * m.stride_f32;
  char* dst = (char*)m.op + (size_t)z * m.stride_op;
  float sc = 1.0f;
  if (prec == kSplitH) {
    MatMeta* mm = (MatMeta*)(m.meta + (size_t)z * m.stride_op);
    const int e = yscale_exp(meta_norm(mm, (n_pad / 64) * (n_pad / 64), &s_nrm), 1.0);
    sc = ldexpf(1.0f, e);
    if (blockIdx.x == 0 && threadIdx.x == 0) mm->scale = e;
  }
  const size_t ngroups = (size_t)n_pad * n_pad / 8;
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < ngroups; g += (size_t)gridDim.x * 256) {
    const size_t r = g / (n_pad / 8);
    const int c0 = (int)(g % (n_pad / 8)) * 8;
    const f32x4 a = *(const f32x4*)(src + r * n_pad + c0);
    const f32x4 b = *(const f32x4*)(src + r * n_pad + c0 + 4);
    const float v[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    store_group8(prec, dst, n_pad, (int)r, c0, v, sc);
  }
}

// Tiled FP16 split copy of one n_pad x n_pad FP32 matrix at the scale 2^e.
__global__ __launch_bounds__(256) void k_split_copy(const float* src, char* dst, int n_pad, float sc) {
  const size_t ngroups = (size_t)n_pad * n_pad / 8;
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < ngroups; g += (size_t)gridDim.x * 256) {
    const size_t r = g / (n_pad / 8);
    const int c0 = (int)(g % (n_pad / 8)) * 8;
    const f32x4 a = *(const f32x4*)(src + r * n_pad + c0);
    const f32x4 b = *(const f32x4*)(src + r * n_pad + c0 + 4);
    const float v[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    store_group8_t<kSplitH>(dst, n_pad / Fmt<kSplitH>::K, (int)r, c0, v, sc);
  }
}

hipError_t launch_split_copy(const float* src, void* dst, int n_pad, int e, hipStream_t s) {
  hipLaunchKernelGGL(k_split_copy, dim3(2048), dim3(256), 0, s, src, (char*)dst, n_pad, ldexpf(1.0f, e));
  return hipGetLastError();
}

// Tiled operand copy (format F) of the n_pad x n_pad zero padding of an
// n_src x n_src row-major FP32 matrix (n_src <= n_pad), scaled by sc
// (kSplitH; a power of two).
template <int F>
__global__ __launch_bounds__(256) void k_copy_src(const float* src, int n_src, char* dst, int n_pad, float sc) {
  const size_t ngroups = (size_t)n_pad * n_pad / 8;
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < ngroups; g += (size_t)gridDim.x * 256) {
    const int r = (int)(g / (n_pad / 8));
    const int c0 = (int)(g % (n_pad / 8)) * 8;
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = c0 + e;
      v[e] = (r < n_src && c < n_src) ? src[(size_t)r * n_src + c] : 0.0f;
    }
    store_group8_t<F>(dst, n_pad / Fmt<F>::K, r, c0, v, sc);
  }
}

hipError_t launch_copy_src(int prec, const float* src, int n_src, void* dst, int n_pad, int e, hipStream_t s) {
  const float sc = ldexpf(1.0f, e);
  switch (prec) {
    case kSplitH: hipLaunchKernelGGL(k_copy_src<kSplitH>, dim3(2048), dim3(256), 0, s, src, n_src, (char*)dst, n_pad, sc); break;
    case kSplit3: hipLaunchKernelGGL(k_copy_src<kSplit3>, dim3(2048), dim3(256), 0, s, src, n_src, (char*)dst, n_pad, sc); break;
    case kSplit2: hipLaunchKernelGGL(k_copy_src<kSplit2>, dim3(2048), dim3(256), 0, s, src, n_src, (char*)dst, n_pad, sc); break;
    case kBF16: hipLaunchKernelGGL(k_copy_src<kBF16>, dim3(2048), dim3(256), 0, s, src, n_src, (char*)dst, n_pad, sc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// FP64 partials of ||M||_F^2 of an n_src x n_src row-major FP32 matrix: one
// per workgroup of a fixed grid of kNormBlocks (summed by the caller in a
// fixed order).
__global__ __launch_bounds__(256) void k_norm2(const float* src, size_t count, double* part) {
  __shared__ double s_red[4];
  double acc = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (size_t)gridDim.x * 256) {
    const double v = src[e];
    acc += v * v;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
}

hipError_t launch_norm2(const float* src, size_t count, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_norm2, dim3(kNormBlocks), dim3(256), 0, s, src, count, part);
  return hipGetLastError();
}

// R = W - W^T with W = V1 + V2 (n_pad x n_pad FP32, V2 nullable), written
// only as the plain BF16 operand copy (tiled layout).  One 64 x 64 block per
// workgroup; the block and its transposed partner are staged through LDS.
__global__ __launch_bounds__(256) void k_antisym_bf16(const float* v1, const float* v2, int n_pad, char* dst) {
  __shared__ float t[64][65];
  __shared__ float tt[64][65];
  const int bi = blockIdx.y, bj = blockIdx.x;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    const size_t o = (size_t)(bi * 64 + r) * n_pad + bj * 64 + c;
    const size_t ot = (size_t)(bj * 64 + r) * n_pad + bi * 64 + c;
    t[r][c] = v1[o] + (v2 ? v2[o] : 0.0f);
    tt[r][c] = v1[ot] + (v2 ? v2[ot] : 0.0f);
  }
  __syncthreads();
  for (int g = threadIdx.x; g < 64 * 8; g += 256) {
    const int r = g >> 3, c0 = (g & 7) * 8;
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = t[r][c0 + e] - tt[c0 + e][r];
    store_group8_t<kBF16>(dst, n_pad / Fmt<kBF16>::K, bi * 64 + r, bj * 64 + c0, v, 1.0f);
  }
}

hipError_t launch_antisym_bf16(const float* v1, const float* v2, int n_pad, void* dst, hipStream_t s) {
  const int nb = n_pad / 64;
  hipLaunchKernelGGL(k_antisym_bf16, dim3(nb, nb), dim3(256), 0, s, v1, v2, n_pad, (char*)dst);
  return hipGetLastError();
}

// y_k += d_k for nmat matrices of n_pad x n_pad FP32 (masters).
__global__ __launch_bounds__(256) void k_add_into(float* y, size_t ys, const float* d, size_t ds, size_t count) {
  const int k = blockIdx.y;
  float* yk = y + (size_t)k * ys;
  const float* dk = d + (size_t)k * ds;
  for (size_t e = ((size_t)blockIdx.x * 256 + threadIdx.x) * 4; e < count; e += (size_t)gridDim.x * 256 * 4) {
    f32x4 a = *(const f32x4*)(yk + e);
    const f32x4 b = *(const f32x4*)(dk + e);
    a += b;
    *(f32x4*)(yk + e) = a;
  }
}

hipError_t launch_add_into(float* y, size_t ys, const float* d, size_t ds, int n_pad, int nmat, hipStream_t s) {
  if (nmat <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_into, dim3(1024, nmat), dim3(256), 0, s, y, ys, d, ds, (size_t)n_pad * n_pad);
  return hipGetLastError();
}

// b <- 2 a - b for every observable (FP32 masters, n_pad x n_pad, one
// rounding as in the step epilogue), with b's operand copy rewritten at the
// scale b's metadata records (kSplitH) and b's norm partials replaced by one
// FP64 partial of ||b||_F^2 per 64 x 64 block.  Grid (n_pad / 64,
// n_pad / 64, observables).
__global__ __launch_bounds__(256) void k_reflect(int prec, MatRef a, MatRef b, int n_pad) {
  __shared__ double s_red[4];
  const int z = blockIdx.z, bi = blockIdx.y, bj = blockIdx.x, nb = gridDim.x;
  const float* ya = a.f32 + (size_t)z * a.stride_f32;
  float* yb = b.f32 + (size_t)z * b.stride_f32;
  char* op = (char*)b.op + (size_t)z * b.stride_op;
  MatMeta* mm = (MatMeta*)(b.meta + (size_t)z * b.stride_op);
  const float sc = prec == kSplitH ? ldexpf(1.0f, mm->scale) : 1.0f;
  double sq = 0.0;
  for (int g = threadIdx.x; g < 64 * 8; g += 256) {
    const int r = bi * 64 + (g >> 3), c0 = bj * 64 + (g & 7) * 8;
    const size_t o = (size_t)r * n_pad + c0;
    const f32x4 a0 = *(const f32x4*)(ya + o), a1 = *(const f32x4*)(ya + o + 4);
    const f32x4 b0 = *(const f32x4*)(yb + o), b1 = *(const f32x4*)(yb + o + 4);
    float v[8];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[e] = 2.0f * a0[e] - b0[e];
      v[4 + e] = 2.0f * a1[e] - b1[e];
    }
    *(f32x4*)(yb + o) = f32x4{v[0], v[1], v[2], v[3]};
    *(f32x4*)(yb + o + 4) = f32x4{v[4], v[5], v[6], v[7]};
    if (prec != kFP32) store_group8(prec, op, n_pad, r, c0, v, sc);
#pragma unroll
    for (int e = 0; e < 8; ++e) sq += (double)v[e] * (double)v[e];
  }
  sq = wave_sum(sq);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    mm->nrm[bi * nb + bj] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
    if (bi == 0 && bj == 0) mm->count = nb * nb;
  }
}

hipError_t launch_reflect(int prec, MatRef a, MatRef b, int n_pad, int nmat, hipStream_t s) {
  if (nmat <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reflect, dim3(n_pad / 64, n_pad / 64, nmat), dim3(256), 0, s, prec, a, b, n_pad);
  return hipGetLastError();
}

hipError_t launch_resplit(int prec, MatRef m, int n_pad, int nmat, hipStream_t s) {
  if (prec == kFP32 || nmat <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_resplit, dim3(1024, nmat), dim3(256), 0, s, prec, m, n_pad);
  return hipGetLastError();
}

// ---------------------------------------------------------------- init

// X_1 = alpha I + beta H (Eq. DM0) and Y_1 = c A_k (c = beta for Eq. DM3 /
// DMSuscept, c = 1 for the start Y_M = A of Eq. DM2), built from the
// symmetric parts (S + S^T)/2 of H and A (exactly symmetric in FP32).  One
// pair of mirror 64 x 64 blocks (bi, bj), (bj, bi) with bi <= bj per
// workgroup: both are read once, row-wise, into LDS, and both output blocks
// are written from them.  Blocks of X emit (Tr, ||.||^2) partials, each
// block its own in a fixed order.
__device__ __forceinline__ void init_block(int prec, const float (*p)[65], const float (*q)[65], int bi, int bj,
                                           int nb, int n, int n_pad, int z, const MatRef& x, const MatRef& y,
                                           double y_scale_mode, Part* part, const Ctl* ctl, double* s_red) {
  // output block (bi, bj): element (r, c) = (p[r][c] + q[c][r]) / 2, p the
  // source block (bi, bj), q the source block (bj, bi)
  const int t = threadIdx.x;
  const double alpha = ctl->alpha, beta = ctl->beta;
  const double ys = y_scale_mode == 0.0 ? beta : y_scale_mode;
  const MatRef& m = z == 0 ? x : y;
  float* o32 = m.f32 + (z == 0 ? 0 : (size_t)(z - 1) * m.stride_f32);
  char* oop = (char*)m.op + (z == 0 ? 0 : (size_t)(z - 1) * m.stride_op);
  // kSplitH: X_1's copy at the fixed 2^14; a Y copy needs the matrix's norm
  // first, so here Y gets only its master and norm partials (k_resplit
  // writes the copy)
  const bool ycopy_later = prec == kSplitH && z != 0;
  // three-term-X^2 option: X_1 gets its three- and two-term copies, Y_1 the two-term one
  const int fmt = prec == kSplit32 ? (z == 0 ? kSplit3 : kSplit2) : prec;
  char* oop2 = prec == kSplit32 && z == 0 ? (char*)x.op2 : nullptr;
  const float sc = prec == kSplitH ? ldexpf(1.0f, kXScaleExp) : 1.0f;
  double tr = 0.0, sq = 0.0;
  // each thread: 2 groups of 8 consecutive columns
  for (int gidx = t; gidx < 64 * 8; gidx += 256) {
    const int r = gidx >> 3, cg = (gidx & 7) * 8;
    const int gi = bi * 64 + r;
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = cg + e, gj = bj * 64 + c;
      const double s = 0.5 * ((double)p[r][c] + (double)q[c][r]);
      double val;
      if (z == 0) {
        val = beta * (double)s + ((gi == gj && gi < n) ? alpha : 0.0);
      } else {
        val = ys * (double)s;
      }
      v[e] = (float)val;
      const double d = v[e];
      sq += d * d;
      if (z == 0 && gi == gj) tr += d;
    }
    float* dst = o32 + (size_t)gi * n_pad + bj * 64 + cg;
    *(f32x4*)dst = f32x4{v[0], v[1], v[2], v[3]};
    *(f32x4*)(dst + 4) = f32x4{v[4], v[5], v[6], v[7]};
    if (!ycopy_later) store_group8(fmt, oop, n_pad, gi, bj * 64 + cg, v, sc);
    if (oop2) store_group8(kSplit2, oop2, n_pad, gi, bj * 64 + cg, v, 1.0f);
  }
  if (ycopy_later) {
    sq = wave_sum(sq);
    if ((t & 63) == 0) s_red[t >> 6] = sq;
    __syncthreads();
    if (t == 0) {
      MatMeta* mm = (MatMeta*)(m.meta + (size_t)(z - 1) * m.stride_op);
      mm->nrm[bi * nb + bj] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
      if (bi == 0 && bj == 0) mm->count = nb * nb;
    }
    __syncthreads();
  }
  if (z == 0) {
    tr = wave_sum(tr);
    sq = wave_sum(sq);
    if ((t & 63) == 0) {
      s_red[2 * (t >> 6)] = tr;
      s_red[2 * (t >> 6) + 1] = sq;
    }
    __syncthreads();
    if (t == 0) {
      double tt = 0.0, qq = 0.0;
      for (int w = 0; w < 4; ++w) {
        tt += s_red[2 * w];
        qq += s_red[2 * w + 1];
      }
      part[bi * nb + bj] = Part{tt, qq, 0.0, 0.0};
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_init(int prec, const float* h, const float* a, int n,
                                              int n_pad, int zoff, MatRef x, MatRef y,
                                              double y_scale_mode, Part* part, Ctl* ctl) {
  __shared__ float tile[64][65];    // block (bi, bj) of the source
  __shared__ float tileT[64][65];   // block (bj, bi) of the source
  __shared__ double s_red[8];
  const int bi = blockIdx.y, bj = blockIdx.x;   // output blocks (bi, bj) and (bj, bi)
  if (bi > bj) return;                          // the workgroup of (bj, bi) writes both
  const int nb = gridDim.x;
  const int z = blockIdx.z + zoff;               // 0: X from H; k >= 1: Y_{k-1} from A_{k-1}
  const float* src = z == 0 ? h : a + (size_t)(z - 1) * n * n;
  const int t = threadIdx.x;
  int bad = 0;
  // stage both blocks row-wise (coalesced)
  for (int e = t; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    const int gi = bi * 64 + r, gj = bj * 64 + c;
    const int ti_ = bj * 64 + r, tj_ = bi * 64 + c;
    float v = 0.0f, w = 0.0f;
    if (gi < n && gj < n) {
      v = src[(size_t)gi * n + gj];
      if (!isfinite(v)) bad = 1;
    }
    if (bi != bj && ti_ < n && tj_ < n) {
      w = src[(size_t)ti_ * n + tj_];
      if (!isfinite(w)) bad = 1;
    }
    tile[r][c] = v;
    tileT[r][c] = w;
  }
  if (bad) ctl->nonfinite = 1;
  __syncthreads();
  if (bi == bj) {
    init_block(prec, tile, tile, bi, bj, nb, n, n_pad, z, x, y, y_scale_mode, part, ctl, s_red);
  } else {
    init_block(prec, tile, tileT, bi, bj, nb, n, n_pad, z, x, y, y_scale_mode, part, ctl, s_red);
    init_block(prec, tileT, tile, bj, bi, nb, n, n_pad, z, x, y, y_scale_mode, part, ctl, s_red);
  }
}

// nobs >= 0: X_1 and nobs observables; nobs < 0: only the -nobs observables.
hipError_t launch_init(int prec, int /*tile*/, const float* h, const float* a, int n, int n_pad,
                       int nobs, const uint32_t* /*jobs*/, int /*njobs*/, MatRef x, MatRef y,
                       double y_scale_mode, Part* part, Ctl* ctl, hipStream_t s) {
  const int nb = n_pad / 64;
  const int zoff = nobs < 0 ? 1 : 0;
  const int nz = nobs < 0 ? -nobs : 1 + nobs;
  hipLaunchKernelGGL(k_init, dim3(nb, nb, nz), dim3(256), 0, s, prec, h, a, n, n_pad, zoff, x, y,
                     y_scale_mode, part, ctl);
  return hipGetLastError();
}

// ---------------------------------------------------------------- outputs

// D = X (n x n), chi_k = c * Y_k with c = scale (times beta from the control
// block if scale_by_beta), and per-block FP64 partials of Tr[A_k D].
__global__ __launch_bounds__(256) void k_output(const float* x32, const float* y32, size_t ystride,
                                                const float* a, int n, int n_pad, int nobs,
                                                float* d_out, float* chi_out, double scale,
                                                int scale_by_beta, double* a0_part, Ctl* ctl) {
  __shared__ double s_red[4];
  const size_t n2 = (size_t)n * n;
  const double c = scale * (scale_by_beta ? ctl->beta : 1.0);
  const int k = blockIdx.y;   // observable (or 0 when nobs == 0)
  double acc = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n2; e += (size_t)gridDim.x * 256) {
    const size_t i = e / n, j = e % n;
    const float dv = x32[i * n_pad + j];
    if (k == 0 && d_out) d_out[e] = dv;
    if (nobs > 0) {
      const float yv = y32[(size_t)k * ystride + i * n_pad + j];
      if (chi_out) chi_out[(size_t)k * n2 + e] = (float)(c * (double)yv);
      acc += (double)dv * (double)a[(size_t)k * n2 + e];
    }
  }
  if (nobs > 0 && a0_part) {
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) a0_part[(size_t)k * gridDim.x + blockIdx.x] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
  }
}

constexpr int kOutBlocks = 1024;

hipError_t launch_output(const float* x32, const float* y32, size_t ystride, const float* a, int n,
                         int n_pad, int nobs, float* d_out, float* chi_out, double scale,
                         int scale_by_beta, const uint32_t*, int, int, double* a0_part, Ctl* ctl,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_output, dim3(kOutBlocks, nobs > 0 ? nobs : 1), dim3(256), 0, s, x32, y32,
                     ystride, a, n, n_pad, nobs, d_out, chi_out, scale, scale_by_beta, a0_part, ctl);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_copy_out(const float* src, int n, int n_pad, float* dst) {
  const size_t n2 = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n2; e += (size_t)gridDim.x * 256)
    dst[e] = src[(e / n) * n_pad + e % n];
}

hipError_t launch_copy_out(const float* src, int n, int n_pad, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_out, dim3(kOutBlocks), dim3(256), 0, s, src, n, n_pad, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------- response

// out[k][p] = sum_e chi_k[e] * H1_p[e]  (Eq. dual), FP64 accumulation.
// Each thread streams float4 chunks of every chi_k and H1_p once; perturbations
// are processed in groups of up to 8 (each group re-reads chi).
constexpr int kRespThreads = 256;

int response_blocks(size_t n2) {
  const size_t v4 = (n2 + 3) / 4;
  size_t b = (v4 + kRespThreads * 8 - 1) / (kRespThreads * 8);
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

template <int K>
__global__ __launch_bounds__(kRespThreads) void k_response(const float* chi, const float* h1, int npert,
                                                           size_t n2, double* part) {
  __shared__ double s_red[kRespThreads / 64][K * 8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const size_t nv4 = n2 / 4;
  for (int p0 = 0; p0 < npert; p0 += 8) {
    const int pc = npert - p0 < 8 ? npert - p0 : 8;
    double acc[K][8];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int p = 0; p < 8; ++p) acc[k][p] = 0.0;
    for (size_t e = (size_t)blockIdx.x * kRespThreads + threadIdx.x; e < nv4; e += (size_t)gridDim.x * kRespThreads) {
      f32x4 c[K];
#pragma unroll
      for (int k = 0; k < K; ++k) c[k] = ((const f32x4*)(chi + (size_t)k * n2))[e];
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        if (p < pc) {
          const f32x4 g = ((const f32x4*)(h1 + (size_t)(p0 + p) * n2))[e];
#pragma unroll
          for (int k = 0; k < K; ++k)
            acc[k][p] += (double)c[k][0] * g[0] + (double)c[k][1] * g[1] + (double)c[k][2] * g[2] +
                         (double)c[k][3] * g[3];
        }
      }
    }
    // scalar tail (n2 not a multiple of 4)
    if (blockIdx.x == 0 && threadIdx.x < (int)(n2 - nv4 * 4)) {
      const size_t e = nv4 * 4 + threadIdx.x;
#pragma unroll
      for (int p = 0; p < 8; ++p)
        if (p < pc)
#pragma unroll
          for (int k = 0; k < K; ++k) acc[k][p] += (double)chi[(size_t)k * n2 + e] * h1[(size_t)(p0 + p) * n2 + e];
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const double v = wave_sum(acc[k][p]);
        if (lane == 0) s_red[wave][k * 8 + p] = v;
      }
    __syncthreads();
    if (threadIdx.x < K * 8) {
      const int k = threadIdx.x / 8, p = threadIdx.x % 8;
      if (p < pc) {
        double t = 0.0;
        for (int w = 0; w < kRespThreads / 64; ++w) t += s_red[w][threadIdx.x];
        part[((size_t)blockIdx.x * K + k) * npert + p0 + p] = t;
      }
    }
    __syncthreads();
  }
}

// out[k * ld + p] = sum over blocks of part[b][k][p] (one output per block,
// fixed summation order).
__global__ __launch_bounds__(64) void k_response_final(const double* part, int nblk, int npert, int kp,
                                                       double* out, int ld) {
  const int idx = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) acc += part[(size_t)b * kp + idx];
  acc = wave_sum(acc);
  if (threadIdx.x == 0) out[(size_t)(idx / npert) * ld + idx % npert] = acc;
}

hipError_t launch_response(const float* chi, int nobs, const float* h1, int npert, size_t n2,
                           double* part, int nblk, double* out_dev, int ld, hipStream_t s) {
  switch (nobs) {
#define DMPT_RESP(K)                                                                      \
  case K:                                                                                 \
    hipLaunchKernelGGL(k_response<K>, dim3(nblk), dim3(kRespThreads), 0, s, chi, h1, npert, n2, part); \
    break;
    DMPT_RESP(1)
    DMPT_RESP(2)
    DMPT_RESP(3)
    DMPT_RESP(4)
    DMPT_RESP(5)
    DMPT_RESP(6)
    DMPT_RESP(7)
    DMPT_RESP(8)
#undef DMPT_RESP
    default:
      return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_response_final, dim3(nobs * npert), dim3(64), 0, s, part, nblk, npert, nobs * npert,
                     out_dev, ld);
  return hipGetLastError();
}

}  // namespace dmpt
