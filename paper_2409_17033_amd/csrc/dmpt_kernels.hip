// gfx950 (CDNA4) kernels for the SP2 recursion and its susceptibility sweep
// (arXiv 2409.17033, Eq. DM0, DM2, DM3, DMSuscept, doubleHalf, MixPrecMult).
//
// Data layout (device workspace)
//   X_n, Y_n   n_pad x n_pad, row-major, full symmetric storage.  Each matrix
//              has an FP32 master copy and, for the low-precision products,
//              an operand copy:
//                kSplit2: per row, groups of 8 consecutive columns stored as
//                         [8 x bf16 hi][8 x bf16 lo]  (hi = RNE_bf16(x),
//                         lo = RNE_bf16(x - hi), Eq. doubleHalf with BF16)
//                kBF16:   plain bf16 row-major.
//   Padding rows/columns (n <= i < n_pad) are zero in X- and Y-space: 0 is a
//   fixed point of x^2 and 2x - x^2 and contributes nothing to any trace.
//
// Step kernel (one launch per SP2 step n)
//   grid = list of jobs; a job is one TILE x TILE output tile (I <= J) of
//     P = X_n X_n                    (kind P; symmetric, so X_n rows serve as
//                                      both operands: P_IJ = X_I X_J^T)
//     Z = Y_n X_n + X_n Y_n          (kind Z; = Y_I X_J^T + X_I Y_J^T)
//   Operands are staged HBM -> LDS with global_load_lds_dwordx4 (no VGPR
//   staging), double-buffered, 64 bytes per row per stage, the four 16-byte
//   slots of a row XOR-swizzled by (row/4)&3 so MFMA operand reads are free of
//   bank conflicts.  Products run on v_mfma_f32_32x32x16_bf16 (split / plain
//   BF16) or v_mfma_f32_32x32x2_f32 (FP32) with FP32 accumulation.
//   Epilogue: X_{n+1} = P (sigma=+1) or 2 X_n - P (sigma=-1), likewise Y;
//   the tile and its mirror are stored (exact symmetry), the operand copy is
//   re-split, and P-jobs emit FP64 partials of Tr X_{n+1} and ||X_{n+1}||_F^2.
//   sigma_n and the stop test are evaluated at kernel start by every
//   workgroup from the FP64 partials of the previous step (fixed reduction
//   order, so every workgroup reaches the same decision); workgroup 0 records
//   it in the control block.  No host round trip per step.
#include <hip/hip_runtime.h>

#include "dmpt_internal.h"
#include "sp2_rule.h"

namespace dmpt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

#define LDS_AS __attribute__((address_space(3)))
#define GLB_AS __attribute__((address_space(1)))

// Bytes per LDS row per pipeline stage: 16 k values of FP32 / packed split-2
// (64 B = 4 slots of 16 B), 32 k values of plain BF16 (64 B), 16 k values of
// packed split-3 (96 B = 6 slots).
template <int PREC> struct Fmt {
  static constexpr int RB = PREC == kSplit3 ? 96 : 64;
  static constexpr int S = RB / 16;
  static constexpr int K = PREC == kBF16 ? 32 : 16;
};

int stage_k(int prec) { return prec == kBF16 ? 32 : 16; }

template <int TILE> struct Geo;
template <> struct Geo<256> {   // 8 waves as 2 x 4, wave tile 128 x 64
  static constexpr int WM = 2, WN = 4, NW = 8, NT = 512;
};
template <> struct Geo<128> {   // 4 waves as 2 x 2, wave tile 64 x 64
  static constexpr int WM = 2, WN = 2, NW = 4, NT = 256;
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ unsigned short bf16_bits(float x) {
  return __builtin_bit_cast(unsigned short, (__bf16)x);   // round to nearest even
}
__device__ __forceinline__ float bf16_val(unsigned short b) {
  return __builtin_bit_cast(float, ((unsigned int)b) << 16);
}
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
template <int PREC> struct Terms { static constexpr int T = PREC == kSplit3 ? 3 : PREC == kSplit2 ? 2 : 1; };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
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

// Issue the direct-to-LDS loads of one panel stage: TILE rows x S*16 bytes.
// `src` points at row 0 of the panel at the stage's byte offset.  The panel
// is TILE*S slots of 16 B; instruction j (of TILE*S/64) fills slots
// [64 j, 64 j + 64), lane i slot q = 64 j + i = (row q / S, physical slot q % S)
// and fetches the logical slot that the swizzle maps there.
template <int TILE, int S>
__device__ __forceinline__ void stage_panel(const char* src, size_t ldb, LDS_AS char* panel,
                                            int wave, int lane) {
  constexpr int NW = Geo<TILE>::NW;
  constexpr int NI = TILE * S / 64;
  static_assert(NI % NW == 0, "panel instructions must split evenly over the waves");
#pragma unroll
  for (int jj = 0; jj < NI / NW; ++jj) {
    const int j = wave + jj * NW;
    const int q = 64 * j + lane;
    const int r = q / S;
    const int ls = phys_slot<S>(r, q % S);   // the XOR swizzle is an involution
    const char* g = src + (size_t)r * ldb + ls * 16;
    __builtin_amdgcn_global_load_lds((const GLB_AS void*)g, (LDS_AS void*)(panel + j * 1024), 16, 0, 0);
  }
}

__device__ __forceinline__ u32x4 lds16(const LDS_AS char* p) { return *(const LDS_AS u32x4*)p; }

__device__ __forceinline__ void wait_vm0() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// ---------------------------------------------------------------- mainloop

template <int TILE> struct Acc {
  static constexpr int BR = TILE / Geo<TILE>::WM / 32, BC = TILE / Geo<TILE>::WN / 32;
};

// One pass: tot[bi][bj] += A_I B_J^T over the full K range, for the wave's
// 32 x 32 blocks.  A_I / B_J are TILE-row panels of the operand copies
// (row-major, ldb bytes per row).  A Z-job is two passes into the same tile
// sum (Y_I X_J^T, then X_I Y_J^T); a P-job is one pass (X_I X_J^T).
// `same` (A and B are the same panel: diagonal P tile) stages only one panel.
//   kSplit3: per 16-k stage, logical slot 3h + p = k-group h, part p (hi, mid,
//            lo); products of order >= 2^-16 kept: hh, hm, mh, hl, lh, mm.
//   kSplit2: per 16-k stage, slot 2h + p; products hh, hl, lh (lo*lo dropped,
//            Eq. MixPrecMult).
//   kBF16:   per 32-k stage, two k16 steps t; slot 2t + h.
//   kFP32:   per 16-k stage, lane half h holds k in {4h..4h+3} (slot h) and
//            {8+4h..8+4h+3} (slot h+2); the same k-permutation on A and B.
// Two-level accumulation (TWO): the MFMA chain runs in `acc` and is added to
// `tot` every `flush` stages, so no FP32 accumulator sees more than
// flush x (products per stage) roundings in a row.
template <int PREC, int TILE, bool TWO>
__device__ __forceinline__ void mainloop_pass(const char* a, const char* b, size_t ldb, int nstages,
                                              bool same, int flush, LDS_AS char* lds,
                                              f32x16 (&acc)[Acc<TILE>::BR][Acc<TILE>::BC],
                                              f32x16 (&tot)[Acc<TILE>::BR][Acc<TILE>::BC]) {
  constexpr int WM = Geo<TILE>::WM, WN = Geo<TILE>::WN;
  constexpr int BR = Acc<TILE>::BR, BC = Acc<TILE>::BC;
  constexpr int S = Fmt<PREC>::S, RB = Fmt<PREC>::RB;
  constexpr int PANEL = TILE * RB;   // bytes per panel per stage
  constexpr int BUF = 2 * PANEL;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = wave / WN, wc = wave % WN;
  const int h = lane >> 5;
  const int rowA = wr * (TILE / WM) + (lane & 31);
  const int rowB = wc * (TILE / WN) + (lane & 31);
  const int offB = same ? 0 : PANEL;

  auto issue = [&](int s, int buf) {
    const size_t kb = (size_t)s * RB;
    LDS_AS char* base = lds + buf * BUF;
    stage_panel<TILE, S>(a + kb, ldb, base, wave, lane);
    if (!same) stage_panel<TILE, S>(b + kb, ldb, base + PANEL, wave, lane);
  };

  issue(0, 0);
  int since = 0;
  for (int s = 0; s < nstages; ++s) {
    const int buf = s & 1;
    wait_vm0();
    __syncthreads();
    const LDS_AS char* pA = lds + buf * BUF;
    const LDS_AS char* pB = pA + offB;

    if constexpr (PREC == kSplit3 || PREC == kSplit2) {
      constexpr int T = Terms<PREC>::T;
      bf16x8 A[BR][T], B[BC][T];
#pragma unroll
      for (int j = 0; j < BC; ++j)
#pragma unroll
        for (int p = 0; p < T; ++p)
          B[j][p] = __builtin_bit_cast(bf16x8, lds16(pB + swz<S>(rowB + 32 * j, T * h + p)));
#pragma unroll
      for (int i = 0; i < BR; ++i)
#pragma unroll
        for (int p = 0; p < T; ++p)
          A[i][p] = __builtin_bit_cast(bf16x8, lds16(pA + swz<S>(rowA + 32 * i, T * h + p)));
      if (s + 1 < nstages) issue(s + 1, buf ^ 1);
#pragma unroll
      for (int i = 0; i < BR; ++i)
#pragma unroll
        for (int j = 0; j < BC; ++j) {
          f32x16 c = acc[i][j];
          // smallest terms first
          if constexpr (T == 3) {
            c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[i][1], B[j][1], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[i][0], B[j][2], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[i][2], B[j][0], c, 0, 0, 0);
          }
          c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[i][0], B[j][1], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[i][1], B[j][0], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[i][0], B[j][0], c, 0, 0, 0);
          acc[i][j] = c;
        }
    } else if constexpr (PREC == kBF16) {
      bf16x8 A[BR][2], B[BC][2];
#pragma unroll
      for (int j = 0; j < BC; ++j)
#pragma unroll
        for (int t = 0; t < 2; ++t)
          B[j][t] = __builtin_bit_cast(bf16x8, lds16(pB + swz<S>(rowB + 32 * j, 2 * t + h)));
#pragma unroll
      for (int i = 0; i < BR; ++i)
#pragma unroll
        for (int t = 0; t < 2; ++t)
          A[i][t] = __builtin_bit_cast(bf16x8, lds16(pA + swz<S>(rowA + 32 * i, 2 * t + h)));
      if (s + 1 < nstages) issue(s + 1, buf ^ 1);
#pragma unroll
      for (int i = 0; i < BR; ++i)
#pragma unroll
        for (int j = 0; j < BC; ++j) {
          f32x16 c = acc[i][j];
          c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[i][0], B[j][0], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[i][1], B[j][1], c, 0, 0, 0);
          acc[i][j] = c;
        }
    } else {  // kFP32
      f32x4 A[BR][2], B[BC][2];
#pragma unroll
      for (int j = 0; j < BC; ++j)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          B[j][q] = __builtin_bit_cast(f32x4, lds16(pB + swz<S>(rowB + 32 * j, h + 2 * q)));
#pragma unroll
      for (int i = 0; i < BR; ++i)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          A[i][q] = __builtin_bit_cast(f32x4, lds16(pA + swz<S>(rowA + 32 * i, h + 2 * q)));
      if (s + 1 < nstages) issue(s + 1, buf ^ 1);
#pragma unroll
      for (int i = 0; i < BR; ++i)
#pragma unroll
        for (int j = 0; j < BC; ++j) {
          f32x16 c = acc[i][j];
#pragma unroll
          for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e)
              c = __builtin_amdgcn_mfma_f32_32x32x2f32(A[i][q][e], B[j][q][e], c, 0, 0, 0);
          acc[i][j] = c;
        }
    }
    if constexpr (TWO) {
      if (++since == flush) {
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
  }
  if constexpr (TWO) {
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
      for (int j = 0; j < BC; ++j) {
        tot[i][j] += acc[i][j];
        acc[i][j] = f32x16{0};
      }
  }
  __syncthreads();   // every wave is done with both buffers before the next pass stages
}

// ---------------------------------------------------------------- step kernel

// Reduce the per-part (Tr, ||.||^2) partials in a fixed order (wave 0), then
// evaluate the controller.  Returns the DecideCode / sigma to every thread.
__device__ int step_controller(const StepArgs& a, int* s_code) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    double tr = 0.0, sq = 0.0;
    for (int t = lane; t < a.nparts; t += 64) {
      const double2 p = a.part_in[t];
      tr += p.x;
      sq += p.y;
    }
    tr = wave_sum(tr);
    sq = wave_sum(sq);
    if (lane == 0) {
      Ctl* c = a.ctl;
      int code;
      if (c->nonfinite) {
        code = kDecideNonfinite;
      } else {
        const double e2 = (a.step >= 3) ? (c->rec[a.step - 2].tr - c->rec[a.step - 2].sq) : 0.0;
        code = sp2_decide(tr, sq, e2, a.step - 1, a.n, a.nocc, a.min_iter, a.idem_tol);
        if ((code == 1 || code == -1) && a.step > a.max_iter) code = kDecideNotConverged;
      }
      if (blockIdx.x == 0) {
        c->rec[a.step].tr = tr;
        c->rec[a.step].sq = sq;
        c->rec[a.step].sigma = (code == 1 || code == -1) ? code : 0;
        if (!(code == 1 || code == -1)) {
          c->m = a.step - 1;
          c->code = code;
          __threadfence();
          c->done = 1;
        }
      }
      *s_code = code;
    }
  }
  __syncthreads();
  return *s_code;
}

// Store the operand copy (split terms) of 4 values at rows row0..row0+3,
// column col, and of their mirror (row col, columns row0..row0+3).
template <int PREC>
__device__ __forceinline__ void store_split4(char* oop, size_t oldb, int row0, int col, const float (&v)[4],
                                             bool mirror) {
  constexpr int T = Terms<PREC>::T;
  constexpr int GB = 16 * T;   // bytes per group of 8 columns
  unsigned short part[4][T];
#pragma unroll
  for (int e = 0; e < 4; ++e) split_terms<T>(v[e], part[e]);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    char* rp = oop + (size_t)(row0 + e) * oldb + (col >> 3) * GB + (col & 7) * 2;
#pragma unroll
    for (int t = 0; t < T; ++t) *(unsigned short*)(rp + 16 * t) = part[e][t];
  }
  if (mirror) {
    char* mp = oop + (size_t)col * oldb + (row0 >> 3) * GB + (row0 & 7) * 2;
#pragma unroll
    for (int t = 0; t < T; ++t)
      *(u32x2*)(mp + 16 * t) = u32x2{part[0][t] | ((unsigned)part[1][t] << 16),
                                     part[2][t] | ((unsigned)part[3][t] << 16)};
  }
}

template <int PREC>
__device__ __forceinline__ void store_split1(char* oop, size_t oldb, int r, int c, float v) {
  constexpr int T = Terms<PREC>::T;
  constexpr int GB = 16 * T;
  unsigned short part[T];
  split_terms<T>(v, part);
  char* rp = oop + (size_t)r * oldb + (c >> 3) * GB + (c & 7) * 2;
#pragma unroll
  for (int t = 0; t < T; ++t) *(unsigned short*)(rp + 16 * t) = part[t];
}

template <int PREC, int TILE, bool TWO>
__global__ __launch_bounds__(Geo<TILE>::NT) __attribute__((amdgpu_waves_per_eu(2))) void k_step(StepArgs a) {
  constexpr int WM = Geo<TILE>::WM, WN = Geo<TILE>::WN, NW = Geo<TILE>::NW;
  constexpr int BR = Acc<TILE>::BR, BC = Acc<TILE>::BC;
  __shared__ __attribute__((aligned(1024))) char lds_raw[2 * 2 * TILE * Fmt<PREC>::RB];
  __shared__ int s_code;
  __shared__ double s_red[2 * NW];
  LDS_AS char* lds = (LDS_AS char*)lds_raw;

  if (a.decide && a.ctl->done) return;
  int sigma;
  if (a.decide) {
    const int code = step_controller(a, &s_code);
    if (!(code == 1 || code == -1)) return;
    sigma = code;
  } else {
    sigma = a.sigma_src ? a.sigma_src[a.step].sigma : a.fixed_sigma;
  }

  const uint32_t job = a.jobs[blockIdx.x];
  const int kind = job & 1;
  const int obs = (job >> 1) & 127;
  const int ti = (job >> 8) & 4095;
  const int tj = (job >> 20) & 4095;
  const bool diag = ti == tj;
  constexpr int opb = operand_bytes(PREC);
  const size_t ldb = (size_t)a.n_pad * opb;
  const int nstages = a.n_pad / Fmt<PREC>::K;

  const char* xop = (const char*)a.x_in.op;
  const char* yop = (const char*)a.y_in.op + obs * a.y_in.stride_op;
  const size_t rowI = (size_t)ti * TILE * ldb, rowJ = (size_t)tj * TILE * ldb;

  f32x16 acc[BR][BC], tot[BR][BC];
#pragma unroll
  for (int i = 0; i < BR; ++i)
#pragma unroll
    for (int j = 0; j < BC; ++j) {
      acc[i][j] = f32x16{0};
      tot[i][j] = f32x16{0};
    }
  if (kind == kJobZ) {
    // Z = Y_I X_J^T + X_I Y_J^T  (both products accumulate into one tile)
    mainloop_pass<PREC, TILE, TWO>(yop + rowI, xop + rowJ, ldb, nstages, false, a.flush, lds, acc, tot);
    mainloop_pass<PREC, TILE, TWO>(xop + rowI, yop + rowJ, ldb, nstages, false, a.flush, lds, acc, tot);
  } else {
    mainloop_pass<PREC, TILE, TWO>(xop + rowI, xop + rowJ, ldb, nstages, diag, a.flush, lds, acc, tot);
  }
  if constexpr (!TWO) {
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
      for (int j = 0; j < BC; ++j) tot[i][j] = acc[i][j];
  }

  // ------------------------------------------------------------ epilogue
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = wave / WN, wc = wave % WN;
  const int h = lane >> 5, l32 = lane & 31;
  const size_t np = a.n_pad;
  const MatRef& in = kind == kJobZ ? a.y_in : a.x_in;
  const MatRef& out = kind == kJobZ ? a.y_out : a.x_out;
  const float* cur = in.f32 + (kind == kJobZ ? obs * in.stride_f32 : 0);
  float* o32 = out.f32 + (kind == kJobZ ? obs * out.stride_f32 : 0);
  char* oop = (char*)out.op + (kind == kJobZ ? obs * out.stride_op : 0);
  const size_t oldb = (size_t)a.n_pad * opb;
  const bool wsplit = a.write_split && PREC != kFP32;
  double tr = 0.0, sq = 0.0;

  // 32x32 MFMA output layout: lane l, register 4g+e holds row 8g + 4(l/32) + e, column l%32.
#pragma unroll
  for (int bi = 0; bi < BR; ++bi)
#pragma unroll
    for (int bj = 0; bj < BC; ++bj) {
      const int col = tj * TILE + wc * (TILE / WN) + bj * 32 + l32;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int row0 = ti * TILE + wr * (TILE / WM) + bi * 32 + 8 * g + 4 * h;
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float p = tot[bi][bj][4 * g + e];
          v[e] = sigma > 0 ? p : 2.0f * cur[(size_t)(row0 + e) * np + col] - p;
        }
        if (!diag) {
#pragma unroll
          for (int e = 0; e < 4; ++e) o32[(size_t)(row0 + e) * np + col] = v[e];
          *(f32x4*)(o32 + (size_t)col * np + row0) = f32x4{v[0], v[1], v[2], v[3]};
          if (wsplit) store_split4<PREC>(oop, oldb, row0, col, v, true);
          if (kind == kJobP) {
#pragma unroll
            for (int e = 0; e < 4; ++e) sq += 2.0 * (double)v[e] * (double)v[e];
          }
        } else {
          // diagonal tile: keep the upper triangle and mirror it (exact symmetry)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int r = row0 + e;
            if (r > col) continue;
            o32[(size_t)r * np + col] = v[e];
            o32[(size_t)col * np + r] = v[e];
            if (wsplit) {
              store_split1<PREC>(oop, oldb, r, col, v[e]);
              if (r != col) store_split1<PREC>(oop, oldb, col, r, v[e]);
            }
            if (kind == kJobP) {
              const double d = v[e];
              if (r == col) {
                tr += d;
                sq += d * d;
              } else {
                sq += 2.0 * d * d;
              }
            }
          }
        }
      }
    }

  if (kind == kJobP) {
    tr = wave_sum(tr);
    sq = wave_sum(sq);
    if (lane == 0) {
      s_red[2 * wave] = tr;
      s_red[2 * wave + 1] = sq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0, q = 0.0;
      for (int w = 0; w < NW; ++w) {
        t += s_red[2 * w];
        q += s_red[2 * w + 1];
      }
      // part index = upper-triangle tile index (row-major over I <= J)
      const int T = a.ntile;
      const int pidx = ti * T - ti * (ti - 1) / 2 + (tj - ti);
      a.part_out[pidx] = double2{t, q};
    }
  }
}

hipError_t launch_step(int prec, int tile, const StepArgs& args, int njobs, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  const bool two = args.flush > 0;
#define DMPT_LAUNCH_STEP(P, T, W)                                                  \
  if (prec == P && tile == T && two == W) {                                        \
    hipLaunchKernelGGL((k_step<P, T, W>), dim3(njobs), dim3(Geo<T>::NT), 0, s, args); \
    return hipGetLastError();                                                      \
  }
  DMPT_LAUNCH_STEP(kFP32, 128, true)
  DMPT_LAUNCH_STEP(kFP32, 128, false)
  DMPT_LAUNCH_STEP(kSplit3, 128, true)
  DMPT_LAUNCH_STEP(kSplit3, 128, false)
  DMPT_LAUNCH_STEP(kSplit2, 256, false)
  DMPT_LAUNCH_STEP(kSplit2, 128, true)
  DMPT_LAUNCH_STEP(kBF16, 256, false)
  DMPT_LAUNCH_STEP(kBF16, 128, true)
#undef DMPT_LAUNCH_STEP
  return hipErrorInvalidValue;
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
    for (int j = lane; j < n; j += 64) {
      const float x = row[j];
      if (!isfinite(x)) bad = 1;
      if (j != i) rs += fabs((double)x);
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
__global__ __launch_bounds__(256) void k_gemv(const float* h, const double* v, double* w, int n) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const float* row = h + (size_t)i * n;
  double acc = 0.0;
  for (int j = lane; j < n; j += 64) acc += (double)row[j] * v[j];
  acc = wave_sum(acc);
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

// Operand copy of 8 consecutive columns c0..c0+7 (c0 % 8 == 0) of one row:
// packed split groups [8 x part_0][8 x part_1]... or plain BF16.
template <int T>
__device__ __forceinline__ void store_group8_t(char* row, int c0, const float (&v)[8]) {
  unsigned short part[8][T];
#pragma unroll
  for (int e = 0; e < 8; ++e) split_terms<T>(v[e], part[e]);
  char* p = row + (c0 >> 3) * (16 * T);
#pragma unroll
  for (int t = 0; t < T; ++t) {
    u32x4 w;
#pragma unroll
    for (int e = 0; e < 4; ++e) w[e] = part[2 * e][t] | ((unsigned)part[2 * e + 1][t] << 16);
    *(u32x4*)(p + 16 * t) = w;
  }
}

__device__ __forceinline__ void store_group8(int prec, char* row, int c0, const float (&v)[8]) {
  if (prec == kSplit2) store_group8_t<2>(row, c0, v);
  else if (prec == kSplit3) store_group8_t<3>(row, c0, v);
  else if (prec == kBF16) {
    u32x4 w;
#pragma unroll
    for (int e = 0; e < 4; ++e) w[e] = bf16_bits(v[2 * e]) | ((unsigned)bf16_bits(v[2 * e + 1]) << 16);
    *(u32x4*)(row + c0 * 2) = w;
  }
}

// Rebuild the operand copy of nmat matrices from their FP32 masters.
__global__ __launch_bounds__(256) void k_resplit(int prec, MatRef m, int n_pad) {
  const int z = blockIdx.y;
  const float* src = m.f32 + (size_t)z * m.stride_f32;
  char* dst = (char*)m.op + (size_t)z * m.stride_op;
  const size_t ldb = (size_t)n_pad * operand_bytes(prec);
  const size_t ngroups = (size_t)n_pad * n_pad / 8;
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < ngroups; g += (size_t)gridDim.x * 256) {
    const size_t r = g / (n_pad / 8);
    const int c0 = (int)(g % (n_pad / 8)) * 8;
    const f32x4 a = *(const f32x4*)(src + r * n_pad + c0);
    const f32x4 b = *(const f32x4*)(src + r * n_pad + c0 + 4);
    const float v[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    store_group8(prec, dst + r * ldb, c0, v);
  }
}

hipError_t launch_resplit(int prec, MatRef m, int n_pad, int nmat, hipStream_t s) {
  if (prec == kFP32 || nmat <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_resplit, dim3(1024, nmat), dim3(256), 0, s, prec, m, n_pad);
  return hipGetLastError();
}

// ---------------------------------------------------------------- init

// X_1 = alpha I + beta H (Eq. DM0) and Y_1 = c A_k (c = beta for Eq. DM3 /
// DMSuscept, c = 1 for the start Y_M = A of Eq. DM2), built from the upper
// triangle of H and A.  One 64 x 64 block per workgroup over the full n_pad
// square; lower blocks read the transposed upper block through LDS so every
// global access is row-contiguous.  Blocks of X emit (Tr, ||.||^2) partials.
__global__ __launch_bounds__(256) void k_init(int prec, const float* h, const float* a, int n,
                                              int n_pad, int zoff, MatRef x, MatRef y,
                                              double y_scale_mode, double2* part, Ctl* ctl) {
  __shared__ float tile[64][65];
  __shared__ double s_red[8];
  const int bi = blockIdx.y, bj = blockIdx.x;   // output block (row, col)
  const int z = blockIdx.z + zoff;               // 0: X from H; k >= 1: Y_{k-1} from A_{k-1}
  const bool lower = bi > bj;
  const int sbi = lower ? bj : bi, sbj = lower ? bi : bj;
  const float* src = z == 0 ? h : a + (size_t)(z - 1) * n * n;
  const int t = threadIdx.x;
  int bad = 0;
  // stage the source block (sbi, sbj) row-wise
  for (int e = t; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    const int gi = sbi * 64 + r, gj = sbj * 64 + c;
    float v = 0.0f;
    if (gi < n && gj < n) {
      // upper triangle only: inside a diagonal block take (min, max)
      const int ui = gi <= gj ? gi : gj, uj = gi <= gj ? gj : gi;
      v = src[(size_t)ui * n + uj];
      if (!isfinite(v)) bad = 1;
    }
    tile[r][c] = v;
  }
  if (bad) ctl->nonfinite = 1;
  __syncthreads();
  const double alpha = ctl->alpha, beta = ctl->beta;
  const double ys = y_scale_mode == 0.0 ? beta : y_scale_mode;
  const MatRef& m = z == 0 ? x : y;
  float* o32 = m.f32 + (z == 0 ? 0 : (size_t)(z - 1) * m.stride_f32);
  char* oop = (char*)m.op + (z == 0 ? 0 : (size_t)(z - 1) * m.stride_op);
  const int opb = operand_bytes(prec);
  const size_t ldb = (size_t)n_pad * opb;
  double tr = 0.0, sq = 0.0;
  // each thread: 2 groups of 8 consecutive columns
  for (int gidx = t; gidx < 64 * 8; gidx += 256) {
    const int r = gidx >> 3, cg = (gidx & 7) * 8;
    const int gi = bi * 64 + r;
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = cg + e, gj = bj * 64 + c;
      const float s = lower ? tile[c][r] : tile[r][c];
      double val;
      if (z == 0) {
        val = beta * (double)s + ((gi == gj && gi < n) ? alpha : 0.0);
      } else {
        val = ys * (double)s;
      }
      v[e] = (float)val;
      if (z == 0) {
        const double d = v[e];
        sq += d * d;
        if (gi == gj) tr += d;
      }
    }
    float* dst = o32 + (size_t)gi * n_pad + bj * 64 + cg;
    *(f32x4*)dst = f32x4{v[0], v[1], v[2], v[3]};
    *(f32x4*)(dst + 4) = f32x4{v[4], v[5], v[6], v[7]};
    store_group8(prec, oop + (size_t)gi * ldb, bj * 64 + cg, v);
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
      part[bi * gridDim.x + bj] = double2{tt, qq};
    }
  }
}

// nobs >= 0: X_1 and nobs observables; nobs < 0: only the -nobs observables.
hipError_t launch_init(int prec, int /*tile*/, const float* h, const float* a, int n, int n_pad,
                       int nobs, const uint32_t* /*jobs*/, int /*njobs*/, MatRef x, MatRef y,
                       double y_scale_mode, double2* part, Ctl* ctl, hipStream_t s) {
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

__global__ __launch_bounds__(64) void k_response_final(const double* part, int nblk, int kp, double* out) {
  const int idx = blockIdx.x;   // one output per block, fixed summation order
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) acc += part[(size_t)b * kp + idx];
  acc = wave_sum(acc);
  if (threadIdx.x == 0) out[idx] = acc;
}

hipError_t launch_response(const float* chi, int nobs, const float* h1, int npert, size_t n2,
                           double* part, int nblk, double* out_dev, hipStream_t s) {
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
  hipLaunchKernelGGL(k_response_final, dim3(nobs * npert), dim3(64), 0, s, part, nblk, nobs * npert, out_dev);
  return hipGetLastError();
}

}  // namespace dmpt
