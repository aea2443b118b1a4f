// Internal interface between the host runtime (dmpt_api.cpp) and the gfx950
// kernels (dmpt_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/dmpt.h"

namespace dmpt {

// Operand formats of the dense products.
enum Prec : int {
  kFP32 = 0,    // FP32 row-major, FP32 MFMA
  kSplit2 = 1,  // packed (hi, lo) BF16 pairs, BF16 MFMA, FP32 accumulate
  kSplit3 = 2,  // packed (hi, mid, lo) BF16 triples, BF16 MFMA, FP32 accumulate
  kBF16 = 3,    // plain BF16 row-major
  kSplit32 = 4, // precision option only (no kernel format): X^2 products in kSplit3, the sweep
                // products in kSplit2; X_n carries both copies (MatRef::op, MatRef::op2)
  kSplitH = 5,  // packed (hi, lo) FP16 pairs of the operand scaled by 2^s, FP16 MFMA,
                // FP32 accumulate; s = kXScaleExp for X, per matrix (MatMeta) for Y
};

// FP16 split (kSplitH): X_n's entries lie in [-1, 1] (spectrum in [0, 1]), so a
// fixed 2^14 keeps them below the FP16 maximum with 4x headroom.  A Y matrix
// carries its own exponent in its MatMeta: the producer of Y_{n+1} picks s
// with 4.5 ||Y_n||_F 2^s <= 2^15, a bound on every entry of Y_{n+1}
// (|Y_{n+1}|_ij <= ||Y_{n+1}||_2 <= (2 + 2 ||X_n||_2) ||Y_n||_2, ||X_n||_2 <= 1).
constexpr int kXScaleExp = 14;
constexpr double kYBound = 4.5;
constexpr double kYTarget = 32768.0;

// Bytes per matrix element in the operand copy of each format.
__host__ __device__ constexpr int operand_bytes(int prec) {
  return prec == kFP32 ? 4 : (prec == kSplit2 || prec == kSplitH) ? 4 : (prec == kSplit3 || prec == kSplit32) ? 6
       : prec == kBF16 ? 2 : 0;
}
// Bytes per element of the second (two-term) operand copy of the kSplit32 option.
__host__ __device__ constexpr int operand2_bytes(int prec) { return prec == kSplit32 ? 4 : 0; }

constexpr int kPadTo = 256;     // n is padded (with zeros in X-space) to a multiple of this
constexpr int kMaxObs = 64;

// Per-step record written by workgroup 0 of the step kernel (step n, 1-based).
struct StepRec {
  double tr;    // Tr X_n
  double sq;    // ||X_n||_F^2
  double eps;   // ||X_n - X_n^2||_F^2 (known one launch later)
  int sigma;    // sigma_n (0 if the recursion stopped at X_n)
  int pad;
};

// Per-tile FP64 partials written by the X-product jobs of step n:
// (Tr X_{n+1}, ||X_{n+1}||_F^2, ||X_n - X_n^2||_F^2, unused).
struct Part {
  double tr, sq, eps, pad;
};

// Job queues of the persistent step kernel: one queue per XCD (queue x holds
// the job-list positions x, x + 8, x + 16, ...), each with a ticket counter
// that workgroups advance with atomic adds.  Counters of one launch are one
// set; sets rotate over kQSets so that launch L can clear the set of launch
// L + 2 (launch L - 2, its last user, has finished and L + 2 starts after L).
// Counters sit kQStride words apart (separate 64-byte lines).
constexpr int kXcdQueues = 8, kQSets = 4, kQStride = 16;

// Device control block (lives at the start of the workspace).
struct Ctl {
  int done;        // recursion finished (stop, error or limit)
  int code;        // DecideCode at the stop (0 = converged)
  int m;           // steps taken (M) when done
  int nonfinite;   // an input matrix held NaN/Inf
  int ystop;       // step k whose Y_k ended the sweep (StepArgs::ytol2; 0: not yet)
  int pad_;
  double emin, emax, alpha, beta;
  double gmin, gmax;   // Gershgorin bounds
  StepRec rec[DMPT_MAX_STEPS + 3];
  unsigned int qhead[kQSets][kXcdQueues * kQStride];
};

// Job = one output tile (I, J), I <= J, of either the X product
// P = X_n X_n (kind 0) or the response product Z = Y_n X_n + X_n Y_n of
// observable `obs` (kind 1).
enum JobKind : uint32_t { kJobP = 0, kJobZ = 1 };

// Bits: 0 kind, 1-6 observable, 7 wide / second half, 8-19 tile row block,
// 20-30 tile column block, 31 split.
inline uint32_t job_pack(uint32_t kind, uint32_t obs, uint32_t ti, uint32_t tj) {
  return kind | (obs << 1) | (ti << 8) | (tj << 20);
}
// Bit 7 of a Z-job (obs < 64 uses bits 1-6): a wide job, one 256 x 256 tile
// (I, J >= I) of Z with tj counting 256-column blocks.
constexpr uint32_t kJobWide = 1u << 7;
// Bit 31: a K-split job of a regular tile, one of two that each run half of
// the tile's pipeline stages (a Z-job's two products, or the first and second
// half of a P-job's K range) and store the partial tile sum in slot
// split_slot[list position] of the split scratch; bit 7 marks the second
// half.  A combine launch (launch_step_combine) adds the two halves and runs
// the tile's epilogue before the next launch reads the outputs.
constexpr uint32_t kJobSplit = 1u << 31;
constexpr uint32_t kJobHalf1 = 1u << 7;
constexpr int kSplitTileFloats = 256 * 128;   // one partial tile sum

// Per-matrix metadata next to each operand copy: the scale exponent of the
// FP16 copy (kSplitH) and FP64 partials of ||M||_F^2 written by the producer
// (`count` of them, fixed order), from which the next producer bounds its output.
struct MatMeta {
  int32_t scale;
  int32_t count;
  double nrm[1];       // count entries
};
inline size_t meta_bytes(int nparts) { return sizeof(int32_t) * 2 + sizeof(double) * (size_t)nparts; }

// One operand matrix set: FP32 master plus (optionally) the operand copy in
// the product format.  `stride_*` separates observables in a batch; the
// metadata of observable k sits at meta + k * stride_op.
struct MatRef {
  float* f32;
  void* op;
  size_t stride_f32;   // elements
  size_t stride_op;    // bytes
  char* meta;
  void* op2 = nullptr; // kSplit3 matrices of the kSplit32 option: their two-term (kSplit2) copy,
                       // written next to the three-term one (same (hi, lo = RNE(x - hi)) terms)
};

struct StepArgs {
  int n, n_pad, ntile;       // ntile = n_pad / TILE
  int step;                  // n: computes X_{n+1}, Y_{n+1} from X_n, Y_n
  int max_iter, min_iter;
  double nocc, idem_tol;
  double unit;               // unit roundoff of X_n^2 for the stopping test (the X product precision)
  double ytol2;              // > 0 (decide == 1): launch k skips its Z-jobs, and every later launch
                             // too, once ||X_{k-1} - X_{k-1}^2||_F^2 <= ytol2; Y_k is the result
  int decide;                // 1: evaluate the controller on the partials of X_n
  int fixed_sigma;           // used when decide == 0 and sigma_src == nullptr
  const StepRec* sigma_src;  // decide == 0: sigma_n read from sigma_src[step].sigma
  int write_split;           // also write the operand copy of the outputs
  int flush;                 // two-level accumulation: add the pass accumulator into the
                             // running tile sum every `flush` groups of 4 stages (FP32
                             // operands: into an FP64 tile sum every `flush` stages)
                             // (0: single level)
  int flush_z;               // Z-jobs of a mixed launch (kSplit32): their own interval (0: flush)
  char* hist;                // P-jobs also write a plain BF16 tiled copy of X_{n+1} at
  size_t hist_stride;        //   hist + (n + 1) hist_stride bytes (nullptr: no copy)
  float oscale;              // tile sums are multiplied by this before the epilogue (0 or 1: none)
  const uint32_t* jobs;
  int njobs;                 // length of the job list
  unsigned int* qhead;       // this launch's queue counters (zero at launch start)
  unsigned int* qclear;      // counter set cleared by this launch for a later one
  MatRef x_in, x_out, y_in, y_out;
  const Part* part_in;       // partials written by the previous step (or X_1's init)
  Part* part_out;
  int nparts;
  Ctl* ctl;
  const uint32_t* split_slot; // kJobSplit jobs: scratch slot of list position p (split_slot[p])
  float* split_buf;           // scratch: slot q, half h at split_buf + (2 q + h) kSplitTileFloats
};

// Launchers (dmpt_kernels.hip).  All return hipError_t of the launch.
hipError_t launch_ctl_reset(Ctl* ctl, hipStream_t s);
hipError_t launch_gershgorin(const float* h, int n, double2* scratch, int nblk, Ctl* ctl,
                             int set_coeffs, hipStream_t s);
int gershgorin_blocks(int n);
hipError_t launch_lanczos_start(double* v, double* vprev, int n, hipStream_t s);
hipError_t launch_lanczos_step(const float* h, int n, double* v, double* vprev, double* w,
                               double* ab, int j, hipStream_t s);
hipError_t launch_set_bounds(Ctl* ctl, double emin, double emax, hipStream_t s);
hipError_t launch_init(int prec, int tile, const float* h, const float* a, int n, int n_pad,
                       int nobs, const uint32_t* jobs, int njobs, MatRef x, MatRef y,
                       double y_scale_mode, Part* part, Ctl* ctl, hipStream_t s);
// Workgroups of a persistent step launch over njobs jobs (one per CU at most).
int persistent_grid(int njobs);
// Step launch: a persistent grid of at most one workgroup per CU working
// through args.jobs[0, njobs) (njobs is stored into the arguments).  The
// caller sets qhead / qclear from step_queue_sets.
// wide: the list may hold wide Z-jobs (kJobWide; kSplit2, kSplit32 and kBF16
// only), which accumulate on one level.
hipError_t launch_step(int prec, StepArgs args, int njobs, hipStream_t s, bool wide = false);
// Queue counter sets of the seq-th step launch since the last queue reset.
inline void step_queue_sets(Ctl* ctl, unsigned seq, StepArgs* a) {
  a->qhead = ctl->qhead[seq % kQSets];
  a->qclear = ctl->qhead[(seq + 2) % kQSets];
}
hipError_t launch_queue_reset(Ctl* ctl, hipStream_t s);
// After a step launch whose list holds K-split jobs: one workgroup per split
// tile (cjobs[q], slot q) adds the two partial sums and runs the tile's
// epilogue with the launch's sigma (nothing when that launch stopped, or for
// Z tiles once the sweep has stopped).  prec as for launch_step with wide.
hipError_t launch_step_combine(int prec, StepArgs args, const uint32_t* cjobs, int ncomb, hipStream_t s);
// Step tiles are 256 rows x 128 columns; tile (I, J) with J >= 2I covers the
// upper triangle.  ntile in StepArgs is the number of 128-column blocks.
constexpr int kStepTM = 256, kStepTN = 128;
inline int step_tile_count(int n_pad) { const int t = n_pad / kStepTM; return t * (t + 1); }
hipError_t launch_output(const float* x32, const float* y32, size_t ystride, const float* a,
                         int n, int n_pad, int nobs, float* d_out, float* chi_out,
                         double scale, int scale_by_beta, const uint32_t* jobs, int njobs,
                         int tile, double* a0_part, Ctl* ctl, hipStream_t s);
// dmpt_response with the caller's workspace (dmpt_api.cpp), shared by the
// entry point that brings its own device scratch (dmpt_static.hip), and the
// error reporter behind dmpt_last_error.
size_t response_workspace_bytes(int32_t nobs, int32_t npert, int32_t n);
dmpt_status response_run(const float* chi, int32_t nobs, const float* H1, int32_t npert, int32_t n,
                         double* out, void* stream, void* workspace, size_t workspace_bytes);
dmpt_status report_error(dmpt_status st, const char* msg);
hipError_t launch_response(const float* chi, int nobs, const float* h1, int npert, size_t n2,
                           double* part, int nblk, double* out_dev, int ld, hipStream_t s);
int response_blocks(size_t n2);
hipError_t launch_copy_out(const float* src, int n, int n_pad, float* dst, hipStream_t s);
// Non-orthonormal basis: C = alpha A B^T (n_pad x n_pad, n_pad % 256 == 0,
// FP32 MFMA) and zero-padded (optionally transposed) copies.
hipError_t launch_gemm_nt(const float* A, const float* B, float* C, int n_pad, float alpha, int flush,
                          hipStream_t s);
// The same for a product known to be symmetric: upper-triangle tiles only,
// then the lower triangle mirrored (exactly symmetric result).
hipError_t launch_gemm_nt_sym(const float* A, const float* B, float* C, int n_pad, float alpha, int flush,
                              hipStream_t s);
// General form: operands FP32 row-major (prec = kFP32) or tiled FP16 split
// copies (prec = kSplitH, written by launch_split_copy); sym as above.
hipError_t launch_gemm_op(int prec, const void* A, const void* B, float* C, int n_pad, float alpha, int flush,
                          int sym, hipStream_t s);
// Tiled FP16 split copy (the kSplitH operand format) of an n_pad x n_pad FP32
// matrix scaled by 2^e.
hipError_t launch_split_copy(const float* src, void* dst, int n_pad, int e, hipStream_t s);
hipError_t launch_pad(const float* src, int n, int n_pad, float* dst, int transpose, hipStream_t s);
// Residual refinement helpers.
//   launch_copy_src: tiled operand copy (prec kSplitH at scale 2^e, kSplit3 or
//     kBF16) of the zero padding of an n_src x n_src row-major FP32 matrix.
//   launch_norm2: kNormBlocks FP64 partials of the squared Frobenius norm of
//     `count` consecutive floats.
//   launch_antisym_bf16: plain BF16 tiled copy of W - W^T, W = V1 + V2.
//   launch_add_into: y_k += d_k over nmat n_pad x n_pad FP32 masters.
constexpr int kNormBlocks = 256;
hipError_t launch_copy_src(int prec, const float* src, int n_src, void* dst, int n_pad, int e, hipStream_t s);
hipError_t launch_norm2(const float* src, size_t count, double* part, hipStream_t s);
hipError_t launch_antisym_bf16(const float* v1, const float* v2, int n_pad, void* dst, hipStream_t s);
hipError_t launch_add_into(float* y, size_t ys, const float* d, size_t ds, int n_pad, int nmat, hipStream_t s);
hipError_t launch_resplit(int prec, MatRef m, int n_pad, int nmat, hipStream_t s);
// b <- 2 a - b for nmat matrices (FP32 masters), rewriting b's operand copy at
// the scale b's metadata holds and b's norm partials.
hipError_t launch_reflect(int prec, MatRef a, MatRef b, int n_pad, int nmat, hipStream_t s);
int stage_k(int prec);   // k values per pipeline stage of the step kernel

}  // namespace dmpt
