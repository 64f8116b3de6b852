// Batched chain for one geometry and many parameter points, with the smearing
// on the matrix cores.
//
// One work-group evaluates a tile of 16 parameter points over all bins:
//   1. point pass: thread (bin group, point n) walks its bins' quadrature
//      points and baselines (Sec. 4.1 probability and its tangents, q = KL/E
//      and f_k staged in LDS) and keeps mu0_j and J0_jc in registers;
//   2. nu = R mu as a block-banded GEMM [n_bins x n_bins] x [n_bins x 16]
//      on 16x16x4 MFMA (FP32 accumulation in mixed mode, FP64 in FP64 mode);
//      R is pre-tiled in MFMA operand order, so each A fetch is one
//      contiguous 64-lane load, and all-zero 16x16 blocks are skipped;
//   3. chi2 and gnu = d chi2 / d nu in FP64 from the accumulators;
//   4. gmu = R^T gnu as a second block-banded GEMM;
//   5. grad_c = norm sum_j gmu_j J0_jc, grad_norm = sum_j gmu_j mu0_j from
//      the registers of step 1 (FP64 sums).
// No global scratch and no inter-group hand-off: one launch, a persistent
// grid over tiles.  Needs n_bins <= 256 and the q / f tables in LDS.
#include <algorithm>
#include <cmath>

#include "gna_internal.h"
#include "gna_math.h"
#include "lanes.h"

namespace gna {
namespace {

constexpr int kScanN = 16;         // parameter points per tile (MFMA N)
// Row stride of the GEMM operand bb in LDS: 16 columns and one of padding,
// so that rows written by neighbouring lanes (one bin each) start in
// different banks, and the MFMA operand reads (4 rows of 16) stay spread.
constexpr int kBRow = 17;
constexpr int kScanMaxBins = 256;  // 16 row tiles of 16
constexpr size_t kScanLdsMax = 64 * 1024;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <class R>
struct Acc;
// Operand layouts on gfx950 (checked with a one-hot probe of each builtin):
// A[i][k] and B[k][j] sit in lane i + 16 k and lane j + 16 k for both
// precisions; the 16x16 accumulator differs:
//   f32: D[i][j] in lane j + 16 (i / 4), register i % 4  (row = 4 (lane/16) + v)
//   f64: D[i][j] in lane j + 16 (i % 4), register i / 4  (row = lane/16 + 4 v)
template <>
struct Acc<float> {
  using T = f32x4;
  __device__ static T mfma(float a, float b, T c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int krow, int v) { return krow * 4 + v; }
};
template <>
struct Acc<double> {
  using T = f64x4;
  __device__ static T mfma(double a, double b, T c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int krow, int v) { return krow + 4 * v; }
};

// acc += sum over column blocks lo <= kb <= hi of A(kb) B(kb), with the A
// operands of one row tile read from global memory in MFMA operand order
// (At: the tile's first block, lane offset included; block kb at
// At + kb * 256) and B from the LDS operand bb.  The A loads of up to
// kGemmBatch blocks go out together before their MFMAs, so a row tile waits
// for memory once per batch, not once per block.  Same MFMAs in the same
// order as one block at a time.
constexpr int kGemmBatch = 6;
template <class R, class A4>
__device__ __forceinline__ void gemm_row_global(const R* __restrict__ At, int lo, int hi,
                                                const R* bb, int krow, int n, A4& acc) {
  for (int kb0 = lo; kb0 <= hi; kb0 += kGemmBatch) {
    R av[kGemmBatch][4];
#pragma unroll
    for (int b = 0; b < kGemmBatch; ++b)
#pragma unroll
      for (int st = 0; st < 4; ++st)
        av[b][st] = (kb0 + b <= hi) ? At[((kb0 + b) * 4 + st) * 64] : R(0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b = 0; b < kGemmBatch; ++b) {
      if (kb0 + b > hi) break;
      const int kb = kb0 + b;
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const R bv = bb[(kb * 16 + st * 4 + krow) * kBRow + n];
        acc = Acc<R>::mfma(av[b][st], bv, acc);
      }
    }
  }
}

template <class R>
struct ScanArgs {
  int32_t B, nb, mt, ppb, nL, nq;
  const double* qtab;  // [nL][nq]  q = (K L_r) / E_k
  const double* logtab;  // [kLogTab][2] table of the chi^2 logarithm
  const R* f;          // [nq]
  const double* wL;    // [nL]
  const double* data;  // [nb]
  const R* RA;         // [mt][mt][4][64]  R in A-operand order
  const R* RT;         // [mt][mt][4][64]  R^T in A-operand order
  // Index tables, contiguous: kbA [mt][2] first / last nonzero k-block of
  // row tile I of R; kbT [mt][2] the same for R^T; kbo [mt] index of row tile
  // I's first block in the band; blkT [mt][mt] band index of block (I, J) at
  // [J][I], or -1 where (I, J) lies outside row tile I's range.
  const int32_t* meta;
  const R* band;       // [nblk][16][kRowPad] the band of R, row tile by row tile
  int32_t nblk;        // blocks in the band (kbA ranges, zero blocks inside included)
  int32_t rlds;        // 1: the band is staged in LDS, 0: A operands come from RA / RT
  const double* params;
  double* chi2;
  double* grad;
  double* pred;
  uint32_t* status;
};

__host__ __device__ inline size_t a16(size_t x) { return (x + 15) & ~size_t(15); }
__host__ __device__ inline int scan_meta_ints(int mt) { return 5 * mt + mt * mt; }

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Logarithm of the chi^2 terms: the table-driven one in the mixed-precision
// kernels (fewer instructions; measured 4% faster there), the series one in
// FP64, whose kernels sit at the register limit (the table's address and
// operands made them spill).
template <class R>
__device__ __forceinline__ double chi2_log(double x, const double* tab) {
  return sizeof(R) == 4 ? log_tab(x, tab) : log_pos(x);
}

// dst[0, bytes) = src[0, bytes) by the work-group, 16 bytes a lane, with
// several loads in flight per lane (both 16-byte aligned; bytes % 16 == 0).
template <int NT>
__device__ __forceinline__ void copy16(void* dst, const void* src, size_t bytes) {
  u32x4* d = reinterpret_cast<u32x4*>(dst);
  const u32x4* g = reinterpret_cast<const u32x4*>(src);
  const int n16 = (int)(bytes >> 4);
#pragma unroll 8
  for (int i = threadIdx.x; i < n16; i += NT) d[i] = g[i];
}

// The same copy with direct-to-LDS loads (global_load_lds_dwordx4): every
// wavefront instruction moves 1 KB (lane l's 16 bytes land at dst + 16 l)
// without passing through registers, and the copy completes in the
// background.  The tail below 1 KB goes through registers.  Before dst is
// read, every wavefront waits for its loads (s_waitcnt vmcnt(0)) and then
// the work-group meets at a barrier.  dst, src and bytes: multiples of 16.
template <int NT>
__device__ __forceinline__ void copy16_async(void* dst, const void* src, size_t bytes) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const size_t nk = bytes >> 10;
  const unsigned char* g = reinterpret_cast<const unsigned char*>(src);
  unsigned char* d = reinterpret_cast<unsigned char*>(dst);
  // The tail first: its register round trip must not wait for the DMA.
  const size_t done = nk << 10;
  if (bytes > done) copy16<NT>(d + done, g + done, bytes - done);
  for (size_t c = wave; c < nk; c += NW)
    __builtin_amdgcn_global_load_lds(
        g + (c << 10) + lane * 16,
        (__attribute__((address_space(3))) void*)(d + (c << 10)), 16, 0, 0);
}

// Per-bin sums of the phase terms that a tile of points with common
// (dm2_21, dm2_31) shares; see the kernel.
constexpr int kTab = 10;
// A 16x16 block of R staged in LDS: row-major with rows padded to 17 entries,
// so that both R[i][k] (lanes along i) and R[k][i] (the transpose, lanes
// along i) read distinct banks.
constexpr int kRowPad = 17;
constexpr int kBlk = 16 * kRowPad;

template <class R>
__host__ __device__ inline size_t scan_lds(int nL, int nq, int mt, int nwaves, int rblocks,
                                           bool share) {
  return a16((size_t)scan_meta_ints(mt) * 4) + a16((size_t)kScanN * 5 * 8) +
         a16((size_t)nL * nq * 8) + a16((size_t)nq * sizeof(R)) + a16((size_t)mt * 16 * 8) +
         a16((size_t)nL * 8) + a16((size_t)mt * 16 * kBRow * sizeof(R)) +
         a16((size_t)nwaves * kScanN * 6 * 8) + (share ? a16((size_t)mt * 16 * kTab * 8) : 0) +
         (sizeof(R) == 4 ? a16((size_t)kLogTab * 16) : 0) +
         a16((size_t)rblocks * kBlk * sizeof(R));
}

// v + (lane l ^ 16) + ..., summed as the butterfly over 16 and 32.
template <class T>
__device__ __forceinline__ T xor_sum_16_32(T v) {
  v += partner<16>(v);
  v += partner<32>(v);
  return v;
}

// WPE: wavefronts per SIMD the register allocation must allow (2 = the
// natural ~240-register allocation of the FP64 gradient variant; 3 and 4
// trade spills of the per-bin sums for occupancy; the autotuner chooses).
//
// SHARE: tiles whose points all have the same (dm2_21, dm2_31) take the
// shared-phase path.  The phases depend only on dm2, E and L (a transformation
// is recomputed only when its own inputs change, Sec. 2), and P_ee and its
// tangents are linear in the per-point coefficients (K0, A, B1, B2 and the
// tangent weights).  So the work-group forms, once per bin j, the sums over
// the bin's quadrature points k and baselines r of f_k w_r times
//   1, cos^2 phi21, cos^2 phi31, cos^2 phi32          (for mu)
//   q sin 2phi21, q sin 2phi31, q sin 2phi32,          (for d/d dm2)
//   sin^2 phi21, sin^2 phi31, sin^2 phi32              (for d/d s12, s13)
// and each point's mu_j and J_jc are a few products of its coefficients with
// that row.  The sums are taken in another order than the per-point path
// (sum, then combine), so results agree to rounding, not bit for bit.  A
// separate instantiation, so that the per-point kernel keeps its own register
// allocation; tiles that do not share still take the per-point path.
template <class R, bool GRAD, int NT, int WPE, bool SHARE>
__global__ void __launch_bounds__(NT, WPE) scan_kernel(ScanArgs<R> a) {
  using A4 = typename Acc<R>::T;
  constexpr int NW = NT / kWave;
  constexpr int NG = NT / kScanN;           // bin groups
  constexpr int PPT = kScanMaxBins / NG;    // bins per thread (upper bound)
  constexpr int TPW = (16 + NW - 1) / NW;   // row tiles per wave (upper bound)
  extern __shared__ __align__(16) unsigned char lds[];
  const int nL = a.nL, nq = a.nq, mt = a.mt, nb = a.nb, nbp = mt * 16;
  unsigned char* cur = lds;
  int32_t* meta = reinterpret_cast<int32_t*>(cur);  // index tables (see ScanArgs)
  cur += a16((size_t)scan_meta_ints(mt) * 4);
  const int32_t* kbA_s = meta;
  const int32_t* kbT_s = meta + 2 * mt;
  const int32_t* kbo_s = meta + 4 * mt;
  const int32_t* blkT_s = meta + 5 * mt;
  double* p_s = reinterpret_cast<double*>(cur);  // [16][5] parameters of the tile
  cur += a16((size_t)kScanN * 5 * 8);
  double* q_s = reinterpret_cast<double*>(cur);
  cur += a16((size_t)nL * nq * 8);
  R* f_s = reinterpret_cast<R*>(cur);
  cur += a16((size_t)nq * sizeof(R));
  double* d_s = reinterpret_cast<double*>(cur);
  cur += a16((size_t)nbp * 8);
  double* w_s = reinterpret_cast<double*>(cur);
  cur += a16((size_t)nL * 8);
  R* bb = reinterpret_cast<R*>(cur);  // [nbp][kBRow] GEMM B operand (16 columns used)
  cur += a16((size_t)nbp * kBRow * sizeof(R));
  double* red = reinterpret_cast<double*>(cur);  // [NW][16][6]
  cur += a16((size_t)NW * kScanN * 6 * 8);
  double* mm = reinterpret_cast<double*>(cur);  // [nbp][kTab] M = R T of a shared tile
  cur += SHARE ? a16((size_t)nbp * kTab * 8) : 0;
  double* lt_s = reinterpret_cast<double*>(cur);  // [kLogTab][2] logarithm table
  cur += sizeof(R) == 4 ? a16((size_t)kLogTab * 16) : 0;  // FP32 kernels only
  R* Rs = reinterpret_cast<R*>(cur);  // [nblk][16][kRowPad] the band of R (if a.rlds)

  const int tid = threadIdx.x;
  const int n = tid & (kScanN - 1);  // parameter point inside the tile (= GEMM column)
  const int ntiles = (a.B + kScanN - 1) / kScanN;
  // Every load of the prologue is independent, so their latencies overlap:
  // the first tile's parameters, the index tables, the band of R (a plain
  // copy: it is stored in its LDS layout) and the per-geometry tables.
  if (tid < kScanN * 5) {
    const int pp = min((int)blockIdx.x * kScanN + tid / 5, a.B - 1);
    p_s[tid] = a.params[5 * (int64_t)pp + tid % 5];
  }
  for (int i = tid; i < scan_meta_ints(mt); i += NT) meta[i] = a.meta[i];
  if ((nL * nq) % 2 == 0)
    copy16<NT>(q_s, a.qtab, (size_t)nL * nq * 8);
  else
    for (int i = tid; i < nL * nq; i += NT) q_s[i] = a.qtab[i];
  for (int i = tid; i < nq; i += NT) f_s[i] = a.f[i];
  for (int i = tid; i < nbp; i += NT) d_s[i] = (i < nb) ? a.data[i] : 0.0;
  for (int i = tid; i < nL; i += NT) w_s[i] = a.wL[i];
  if (sizeof(R) == 4) copy16<NT>(lt_s, a.logtab, (size_t)kLogTab * 16);
  // The GEMM operand starts at zero (its padding rows and, for shared tiles,
  // columns kTab..15 stay zero until a per-point tile writes them).
  for (int i = tid; i < nbp * kBRow; i += NT) bb[i] = R(0);
  __syncthreads();
  // The band is needed only from the smearing on: its copy runs while the
  // point pass computes (issued after the barrier, which would wait for it).
  if (a.rlds) copy16_async<NT>(Rs, a.band, (size_t)a.nblk * kBlk * sizeof(R));

  const int bg = tid >> 4;           // bin group
  const int lane = tid & (kWave - 1), wave = tid >> 6;
  const int krow = lane >> 4;        // k index of this lane in an MFMA operand
  // Lanes per bin for the shared sums: the largest power of two, at most 16,
  // with which one pass over the bins covers them all (G nb <= NT).
  int G = 1;
  while (G < 16 && 2 * G * nb <= NT) G *= 2;
  const int items = a.ppb * nL;
  const int gq = G / nL, gr = G - gq * nL;

  bool bb_clean = true;  // columns kTab..15 of bb are zero (work-group uniform)
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int p_raw = tile * kScanN + n;
    const bool valid = p_raw < a.B;
    const int p = valid ? p_raw : a.B - 1;
    double thv[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) thv[c] = p_s[5 * n + c];
    const PeeCoef<R> k = pee_coef<R>(thv);
    const double norm = thv[4];

    // Each 16-lane group holds all 16 points of the tile, so a wave vote
    // decides for the whole work-group (lanes past the end of the batch
    // repeat its last point).
    bool shared = false;
    if (SHARE) shared = __all(thv[0] == p_s[0] && thv[1] == p_s[1]) != 0;

    // ---- 1. point pass ------------------------------------------------------
    R mu0[PPT];
    R J0[PPT][4];
    if (SHARE && shared) {
      // Per-bin phase sums: G lanes split the bin's (k, r) items, then fold.
      // Each lane takes its items three at a time (independent chains that
      // can overlap); slots past the end carry weight 0 and add exact zeros.
      const int nslot = (items + G - 1) / G;
      for (int j0 = 0; j0 < nb; j0 += NT / G) {
        const int j = j0 + tid / G, sub = tid & (G - 1);
        const bool jin = j < nb;
        const int jc = jin ? j : nb - 1;
        R sum[kTab];
#pragma unroll
        for (int c = 0; c < kTab; ++c) sum[c] = R(0);
        // Item it = kk nL + r; a lane's items step by G = gq nL + gr.
        int kk = sub / nL, r = sub - kk * nL;
        for (int s0 = 0; s0 < nslot; s0 += 3) {
          int kks[3], rs[3];
          bool ok[3];
#pragma unroll
          for (int u = 0; u < 3; ++u) {
            ok[u] = jin && sub + (s0 + u) * G < items;
            kks[u] = ok[u] ? kk : 0;
            rs[u] = ok[u] ? r : 0;
            kk += gq;
            r += gr;
            if (r >= nL) {
              r -= nL;
              ++kk;
            }
          }
#pragma unroll
          for (int u = 0; u < 3; ++u) {
            const int kq = jc * a.ppb + kks[u];
            const double q = q_s[rs[u] * nq + kq];
            const R fw = ok[u] ? f_s[kq] * (R)w_s[rs[u]] : R(0);
            const PhaseTerms<R> t21 = phase_terms<R>(k.dm21 * q);
            const PhaseTerms<R> t31 = phase_terms<R>(k.dm31 * q);
            PhaseTerms<R> t32;
            if constexpr (sizeof(R) == 8)
              t32 = phase_terms_diff64<R>(t21, t31, q, k);
            else
              t32 = phase_terms_diff<R>(t21, t31);
            sum[0] += fw;
            sum[1] = rfma_t<R>(fw, t21.C, sum[1]);
            sum[2] = rfma_t<R>(fw, t31.C, sum[2]);
            sum[3] = rfma_t<R>(fw, t32.C, sum[3]);
            if (GRAD) {
              const R fq = fw * to_r<R>(q);
              sum[4] = rfma_t<R>(fq, t21.T, sum[4]);
              sum[5] = rfma_t<R>(fq, t31.T, sum[5]);
              sum[6] = rfma_t<R>(fq, t32.T, sum[6]);
              sum[7] = rfma_t<R>(fw, t21.S, sum[7]);
              sum[8] = rfma_t<R>(fw, t31.S, sum[8]);
              sum[9] = rfma_t<R>(fw, t32.S, sum[9]);
            }
          }
        }
        group_sums(sum, G);  // the G lanes of a bin (G <= 16)
        if (j < nb && sub == 0) {
          // Row j of the operand in 16-byte stores (fewer, wider LDS writes
          // than one per sum: the rows of neighbouring lanes share banks).
          R* row = bb + j * kBRow;
#pragma unroll
          for (int c = 0; c < kTab; ++c) row[c] = sum[c];
        }
      }
      // The rest of the operand (columns kTab..15) is zero unless a per-point
      // tile of this work-group wrote it.
      if (!bb_clean) {
        for (int i = tid; i < nb * kBRow; i += NT)
          if (i % kBRow >= kTab) bb[i] = R(0);
        bb_clean = true;
      }
    } else {
      // Per-point phases.  The SHARE kernel keeps only mu here and recomputes
      // the tangents in the gradient pass, which keeps its registers for the
      // shared path; the per-point kernel keeps the tangents in registers.
      constexpr bool KEEP_J = GRAD && !SHARE;
#pragma clang loop unroll(full)
      for (int m = 0; m < PPT; ++m) {
        const int j = bg + NG * m;
        R mu = R(0);
        R J[4] = {R(0), R(0), R(0), R(0)};
        if (j < nb) {
          for (int kk = 0; kk < a.ppb; ++kk) {
            const int kq = j * a.ppb + kk;
            const R fk = f_s[kq];
            R pb = R(0);
            R dpb[4] = {R(0), R(0), R(0), R(0)};
            for (int r = 0; r < nL; ++r) {
              R P, dP[4];
              pee_point<R, KEEP_J>(k, q_s[r * nq + kq], P, dP);
              const R wr = (R)w_s[r];
              pb = rfma_t<R>(wr, P, pb);
              if (KEEP_J) {
#pragma unroll
                for (int c = 0; c < 4; ++c) dpb[c] = rfma_t<R>(wr, dP[c], dpb[c]);
              }
            }
            mu = rfma_t<R>(fk, pb, mu);
            if (KEEP_J) {
#pragma unroll
              for (int c = 0; c < 4; ++c) J[c] = rfma_t<R>(fk, dpb[c], J[c]);
            }
          }
        }
        mu0[m] = mu;
        if (KEEP_J) {
#pragma unroll
          for (int c = 0; c < 4; ++c) J0[m][c] = J[c];
        }
        if (j < nbp) bb[j * kBRow + n] = (R)norm * mu;  // padded rows: 0
      }
      bb_clean = false;
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wavefront's band copy
    __syncthreads();

    // ---- 2. nu = R mu ---------------------------------------------------------
    A4 acc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
      acc[u] = A4{R(0), R(0), R(0), R(0)};
      const int I = wave + u * NW;
      if (I < mt) {
        const int lo = kbA_s[2 * I], hi = kbA_s[2 * I + 1];
        if (a.rlds) {
          // A[i][k] = R[16 I + i][16 kb + k], i = lane & 15, k = 4 st + krow.
          const R* Ab = Rs + kbo_s[I] * kBlk + (lane & 15) * kRowPad + krow;
          for (int kb = lo; kb <= hi; ++kb) {
#pragma unroll
            for (int st = 0; st < 4; ++st) {
              const R av = Ab[(kb - lo) * kBlk + 4 * st];
              const R bv = bb[(kb * 16 + st * 4 + krow) * kBRow + n];
              acc[u] = Acc<R>::mfma(av, bv, acc[u]);
            }
          }
        } else {
          gemm_row_global<R>(a.RA + ((int64_t)I * mt) * 256 + lane, lo, hi, bb, krow, n, acc[u]);
        }
      }
    }
    __syncthreads();  // every wave is done reading the GEMM operand

    double chi = 0.0;
    bool badnu = false;
    double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (SHARE && shared) {
      // ---- 3s. shared tiles: the accumulators hold M = R T, T the per-bin
      // phase sums.  With c = (K0, A, B1, B2) of a point, nu = norm M c; with
      // gnu = d chi2 / d nu, the gradient needs only the projections
      // G_t = sum_i M_it gnu_i: gmu = R^T gnu and sum_j gmu_j T_jt = G_t, and
      // mu_j and J_jc are linear in T_j.  Sums in FP64 (the products of FP32
      // values are exact there).
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        const int I = wave + u * NW;
        if (I < mt && n < kTab) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            mm[(I * 16 + Acc<R>::row(krow, v)) * kTab + n] = (double)acc[u][v];
        }
      }
      __syncthreads();
      const double c0 = (double)k.K0, c1 = (double)k.A, c2 = (double)k.B1, c3 = (double)k.B2;
      // Gp[0] = sum_i gnu_i s_i with s = M c (= nu / norm); Gp[t] = G_t for t >= 4.
      double Gp[kTab];
#pragma unroll
      for (int t = 0; t < kTab; ++t) Gp[t] = 0.0;
      double nus[PPT];
      // Branch-free over the bins (rows past nb are masked), so that the
      // bins' division and logarithm chains can overlap (four at a time:
      // more would not fit the registers).
#pragma unroll 4
      for (int m = 0; m < PPT; ++m) {
        const int i = bg + NG * m;
        const bool in = i < nb;
        const double* Mi = mm + (in ? i : 0) * kTab;
        const double si = dfma(c3, Mi[3], dfma(c2, Mi[2], dfma(c1, Mi[1], c0 * Mi[0])));
        const double nu = norm * si;
        const double d = in ? d_s[i] : 0.0;
        badnu |= in && !(nu > 0.0 && nu < __builtin_huge_val());
        const double ratio = quot_pos(d, nu);
        const double term = dfma(d, chi2_log<R>(d > 0.0 ? ratio : 1.0, lt_s), nu - d);
        chi += in ? term : 0.0;
        if (GRAD) {
          const double gn = in ? 2.0 * (1.0 - ratio) : 0.0;
          Gp[0] = dfma(si, gn, Gp[0]);
#pragma unroll
          for (int t = 4; t < kTab; ++t) Gp[t] = dfma(Mi[t], gn, Gp[t]);
        }
        nus[m] = nu;
      }
      if (a.pred && valid) {
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
          const int i = bg + NG * m;
          if (i < nb) a.pred[(int64_t)p * nb + i] = nus[m];
        }
      }
      if (badnu && valid)
        __hip_atomic_fetch_or(a.status, (uint32_t)kBadPrediction, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
      if (GRAD) {
        const double b = (double)k.B;
        g[0] = dfma(c3, Gp[6], -(c1 * Gp[4]));
        g[1] = -dfma(c2, Gp[5], c3 * Gp[6]);
        g[2] = dfma(b, Gp[8], -((double)k.dA12 * Gp[7])) - b * Gp[9];
        g[3] = -((double)k.dA13 * Gp[7]) -
               (double)k.dB13 * dfma((double)k.c12, Gp[8], (double)k.s12 * Gp[9]);
        g[4] = Gp[0];
#pragma unroll
        for (int c = 0; c < 5; ++c) g[c] = xor_sum_16_32(g[c]);
      }
      chi = xor_sum_16_32(chi);
      if (lane < kScanN) {
        red[(wave * kScanN + n) * 6] = chi;
        if (GRAD) {
#pragma unroll
          for (int c = 0; c < 5; ++c) red[(wave * kScanN + n) * 6 + 1 + c] = g[c];
        }
      }
      __syncthreads();
    } else {
      // ---- 3. chi2 and gnu --------------------------------------------------------
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        const int I = wave + u * NW;
        if (I < mt) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            // Branch-free over the padded rows (i >= nb: d = 0, nu = 0),
            // which are masked; d = 0 takes ln 1 = 0.
            const int i = I * 16 + Acc<R>::row(krow, v);
            const bool in = i < nb;
            const double nu = (double)acc[u][v];
            const double d = d_s[i];
            badnu |= in && !(nu > 0.0 && nu < __builtin_huge_val());
            const double ratio = quot_pos(d, nu);
            const double term = dfma(d, chi2_log<R>(d > 0.0 ? ratio : 1.0, lt_s), nu - d);
            chi += in ? term : 0.0;
            bb[i * kBRow + n] = in ? (R)(2.0 * (1.0 - ratio)) : R(0);
          }
        }
      }
      if (a.pred && valid) {
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
          const int I = wave + u * NW;
          if (I < mt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int i = I * 16 + Acc<R>::row(krow, v);
              if (i < nb) a.pred[(int64_t)p * nb + i] = (double)acc[u][v];
            }
          }
        }
      }
      if (badnu && valid)
        __hip_atomic_fetch_or(a.status, (uint32_t)kBadPrediction, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
      chi = xor_sum_16_32(chi);
      if (lane < kScanN) red[(wave * kScanN + n) * 6] = chi;
      __syncthreads();

      if (GRAD) {
        // ---- 4. gmu = R^T gnu ---------------------------------------------------
        A4 acc2[TPW];
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
          acc2[u] = A4{R(0), R(0), R(0), R(0)};
          const int J = wave + u * NW;
          if (J < mt) {
            const int lo = kbT_s[2 * J], hi = kbT_s[2 * J + 1];
            if (a.rlds) {
              // A[i][k] = R^T[16 J + i][16 kb + k] = R[16 kb + k][16 J + i]: block
              // (kb, J) of the band, read transposed; blocks outside row tile
              // kb's range are zero.
              for (int kb = lo; kb <= hi; ++kb) {
                const int bi = blkT_s[J * mt + kb];
                if (bi < 0) continue;
                const R* Ab = Rs + bi * kBlk + krow * kRowPad + (lane & 15);
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                  const R av = Ab[4 * st * kRowPad];
                  const R bv = bb[(kb * 16 + st * 4 + krow) * kBRow + n];
                  acc2[u] = Acc<R>::mfma(av, bv, acc2[u]);
                }
              }
            } else {
              gemm_row_global<R>(a.RT + ((int64_t)J * mt) * 256 + lane, lo, hi, bb, krow, n,
                                 acc2[u]);
            }
          }
        }
        __syncthreads();  // every wave is done reading gnu
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
          const int J = wave + u * NW;
          if (J < mt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) bb[(J * 16 + Acc<R>::row(krow, v)) * kBRow + n] = acc2[u][v];
          }
        }
        __syncthreads();

        // ---- 5. gradient from the point-pass registers (or recomputed) -----------
        if (SHARE) {
          // Tangents recomputed (same operations and order as the per-point
          // kernel's point pass, so the same values).
#pragma clang loop unroll(full)
          for (int m = 0; m < PPT; ++m) {
            const int j = bg + NG * m;
            if (j < nb) {
              R J[4] = {R(0), R(0), R(0), R(0)};
              for (int kk = 0; kk < a.ppb; ++kk) {
                const int kq = j * a.ppb + kk;
                const R fk = f_s[kq];
                R dpb[4] = {R(0), R(0), R(0), R(0)};
                for (int r = 0; r < nL; ++r) {
                  R P, dP[4];
                  pee_point<R, true>(k, q_s[r * nq + kq], P, dP);
                  const R wr = (R)w_s[r];
#pragma unroll
                  for (int c = 0; c < 4; ++c) dpb[c] = rfma_t<R>(wr, dP[c], dpb[c]);
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) J[c] = rfma_t<R>(fk, dpb[c], J[c]);
              }
              const double gm = (double)bb[j * kBRow + n];
#pragma unroll
              for (int c = 0; c < 4; ++c) g[c] = dfma(gm, (double)J[c], g[c]);
              g[4] = dfma(gm, (double)mu0[m], g[4]);
            }
          }
        } else {
#pragma clang loop unroll(full)
          for (int m = 0; m < PPT; ++m) {
            const int j = bg + NG * m;
            if (j < nb) {
              const double gm = (double)bb[j * kBRow + n];
#pragma unroll
              for (int c = 0; c < 4; ++c) g[c] = dfma(gm, (double)J0[m][c], g[c]);
              g[4] = dfma(gm, (double)mu0[m], g[4]);
            }
          }
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) g[c] = xor_sum_16_32(g[c]);
        if (lane < kScanN) {
#pragma unroll
          for (int c = 0; c < 5; ++c) red[(wave * kScanN + n) * 6 + 1 + c] = g[c];
        }
        __syncthreads();
      }
    }

    if (tid < kScanN && valid) {
      double cs = 0.0, gs[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      for (int w = 0; w < NW; ++w) {
        cs += red[(w * kScanN + n) * 6];
        if (GRAD) {
#pragma unroll
          for (int c = 0; c < 5; ++c) gs[c] += red[(w * kScanN + n) * 6 + 1 + c];
        }
      }
      if (k.bad)
        __hip_atomic_fetch_or(a.status, (uint32_t)kBadMixing, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
      a.chi2[p] = k.bad ? NAN : 2.0 * cs;
      if (GRAD && a.grad) {
#pragma unroll
        for (int c = 0; c < 4; ++c) a.grad[5 * (int64_t)p + c] = k.bad ? NAN : norm * gs[c];
        a.grad[5 * (int64_t)p + 4] = k.bad ? NAN : gs[4];
      }
    }
    // Parameters of this group's next tile (every lane read p_s at the top).
    if (tid < kScanN * 5) {
      const int pn = min((tile + (int)gridDim.x) * kScanN + tid / 5, a.B - 1);
      p_s[tid] = a.params[5 * (int64_t)pn + tid % 5];
    }
    __syncthreads();  // LDS is reused by the next tile
  }
}

// ---- configuration-stage tables -------------------------------------------
__global__ void qtab_kernel(const double* __restrict__ E, const double* __restrict__ L, int nL,
                            int nq, double* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nL * nq) return;
  const int r = (int)(i / nq), k = (int)(i - (int64_t)r * nq);
  q[i] = (kPhase * L[r]) / E[k];
}

// A-operand tiles of R (transpose = 0) or R^T (transpose = 1):
// tile (I, kb), step st, lane l holds M[I*16 + (l & 15)][kb*16 + 4 st + (l >> 4)].
template <class R>
__global__ void tile_kernel(const SliceDev* __restrict__ slices, const R* __restrict__ Rv, int nb,
                            int mt, int transpose, R* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)mt * mt * 256) return;
  const int l = (int)(idx & 63);
  const int st = (int)((idx >> 6) & 3);
  const int64_t t = idx >> 8;
  const int kb = (int)(t % mt), I = (int)(t / mt);
  const int a = I * 16 + (l & 15), b = kb * 16 + st * 4 + (l >> 4);
  const int i = transpose ? b : a;  // row of R
  const int j = transpose ? a : b;  // column of R
  R v = R(0);
  if (i < nb && j < nb) {
    const SliceDev sd = slices[i / kSlice];
    const int d = j - i;
    if (d >= sd.dlo && d < sd.dlo + sd.nd) v = Rv[sd.off + (int64_t)(d - sd.dlo) * kSlice + (i % kSlice)];
  }
  out[idx] = v;
}

// Block (I, J) of R, listed in blist, into the band in its LDS layout
// (row-major, rows padded to kRowPad; pads are 0).
template <class R>
__global__ void pack_band_kernel(const R* __restrict__ RA, const int32_t* __restrict__ blist,
                                 int nblk, int mt, R* __restrict__ band) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nblk * kBlk) return;
  const int b = (int)(idx / kBlk), w = (int)(idx % kBlk);
  const int row = w / kRowPad, col = w % kRowPad;
  R v = R(0);
  if (col < 16) {
    const int I = blist[2 * b], J = blist[2 * b + 1];
    // RA holds A[i][k] = R[16 I + i][16 J + k] at step k / 4, lane i + 16 (k % 4).
    v = RA[((int64_t)(I * mt + J) * 4 + col / 4) * 64 + row + 16 * (col % 4)];
  }
  band[idx] = v;
}

struct ScanLayout {
  size_t RA, RT, meta, blist, band, qtab, logtab, total;
};

ScanLayout scan_layout(const gna_plan* p) {
  ScanLayout L{};
  const ProbDev& pd = p->probs[0];
  const int mt = (pd.n_bins + 15) / 16;
  const size_t rs = (p->prec == GNA_FP64) ? 8 : 4;
  const int64_t nq = (int64_t)pd.n_bins * pd.ppb;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t at = off;
    off = align_up(off + std::max<size_t>(b, 1), 256);
    return at;
  };
  L.RA = take((size_t)mt * mt * 256 * rs);
  L.RT = take((size_t)mt * mt * 256 * rs);
  L.meta = take((size_t)scan_meta_ints(mt) * 4);
  L.blist = take((size_t)mt * mt * 2 * 4);
  L.band = take((size_t)mt * mt * kBlk * rs);
  L.qtab = take((size_t)pd.n_L * nq * 8);
  L.logtab = take((size_t)kLogTab * 16);
  L.total = off;
  return L;
}


template <class R, bool GRAD, int NT, int WPE, bool SHARE>
int launch_scan_k(gna_plan* p, const ScanArgs<R>& a, const gna_plan::LaunchCache& lc,
                  hipStream_t s) {
  const int ntiles = (a.B + kScanN - 1) / kScanN;
  const int grid = std::max(1, std::min(ntiles, lc.occ * p->cu_count));
  hipLaunchKernelGGL((scan_kernel<R, GRAD, NT, WPE, SHARE>), dim3(grid), dim3(NT), lc.lds, s, a);
  return check_hip(hipGetLastError(), "scan_kernel launch");
}

template <class R, bool GRAD, int NT, int WPE, bool SHARE>
bool scan_lds_ok(const gna_plan* p, size_t bytes) {
  if (bytes > p->lds_device) return false;
  if (bytes <= 64 * 1024) return true;
  if (hipFuncSetAttribute((const void*)scan_kernel<R, GRAD, NT, WPE, SHARE>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess)
    return true;
  (void)hipGetLastError();
  return false;
}

template <class R, bool GRAD, int NT, int WPE>
int launch_scan_t(gna_plan* p, ScanArgs<R> a, hipStream_t s) {
  gna_plan::LaunchCache& lc = p->launch_cache[GRAD];
  if (!lc.ready) {
    // The shared-phase kernel needs an FP64 copy of M = R T in LDS, and the
    // band of R is staged in LDS when it fits; beyond 64 KB the kernel asks
    // for the LDS (up to the device's per-work-group limit), else goes without.
    const int nw = NT / 64;
    lc.share = p->share_phases;
    const size_t with_r = scan_lds<R>(a.nL, a.nq, a.mt, nw, a.nblk, lc.share);
    lc.rlds = a.nblk > 0 && (lc.share ? scan_lds_ok<R, GRAD, NT, WPE, true>(p, with_r)
                                      : scan_lds_ok<R, GRAD, NT, WPE, false>(p, with_r));
    lc.lds = scan_lds<R>(a.nL, a.nq, a.mt, nw, lc.rlds ? a.nblk : 0, lc.share);
    if (!lc.rlds && lc.share && !scan_lds_ok<R, GRAD, NT, WPE, true>(p, lc.lds)) {
      lc.share = 0;
      lc.lds = scan_lds<R>(a.nL, a.nq, a.mt, nw, 0, false);
    }
    lc.occ = 0;
    const hipError_t e =
        lc.share ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                       &lc.occ, scan_kernel<R, GRAD, NT, WPE, true>, NT, lc.lds)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                       &lc.occ, scan_kernel<R, GRAD, NT, WPE, false>, NT, lc.lds);
    if (e != hipSuccess || lc.occ < 1) lc.occ = 1;
    lc.ready = 1;
  }
  a.rlds = lc.rlds;
  return lc.share ? launch_scan_k<R, GRAD, NT, WPE, true>(p, a, lc, s)
                  : launch_scan_k<R, GRAD, NT, WPE, false>(p, a, lc, s);
}

template <class R>
int launch_scan_r(gna_plan* p, const double* params, int32_t B, double* chi2, double* grad,
                  double* pred, hipStream_t s) {
  const ScanLayout SL = scan_layout(p);
  const ProbDev& pd = p->probs[0];
  unsigned char* w = p->ws;
  unsigned char* base = w + p->lay.Rdense;
  ScanArgs<R> a{};
  a.B = B;
  a.nb = pd.n_bins;
  a.mt = (pd.n_bins + 15) / 16;
  a.ppb = pd.ppb;
  a.nL = pd.n_L;
  a.nq = pd.n_bins * pd.ppb;
  a.qtab = (const double*)(base + SL.qtab);
  a.logtab = (const double*)(base + SL.logtab);
  a.f = (const R*)(w + p->lay.f);
  a.wL = (const double*)(w + p->lay.wL);
  a.data = (const double*)(w + p->lay.data);
  a.RA = (const R*)(base + SL.RA);
  a.RT = (const R*)(base + SL.RT);
  a.meta = (const int32_t*)(base + SL.meta);
  a.band = (const R*)(base + SL.band);
  a.nblk = p->scan_nblk;
  a.params = params;
  a.chi2 = chi2;
  a.grad = grad;
  a.pred = pred;
  a.status = (uint32_t*)(w + p->lay.status);
  const int nt = scan_threads(p);
  if (nt != 512) return fail(GNA_E_UNSUPPORTED, "scan kernel does not fit in LDS");
  switch (p->shape.mfma) {
    case 2:
      return grad ? launch_scan_t<R, true, 512, 3>(p, a, s) : launch_scan_t<R, false, 512, 3>(p, a, s);
    case 3:
      return grad ? launch_scan_t<R, true, 512, 4>(p, a, s) : launch_scan_t<R, false, 512, 4>(p, a, s);
    default:
      return grad ? launch_scan_t<R, true, 512, 2>(p, a, s) : launch_scan_t<R, false, 512, 2>(p, a, s);
  }
}

}  // namespace

int scan_threads(const gna_plan* p) {
  const ProbDev& pd = p->probs[0];
  const int mt = (pd.n_bins + 15) / 16;
  const int nq = pd.n_bins * pd.ppb;
  const bool fp64 = p->prec == GNA_FP64;
  // 512 lanes: the gradient variant keeps mu0 / J0 of 8 bins in registers
  // (~240 VGPRs in FP64) without spilling; 1024 lanes would cap it at 128.
  for (int nt : {512}) {
    const size_t b = fp64 ? scan_lds<double>(pd.n_L, nq, mt, nt / 64, 0, false)
                          : scan_lds<float>(pd.n_L, nq, mt, nt / 64, 0, false);
    if (b <= std::min(kScanLdsMax, p->lds_limit)) return nt;
  }
  return 0;
}

bool scan_supported(const gna_plan* p) {
  if (p->kind != kChain || p->probs.empty()) return false;
  const ProbDev& pd = p->probs[0];
  if (pd.n_bins > kScanMaxBins) return false;
  return scan_threads(p) != 0;
}

size_t scan_dense_bytes(const gna_plan* p) {
  if (!scan_supported(p)) return 0;
  return scan_layout(p).total;
}

int build_scan_tables(gna_plan* p, hipStream_t s) {
  const ScanLayout SL = scan_layout(p);
  const ProbDev& pd = p->probs[0];
  const int nb = pd.n_bins, mt = (nb + 15) / 16;
  unsigned char* w = p->ws;
  unsigned char* base = w + p->lay.Rdense;
  // Block-band extents from the slices: row i holds columns
  // [i + dlo, i + dlo + nd - 1] of its slice, clipped to the matrix.
  std::vector<int32_t> kbA(2 * mt), kbT(2 * mt);
  std::vector<int> colA_lo(mt, 1 << 30), colA_hi(mt, -1), rowT_lo(mt, 1 << 30), rowT_hi(mt, -1);
  for (int i = 0; i < nb; ++i) {
    const SliceDev& sd = p->slices[pd.slice_off + i / kSlice];
    const int c0 = std::max(0, i + sd.dlo), c1 = std::min(nb - 1, i + sd.dlo + sd.nd - 1);
    if (c1 < c0) continue;
    const int I = i / 16;
    colA_lo[I] = std::min(colA_lo[I], c0);
    colA_hi[I] = std::max(colA_hi[I], c1);
    for (int J = c0 / 16; J <= c1 / 16; ++J) {
      rowT_lo[J] = std::min(rowT_lo[J], i);
      rowT_hi[J] = std::max(rowT_hi[J], i);
    }
  }
  std::vector<int32_t> kbo(mt), blist, blkT((size_t)mt * mt, -1);
  for (int I = 0; I < mt; ++I) {
    kbA[2 * I] = colA_hi[I] >= 0 ? colA_lo[I] / 16 : 0;
    kbA[2 * I + 1] = colA_hi[I] >= 0 ? colA_hi[I] / 16 : -1;
    kbT[2 * I] = rowT_hi[I] >= 0 ? rowT_lo[I] / 16 : 0;
    kbT[2 * I + 1] = rowT_hi[I] >= 0 ? rowT_hi[I] / 16 : -1;
    // The band's blocks, row tile by row tile, for staging in LDS.
    kbo[I] = (int32_t)(blist.size() / 2);
    for (int J = kbA[2 * I]; J <= kbA[2 * I + 1]; ++J) {
      blkT[(size_t)J * mt + I] = (int32_t)(blist.size() / 2);
      blist.push_back(I);
      blist.push_back(J);
    }
  }
  const int nblk = (int)(blist.size() / 2);
  p->scan_nblk = nblk;
  std::vector<int32_t> meta;
  meta.insert(meta.end(), kbA.begin(), kbA.end());
  meta.insert(meta.end(), kbT.begin(), kbT.end());
  meta.insert(meta.end(), kbo.begin(), kbo.end());
  meta.insert(meta.end(), blkT.begin(), blkT.end());
  int rc = check_hip(hipMemcpyAsync(base + SL.meta, meta.data(), meta.size() * 4,
                                    hipMemcpyHostToDevice, s), "hipMemcpyAsync (scan index tables)");
  if (rc) return rc;
  // Logarithm table (log_tab): r_k = 362 / (k + 256) rounded once, and
  // -ln r_k from a long-double logarithm, rounded once.
  std::vector<double> lt(2 * kLogTab);
  for (int k = 0; k < kLogTab; ++k) {
    lt[2 * k] = 362.0 / (double)(k + 256);
    lt[2 * k + 1] = (double)(-std::log((long double)lt[2 * k]));
  }
  rc = check_hip(hipMemcpyAsync(base + SL.logtab, lt.data(), lt.size() * 8, hipMemcpyHostToDevice,
                                s), "hipMemcpyAsync (logarithm table)");
  if (rc) return rc;
  if (nblk > 0) {
    rc = check_hip(hipMemcpyAsync(base + SL.blist, blist.data(), blist.size() * 4,
                                  hipMemcpyHostToDevice, s), "hipMemcpyAsync (blist)");
    if (rc) return rc;
  }
  const int64_t nq = (int64_t)nb * pd.ppb;
  const int64_t nqt = nq * pd.n_L;
  hipLaunchKernelGGL(qtab_kernel, dim3((unsigned)((nqt + 255) / 256)), dim3(256), 0, s,
                     (const double*)(w + p->lay.E), (const double*)(w + p->lay.L), pd.n_L,
                     (int)nq, (double*)(base + SL.qtab));
  if ((rc = check_hip(hipGetLastError(), "qtab_kernel"))) return rc;
  const int64_t nt = (int64_t)mt * mt * 256;
  const unsigned g = (unsigned)((nt + 255) / 256);
  const SliceDev* dsl = (const SliceDev*)(w + p->lay.slices) + pd.slice_off;
  for (int tr = 0; tr < 2; ++tr) {
    if (p->prec == GNA_FP64)
      hipLaunchKernelGGL(tile_kernel<double>, dim3(g), dim3(256), 0, s, dsl,
                         (const double*)(w + p->lay.Rv), nb, mt, tr,
                         (double*)(base + (tr ? SL.RT : SL.RA)));
    else
      hipLaunchKernelGGL(tile_kernel<float>, dim3(g), dim3(256), 0, s, dsl,
                         (const float*)(w + p->lay.Rv), nb, mt, tr,
                         (float*)(base + (tr ? SL.RT : SL.RA)));
    if ((rc = check_hip(hipGetLastError(), "tile_kernel"))) return rc;
  }
  if (nblk > 0) {
    const int64_t nbe = (int64_t)nblk * kBlk;
    const unsigned gb = (unsigned)((nbe + 255) / 256);
    if (p->prec == GNA_FP64)
      hipLaunchKernelGGL(pack_band_kernel<double>, dim3(gb), dim3(256), 0, s,
                         (const double*)(base + SL.RA), (const int32_t*)(base + SL.blist), nblk,
                         mt, (double*)(base + SL.band));
    else
      hipLaunchKernelGGL(pack_band_kernel<float>, dim3(gb), dim3(256), 0, s,
                         (const float*)(base + SL.RA), (const int32_t*)(base + SL.blist), nblk,
                         mt, (float*)(base + SL.band));
    if ((rc = check_hip(hipGetLastError(), "pack_band_kernel"))) return rc;
  }
  // The host vectors die here.
  return check_hip(hipStreamSynchronize(s), "hipStreamSynchronize (scan tables)");
}

int launch_scan(gna_plan* p, const double* params, int32_t B, double* chi2, double* grad,
                double* pred, hipStream_t s) {
  if (!scan_supported(p)) return fail(GNA_E_UNSUPPORTED, "plan does not support the scan kernel");
  if (p->prec == GNA_FP64) return launch_scan_r<double>(p, params, B, chi2, grad, pred, s);
  return launch_scan_r<float>(p, params, B, chi2, grad, pred, s);
}

}  // namespace gna
