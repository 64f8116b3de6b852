// Internal declarations of libgna_hip.so (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gna_hip.h"

namespace gna {

// ---- limits ----------------------------------------------------------------
constexpr int kMaxBins = 4096;      // LDS holds mu and d chi2/d nu of one problem
constexpr int kMaxOrder = 64;       // Gauss-Legendre order
constexpr int kMaxPPB = 65536;      // points per bin
constexpr int kMaxBaselines = 64;
constexpr int kSlice = 64;          // rows per smearing-band slice (one wavefront)
constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kGLTable = kMaxOrder * (kMaxOrder + 1) / 2;  // rules of order 1..64
constexpr double kBandZ = 6.0;      // erf(z) == +-1 in FP64 beyond |z| = 5.93
// Queued tail: a fit's tail item sits at least this many wavefronts per CU
// of queue entries after its last tile (with the CU count and the
// work-group size: about one turnover of the resident work-groups).
constexpr int kQueuedLagWaves = 16;
// Lanes of the per-point tail launch of a two-launch chain plan.
constexpr int kChainTailThreads = 512;

// ---- device-side descriptors (live in the workspace) -----------------------
struct ProbDev {
  int32_t n_bins;
  int32_t ppb;            // quadrature points per bin = order * n_sub
  int32_t n_L;
  int32_t order;
  int32_t n_sub;
  int32_t G;              // lanes per bin
  int32_t C;              // chunks per bin
  int32_t bins_per_tile;  // threads / G
  int32_t n_bin_blocks;
  int32_t n_slices;
  int32_t by_item;        // lanes and chunks split (point, baseline) items, not points
  int32_t pad_;
  int64_t pt_off;         // first quadrature point (E, f arrays)
  int64_t bin_off;        // first bin in data / pred (fitset) arrays
  int64_t edge_off;       // first edge
  int64_t L_off;          // first baseline
  int64_t slice_off;      // first band slice
  int64_t scratch_off;    // fitset: first scratch element of this fit
};

// One 64-row slice of the banded smearing matrix: rows i = 64 s + l, l < 64,
// diagonals d = dlo .. dlo + nd - 1 hold R[i][i + d] at off + (d - dlo) * 64 + l.
struct SliceDev {
  int32_t dlo;
  int32_t nd;
  int64_t off;
};

struct TileDev {
  int32_t point;  // parameter point (fitset: fit index)
  int32_t prob;   // problem index
  int32_t bb;     // bin block
  int32_t chunk;  // chunk of each bin's points
};

// Arguments of the generic tile kernel (by value).
template <class R>
struct ChainArgs {
  const ProbDev* probs;
  const TileDev* tiles;      // NULL: chain plan, tiles decoded from the index
  int64_t n_tiles;
  int32_t tiles_per_point;   // chain plan only
  int32_t want_grad;
  int64_t scratch_stride;    // chain plan: scratch elements per parameter point
  const double* E;
  const R* f;
  const double* L;
  const double* wL;
  const double* data;
  const SliceDev* slices;
  const R* Rv;
  const double* params;      // [B][5] on the device; NULL: one point, given in pin
  double pin[5];             // the one point's parameters, by value (params == NULL)
  R* scratch;
  uint32_t* counters;
  uint32_t* status;
  uint32_t* queue;
  double* chi2;
  double* grad;
  double* pred;
  // Queued tail (uneven batches, one launch): the queue (entry >= 0: a tile
  // index; < 0: the tail of fit -1 - entry), the fit of each slice and the
  // per-slice partial sums (counters holds the per-fit count of finished
  // tiles).
  const int32_t* q_items;
  int64_t n_items;
  const int32_t* slice_prob;
  double* part;
  uint32_t spin_limit;  // sleeps before a tail's wait gives up
  uint32_t need_extra;  // tiles a tail waits for beyond its fit's (0; tests of the bound)
};

// kSpinTimeout: a queued tail waited longer than its bound for a fit's point
// tiles (its results are not valid).
enum StatusBits : uint32_t { kBadMixing = 1u, kBadPrediction = 2u, kSpinTimeout = 4u };

// ---- host-side plan ---------------------------------------------------------
enum PlanKind { kChain = 0, kFitset = 1 };

struct Layout {
  size_t probs = 0, slices = 0, slice_prob = 0, tiles = 0, E = 0, f = 0, L = 0, wL = 0,
         edges = 0, data = 0, gl = 0, Rv = 0, scratch = 0, counters = 0, queue = 0, status = 0,
         Rdense = 0, tailpart = 0, fwd_order = 0, q_items = 0, total = 0;
};

struct Shape {
  int threads = 256, G = 1, C = 1, persistent = 0, mfma = 0;
  int share = 1;  // MFMA kernel: tiles with common dm2 share their phases (if the plan allows)
  // Uneven batch: 0 = each fit's tail in the work-group that finishes its
  // last tile; 1 = the tails in two more launches, wide over the GPU;
  // 2 = queued tail: one tail item per fit in the one persistent launch's
  // queue, interleaved with the point tiles (a fit's tail some way after its
  // last tile).
  int split = 0;
};

}  // namespace gna

struct gna_plan {
  int kind;
  int prec;
  int n_probs;
  int n_points;           // chain: max_batch; fitset: n_fits
  int64_t total_pts;
  int64_t total_bins;
  int64_t total_slices;
  int64_t total_band;     // stored band entries
  int max_bins;
  int ccap;               // largest chunk count the scratch is sized for
  int64_t tile_capacity;  // fitset: tile-list capacity
  int64_t scratch_elems;
  gna::Shape shape;
  int64_t n_tiles;        // fitset: tiles in the queue; chain: tiles per point
  int64_t n_qitems;       // queued tail: queue entries (tiles and fit tails)
  int tail_pin;           // fitset: opts.split_tail (nonzero: the autotuner keeps that tail)
  uint32_t q_spin_limit;  // queued tail: 0 = the default bound (gna_debug_queued_wait)
  uint32_t q_need_extra;
  int cu_count;
  size_t lds_limit;       // LDS budget of the generic kernel (64 KB)
  size_t lds_device;      // LDS per work-group the device allows (160 KB on gfx950)
  int share_allowed;      // the plan's options allow phase sharing across a tile
  int share_phases;       // the current shape shares (share_allowed && shape.share)
  // Launch decisions that depend only on the plan and its shape (dynamic LDS,
  // work-groups per CU, whether the shared-phase scan kernel got its LDS),
  // made at the first launch without / with the gradient; apply_shape clears
  // them.  Keeps attribute and occupancy queries off the evaluation path.
  struct LaunchCache {
    int ready;
    int share;
    int rlds;
    size_t lds;
    int occ;
  } launch_cache[2];
  int scan_nblk;          // 16x16 blocks in the band of R (scan kernel)
  char arch[64];
  unsigned char* ws;
  size_t ws_bytes;
  gna::Layout lay;
  gna_model model;
  std::vector<gna::ProbDev> probs;     // host copy of the device descriptors
  std::vector<gna::SliceDev> slices;   // host copy
  std::vector<int32_t> fwd_order;      // fitset: slices, most diagonals first
  std::vector<double> edges_host;      // concatenated edges
  // The rest of the configuration, kept on the host so that the
  // configuration stage can be run again into the same workspace
  // (gna_plan_rebuild): baselines, weights, data, slice owners.
  std::vector<double> L_host, wL_host, data_host;
  std::vector<int32_t> slice_prob_host;
};

namespace gna {

// ---- error plumbing ----------------------------------------------------------
int fail(int code, const char* fmt, ...);
int check_hip(hipError_t e, const char* what);
void clear_error();

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Launch helpers implemented in the .hip files.
// params: [B][5] on the device, or NULL with B = 1 and the point's five
// parameters in host_params (passed by value to the kernel: no upload).
int launch_chain(gna_plan* p, const double* params, int32_t B, double* chi2, double* grad,
                 double* pred, hipStream_t s, const double* host_params = nullptr);
int launch_scan(gna_plan* p, const double* params, int32_t B, double* chi2, double* grad,
                double* pred, hipStream_t s);
int build_scan_tables(gna_plan* p, hipStream_t s);
bool scan_supported(const gna_plan* p);
// Lanes per work-group of the MFMA scan kernel for this plan (0: it does not fit).
int scan_threads(const gna_plan* p);
size_t scan_dense_bytes(const gna_plan* p);
// Dynamic LDS of the generic kernel: vs = LDS stride of the point's vectors
// (0: they stay in the scratch region), kf_cap = largest number of diagonal
// chunks per slice, bytes = total.
struct ChainLds {
  int vs = 0, kf_cap = 1;
  size_t bytes = 0;
};
ChainLds chain_lds(const gna_plan* p, const Shape& sh);
size_t chain_lds_bytes(const gna_plan* p, const Shape& sh);
// LDS a shape may use: 64 KB for the generic kernel, the device's limit for
// the queued-tail kernel.
size_t shape_lds_limit(const gna_plan* p, const Shape& sh);
// Dynamic LDS of the queued-tail kernel: one staging window per wavefront.
size_t queued_lds_bytes(const gna_plan* p, const Shape& sh);
// Sets the per-problem tiling of `sh` (and, for a fitset, rebuilds and
// uploads the tile list when the plan has a workspace).
int apply_shape(gna_plan* p, const Shape& sh, hipStream_t s);
std::vector<Shape> shape_candidates(const gna_plan* p);

// Coefficients of P_ee in the all-positive form P = K0 + A cos^2 phi21 +
// B1 cos^2 phi31 + B2 cos^2 phi32 (Sec. 4.1 with alpha = beta = e):
// A = 4 s12 (1-s12) (1-s13)^2, B = 4 s13 (1-s13), B1 = B (1-s12), B2 = B s12,
// K0 = 1 - A - B.  Host code (pee.hip).
void pee_coefficients(double s12, double s13, double* K0, double* A, double* B1, double* B2);

// Coefficients of the Sec. 4.1 probability for flavours a -> b (0 = e, 1 = mu,
// 2 = tau): P = delta + sum_t re[t] sin^2 phi_t + im[t] sin 2phi_t over the
// pairs t = (21, 31, 32), re = -4 Re X, im = 2 Im X, X_ij = V*_ai V_bi V_aj
// V*_bj, V the PMNS matrix of the angles ang = (th12, th13, th23, delta_CP)
// (delta -> -delta for antineutrinos).  Host code (prob.hip).
void prob_coefficients(int a, int b, int anti, const double* ang, double* delta, double re[3],
                       double im[3]);

}  // namespace gna
