// Internal declarations of the umbir HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>
#include <string>
#include <vector>

#include "umbir.h"

namespace umbir {

constexpr int kMaxLayers = UMBIR_MAX_LAYERS;
constexpr double kTwo32 = 4294967296.0;

// One-way leg record: delay in Q32.32 fixed-point samples and cos^beta of
// the leg's angle sum, stored row-major [nz][n_off].  Within a row the lattice
// offsets are split by parity (even offsets first, then odd): one transducer
// only ever uses offsets of one parity, so neighbouring columns read
// neighbouring records.  n_off is even.  With attenuation a second table of
// the same layout holds each leg's path attenuation in template bins
// (float64, Gamma_leg / dgamma).
struct __align__(16) Leg {
  int64_t delay;
  float apod;
  int spare;  // 0
};

// Attenuation bins: a (trace, voxel) pair whose legs carry u_tx and u_rx
// template bins of attenuation uses the nearest template,
// floor(u_tx + u_rx + 1/2) in float64, at most n_gamma - 1.
constexpr int kMaxGamma = 64;
__host__ __device__ __forceinline__ int gamma_bin(double u, int last) {
  const double b = floor(u + 0.5);
  return b < double(last) ? int(b) : last;
}

// Template occupancy (attenuation): one 64-bit mask per (trace, block of
// 2^kMaskShift fine positions), bit g set when some voxel of template g puts
// weight on a position of the block.
constexpr int kMaskShift = 10;

__host__ __device__ __forceinline__ int leg_slot(int o, int half) { return (o >> 1) + (o & 1) * half; }

// The windowed gather (FP32 fine grid): voxel tiles of kGatherTileRows x
// kGatherTileCols, and for every (tile, trace) the window of fine positions
// its voxels read, staged in LDS when it fits kGatherWinBytes (16384 FP32 or
// 32768 16-bit positions); windows start and end on 16-byte boundaries
// (gather_window_align positions).
constexpr int kGatherTileRows = 32, kGatherTileCols = 64, kGatherWinBytes = 65536;
inline int gather_window_align(int storage) { return storage == UMBIR_STORAGE_F32 ? 4 : 8; }
inline long gather_tiles(int nx, int nz) {
  return long((nx + kGatherTileCols - 1) / kGatherTileCols) * ((nz + kGatherTileRows - 1) / kGatherTileRows);
}
// Its blocks per trace group: one generation of at most 512 blocks (two per
// CU, 64 KiB of window each) over the tiles; *tiles_per_block receives each
// block's share.
inline int gather_lds_blocks(int nx, int nz, int groups, int* tiles_per_block) {
  const long tiles = gather_tiles(nx, nz);
  long nb = tiles < 512 / groups ? tiles : 512 / groups;
  if (nb < 1) nb = 1;
  *tiles_per_block = int((tiles + nb - 1) / nb);
  return int((tiles + *tiles_per_block - 1) / *tiles_per_block);
}
// Bytes of the window table ([tiles][traces] of {first position, count}),
// 0 where the windowed gather does not apply: a record of fine positions not
// a multiple of gather_window_align, more tiles than a grid dimension holds or
// a table over 64 MiB.
inline size_t gather_window_bytes(int nx, int nz, long traces, long fine_per_trace, int storage) {
  const long tiles = gather_tiles(nx, nz);
  const size_t bytes = size_t(tiles) * size_t(traces) * 8;
  if (fine_per_trace % gather_window_align(storage) != 0 || tiles > 65535 || bytes > (size_t(64) << 20)) return 0;
  return bytes;
}
// The default gather form where the table exists: windowed when its blocks
// (groups x tiles, two tiles a block beyond 512) fill at least three quarters
// of one generation; with fewer, one block per CU leaves the window loads'
// latency exposed and the row-wise gather is faster (measured at 352 x 352
// and 384 x 384 with 8 groups, 264 and 288 blocks: 0.43 against 0.33 and
// 0.42 against 0.37 ms per adjoint).
inline bool gather_windowed_default(int nx, int nz, int groups) {
  int tpb;
  return 4L * groups * gather_lds_blocks(nx, nz, groups, &tpb) >= 3L * 512;
}

// LDS of one splat workgroup: all 160 KiB of a gfx950 CU, one workgroup of
// 16 waves per CU (measured against 64 KiB and 80 KiB, two workgroups per CU:
// the larger tiles need fewer passes over the row pointers and fewer partly
// used row blocks; 120 us against 130 us at 256 x 256, 1.49 ms against
// 1.80 ms at 512 x 512).
constexpr long kSplatLdsBytes = 163840;

// Rows per lattice position (per column) of the splat's transposed tables:
// nz rounded up to a multiple of 8 (one 128-byte line of leg records per
// 8-row block), and to an odd number of such blocks, so that the columns of
// one wave step (8 positions apart by whole tables rows) do not all fall on
// addresses a power of two apart.
inline int padded_rows(int nz) {
  int p = (nz + 7) & ~7;
  if (((p >> 3) & 1) == 0) p += 8;
  return p;
}

// Blocks of the forward's image prescale: each leaves its max|tau x| for the
// splat, which takes the largest (no atomic, nothing to clear first).
constexpr int kPrescaleBlocks = 128;

// Row ranges of the layers the grid reaches: rows [lo[s], hi[s]) of layer
// segment s, for the n segments the grid reaches.
struct Segments {
  int n;
  int lo[kMaxLayers];
  int hi[kMaxLayers];
};

// Constants of the QGGMRF prior update (Eqs. (15)-(17)) and the noise level.
struct PriorConst {
  float inv_sigma2;
  float p;
  float T;
  float T_pm2;  // T^(p - 2)
  float sigma0;
  double m, a;
  double z0, dz;
};

// Planar layer stack passed to kernels by value.  top/bottom are depths of
// each layer's faces; the last bottom is +inf.
struct Layers {
  int n;
  double speed[kMaxLayers];
  double atten[kMaxLayers];  // alpha_l [s/m]
  double top[kMaxLayers];
  double bottom[kMaxLayers];
};

// Records `msg` as the calling thread's last error and returns `status`.
int fail(int status, const std::string& msg);

// Returns UMBIR_EDEVICE (with the HIP error text) if `e` is not hipSuccess.
int check_hip(hipError_t e, const char* what);

// Optional per-kernel timing (umbir_profile_enable): when on, every launch is
// bracketed by two events on its stream; umbir_profile_collect sums them.
bool prof_on(const char* name);  // profiling on and `name` selected
hipEvent_t prof_start(hipStream_t s);
void prof_stop(const char* name, hipStream_t s, hipEvent_t start);

#define UMBIR_LAUNCH(name, kernel, grid, block, shmem, stream, ...)          \
  do {                                                                       \
    hipEvent_t umbir_e0_ = umbir::prof_on(name) ? umbir::prof_start(stream) : nullptr; \
    hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);     \
    if (umbir_e0_) umbir::prof_stop(name, stream, umbir_e0_);                \
  } while (0)

// Workspace carved out of one device buffer; offsets are 256-byte aligned.
struct Carve {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

// Block-wide copy into LDS: store(i, load(i)) for i < n, with eight loads in
// flight per thread.  The stores are branch-free (a slot past the end repeats
// element n - 1, with its own value), so the compiler keeps every load of a
// batch ahead of its stores instead of waiting on each in turn.
template <typename T, typename Load, typename StoreF>
__device__ __forceinline__ void stage_block(int n, Load load, StoreF store) {
  constexpr int U = 8;
  for (int i0 = threadIdx.x; i0 < n; i0 += U * int(blockDim.x)) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = load(min(i0 + u * int(blockDim.x), n - 1));
#pragma unroll
    for (int u = 0; u < U; ++u) store(min(i0 + u * int(blockDim.x), n - 1), v[u]);
  }
}

// Owns a workspace: the caller's buffer, or one allocated in stream order.
struct Workspace {
  void* ptr = nullptr;
  bool owned = false;
  hipStream_t stream = nullptr;
  int acquire(void* user, size_t user_bytes, size_t need, hipStream_t s);
  ~Workspace();
};

}  // namespace umbir

struct umbir_geometry {
  int device = -1;
  // problem, as validated
  umbir::Layers layers{};
  double density[umbir::kMaxLayers] = {};
  int nx = 0, nz = 0;
  double dx = 0, dz = 0, x0 = 0, z0 = 0;
  int P = 0, K = 0, beta = 0;
  std::vector<double> tx_x, rx_off;
  int M = 0, Q = 0, Lh = 0;
  double fs = 0, f_c = 0, sigma_t = 0, t_win = 0;
  // derived
  int storage = UMBIR_STORAGE_F32;  // element type of traces, fine grid and taps in the sweeps
  int n_off = 0;        // lattice positions per leg-table row
  int trace_groups = 1; // traces are split into this many groups in voxel-parallel kernels
  // rows of each layer: [seg_lo[s], seg_hi[s]) for the n_seg layers the grid reaches;
  // within one segment a voxel's delay grows strictly with its row
  int n_seg = 0;
  int seg_lo[umbir::kMaxLayers] = {}, seg_hi[umbir::kMaxLayers] = {};
  // fine-grid sweep of the splat: each trace is cut into `chunks` ranges of
  // chunk_bins fine positions, swept in LDS tiles of tile_bins
  int chunks = 1;
  long chunk_bins = 0;
  int tile_bins = 0;
  // tunable launch shapes (umbir_tuning)
  int splat_blocks = 512;      // target splat workgroups; sets chunks, chunk_bins, tile_bins
  int gather_batch_kb = 4096;  // fine-grid KiB per trace group per gather launch
  int conv_grid = 1;           // matrix-core convolution grid: 1 trace tiles fastest, 2 sample tiles fastest
  int conv_tiles = 2;          // 32-sample output tiles per matrix-core convolution workgroup (1, 2 or 4; by size)
  int corr_tiles = 4;          // 32-row tiles per wave of the matrix-core correlation (1, 2 or 4)
  int corr_blocks = 1024;      // target workgroups of the correlation (sets row blocks per workgroup)
  int form = 1;                // operator form: 1 factored (splat + convolution), 2 direct (Eq. (13) tap by tap)
  int split = 1;               // FP32 matrix-core products: 1 as three bf16 pieces each, 0 as FP32 products
  // attenuation: n_gamma templates at gamma_g = g * gamma_step (1 without)
  int n_gamma = 1;
  double gamma_step = 0.0;
  unsigned long long* gmask = nullptr;  // [P*K][mask_blocks] template occupancy (n_gamma > 1)
  double* gunit = nullptr;  // [nz][n_off] leg path attenuation / gamma_step, laid out as legs (n_gamma > 1)
  double* gunit_t = nullptr;  // [n_off][nzp] the same, laid out as legs_t (n_gamma > 1)
  int mask_blocks = 0;
  // resident device tables
  umbir::Leg* legs = nullptr;  // [nz][n_off] one-way legs (delay Q32.32, cos^beta), parity-split rows
  // the same legs by lattice position, the rows of one position contiguous
  // ([n_off][nzp], rows nz .. nzp - 1 zero), delays times Q (Q32.32 in fine
  // positions): the splat's table, where one wave step reads 8 consecutive
  // rows of a position as one aligned 128-byte line
  umbir::Leg* legs_t = nullptr;
  int nzp = 0;  // rows per position of legs_t and per column of tau x: padded_rows(nz)
  float* tau = nullptr;      // [nz] transmittance product of the row's layer
  int* base = nullptr;       // [P + P*K] lattice base: offset index = |base + 2 col|
  float* bank = nullptr;     // [n_gamma][Q*Lh + 2] tabulated windowed responses, zero padded
  float* h = nullptr;        // [n_gamma][Lh][Q] polyphase taps h_t[k] = bank[(k+1)Q - t]
  float* habs = nullptr;     // [n_gamma][Lh][Q] |h|
  float* dbasis = nullptr;   // [P*K][M] direct-arrival columns of D
  float* dnorm = nullptr;    // [P*K] squared norms of the columns of D
  int2* gwin = nullptr;      // [gather tiles][P*K] windowed gather's {first fine position, count} (or absent)
  int gather_form = 1;       // 1 row-wise gather, 2 windowed (needs gwin)
  size_t bytes = 0;

  int traces() const { return P * K; }
  int voxels() const { return nx * nz; }
  size_t fine_per_trace() const { return size_t(M) * Q; }
  size_t elem() const { return storage == UMBIR_STORAGE_F32 ? 4 : 2; }
  // fine-grid workspace: P K M Q elements, then the splat's prescaled image
  // (nx nzp floats, by column: xt[col * nzp + row]), then the prescale
  // blocks' maxima
  size_t fine_grid_bytes() const { return (size_t(traces()) * fine_per_trace() * elem() + 15) & ~size_t(15); }
  // with attenuation every template's grid is kept resident when one trace's
  // grids fit 32-bit offsets (the forward writes them [template][trace]
  // [position], the adjoint [trace][template][position])
  bool multi_grid() const {
    return n_gamma > 1 && storage == UMBIR_STORAGE_F32 &&
           size_t(n_gamma) * fine_per_trace() * elem() < (size_t(1) << 31);
  }
  // the fine grid(s): one, or with multi_grid() one per template
  size_t grids_bytes() const {
    return multi_grid() ? (size_t(traces()) * n_gamma * fine_per_trace() * elem() + 15) & ~size_t(15)
                        : fine_grid_bytes();
  }
  // the fine-grid workspace: the grid(s), then the forward's prescaled image
  // and the prescale blocks' maxima
  size_t fine_bytes() const {
    return grids_bytes() + ((size_t(nx) * nzp * 4 + 15) & ~size_t(15)) + 4 * umbir::kPrescaleBlocks;
  }
  size_t trace_bytes() const { return size_t(traces()) * M * elem(); }
  size_t taps_per_bin() const { return size_t(Q) * Lh; }
};

namespace umbir {

void apply_splat_blocks(umbir_geometry* G, long target);

// Kernel launchers shared between translation units.  All return a status.
int launch_fill(float* p, size_t n, float v, hipStream_t s);
int launch_copy(float* dst, const float* src, size_t n, hipStream_t s);

// The MAP cost of Eq. (18) of the previous iteration, computed inside the
// next forward's first kernel instead of a launch of its own: out = inv_2s2
// sum(ess[0 .. n_ess)) + sum(pcost[0 .. n_p)), summed in the same order as
// the solver's cost kernel (256 strided partial sums, then a halving tree),
// so both give bitwise the same value.
struct CostFold {
  const double* ess;
  int n_ess;
  const double* pcost;
  int n_p;
  double inv_2s2;
  double* out;
};

// y = base + sign * A x - g D   (base, g may be NULL; x NULL means all ones).
// `abs_op` builds the operator from |W| and |h|.  Trace buffers (out, base) hold
// the geometry's storage type; fine: G.fine_bytes() of workspace.  With
// pre_max the workspace already holds tau x for this x (as
// run_prescale_blocks or the prior update leaves it), whose largest |tau x|
// is the largest of the n_pre_max words at pre_max, and x is not read.  With
// fold, its cost is also computed (before any of the forward's writes).
int run_forward(const umbir_geometry& G, const float* x, void* out, const void* base,
                float sign, const float* g, bool abs_op, void* fine, hipStream_t s,
                const unsigned* pre_max = nullptr, int n_pre_max = 0, const CostFold* fold = nullptr);

// Can the direct form serve this geometry (FP32 storage, one template, the
// forward's sample accumulators and template within 64 KiB of LDS)?
bool direct_eligible(const umbir_geometry& G);

// tau x into the forward's workspace `fine` and, per block of 64 voxels, the
// largest |tau x| into maxima[blocks] (blocks * 64 >= the voxel count).
int run_prescale_blocks(const umbir_geometry& G, const float* x, void* fine, unsigned* maxima, int blocks,
                        hipStream_t s);

// out = scale * A^T r (r in the storage type).  partial: trace_groups * N floats.
int run_adjoint(const umbir_geometry& G, const void* r, float* out, float scale, bool abs_op,
                void* fine, float* partial, hipStream_t s);

// A^T r left as the trace_groups partial images (partial[g][v]); their sum in
// the order g = 0, 1, ... is run_adjoint's result with scale 1.
int run_adjoint_partial(const umbir_geometry& G, const void* r, bool abs_op, void* fine, float* partial,
                        hipStream_t s);

// y = D g (or y += D g), y in the storage type.
int launch_direct(const umbir_geometry& G, const float* g, void* y, int accumulate, hipStream_t s);

int log2_int(int q);  // smallest k with 2^k >= q

// Voxels per block of the prior update (four lanes per voxel): the number of
// per-block prior-cost partials is ceil(N / kPriorVox).
constexpr int kPriorVox = 64;

size_t forward_work_bytes(const umbir_geometry& G);
size_t adjoint_work_bytes(const umbir_geometry& G);

// ---- work-list batches: one launch per stage of a surrogate iteration for
// many problems at once, each block walking a work list of items
// (problem, block index x, block index y of that problem's own launch).

// One problem of a work-list batch (FP32 storage, one template, Q = 32 or
// 64): what every stage of its iteration reads, set from its geometry and
// its session's buffers.
struct BatchProb {
  // geometry
  const Leg* legs;
  const Leg* legs_t;  // [n_off][nzp]
  const int* base;
  const float* tau;
  const float* h;       // polyphase taps [Lh][Q]
  const float* dbasis;  // [P K][M]
  const float* dnorm;   // [P K]
  int nx, nz, nzp, n_off, P, K, M, Q, qs, Lh, MQ;
  Segments seg;
  // launch shapes of the sweeps
  int chunk_bins, tile_bins, wide;  // splat
  int conv_tiles;                   // output tiles per convolution block
  int conv_split, corr_split;       // products of the dense sweeps as bf16 pieces (umbir_geometry::split)
  int conv_waves;                   // waves sharing a convolution block's window
  int corr_per;                     // row blocks per correlation block
  int groups, tpg, gbatch, vpb;     // gather: trace groups, traces per group and launch, voxels per block
                                    // (row-wise) or voxel tiles per block (windowed)
  const int2* gwin;                 // windowed gather: the geometry's window table
  int nblk;                         // prior-update blocks
  // session state
  const float* y;
  float* e;
  float* fine;
  float* xt;  // tau x of the current image by column ([nx][nzp], the splat's input), kept by the prior update
  float* partial;
  float* den;
  double* ess;
  double* pcost;
  unsigned* pmax;  // per prior-update block (nblk) the largest |tau x| of its voxels
  float* x[2];  // the image before the batch's step 0, and the other buffer
  float* g;
  double* cost;
  int* counter;
  PriorConst pc;
  double inv_2s2;
  int est;
};

// Stages of one iteration, in launch order.
enum BatchStage { kStPrescale = 0, kStSplat, kStConv, kStGstep, kStCorr, kStGather, kStGatherW, kStPrior, kStCost, kStages };

// A stage's launch: its items, grid (blocks walk the items with a stride of
// the grid) and dynamic LDS bytes.
struct StageLaunch {
  const int4* items = nullptr;
  int n_items = 0;
  int grid = 0;
  size_t lds = 0;
};

// Fills the sweep fields of bp from G (the launch shapes of the plain path)
// and appends problem pi's items of the sweep stages (splat, conv, corr,
// gather) to items[stage]; lds[stage] grows to what the problem needs.
// Gather items carry the index of their launch (batch of traces) in .w.
void plan_sweeps(const umbir_geometry& G, int pi, BatchProb& bp, std::vector<int4>* items, size_t* lds);

// Launches one sweep stage (splat, conv, corr, gather) over the batch; items
// of problem i run only while active[i] is nonzero.
int launch_sweep_stage(int stage, int Q, const BatchProb* probs, const int* active, const StageLaunch& L, int which,
                       hipStream_t s);

}  // namespace umbir
