// The system matrix A of Eq. (13) and its transpose, matrix-free.
//
// Entry (trace ij, sample m; voxel v) of A is W_ij(v) * I((m - D) Q), where
// D = fs T_ij(v) is the voxel's delay in samples, W = tau(v) phi^(beta)(v), and
// I linearly interpolates the tabulated windowed pulse b[n] = h~(n / (Q fs))
// (Eq. (10)), which is zero at both ends of its window.  Writing
// D Q = J + phi (J integer, 0 <= phi < 1), the interpolation weights fall on
// the two fine-grid positions J and J + 1:
//     I((m - D) Q) = (1 - phi) b[mQ - J] + phi b[mQ - J - 1].
// So A = C o S, exactly:
//   S (splat): each voxel deposits W x (1 - phi) at fine position J and
//      W x phi at J + 1 of its trace's fine-grid signal s[J], J < M Q;
//   C (polyphase convolution): y[m] = sum_J s[J] b[mQ - J]
//      = sum_{t<Q} sum_{k<L_h} s[(m-1-k) Q + t] h_t[k],  h_t[k] = b[(k+1) Q - t].
// The transpose is A^T = S^T o C^T:
//   C^T (polyphase correlation): c[nQ + t] = sum_{k<L_h} r[n+1+k] h_t[k];
//   S^T (gather): (A^T r)(v) = sum_ij W ((1 - phi) c[J] + phi c[J+1]).
// C and C^T are dense, register-blocked and coalesced; S and S^T touch two
// fine-grid positions per (trace, voxel) pair.  Delays are Q32.32 fixed point
// (sum of two one-way legs, added exactly as integers), so J and phi are exact.

#include <algorithm>
#include <vector>
#include <cmath>

#include "internal.h"
#include "storage.h"

namespace umbir {
namespace {

constexpr int kR = 16;  // outputs per lane in the dense kernels (register block)

__global__ void k_fill(float* __restrict__ p, size_t n, float v) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  float4* p4 = reinterpret_cast<float4*>(p);
  const size_t n4 = n / 4;
  const float4 v4 = make_float4(v, v, v, v);
  for (size_t k = i; k < n4; k += stride) p4[k] = v4;
  for (size_t k = n4 * 4 + i; k < n; k += stride) p[k] = v;
}

__global__ void k_copy(float* __restrict__ d, const float* __restrict__ s, size_t n) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += stride) d[k] = s[k];
}

constexpr float kTwoM32 = 2.3283064365386963e-10f;  // 2^-32

// The splat's input image with the row transmittance folded in, xt = tau x
// (x == NULL means x = 1), stored by column (xt[col * nzp + row]), and per
// block the largest |xt| as float bits (non-negative floats order like their
// bits) for the fixed-point scale of the splat: out[blockIdx.x], gridDim.x <=
// kPrescaleBlocks.
__device__ __forceinline__ void prescale_body(int bx, int gx, const float* __restrict__ x,
                                              const float* __restrict__ tau, int nx, int nzp, int n,
                                              float* __restrict__ xt, unsigned* __restrict__ out) {
  unsigned m = 0;
  for (int i = bx * blockDim.x + threadIdx.x; i < n; i += gx * blockDim.x) {
    const int row = i / nx;
    const float v = tau[row] * (x ? x[i] : 1.0f);
    xt[size_t(i - row * nx) * nzp + row] = v;
    m = max(m, __float_as_uint(fabsf(v)));
  }
  for (int off = 32; off >= 1; off >>= 1) m = max(m, unsigned(__shfl_xor(int(m), off)));
  __shared__ unsigned wmax[16];
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < int(blockDim.x >> 6); ++w) m = max(m, wmax[w]);
    out[bx] = m;
  }
}

__global__ void k_prescale(const float* __restrict__ x, const float* __restrict__ tau, int nx, int nzp, int n,
                           float* __restrict__ xt, unsigned* __restrict__ out) {
  prescale_body(blockIdx.x, gridDim.x, x, tau, nx, nzp, n, xt, out);
}

// Fixed-point exponent of the splat: contributions are scaled by 2^k with
// 2^k * max|xt| * N <= 2^62, so no tile position can overflow int64 even if
// every voxel of the trace landed on it (the two apodisations and the two
// interpolation weights of a voxel are at most 1).  Power-of-two scaling is
// exact in both directions.
__device__ __forceinline__ int splat_exponent(unsigned maxbits, int n_vox) {
  int e = 0;
  (void)frexpf(__uint_as_float(maxbits), &e);  // max|xt| < 2^e
  int lg = 0;
  while ((1 << lg) < n_vox) ++lg;
  return 62 - lg - e;
}

// One contribution v * scale as a 64-bit integer.  For N > 1024 voxels
// |v * scale| < 2^51 and the sum with 1.5 * 2^52 in double precision, which
// has unit spacing there, leaves the value rounded to the nearest integer in
// its low mantissa bits in two's complement (the constant's low word is zero,
// so the subtraction touches only the high word): three instructions.  Small
// problems (WIDE) use the general conversion, truncating toward zero.
template <bool WIDE>
__device__ __forceinline__ unsigned long long to_fixed(float v, double scale) {
  if (WIDE) return (unsigned long long)(long long)(double(v) * scale);
  const double d = fma(double(v), scale, 6755399441055744.0);
  return (unsigned long long)(__double_as_longlong(d) - 0x4338000000000000ll);
}
constexpr int kSplatNarrowMin = 1025;  // voxels from which to_fixed<false> is exact

// A tile sum v (64-bit two's complement) times 2^-k as FP32, with s_hi =
// 2^(32 - k) and s_lo = 2^-k: the two 32-bit halves are exact in FP64 and so
// are their scaled values, the FMA adds them with one rounding (none for
// |v| < 2^53), and the conversion to FP32 rounds once more, so the result is
// v 2^-k rounded to nearest whenever |v| < 2^53.  Five instructions, against
// about a dozen for an integer-to-float conversion of 64 bits.
__device__ __forceinline__ float fixed_to_float(unsigned long long v, double s_hi, double s_lo) {
  const double hi = double(int(uint32_t(v >> 32)));
  const double lo = double(uint32_t(v));
  return float(fma(hi, s_hi, lo * s_lo));
}

// A tile sum as a stored element.  For FP16 the FP32 value is pinned in a
// register first: the compiler would otherwise merge the two conversions into
// one emulated FP64 -> FP16 conversion of some twenty instructions.
template <int ST>
__device__ __forceinline__ typename Store<ST>::T fixed_to_store(unsigned long long v, double s_hi, double s_lo) {
  float f = fixed_to_float(v, s_hi, s_lo);
  if constexpr (ST == UMBIR_STORAGE_F16) asm("" : "+v"(f));
  return Store<ST>::put(f);
}

// Two neighbouring elements of a storage type, for one paired store.
template <typename T>
struct alignas(2 * sizeof(T)) Pair2 {
  T a, b;
};

constexpr int kSplatWaves = 16;  // waves per splat workgroup (one workgroup per CU)
constexpr int kNoRow = 0x7fffffff;
// Word 3 of a raw buffer resource on CDNA: 32-bit data format, no swizzle.
constexpr int kBufferWord3 = 0x00020000;

// S: the fine-grid signal of one trace, one chunk of fine positions per
// workgroup, built in LDS tiles without global atomics.  Within a layer a
// voxel's delay grows strictly with depth, so for each (column, layer) the
// voxels reach the fine grid in row order: one pointer per (column, layer)
// moves forward through the rows as the tiles advance, and every voxel is
// visited once.  Beside the pointer the block keeps the fine position of the
// row it points at, so a (column, layer) with nothing in the current tile
// costs no load, and per layer the range of positions its voxels reach, so a
// layer outside the tile is skipped whole.  A wave takes 8 neighbouring
// columns x 8 consecutive rows per step (the 8 columns of a row read
// neighbouring leg records) and loads the next step's rows while the current
// one is added: a column continues only after all 8 of its rows fell in the
// tile, so the next rows are known in advance.  The rows of a column that fall
// in the tile are a prefix of the 8, counted with a ballot.  A voxel at
// position J adds W x (1 - phi) to J and W x phi to J + 1; the tile keeps one
// extra slot for J + 1 = the next tile's first position.  The tile
// accumulates in 64-bit fixed point (integer LDS atomics: the sum does not
// depend on the order of the adds, so the result is bitwise reproducible),
// scaled by 2^k from splat_exponent.  Tiles are written out whole
// (coalesced), so the fine buffer needs no clearing.
// First row of a layer segment [lo, hi) whose fine position pos(r) is
// >= target, given jl = pos(lo) and jh = pos(hi - 1); *jfirst receives its
// position (kNoRow if none).  pos is nondecreasing in r and close to linear,
// so each round probes the interpolated row and its successor together (two
// loads in flight); every other round bisects instead, which bounds the
// rounds by twice those of a plain bisection.
// A template pass may skip fine-grid ranges that no voxel of its template
// reaches: mask NULL means no skipping.
struct BinSkip {
  const unsigned long long* mask;  // [traces][nb]
  int nb, gbin;
};

// The skipping of attenuation template gbin's pass (gbin < 0: none)
BinSkip bin_skip(const umbir_geometry& G, int gbin) {
  BinSkip bs;
  bs.mask = (G.n_gamma > 1 && gbin >= 0) ? G.gmask : nullptr;
  bs.nb = G.mask_blocks;
  bs.gbin = gbin < 0 ? 0 : gbin;
  return bs;
}

// Does template bs.gbin reach fine positions [lo, hi) of trace t?
__device__ __forceinline__ bool bin_reaches(const BinSkip& bs, int t, long lo, long hi) {
  if (!bs.mask) return true;
  lo = lo < 0 ? 0 : lo;
  const long b1 = min((hi - 1) >> kMaskShift, long(bs.nb) - 1);
  const unsigned long long* m = bs.mask + size_t(t) * bs.nb;
  for (long b = lo >> kMaskShift; b <= b1; ++b)
    if ((m[b] >> bs.gbin) & 1ull) return true;
  return false;
}

template <typename Pos>
__device__ __forceinline__ int first_row_at(Pos pos, int lo, int hi, int jl, int jh, int target, int* jfirst) {
  if (jl >= target) { *jfirst = jl; return lo; }
  if (jh < target) { *jfirst = kNoRow; return hi; }
  int a = lo, b = hi - 1, ja = jl, jb = jh;  // pos(a) < target <= pos(b)
  for (int round = 0; b - a > 1; ++round) {
    int m = (round & 1) ? ((a + b) >> 1)
                        : a + int((long long)(target - ja) * (b - a) / max(jb - ja, 1));
    m = min(max(m, a + 1), b - 1);
    const int jm = pos(m);
    const int jn = m + 1 < b ? pos(m + 1) : jb;
    if (jm >= target) { b = m; jb = jm; }
    else if (jn >= target) { a = m; ja = jm; b = m + 1; jb = jn; }
    else { a = m + 1; ja = jn; }
  }
  *jfirst = jb;
  return b;
}

// S: the fine-grid signal of one trace, one chunk of fine positions per
// workgroup, built in LDS tiles without global atomics.  Within a layer a
// voxel's delay grows strictly with depth, so for each (column, layer) the
// voxels reach the fine grid in row order: one pointer per (column, layer)
// moves forward through the rows as the tiles advance, and every voxel is
// visited once.  Beside the pointer the block keeps the fine position of the
// row it points at, so a (column, layer) with nothing in the current tile
// costs no load, and per layer the range of positions its voxels reach, so a
// layer outside the tile is skipped whole.  A wave takes 8 neighbouring
// columns x one aligned block of 8 rows per step (rows 8b .. 8b + 7; in the
// first block of a column the rows above its pointer are done already) and
// loads the next block into a second register set while the current one is
// added: a column continues only after all its rows of a block fell in the
// tile, so the next rows are known in advance.  The splat's tables hold the
// rows of one lattice position (legs_t, gunit_t) and of one column (tau x)
// contiguously, so a block of 8 rows is one aligned 128-byte line of leg
// records and 32 bytes of the image, read by 8 consecutive lanes: the L1
// (whose access rate bounds the splat) serves each load of a column's block
// as one access.  The rows of a column that fall
// in the tile are a prefix of its rows in the block, counted with a ballot.
// A voxel at position J adds W x (1 - phi) to J and W x phi to J + 1; the tile keeps one extra slot for J + 1 = the next tile's first
// position and one never-read slot that takes the J part of a voxel at J0 - 1
// (added in the previous tile).  The tile accumulates in 64-bit fixed point
// (integer LDS atomics: the sum does not depend on the order of the adds, so
// the result is bitwise reproducible), scaled by 2^k from splat_exponent.
// Tiles are written out whole (coalesced), so the fine buffer needs no
// clearing.  With ATT only the voxels whose attenuation bin (from the two
// legs' units) is `gbin` are added: one pass per template.  With MT (and ATT)
// the block keeps one tile per template (glast + 1 of them) and every voxel
// is added to its own template's tile: one pass serves all templates, whose
// grids are written [template][trace][position] (each template's grid as the
// convolution reads it).
template <bool ABSW, bool WIDE, int ST, bool ATT, bool MT>
__device__ __forceinline__ void splat_body(int bx, int by,
    const float* __restrict__ xt, int nx, int nzp, int n_off, const Leg* __restrict__ legs_t,
    const double* __restrict__ gunit_t,
    const int* __restrict__ base, int P, int K, int qs, int MQ, const Segments& seg, int chunk_bins, int tile_bins,
    const unsigned* __restrict__ xmax, int n_xmax,
    int gbin, int glast, BinSkip bs, typename Store<ST>::T* __restrict__ fine) {
  extern __shared__ __align__(16) unsigned long long smem[];
  const int NT = MT ? glast + 1 : 1;                                 // tiles
  // A tile's slots: 0 takes the part at J0 - 1 (never read), 1 + k position
  // J0 + k, n + 1 the carry (position J1, the next tile's first).  The tiles
  // start one word into the LDS, so that slots 1 + 2i are 16-byte aligned.
  const int TS = tile_bins + 2;
  unsigned long long* tile = smem + 1;                               // [NT][TS]
  int2* pn = reinterpret_cast<int2*>(smem + 1 + NT * TS);            // [seg.n][nx] {next row, its position}
  int2* colofs = pn + seg.n * nx;                                    // [nx] byte offsets of the columns' legs_t rows
  __shared__ int lay_lo[kMaxLayers], lay_hi[kMaxLayers];             // positions a layer reaches
  const int ij = by;
  const int J_begin = bx * chunk_bins;
  const int J_end = min(J_begin + chunk_bins, MQ);
  if (J_begin >= J_end) return;  // uniform over the block
  const int btx = base[ij / K];
  const int brx = base[P + ij];
  const int half = n_off / 2;
  // legs_t holds the delays times Q (Q32.32 in fine positions): the fine
  // position of a pair is the high word of the sum, its fraction the low word
  typename Store<ST>::T* out = fine + size_t(ij) * MQ;
  if (ATT && !MT && !bin_reaches(bs, ij, J_begin, J_end)) {  // uniform: no voxel of the template here
    for (int k = J_begin + threadIdx.x; k < J_end; k += blockDim.x) out[k] = Store<ST>::put(0.0f);
    return;
  }

  // Set-up in two phases: first the largest |tau x| over the prescale blocks'
  // maxima, the column offsets, and the positions of the first and last row
  // of each (column, layer), parked in its pointer slot (a thread's first
  // slot is loaded before the maxima, so that their loads are in flight
  // together); then the scale, the layer ranges and each (column, layer)'s
  // first row at or after J_begin - 1.
  __shared__ unsigned wave_max[kSplatWaves];
  auto col_ofs = [&](int c) {
    return make_int2(leg_slot(abs(btx + 2 * c), half) * nzp * int(sizeof(Leg)),
                     leg_slot(abs(brx + 2 * c), half) * nzp * int(sizeof(Leg)));
  };
  auto pos_at = [&](int2 co, int r) {
    return int(uint64_t(legs_t[co.x / int(sizeof(Leg)) + r].delay + legs_t[co.y / int(sizeof(Leg)) + r].delay) >> 32);
  };
  {
    auto ends = [&](int i) {  // segments are never empty
      const int sg = i / nx;
      const int2 co = col_ofs(i - sg * nx);
      return make_int2(pos_at(co, seg.lo[sg]), pos_at(co, seg.hi[sg] - 1));
    };
    const int n_slots = seg.n * nx;
    const int i0 = min(int(threadIdx.x), n_slots - 1);
    const int2 e0 = ends(i0);
    unsigned m = 0u;
    for (int i = threadIdx.x; i < n_xmax; i += blockDim.x) m = max(m, xmax[i]);
    if (int(threadIdx.x) < n_slots) pn[i0] = e0;
    for (int i = threadIdx.x + blockDim.x; i < n_slots; i += blockDim.x) pn[i] = ends(i);
    if (threadIdx.x < kMaxLayers) {
      lay_lo[threadIdx.x] = kNoRow;
      lay_hi[threadIdx.x] = -kNoRow;
    }
    for (int c = threadIdx.x; c < nx; c += blockDim.x) colofs[c] = col_ofs(c);
    {  // clear the tiles (and the alignment word), 16 bytes per store
      ulonglong2* t2 = reinterpret_cast<ulonglong2*>(smem);
      for (int k = threadIdx.x; k < (1 + NT * TS) / 2; k += blockDim.x) t2[k] = make_ulonglong2(0ull, 0ull);
      if (((1 + NT * TS) & 1) && threadIdx.x == 0) smem[NT * TS] = 0ull;
    }
    for (int off = 32; off >= 1; off >>= 1) m = max(m, unsigned(__shfl_xor(int(m), off)));
    if ((threadIdx.x & 63) == 0) wave_max[threadIdx.x >> 6] = m;
  }
  __syncthreads();
  unsigned maxbits = 0;
  for (int w = 0; w < int(blockDim.x >> 6); ++w) maxbits = max(maxbits, wave_max[w]);
  const int kx = splat_exponent(maxbits, nx * (seg.hi[seg.n - 1] - seg.lo[0]));
  const double scale = ldexp(1.0, kx);
  const double s_hi = ldexp(1.0, 32 - kx), s_lo = ldexp(1.0, -kx);  // back from fixed point
  // first row of each (column, layer) whose position is >= J_begin - 1 (the
  // same thread wrote the slot's two positions above).  The layer ranges are
  // reduced over the wave first when its 64 slots share a layer (atomics of a
  // whole wave on one LDS word run one lane at a time).
  for (int b0 = 0; b0 < seg.n * nx; b0 += blockDim.x) {
    const int i = b0 + threadIdx.x;
    const bool valid = i < seg.n * nx;
    const int iv = valid ? i : seg.n * nx - 1;  // past the end: the last slot's layer, neutral range
    const int sg = iv / nx, c = iv - sg * nx;
    const int2 jlh = valid ? pn[i] : make_int2(kNoRow, -kNoRow);
    if (__shfl(sg, 0) == __shfl(sg, 63)) {  // every lane is here (blockDim is a multiple of 64)
      int lo_v = jlh.x, hi_v = jlh.y;
      for (int off = 32; off >= 1; off >>= 1) {
        lo_v = min(lo_v, __shfl_xor(lo_v, off));
        hi_v = max(hi_v, __shfl_xor(hi_v, off));
      }
      if ((threadIdx.x & 63) == 0) {
        atomicMin(&lay_lo[sg], lo_v);
        atomicMax(&lay_hi[sg], hi_v);
      }
    } else if (valid) {
      atomicMin(&lay_lo[sg], jlh.x);
      atomicMax(&lay_hi[sg], jlh.y);
    }
    if (valid) {
      const int2 co = colofs[c];
      int jf;
      const int first = first_row_at([&](int r) { return pos_at(co, r); }, seg.lo[sg], seg.hi[sg], jlh.x, jlh.y,
                                     J_begin - 1, &jf);
      pn[i] = make_int2(first, jf);
    }
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // lanes 8 cc .. 8 cc + 7 take the 8 rows of column cc: consecutive lanes
  // read consecutive records of one line, which the L1 serves as one access
  const int cc = lane >> 3, rr = lane & 7;
  const unsigned long long colmask = 0xffull << (8 * cc);
  const int n_groups = (nx + 7) >> 3;
  // The step loads are raw buffer loads: unconditional (so the next step's
  // loads never wait behind a branch), with 32-bit byte offsets, and the
  // hardware range check returns zeros past the end of a table.  Rows outside
  // the layer (above the pointer or past the layer's end, into the next
  // position's rows) are read too but never used.
  const __amdgpu_buffer_rsrc_t leg_rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<Leg*>(legs_t), 0, n_off * nzp * int(sizeof(Leg)), kBufferWord3);
  const __amdgpu_buffer_rsrc_t xt_rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(xt), 0, nx * nzp * 4, kBufferWord3);
  // ATT: the legs' attenuation in template bins, 8 bytes per leg (byte
  // offset half that of the leg record)
  const __amdgpu_buffer_rsrc_t gu_rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<double*>(ATT ? gunit_t : reinterpret_cast<const double*>(legs_t)), 0, n_off * nzp * 8,
      kBufferWord3);
  constexpr unsigned lstep = 8u * unsigned(sizeof(Leg));  // bytes between a lane's steps: one block of rows
  constexpr unsigned xstep = 8u * 4u;
  struct Rows {
    int64_t da, db;
    float pa, pb, xv;
    double ua, ub;
  };
  for (int J0 = J_begin; J0 < J_end; J0 += tile_bins) {
    const int J1 = min(J0 + tile_bins, J_end);
    for (int sg = 0; sg < seg.n; ++sg) {
      if (lay_lo[sg] >= J1 || lay_hi[sg] < J0 - 1) continue;  // uniform: no voxel of the layer here
      const int hi = seg.hi[sg];
      for (int grp = wave; grp < n_groups; grp += kSplatWaves) {
        const int c = grp * 8 + cc;
        const int slot = sg * nx + c;
        const int2 pv = c < nx ? pn[slot] : make_int2(hi, kNoRow);
        bool live = pv.x < hi && pv.y < J1;
        if (!__any(live)) continue;
        const int cl = min(c, nx - 1);  // addresses of lanes past the last column stay in the tables
        const int2 co = colofs[cl];
        const int p0 = pv.x;                 // the column's first row not yet added
        int r = (p0 & ~7) + rr;              // this lane's row of the column's current block
        int k0 = p0 & 7;                     // rows of the block above the pointer (first block only)
        unsigned oa = unsigned(co.x) + unsigned(r) * unsigned(sizeof(Leg));
        unsigned ob = unsigned(co.y) + unsigned(r) * unsigned(sizeof(Leg));
        unsigned ox = (unsigned(cl) * unsigned(nzp) + unsigned(r)) * 4u;
        auto load = [&](Rows& v, unsigned k) {  // rows r + 8 k of this lane
          // delay and apodisation as a 64-bit and a 32-bit load (the compiler
          // merges them into one 12-byte load)
          const int ka = int(oa + k * lstep), kb = int(ob + k * lstep);
          const auto a = __builtin_amdgcn_raw_buffer_load_b64(leg_rs, ka, 0, 0);
          const auto b = __builtin_amdgcn_raw_buffer_load_b64(leg_rs, kb, 0, 0);
          v.pa = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(leg_rs, ka + 8, 0, 0));
          v.pb = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(leg_rs, kb + 8, 0, 0));
          if constexpr (ATT) {  // the legs' attenuation in template bins
            v.ua = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(gu_rs, ka >> 1, 0, 0));
            v.ub = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(gu_rs, kb >> 1, 0, 0));
          }
          v.xv = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(xt_rs, int(ox + k * xstep), 0, 0));
          v.da = int64_t((uint64_t(a[1]) << 32) | a[0]);
          v.db = int64_t((uint64_t(b[1]) << 32) | b[0]);
        };
        // adds this lane's row r; false once no column of the wave continues.
        // The first lane of a column left out of the tile stores that row and
        // its position for the next tile.
        auto add = [&](const Rows& v) {
          const bool have = live && rr >= k0 && r < hi;  // rows above the pointer: first block only
          const uint64_t D = uint64_t(v.da + v.db);
          const int J = int(D >> 32);
          const bool in = have && J < J1;
          // J + 1 >= J0 holds while delays grow with depth within a layer
          bool mine = true;
          int tb = 0;  // MT: the tile of the voxel's template
          if constexpr (ATT) {
            const int b = gamma_bin(v.ua + v.ub, glast);
            if constexpr (MT) tb = b * TS;
            else mine = b == gbin;
          }
          if (in && mine && v.xv != 0.0f && J + 1 >= J0) {
            float w = v.xv * (v.pa * v.pb);
            if (ABSW) w = fabsf(w);
            const float phi = float(uint32_t(D)) * kTwoM32;
            const float w1 = w * phi;
            unsigned long long* t = tile + tb + (J + 1 - J0);  // slot of position J (J = J0 - 1: slot 0)
            atomicAdd(t, to_fixed<WIDE>(w - w1, scale));
            atomicAdd(t + 1, to_fixed<WIDE>(w1, scale));
          }
          // rows of column c taken: a prefix of its rows in the block from k0
          const int nxt = k0 + __popcll(__ballot(in) & colmask);
          if (live && rr == nxt) pn[slot] = make_int2(r, have ? J : kNoRow);
          live = live && nxt == 8;
          k0 = 0;
          r += 8;
          oa += lstep;
          ob += lstep;
          ox += xstep;
          return __any(live);
        };
        Rows s0, s1;
        load(s0, 0);
        while (true) {
          load(s1, 1);
          if (!add(s0)) break;
          load(s0, 1);
          if (!add(s1)) break;
        }
      }
    }
    __syncthreads();
    // flush: write the tile out and clear it in one pass; the carry slot n is
    // outside the pass and becomes the next tile's first position
    const int n = J1 - J0;
    if constexpr (MT) {
      const unsigned long long carry = threadIdx.x < NT ? tile[threadIdx.x * TS + n + 1] : 0ull;
      for (int i = threadIdx.x; i < NT * n; i += blockDim.x) {
        const int g = i / n, k = i - g * n;
        out[size_t(g) * P * K * MQ + J0 + k] = fixed_to_store<ST>(tile[g * TS + 1 + k], s_hi, s_lo);
        tile[g * TS + 1 + k] = 0ull;
      }
      __syncthreads();
      if (threadIdx.x < NT) {
        tile[threadIdx.x * TS + 1] = carry;
        tile[threadIdx.x * TS + n + 1] = 0ull;
      }
    } else {
      const unsigned long long carry = tile[n + 1];
      typename Store<ST>::T* o = out + J0;
      if ((reinterpret_cast<uintptr_t>(o) & (2 * sizeof(*o) - 1)) == 0) {  // uniform
        // two positions per thread: one 16-byte LDS read and clear, one paired
        // store; an odd last position by the last thread
        for (int i = threadIdx.x; i < n / 2; i += blockDim.x) {
          ulonglong2* tp = reinterpret_cast<ulonglong2*>(tile + 1) + i;
          const ulonglong2 v = *tp;
          *tp = make_ulonglong2(0ull, 0ull);
          *reinterpret_cast<Pair2<typename Store<ST>::T>*>(o + 2 * i) = {fixed_to_store<ST>(v.x, s_hi, s_lo),
                                                                         fixed_to_store<ST>(v.y, s_hi, s_lo)};
        }
        if ((n & 1) && threadIdx.x == blockDim.x - 1) {
          o[n - 1] = fixed_to_store<ST>(tile[n], s_hi, s_lo);
          tile[n] = 0ull;
        }
      } else {
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
          o[k] = fixed_to_store<ST>(tile[1 + k], s_hi, s_lo);
          tile[1 + k] = 0ull;
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        tile[1] = carry;
        tile[n + 1] = 0ull;
      }
    }
    __syncthreads();
  }
}

// CostFold's sums by the first 256 threads of a block of at least 256; sh:
// 256 doubles of LDS, free before and after.
__device__ void fold_cost(const CostFold& f, double* sh) {
  const int t = threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (t < 256) {
    for (int i = t; i < f.n_ess; i += 256) v[0] += f.ess[i];
    for (int i = t; i < f.n_p; i += 256) v[1] += f.pcost[i];
  }
  double r[2];
  for (int k = 0; k < 2; ++k) {
    if (t < 256) sh[t] = v[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) sh[t] += sh[t + w];
      __syncthreads();
    }
    r[k] = sh[0];
    __syncthreads();
  }
  if (t == 0) *f.out = r[0] * f.inv_2s2 + r[1];
}

__global__ __launch_bounds__(256) void k_fold_cost(CostFold f) {
  __shared__ double sh[256];
  fold_cost(f, sh);
}

template <bool ABSW, bool WIDE, int ST, bool ATT, bool MT>
__global__ __launch_bounds__(64 * kSplatWaves) void k_splat(
    const float* __restrict__ xt, int nx, int nzp, int n_off, const Leg* __restrict__ legs_t,
    const double* __restrict__ gunit_t,
    const int* __restrict__ base, int P, int K, int qs, int MQ, Segments seg, int chunk_bins, int tile_bins,
    const unsigned* __restrict__ xmax, int n_xmax,
    int gbin, int glast, BinSkip bs, typename Store<ST>::T* __restrict__ fine, CostFold fold) {
  if (fold.out && blockIdx.x == 0 && blockIdx.y == 0) {  // uniform: the block's LDS is free until the walk
    extern __shared__ __align__(16) unsigned long long smem[];
    fold_cost(fold, reinterpret_cast<double*>(smem));
  }
  splat_body<ABSW, WIDE, ST, ATT, MT>(blockIdx.x, blockIdx.y, xt, nx, nzp, n_off, legs_t, gunit_t, base, P, K, qs,
                                      MQ, seg, chunk_bins, tile_bins, xmax, n_xmax, gbin, glast, bs, fine);
}

// ---- the direct (unfactored) form of Eq. (13), an alternative for small
// problems: every (trace, voxel) pair sums its own window of L_h taps, as the
// equation is written, instead of the splat + polyphase convolution.  With
// z = (m - D) Q = n - phi, n = m Q - J, the tap is
//     I = (1 - phi) b[n] + phi b[n - 1],   1 <= n <= Q L_h
// (b is zero at both ends of its window), the same interpolation as the
// factored form, only summed in another order.

// Bytes of LDS the direct forward needs (64-bit sample accumulators and the
// template); the direct form is offered when this fits 64 KiB.
size_t direct_fwd_lds(const umbir_geometry& G) {
  return size_t(G.M) * sizeof(unsigned long long) + (size_t(G.Q) * G.Lh + 2) * sizeof(float);
}

// A = direct: one block per trace; the trace's M samples accumulate in LDS in
// 64-bit fixed point (scale 2^k from max|tau x| as the splat's, so the sum is
// exact and independent of the order of the adds), then
//   out[m] = (base ? base[m] : 0) + sign * y[m] - (g ? g[ij] d_ij[m] : 0).
template <bool ABSW, bool WIDE>
__global__ __launch_bounds__(1024) void k_fwd_direct(
    const float* __restrict__ xt, int nx, int rows, int nzp, int n_off, const Leg* __restrict__ legs,
    const int* __restrict__ base_off, int P, int K, int qs, int Lh, int M, const float* __restrict__ bank,
    const unsigned* __restrict__ xmax, int n_xmax, const float* ybase, float sign, const float* __restrict__ g,
    const float* __restrict__ dbasis, float* out) {
  extern __shared__ unsigned long long dsm[];
  unsigned long long* acc = dsm;                           // [M]
  float* b = reinterpret_cast<float*>(dsm + M);            // [Q Lh + 2]
  const int Q = 1 << qs;
  const int QLh = Q * Lh;
  const int ij = blockIdx.x;
  const int btx = base_off[ij / K], brx = base_off[P + ij];
  const int half = n_off / 2;
  const int N = nx * rows;
  __shared__ unsigned wave_max[16];
  {
    unsigned m = 0;
    for (int i = threadIdx.x; i < n_xmax; i += blockDim.x) m = max(m, xmax[i]);
    for (int off = 32; off >= 1; off >>= 1) m = max(m, unsigned(__shfl_xor(int(m), off)));
    if ((threadIdx.x & 63) == 0) wave_max[threadIdx.x >> 6] = m;
  }
  for (int i = threadIdx.x; i < M; i += blockDim.x) acc[i] = 0ull;
  for (int i = threadIdx.x; i < QLh + 2; i += blockDim.x) b[i] = ABSW ? fabsf(bank[i]) : bank[i];
  __syncthreads();
  unsigned maxbits = 0;
  for (int w = 0; w < int(blockDim.x >> 6); ++w) maxbits = max(maxbits, wave_max[w]);
  const int kx = splat_exponent(maxbits, N);
  const double scale = ldexp(1.0, kx);
  for (int v = threadIdx.x; v < N; v += blockDim.x) {
    const int row = v / nx, col = v - row * nx;
    const float xv = xt[size_t(col) * nzp + row];  // tau x by column
    if (xv == 0.0f) continue;
    const Leg a = legs[size_t(row) * n_off + leg_slot(abs(btx + 2 * col), half)];
    const Leg c = legs[size_t(row) * n_off + leg_slot(abs(brx + 2 * col), half)];
    const uint64_t D = uint64_t(a.delay + c.delay);
    const long J = long(D >> (32 - qs));
    const float phi = float(uint32_t(D) << qs) * kTwoM32;
    float w = xv * (a.apod * c.apod);
    if (ABSW) w = fabsf(w);
    const long m_lo = max((J + Q) >> qs, 0L);                 // first m with n = m Q - J >= 1
    const long m_hi = min((J + QLh) >> qs, long(M) - 1);      // last m with n <= Q L_h
    for (long m = m_lo; m <= m_hi; ++m) {
      const int n = int(m * Q - J);
      const float tap = fmaf(phi, b[n - 1] - b[n], b[n]);
      atomicAdd(&acc[m], to_fixed<WIDE>(w * tap, scale));
    }
  }
  __syncthreads();
  const float gv = g ? g[ij] : 0.0f;
  for (int m = threadIdx.x; m < M; m += blockDim.x) {
    const size_t idx = size_t(ij) * M + m;
    float val = sign * ldexpf(float((long long)acc[m]), -kx);
    if (ybase) val += ybase[idx];
    if (g) val -= gv * dbasis[idx];
    out[idx] = val;
  }
}

// A^T = direct: per voxel, over the traces of group blockIdx.x, W times the
// window's sum of r[m] times the tap; one partial image per group (summed in
// a fixed order like the gather's).  The template sits in LDS.
template <bool ABSW, int VPT>
__global__ __launch_bounds__(256) void k_adj_direct(
    const float* __restrict__ rt, int nx, int nz, int n_off, const Leg* __restrict__ legs,
    const float* __restrict__ tau, const int* __restrict__ base_off, int P, int K, int qs, int Lh, int M,
    const float* __restrict__ bank, int tpg, int vox_per_block, float* __restrict__ partial) {
  extern __shared__ float bsm[];  // [Q Lh + 2]
  const int Q = 1 << qs;
  const int QLh = Q * Lh;
  for (int i = threadIdx.x; i < QLh + 2; i += blockDim.x) bsm[i] = ABSW ? fabsf(bank[i]) : bank[i];
  __syncthreads();
  const int N = nx * nz;
  const int PK = P * K;
  const int half = n_off / 2;
  const int v_begin = blockIdx.y * vox_per_block;
  const int v_end = min(N, v_begin + vox_per_block);
  const int t0 = blockIdx.x * tpg, t1 = min(t0 + tpg, PK);
  for (int vc = v_begin; vc < v_end; vc += blockDim.x * VPT) {
    float acc[VPT];
    int row[VPT], col2[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int v = min(vc + u * int(blockDim.x) + int(threadIdx.x), v_end - 1);
      row[u] = v / nx;
      col2[u] = 2 * (v - row[u] * nx);
      acc[u] = 0.0f;
    }
    for (int t = t0; t < t1; ++t) {
      const int btx = base_off[t / K], brx = base_off[P + t];
      const float* r = rt + size_t(t) * M;
#pragma unroll
      for (int u = 0; u < VPT; ++u) {
        const Leg a = legs[size_t(row[u]) * n_off + leg_slot(abs(btx + col2[u]), half)];
        const Leg c = legs[size_t(row[u]) * n_off + leg_slot(abs(brx + col2[u]), half)];
        const uint64_t D = uint64_t(a.delay + c.delay);
        const long J = long(D >> (32 - qs));
        const float phi = float(uint32_t(D) << qs) * kTwoM32;
        float w = a.apod * c.apod;
        if (ABSW) w = fabsf(w);
        const long m_lo = max((J + Q) >> qs, 0L);
        const long m_hi = min((J + QLh) >> qs, long(M) - 1);
        float s = 0.0f;
        for (long m = m_lo; m <= m_hi; ++m) {
          const int n = int(m * Q - J);
          s = fmaf(r[m], fmaf(phi, bsm[n - 1] - bsm[n], bsm[n]), s);
        }
        acc[u] = fmaf(w, s, acc[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int v = vc + u * int(blockDim.x) + int(threadIdx.x);
      if (v < v_end) {
        float tr = tau[v / nx];
        if (ABSW) tr = fabsf(tr);
        partial[size_t(blockIdx.x) * N + v] = acc[u] * tr;
      }
    }
  }
}

// One fine-grid sample through a buffer resource over one trace: positions
// past the record read as zero.
template <int ST>
__device__ __forceinline__ float fine_at(__amdgpu_buffer_rsrc_t rs, unsigned off);
template <>
__device__ __forceinline__ float fine_at<UMBIR_STORAGE_F32>(__amdgpu_buffer_rsrc_t rs, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, int(off * 4u), 0, 0));
}
template <>
__device__ __forceinline__ float fine_at<UMBIR_STORAGE_F16>(__amdgpu_buffer_rsrc_t rs, unsigned off) {
  return float(__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(rs, int(off * 2u), 0, 0)));
}
template <>
__device__ __forceinline__ float fine_at<UMBIR_STORAGE_BF16>(__amdgpu_buffer_rsrc_t rs, unsigned off) {
  return __uint_as_float(uint32_t(__builtin_amdgcn_raw_buffer_load_b16(rs, int(off * 2u), 0, 0)) << 16);
}

// S^T: per voxel, sum over the traces of group blockIdx.x of W ((1 - phi) c[J]
// + phi c[J + 1]); one partial image per group, summed in a fixed order (by
// k_reduce_groups, or by the prior update in an iteration).  The group is the
// fastest block index, so group g runs on XCD g mod 8 and that XCD's L2 only
// ever holds its own traces' fine-grid data.  One launch covers a batch of
// each group's traces (4 MiB of fine-grid data per group by default, read by
// every block of the XCD while the batch is
// warm in L2 and the last-level cache; blocks cannot be kept in step within a
// launch, but launch boundaries are barriers), and the partial images
// accumulate across launches in a fixed order.  The grid is one generation (at
// most four blocks per CU).  A thread accumulates VPT voxels (row-major, so neighbouring threads read
// neighbouring leg records).  The trace loop is a three-stage pipeline over
// two register sets in turn: while trace t accumulates, the fine-grid samples
// of trace t + 1 and the legs of trace t + 2 are in flight.  All loads are raw
// buffer loads (unconditional; a per-trace resource makes positions outside
// the record read as zero); traces past the batch are read at its last trace
// and weighted by zero.  With ATT only the pairs whose attenuation bin is
// `gbin` are weighted (one pass per template), and with `accum` the first
// launch adds to the partial image too.  ONE: every group's traces in this
// launch belong to one scan position, so the transmit legs are loaded once per
// voxel chunk and only the receive legs per trace.  MULTI (with ATT): the
// fine grids of all glast + 1 templates are resident, laid out
// [trace][template][position], and every pair reads the grid of its own
// template, so one pass serves all templates.
template <bool ABSW, int VPT, int ST, bool ATT, bool ONE, bool MULTI>
__device__ __forceinline__ void gather_body(int bx, int by, 
    const typename Store<ST>::T* __restrict__ fine, int nx, int nz, int n_off, const Leg* __restrict__ legs,
    const double* __restrict__ gunit, const float* __restrict__ tau, const int* __restrict__ base, int P, int K, int qs, int MQ,
    int tpg, int t_off, int t_cnt, int vox_per_block, int gbin, int glast, int accum,
    float* __restrict__ partial) {
  const int N = nx * nz;
  const int v_begin = by * vox_per_block;
  const int v_end = min(N, v_begin + vox_per_block);
  const int PK = P * K;
  // this launch covers traces [t_off, t_off + t_cnt) of each group; the first
  // launch writes the partial image, later ones add to it
  const int g_end = min((bx + 1) * tpg, PK);
  const int t0 = bx * tpg + t_off;
  const int t1 = min(t0 + t_cnt, g_end);
  if (t0 >= t1 && (t_off > 0 || accum)) return;  // uniform over the block: nothing to add
  const int sh = 32 - qs;
  const int half = n_off / 2;
  const __amdgpu_buffer_rsrc_t leg_rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<Leg*>(legs), 0, nz * n_off * int(sizeof(Leg)), kBufferWord3);
  // ATT: the legs' attenuation in template bins (byte offset half the record's)
  const __amdgpu_buffer_rsrc_t gu_rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<double*>(ATT ? gunit : reinterpret_cast<const double*>(legs)), 0, nz * n_off * 8, kBufferWord3);
  const int grid_elems = MULTI ? (glast + 1) * MQ : MQ;  // one trace's fine data
  const int fine_bytes = grid_elems * int(sizeof(typename Store<ST>::T));
  struct Legs { int64_t da[VPT], db[VPT]; float pa[VPT], pb[VPT]; double ua[VPT], ub[VPT]; };
  struct Taps { unsigned J[VPT], J1[VPT]; float phi[VPT], w[VPT]; };
  struct Samples { float c0[VPT], c1[VPT]; };
  for (int vc = v_begin; vc < v_end; vc += blockDim.x * VPT) {
    int col2[VPT], rowoff[VPT];
    bool ok[VPT];
    float acc[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int v = vc + u * blockDim.x + threadIdx.x;
      ok[u] = v < v_end;
      const int vv = ok[u] ? v : v_begin;
      const int row = vv / nx;
      col2[u] = 2 * (vv - row * nx);
      rowoff[u] = row * n_off;
      acc[u] = 0.0f;
    }
    // one leg record (delay, apodisation; with ATT the attenuation in
    // template bins) per voxel of the thread for the transducer with lattice
    // base bt
    auto load_leg = [&](int bt, int64_t (&d)[VPT], float (&p)[VPT], double (&ua)[VPT]) {
#pragma unroll
      for (int u = 0; u < VPT; ++u) {
        const int o = (rowoff[u] + leg_slot(abs(bt + col2[u]), half)) * int(sizeof(Leg));
        const auto a = __builtin_amdgcn_raw_buffer_load_b64(leg_rs, o, 0, 0);
        p[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(leg_rs, o + 8, 0, 0));
        if constexpr (ATT) ua[u] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(gu_rs, o >> 1, 0, 0));
        d[u] = int64_t((uint64_t(a[1]) << 32) | a[0]);
      }
    };
    Legs TX;  // ONE: the transmit legs of the launch's scan position
    if constexpr (ONE) load_leg(base[min(t0, t1 - 1) / K], TX.da, TX.pa, TX.ua);
    auto load_legs = [&](Legs& L, int t) {
      t = min(t, t1 - 1);
      if constexpr (!ONE) load_leg(base[t / K], L.da, L.pa, L.ua);
      load_leg(base[P + t], L.db, L.pb, L.ub);
    };
    auto taps_of = [&](const Legs& L, Taps& T, int t) {
      const float live = t < t1 ? 1.0f : 0.0f;  // steps past the batch add nothing
#pragma unroll
      for (int u = 0; u < VPT; ++u) {
        const int64_t da = ONE ? TX.da[u] : L.da[u];
        const uint64_t D = uint64_t(da + L.db[u]);
        // positions past the record (or past 2^31) clamp to MQ and read zero
        const unsigned J = unsigned(min(D >> sh, uint64_t(MQ)));
        if constexpr (MULTI) {  // the grid of the pair's template; past its record: past the trace's data
          const unsigned off = unsigned(gamma_bin((ONE ? TX.ua[u] : L.ua[u]) + L.ub[u], glast)) * unsigned(MQ);
          T.J[u] = J < unsigned(MQ) ? off + J : unsigned(grid_elems);
          T.J1[u] = J + 1u < unsigned(MQ) ? off + J + 1u : unsigned(grid_elems);
        } else {
          T.J[u] = J;
          T.J1[u] = J + 1u;
        }
        T.phi[u] = float(uint32_t(D) << qs) * kTwoM32;
        float w = (ONE ? TX.pa[u] : L.pa[u]) * L.pb[u];
        if (ABSW) w = fabsf(w);
        if constexpr (ATT && !MULTI) w = gamma_bin((ONE ? TX.ua[u] : L.ua[u]) + L.ub[u], glast) == gbin ? w : 0.0f;
        T.w[u] = w * live;
      }
    };
    auto load_samples = [&](const Taps& T, Samples& S, int t) {
      t = min(t, t1 - 1);
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<typename Store<ST>::T*>(fine + size_t(t) * grid_elems), 0, fine_bytes, kBufferWord3);
#pragma unroll
      for (int u = 0; u < VPT; ++u) {
        S.c0[u] = fine_at<ST>(rs, T.J[u]);
        S.c1[u] = fine_at<ST>(rs, T.J1[u]);
      }
    };
    auto add = [&](const Taps& T, const Samples& S) {
#pragma unroll
      for (int u = 0; u < VPT; ++u) acc[u] = fmaf(T.w[u], fmaf(T.phi[u], S.c1[u] - S.c0[u], S.c0[u]), acc[u]);
    };
    if (t0 < t1) {
      Legs L0, L1;
      Taps T0, T1;
      Samples S0, S1;
      load_legs(L0, t0);
      taps_of(L0, T0, t0);
      // issued in the loop's steady-state order (legs, then samples), so the
      // waits at the loop head stay partial
      load_legs(L1, t0 + 1);
      load_samples(T0, S0, t0);
      // the scheduling barriers keep each stage's loads ahead of the waits of
      // the stages after it
      for (int t = t0; t < t1; t += 2) {
        // trace t: T0 / S0 (in flight); trace t + 1: L1 (in flight)
        load_legs(L0, t + 2);
        __builtin_amdgcn_sched_barrier(0);
        taps_of(L1, T1, t + 1);
        load_samples(T1, S1, t + 1);
        __builtin_amdgcn_sched_barrier(0);
        add(T0, S0);
        __builtin_amdgcn_sched_barrier(0);
        // trace t + 1: T1 / S1 (in flight); trace t + 2: L0 (in flight)
        load_legs(L1, t + 3);
        __builtin_amdgcn_sched_barrier(0);
        taps_of(L0, T0, t + 2);
        load_samples(T0, S0, t + 2);
        __builtin_amdgcn_sched_barrier(0);
        add(T1, S1);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int v = vc + u * blockDim.x + threadIdx.x;
      if (ok[u]) {
        float tr = tau[v / nx];
        if (ABSW) tr = fabsf(tr);
        float* pv = partial + size_t(bx) * N + v;
        *pv = (t_off == 0 && !accum) ? acc[u] * tr : fmaf(acc[u], tr, *pv);
      }
    }
  }
}

template <bool ABSW, int VPT, int ST, bool ATT, bool ONE, bool MULTI>
__global__ __launch_bounds__(256) void k_gather(
    const typename Store<ST>::T* __restrict__ fine, int nx, int nz, int n_off, const Leg* __restrict__ legs,
    const double* __restrict__ gunit, const float* __restrict__ tau, const int* __restrict__ base, int P, int K, int qs, int MQ,
    int tpg, int t_off, int t_cnt, int vox_per_block, int gbin, int glast, int accum,
    float* __restrict__ partial) {
  gather_body<ABSW, VPT, ST, ATT, ONE, MULTI>(blockIdx.x, blockIdx.y, fine, nx, nz, n_off, legs, gunit, tau, base, P, K, qs, MQ, tpg, t_off, t_cnt, vox_per_block, gbin, glast, accum, partial);
}

// One position of the window in LDS, as the storage type's sample reads it
// (the value fine_at gives).
template <int ST>
__device__ __forceinline__ float win_at(const uint4* w, int i) {
  return Store<ST>::get(reinterpret_cast<const typename Store<ST>::T*>(w)[i]);
}

// S^T with the fine-grid window in LDS (one template; same pairs,
// same arithmetic and the same per-voxel order over the traces as k_gather,
// so the same results).  A trace's delays change by several 128-byte lines of
// the fine grid from one voxel to the next, so in k_gather nearly every lane's
// sample is a line of its own, fetched from L2 (0.65 fetches per (voxel,
// trace) pair at 256 x 256).  Here a block takes voxel tiles of 32 x 64 and
// for each trace first copies the tile's window of fine positions (from the
// table k_gather_windows builds: 0.2 lines per pair on average at 256 x 256)
// into LDS with coalesced 16-byte loads, then every voxel reads its two taps
// from LDS.  A trace whose window exceeds 64 KiB (16384 FP32 or 32768 16-bit
// positions; about one FP32 window in ten there: tiles near the array, where
// the delays spread most) reads its taps from global memory as k_gather
// does.  The window of trace t + 1 and the legs of trace t + 2 are in flight
// while trace t accumulates.  Wave w's load u covers row 8 u + w of the tile,
// one lane per column (neighbouring leg records).  ONE and the arguments as
// for k_gather.
template <bool ABSW, bool ONE, int ST = UMBIR_STORAGE_F32>
__device__ __forceinline__ void gather_lds_body(int bx, int by,
    const typename Store<ST>::T* __restrict__ fine, int nx, int nz, int n_off, const Leg* __restrict__ legs,
    const float* __restrict__ tau, const int* __restrict__ base, int P, int K, int qs, int MQ, int tpg, int t_off,
    int t_cnt, const int2* __restrict__ gwin, int tiles_per_block, float* __restrict__ partial) {
  using T16 = typename Store<ST>::T;
  extern __shared__ uint4 wlds[];  // the window: kGatherWinBytes
  constexpr int VPT = kGatherTileRows / 8;
  constexpr int ES = int(sizeof(T16));                // bytes per position
  constexpr int EPC = 16 / ES;                        // positions per 16-byte load
  constexpr int kWin = kGatherWinBytes / ES;          // window capacity in positions
  constexpr int kStage = kGatherWinBytes / 16 / 512;  // 16-byte loads per thread per window
  const int N = nx * nz;
  const int PK = P * K;
  const int g_end = min((bx + 1) * tpg, PK);
  const int t0 = bx * tpg + t_off;
  const int t1 = min(t0 + t_cnt, g_end);
  if (t0 >= t1 && t_off > 0) return;  // uniform over the block: nothing to add
  const int tiles_x = (nx + kGatherTileCols - 1) / kGatherTileCols;
  const int n_tiles = tiles_x * ((nz + kGatherTileRows - 1) / kGatherTileRows);
  const int tile_end = min(n_tiles, (by + 1) * tiles_per_block);
  const int sh = 32 - qs;
  const int half = n_off / 2;
  const int wave = int(threadIdx.x >> 6), lane = int(threadIdx.x & 63);
  const __amdgpu_buffer_rsrc_t leg_rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<Leg*>(legs), 0, nz * n_off * int(sizeof(Leg)), kBufferWord3);
  struct Legs { int64_t d[VPT]; float p[VPT]; };
  struct Taps { unsigned J[VPT]; float phi[VPT], w[VPT]; };
  for (int tile = by * tiles_per_block; tile < tile_end; ++tile) {
    const int tz = tile / tiles_x;
    const int tx = tile - tz * tiles_x;
    int col2[VPT], rowoff[VPT], vox[VPT];
    bool ok[VPT];
    float acc[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int row = tz * kGatherTileRows + 8 * u + wave;
      const int col = tx * kGatherTileCols + lane;
      ok[u] = row < nz && col < nx;
      const int r = min(row, nz - 1), c = min(col, nx - 1);  // outside the grid: a voxel of the grid, unused
      vox[u] = r * nx + c;
      col2[u] = 2 * c;
      rowoff[u] = r * n_off;
      acc[u] = 0.0f;
    }
    const int2* wt = gwin + size_t(tile) * PK;
    auto load_leg = [&](int bt, int64_t (&d)[VPT], float (&p)[VPT]) {
#pragma unroll
      for (int u = 0; u < VPT; ++u) {
        const int o = (rowoff[u] + leg_slot(abs(bt + col2[u]), half)) * int(sizeof(Leg));
        const auto a = __builtin_amdgcn_raw_buffer_load_b64(leg_rs, o, 0, 0);
        p[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(leg_rs, o + 8, 0, 0));
        d[u] = int64_t((uint64_t(a[1]) << 32) | a[0]);
      }
    };
    Legs TX;
    if constexpr (ONE) load_leg(base[min(t0, t1 - 1) / K], TX.d, TX.p);
    Legs TXt;  // !ONE: the transmit legs of the trace being loaded
    auto load_legs = [&](Legs& L, Legs& LT, int t) {
      t = min(t, t1 - 1);
      if constexpr (!ONE) load_leg(base[t / K], LT.d, LT.p);
      load_leg(base[P + t], L.d, L.p);
    };
    auto taps_of = [&](const Legs& L, const Legs& LT, Taps& T) {
#pragma unroll
      for (int u = 0; u < VPT; ++u) {
        const int64_t da = ONE ? TX.d[u] : LT.d[u];
        const uint64_t D = uint64_t(da + L.d[u]);
        T.J[u] = unsigned(min(D >> sh, uint64_t(MQ)));  // past the record: MQ
        T.phi[u] = float(uint32_t(D) << qs) * kTwoM32;
        float w = (ONE ? TX.p[u] : LT.p[u]) * L.p[u];
        if (ABSW) w = fabsf(w);
        T.w[u] = w;
      }
    };
    // the window of trace t into registers: 16-byte loads of the trace's fine
    // data, positions past the record (and loads past the window) read zero
    auto stage_load = [&](int2 W, int t, uint4 (&R)[kStage]) {
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<T16*>(fine + size_t(t) * MQ), 0, MQ * ES, kBufferWord3);
      const int nq = W.y / EPC;
#pragma unroll
      for (int k = 0; k < kStage; ++k) {
        const int c = int(threadIdx.x) + 512 * k;
        const int off = c < nq ? (W.x + EPC * c) * ES : 0x7ffffff0;
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        R[k] = make_uint4(v[0], v[1], v[2], v[3]);
      }
    };
    auto stage_store = [&](int2 W, const uint4 (&R)[kStage]) {
      const int nq = W.y / EPC;
#pragma unroll
      for (int k = 0; k < kStage; ++k) {
        const int c = int(threadIdx.x) + 512 * k;
        if (c < nq) wlds[c] = R[k];
      }
    };
    // trace t's taps from the window in LDS (fits) or from global memory
    auto add = [&](const Taps& T, int2 W, bool fits, int t) {
      if (fits) {
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
          // a voxel whose J lies in the record has J, J + 1 inside the window;
          // others (past the record, or outside the grid) read a clamped
          // position and add nothing
          const int i = int(T.J[u]) - W.x;
          const bool in = T.J[u] < unsigned(MQ) && i >= 0 && i <= W.y - 2;
          const int ic = in ? i : 0;
          const float c0 = in ? win_at<ST>(wlds, ic) : 0.0f;
          const float c1 = in ? win_at<ST>(wlds, ic + 1) : 0.0f;
          acc[u] = fmaf(T.w[u], fmaf(T.phi[u], c1 - c0, c0), acc[u]);
        }
      } else {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<T16*>(fine + size_t(t) * MQ), 0, MQ * ES, kBufferWord3);
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
          const float c0 = fine_at<ST>(rs, T.J[u]);
          const float c1 = fine_at<ST>(rs, T.J[u] + 1u);
          acc[u] = fmaf(T.w[u], fmaf(T.phi[u], c1 - c0, c0), acc[u]);
        }
      }
    };
    if (t0 < t1) {
      Legs La, Lb, LTa, LTb;
      Taps T;
      uint4 R[kStage];
      int2 W = wt[t0];
      load_legs(La, LTa, t0);
      load_legs(Lb, LTb, t0 + 1);
      if (W.y <= kWin) stage_load(W, t0, R);
      taps_of(La, LTa, T);
      // one step: trace t accumulates from (T, W); L holds the legs of t + 1
      // (in flight), Lf is free for those of t + 2
      auto step = [&](int t, Legs& L, Legs& LT, Legs& Lf, Legs& LTf) {
        const bool fits = W.y <= kWin;
        __syncthreads();  // every wave has read the previous window
        if (fits) stage_store(W, R);
        __syncthreads();
        const int2 Wn = wt[min(t + 1, t1 - 1)];
        if (t + 1 < t1 && Wn.y <= kWin) stage_load(Wn, t + 1, R);
        load_legs(Lf, LTf, t + 2);
        add(T, W, fits, t);
        taps_of(L, LT, T);
        W = Wn;
      };
      for (int t = t0; t < t1; t += 2) {
        step(t, Lb, LTb, La, LTa);
        if (t + 1 < t1) step(t + 1, La, LTa, Lb, LTb);
      }
    }
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int v = vox[u];
      if (ok[u]) {
        float tr = tau[v / nx];
        if (ABSW) tr = fabsf(tr);
        float* pv = partial + size_t(bx) * N + v;
        *pv = t_off == 0 ? acc[u] * tr : fmaf(acc[u], tr, *pv);
      }
    }
  }
}

template <bool ABSW, bool ONE, int ST>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_gather_lds(
    const typename Store<ST>::T* __restrict__ fine, int nx, int nz, int n_off, const Leg* __restrict__ legs,
    const float* __restrict__ tau, const int* __restrict__ base, int P, int K, int qs, int MQ, int tpg, int t_off,
    int t_cnt, const int2* __restrict__ gwin, int tiles_per_block, float* __restrict__ partial) {
  gather_lds_body<ABSW, ONE, ST>(blockIdx.x, blockIdx.y, fine, nx, nz, n_off, legs, tau, base, P, K, qs, MQ, tpg, t_off,
                             t_cnt, gwin, tiles_per_block, partial);
}

__global__ void k_reduce_groups(const float* __restrict__ partial, int groups, int N, float scale,
                                float* __restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  float acc = 0.0f;
  for (int g = 0; g < groups; ++g) acc += partial[size_t(g) * N + v];
  out[v] = acc * scale;
}

// Stage the polyphase taps [L_h][Q] into LDS, zero-padded to LhPad rows.
__device__ __forceinline__ void stage_taps(float* sh, const float* __restrict__ hq, int Lh, int LhPad,
                                           int Q) {
  const int n = Lh * Q;
  stage_block<float>(LhPad * Q, [&](int i) { return hq[min(i, n - 1)]; },
                     [&](int i, float v) { sh[i] = i < n ? v : 0.0f; });
  __syncthreads();
}

// C: y[m] = sum_t sum_k s[(m-1-k)Q + t] h_t[k].  Lane = (phase t, block of R
// outputs); the phase sum is a cross-lane reduction at the end.
//   out[m] = (base ? base[m] : 0) + sign * y[m] - (g ? g[ij] d_ij[m] : 0)
// base may alias out.
template <int Q>
__global__ __launch_bounds__(256) void k_conv(const float* __restrict__ fine,
                                              const float* __restrict__ hq, int M, int Lh, int LhPad,
                                              const float* base, float sign,
                                              const float* __restrict__ g,
                                              const float* __restrict__ dbasis, float* out, long tstride) {
  constexpr int R = kR;
  constexpr int MB = 64 / Q;
  constexpr int PER_WAVE = MB * R;
  extern __shared__ float sh[];
  stage_taps(sh, hq, Lh, LhPad, Q);
  const int ij = blockIdx.x;  // trace fastest: all blocks of a trace share an XCD and its L2
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = lane & (Q - 1), mb = lane / Q;
  const int m0 = blockIdx.y * (4 * PER_WAVE) + wave * PER_WAVE + mb * R;
  const float* s = fine + size_t(ij) * tstride + t;  // trace ij's fine-grid signal
  auto ld = [&](int n) -> float { return (n >= 0 && n < M) ? s[size_t(n) * Q] : 0.0f; };
  float acc[R];
  float buf[2 * R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0f;
  // buf[q] holds s at n = m0 - k0 - R + q for the current tap block k0
#pragma unroll
  for (int q = 0; q < 2 * R - 1; ++q) buf[q] = ld(m0 - R + q);
  for (int k0 = 0; k0 < LhPad; k0 += R) {
#pragma unroll
    for (int kk = 0; kk < R; ++kk) {
      const float hv = sh[(k0 + kk) * Q + t];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = fmaf(buf[r - kk + R - 1], hv, acc[r]);
    }
#pragma unroll
    for (int q = R - 2; q >= 0; --q) buf[q + R] = buf[q];
    const int nb = m0 - k0 - 2 * R;
#pragma unroll
    for (int q = 0; q < R; ++q) buf[q] = ld(nb + q);
  }
#pragma unroll
  for (int off = Q / 2; off >= 1; off >>= 1) {
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] += __shfl_xor(acc[r], off);
  }
  const float gv = g ? g[ij] : 0.0f;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int m = m0 + r;
    if ((r & (Q - 1)) == t && m < M) {
      const size_t idx = size_t(ij) * M + m;
      float val = sign * acc[r];
      if (base) val += base[idx];
      if (g) val -= gv * dbasis[idx];
      out[idx] = val;
    }
  }
}

// C^T: c[nQ + t] = sum_k r[n+1+k] h_t[k], for n < M.  Lane = (phase t, block
// of R consecutive n); writes are coalesced along t.  Trace ij's output
// starts tstride elements after trace ij - 1's.
template <int Q>
__global__ __launch_bounds__(256) void k_corr(const float* __restrict__ rt,
                                              const float* __restrict__ hq, int M, int Lh, int LhPad,
                                              float* __restrict__ fine, long tstride) {
  constexpr int R = kR;
  constexpr int NB = 64 / Q;
  constexpr int PER_WAVE = NB * R;
  extern __shared__ float sh[];
  stage_taps(sh, hq, Lh, LhPad, Q);
  const int ij = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = lane & (Q - 1), nb = lane / Q;
  const int n0 = blockIdx.y * (4 * PER_WAVE) + wave * PER_WAVE + nb * R;
  const float* r = rt + size_t(ij) * M;
  auto ld = [&](int m) -> float { return m < M ? r[m] : 0.0f; };
  float acc[R];
  float buf[2 * R];
#pragma unroll
  for (int q = 0; q < R; ++q) acc[q] = 0.0f;
  // buf[p] holds r[n0 + 1 + k0 + p] for the current tap block k0
#pragma unroll
  for (int p = 0; p < 2 * R - 1; ++p) buf[p] = ld(n0 + 1 + p);
  for (int k0 = 0; k0 < LhPad; k0 += R) {
#pragma unroll
    for (int kk = 0; kk < R; ++kk) {
      const float hv = sh[(k0 + kk) * Q + t];
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] = fmaf(buf[q + kk], hv, acc[q]);
    }
#pragma unroll
    for (int p = 0; p < R - 1; ++p) buf[p] = buf[p + R];
    const int mb = n0 + 1 + k0 + R;
#pragma unroll
    for (int p = R - 1; p < 2 * R - 1; ++p) buf[p] = ld(mb + p);
  }
  float* c = fine + size_t(ij) * tstride + t;
#pragma unroll
  for (int q = 0; q < R; ++q)
    if (n0 + q < M) c[size_t(n0 + q) * Q] = acc[q];
}

// C^T on the matrix cores, for Q a multiple of 32: per trace the correlation
// is a dense product c[n][t] = sum_k R[n][k] H[k][t] with the Hankel matrix
// R[n][k] = r[n+1+k] and the taps H[k][t] = h_t[k], so it runs as FP32 MFMA
// (v_mfma_f32_32x32x2f32: A lane l = R[l%32][l/32], B lane l = H[l/32][l%32],
// D register i of lane l = row 8(i/4) + 4(l/32) + i%4, column l%32).  A wave
// computes NT tiles of 32 rows x Q phases; the block stages its trace segment
// and the taps (zero-padded to 2 CorrHalf) in LDS.  The contraction index is
// labelled so that lane half lk takes taps k in [lk H, lk H + H): each lane
// then walks its own run of consecutive k, and the operands of the next four
// k are read while the current four multiply.  The second half of the taps
// and a second copy of the segment (shifted by H) sit 32 banks away from the
// first, so the two lane halves never read the same bank.  Writes are
// coalesced along t.
typedef float floatx16 __attribute__((ext_vector_type(16)));

// Half the padded tap count of k_corr_mfma: a multiple of 8 with 2 H >= Lh.
__host__ __device__ inline int corr_half(int Lh) { return (Lh + 15) / 16 * 8; }
// LDS words of k_corr_mfma: taps (two halves, 32 words apart), then the two
// segment copies (the second one 32 banks from the first).
__host__ __device__ inline int corr_seg_len(int rows, int H) { return rows + H; }
__host__ __device__ inline int corr_seg_gap(int rows, int H) { return (rows + H + 63) / 64 * 64 + 32; }
// one segment buffer (both halves), a multiple of 64 words so the two
// buffers have the same bank layout
__host__ __device__ inline int corr_seg_words(int rows, int H) {
  return (corr_seg_gap(rows, H) + corr_seg_len(rows, H) + 63) / 64 * 64;
}
__host__ __device__ inline int corr_lds_words(int Q, int rows, int H) {
  return 2 * H * Q + 32 + 2 * corr_seg_words(rows, H);
}

template <int QT, int NT>
__device__ __forceinline__ void corr_mfma_body(int bx, int by, const float* __restrict__ rt,
                                                   const float* __restrict__ hq, int M, int Lh, int rb_per_block,
                                                   float* __restrict__ fine, long tstride, BinSkip bs) {
  constexpr int Q = 32 * QT;
  constexpr int ROWS = 4 * NT * 32;  // n per row block
  constexpr int KB = 4;              // k per lane per step
  extern __shared__ __align__(16) float sm[];
  const int H = corr_half(Lh);
  const int SL = corr_seg_len(ROWS, H);
  float* taps0 = sm;                                   // taps rows [0, H)
  float* taps1 = sm + H * Q + 32;                      // taps rows [H, 2H)
  // two segment buffers, used by alternate row blocks: in buffer b,
  // seg0(b)[x] = r[n_blk + 1 + x] and seg1(b)[x] = r[n_blk + 1 + H + x]
  float* const segs = taps1 + H * Q;
  const int SW = corr_seg_words(ROWS, H), SG = corr_seg_gap(ROWS, H);
  const int ij = bx;
  const float* r = rt + size_t(ij) * M;
  float* c = fine + size_t(ij) * tstride;  // trace ij's output (tstride = M Q, or more between templates' grids)
  {
    // tap rows [0, 2 H), zero from Lh on, with 16-byte loads, several in
    // flight per thread; a slot past the end writes into the gap between the
    // halves (no branch, so the loads stay ahead of every store)
    const int n4 = 2 * H * Q / 4, h4 = H * Q / 4, l4 = Lh * Q / 4;
    const float4* g4 = reinterpret_cast<const float4*>(hq);
    constexpr int U = 8;
    for (int i0 = threadIdx.x; i0 < n4; i0 += U * blockDim.x) {
      float4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = g4[min(i0 + u * int(blockDim.x), l4 - 1)];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * blockDim.x;
        float* dst = i >= n4 ? taps0 + H * Q : (i < h4 ? taps0 + 4 * i : taps1 + 4 * (i - h4));
        *reinterpret_cast<float4*>(dst) = i < l4 ? v[u] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
    }
  }
  // the block's row blocks, in order; each thread carries its share of the
  // next segment in registers while the current one multiplies
  const int rb0 = by * rb_per_block;
  const int rb_end = min(rb0 + rb_per_block, (M + ROWS - 1) / ROWS);
  constexpr int SEG_PER_THREAD = 4;  // ceil((ROWS + H) / 256) for H <= 768
  float s0[SEG_PER_THREAD], s1[SEG_PER_THREAD];
  auto seg_load = [&](int rb) {
    const int n_blk = rb * ROWS;
#pragma unroll
    for (int u = 0; u < SEG_PER_THREAD; ++u) {
      const int x = threadIdx.x + u * 256;
      const int m = n_blk + 1 + x;
      s0[u] = x < SL && m < M ? r[m] : 0.0f;
      s1[u] = x < SL && m + H < M ? r[m + H] : 0.0f;
    }
  };
  auto seg_store = [&](int b) {
    float* seg0 = segs + b * SW;
#pragma unroll
    for (int u = 0; u < SEG_PER_THREAD; ++u) {
      const int x = threadIdx.x + u * 256;
      if (x < SL) {
        seg0[x] = s0[u];
        seg0[SG + x] = s1[u];
      }
    }
  };
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 31, lk = lane >> 5;
  const int row0 = wave * NT * 32;
  const float* sa0 = segs + (lk ? SG : 0) + row0 + li;  // + buffer SW + a 32 + j
  const float* sb = (lk ? taps1 : taps0) + li;       // + j Q + b 32
  if (rb0 < rb_end) seg_load(rb0);
  int sbuf = 0;  // segment buffer: alternates over the row blocks processed
  for (int rb = rb0; rb < rb_end; ++rb) {
    // a template pass leaves the rows its template never reaches unwritten:
    // the gather of that template reads none of them (uniform over the block)
    if (!bin_reaches(bs, ij, long(rb) * ROWS * Q, long(min((rb + 1) * ROWS, M)) * Q)) {
      if (rb + 1 < rb_end) seg_load(rb + 1);
      continue;
    }
    // buffer sbuf was last read two processed row blocks ago, which every wave
    // finished before the barrier of the previous one: one barrier per block
    seg_store(sbuf);
    __syncthreads();
    if (rb + 1 < rb_end) seg_load(rb + 1);
    const float* sa = sa0 + sbuf * SW;
    sbuf ^= 1;
    floatx16 acc[NT][QT];
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int b = 0; b < QT; ++b)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;
    float av[2][NT][KB], bv[2][QT][KB];
    auto load = [&](int buf, int j) {
#pragma unroll
      for (int t = 0; t < KB; ++t) {
#pragma unroll
        for (int a = 0; a < NT; ++a) av[buf][a][t] = sa[a * 32 + j + t];
#pragma unroll
        for (int b = 0; b < QT; ++b) bv[buf][b][t] = sb[(j + t) * Q + b * 32];
      }
    };
    auto multiply = [&](int buf) {
#pragma unroll
      for (int t = 0; t < KB; ++t)
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
          for (int b = 0; b < QT; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[buf][a][t], bv[buf][b][t], acc[a][b], 0, 0, 0);
    };
    // H is a multiple of 2 KB: the steps pair up; loads past the end are
    // clamped to the last step (read, never used)
    load(0, 0);
    for (int j = 0; j < H; j += 2 * KB) {
      load(1, j + KB);
      multiply(0);
      load(0, min(j + 2 * KB, H - KB));
      multiply(1);
    }
    const int n_blk = rb * ROWS;
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int n = n_blk + row0 + a * 32 + 8 * (i >> 2) + 4 * lk + (i & 3);
        if (n < M) {
#pragma unroll
          for (int b = 0; b < QT; ++b) c[size_t(n) * Q + b * 32 + li] = acc[a][b][i];
        }
      }
  }
}

// C^T with the products as three bf16 pieces each (v_mfma_f32_32x32x16_bf16,
// six per 16 contraction indices; split8_bf16x3).  The contraction index of
// product s is labelled as in the FP32 kernel, lane half lk holding
// k = lk H + 8 s + e (e < 8), so a lane reads 8 consecutive taps of its
// column and 8 consecutive segment samples of its row as one 16-byte word.
// The Hankel rows would put those 8 samples at every alignment, so a tile's
// 32 rows are n_blk + 8 i + rho (i < 32) for one residue rho: lane i reads
// segment positions 8 (i + s) + lk H + e of the copy shifted by rho.
// A row block is 256 rows, the 8 residues, two per wave; the block stages
// eight shifted copies of its segment, split into pieces, and the taps once,
// split and transposed ([piece][t][k], H + 4 words per t: 8 lanes' 16-byte
// reads on distinct banks).  Writes stay coalesced along t.
constexpr int kCorrX3Rows = 256;
constexpr int kCorrX3SegItems = 4;  // segment items (8 positions of one shifted copy) per thread, 256 threads

__host__ __device__ inline int corr_x3_tap_words(int H) { return H + 4; }
__host__ __device__ inline int corr_x3_seg_words(int H) { return (2 * H + kCorrX3Rows) / 2 + 4; }
__host__ __device__ inline int corr_x3_lds_words(int Q, int H) {
  return 3 * Q * corr_x3_tap_words(H) + 8 * 3 * corr_x3_seg_words(H);
}

// The bf16-piece forms where their LDS fits a workgroup (long templates keep
// the FP32 products).
constexpr size_t kMaxWorkgroupLds = 163840;
inline bool conv_split(const umbir_geometry& G) {
  return G.split && size_t(G.Lh + 1) * (3 * G.Q / 2 + 4) * sizeof(float) <= kMaxWorkgroupLds;
}
inline bool corr_split(const umbir_geometry& G) {
  const int H = corr_half(G.Lh);
  return G.split && size_t(corr_x3_lds_words(G.Q, H)) * sizeof(float) <= kMaxWorkgroupLds &&
         2 * H + kCorrX3Rows <= 256 * kCorrX3SegItems;
}

template <int QT>
__device__ __forceinline__ void corr_x3_body(int bx, int by, const float* __restrict__ rt,
                                             const float* __restrict__ hq, int M, int Lh, int rb_per_block,
                                             float* __restrict__ fine, long tstride, BinSkip bs) {
  constexpr int Q = 32 * QT;
  constexpr int ROWS = kCorrX3Rows;
  extern __shared__ __align__(16) float sm[];
  const int H = corr_half(Lh);
  const int TW = corr_x3_tap_words(H), SW = corr_x3_seg_words(H);
  const int SX = 2 * H + ROWS;  // segment positions a row block reads
  unsigned* taps3 = reinterpret_cast<unsigned*>(sm);  // [3][Q][TW]: piece, column t, taps k in pairs
  unsigned* seg3 = taps3 + 3 * Q * TW;                // [8][3][SW]: shift rho, piece, positions in pairs
  const int ij = bx;
  const float* r = rt + size_t(ij) * M;
  float* c = fine + size_t(ij) * tstride;
  // taps: pairs (k, k + 1) of column t, zero from Lh on and in the padding;
  // consecutive threads take consecutive t of one tap row, U pairs per thread
  // in flight
  {
    constexpr int U = 8;
    for (int i0 = threadIdx.x; i0 < Q * TW; i0 += U * blockDim.x) {
      float h[U][2];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * blockDim.x;
        const int kp = i / Q, t = i - kp * Q, k = 2 * kp;
        h[u][0] = i < Q * TW && k < Lh && kp < H ? hq[size_t(k) * Q + t] : 0.0f;
        h[u][1] = i < Q * TW && k + 1 < Lh && kp < H ? hq[size_t(k + 1) * Q + t] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * blockDim.x;
        if (i < Q * TW) {
          const int kp = i / Q, t = i - kp * Q;
          unsigned p1, p2, p3;
          split_pair_bf16x3(h[u][0], h[u][1], p1, p2, p3);
          taps3[(0 * Q + t) * TW + kp] = p1;
          taps3[(1 * Q + t) * TW + kp] = p2;
          taps3[(2 * Q + t) * TW + kp] = p3;
        }
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 31, lk = lane >> 5;
  const int rb0 = by * rb_per_block;
  const int rb_end = min(rb0 + rb_per_block, (M + ROWS - 1) / ROWS);
  // copy rho of a row block's segment holds r[n_blk + 1 + rho + x] at
  // position x < SX, split: item i = (rho, 8 positions), SX items, at most
  // kCorrX3SegItems per thread (corr_split), loaded into registers one row
  // block ahead
  float sv[kCorrX3SegItems][8];
  auto seg_load = [&](int rb) {
    const int n_blk = rb * ROWS;
#pragma unroll
    for (int u = 0; u < kCorrX3SegItems; ++u) {
      const int i = threadIdx.x + u * blockDim.x;
      const int rho = i / (SX / 8), x8 = i - rho * (SX / 8);
      const int m0 = n_blk + 1 + rho + 8 * x8;
#pragma unroll
      for (int e = 0; e < 8; ++e) sv[u][e] = i < SX && m0 + e < M ? r[m0 + e] : 0.0f;
    }
  };
  if (rb0 < rb_end) seg_load(rb0);
  for (int rb = rb0; rb < rb_end; ++rb) {
    const int n_blk = rb * ROWS;
    if (!bin_reaches(bs, ij, long(n_blk) * Q, long(min(n_blk + ROWS, M)) * Q)) {  // uniform
      if (rb + 1 < rb_end) seg_load(rb + 1);
      continue;
    }
    __syncthreads();  // the previous row block's segment copies are read
#pragma unroll
    for (int u = 0; u < kCorrX3SegItems; ++u) {
      const int i = threadIdx.x + u * blockDim.x;
      if (i < SX) {
        const int rho = i / (SX / 8), x8 = i - rho * (SX / 8);
        const Pieces8 pc = split8_bf16x3(make_float4(sv[u][0], sv[u][1], sv[u][2], sv[u][3]),
                                         make_float4(sv[u][4], sv[u][5], sv[u][6], sv[u][7]));
#pragma unroll
        for (int tau = 0; tau < 3; ++tau)
          reinterpret_cast<uint4*>(seg3 + (rho * 3 + tau) * SW)[x8] = pc.p[tau];
      }
    }
    __syncthreads();
    if (rb + 1 < rb_end) seg_load(rb + 1);
    floatx16 acc[2][QT];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < QT; ++b)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;
    const int rho0 = 2 * wave;
    const uint4* sa = reinterpret_cast<const uint4*>(seg3) + li + lk * (H / 8);  // + copy (rho, piece) + s
    const uint4* sb = reinterpret_cast<const uint4*>(taps3) + lk * (H / 8);      // + (piece, t) + s
    for (int st = 0; st < H / 8; ++st) {
      uint4 bq[QT][3];
#pragma unroll
      for (int b = 0; b < QT; ++b)
#pragma unroll
        for (int tau = 0; tau < 3; ++tau) bq[b][tau] = sb[((tau * Q + b * 32 + li) * TW) / 4 + st];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        uint4 aq[3];
#pragma unroll
        for (int tau = 0; tau < 3; ++tau) aq[tau] = sa[((rho0 + a) * 3 + tau) * (SW / 4) + st];
#pragma unroll
        for (int b = 0; b < QT; ++b) acc[a][b] = mfma_bf16x3(aq, bq[b], acc[a][b]);
      }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int n = n_blk + 8 * (8 * (i >> 2) + 4 * lk + (i & 3)) + rho0 + a;
        if (n < M) {
#pragma unroll
          for (int b = 0; b < QT; ++b) c[size_t(n) * Q + b * 32 + li] = acc[a][b][i];
        }
      }
  }
}

template <int QT>
__global__ __launch_bounds__(256) void k_corr_x3(const float* __restrict__ rt, const float* __restrict__ hq, int M,
                                                 int Lh, int rb_per_block, float* __restrict__ fine, long tstride,
                                                 BinSkip bs) {
  corr_x3_body<QT>(blockIdx.x, blockIdx.y, rt, hq, M, Lh, rb_per_block, fine, tstride, bs);
}

template <int QT, int NT>
__global__ __launch_bounds__(256) void k_corr_mfma(const float* __restrict__ rt,
                                                   const float* __restrict__ hq, int M, int Lh, int rb_per_block,
                                                   float* __restrict__ fine, long tstride, BinSkip bs) {
  corr_mfma_body<QT, NT>(blockIdx.x, blockIdx.y, rt, hq, M, Lh, rb_per_block, fine, tstride, bs);
}

// Chunk order of the banded convolutions on the matrix cores.  The rows n a
// block needs are its window [m0 - Lh, m0 + 30], walked in chunks of CN rows.
// Every block walks a window of the same length, P chunks from m0 - Lh,
// rotated so that at step s it reads rows congruent to s CN modulo P CN: the
// blocks of one trace tile, resident together on one XCD, then read the same
// rows at about the same time, and the L2 serves the repeats that a plain
// order leaves to memory.  Rows outside [0, M) read as zero.

struct ChunkOrder {
  int v_lo, P, rot, CN;
  __device__ ChunkOrder(int m0, int Lh, int cn) : CN(cn) {
    v_lo = m0 - Lh;
    P = (Lh + 31 + CN - 1) / CN;
    const int fl = v_lo >= 0 ? v_lo / CN : -((-v_lo + CN - 1) / CN);  // floor(v_lo / CN)
    rot = ((-fl) % P + P) % P;
  }
  __device__ int row(int s) const { return v_lo + ((s + rot) % P) * CN; }
};

// C on the matrix cores, for Q in {32, 64}: the convolution of one trace has a
// single output column, so traces are batched as the N dimension:
//   Y[m][tr] = sum_{(n,t)} H[m-1-n][t] S_tr[n Q + t],
// A = the banded Toeplitz tile built from the taps (zero where m - 1 - n is
// outside the window), B = the fine-grid signals of 32 traces.  A block owns a
// 32 (m) x 32 (trace) output tile; its nw waves take the window's 64-wide
// chunks of (n, t) in turn (ChunkOrder) and their partial tiles are summed in
// LDS at the end.  The contraction index of the 32x32x2 product is labelled
// so that lane half lk holds chunk positions [32 lk, 32 lk + 32): a lane's A
// values are then 32 consecutive taps of one row (read as 16-byte LDS words)
// and its B values 32 consecutive fine-grid samples of one trace, loaded from
// memory straight into registers one chunk ahead, with no staging.  Taps are
// kept with one zero row after the window, which a lane reads for any row
// outside it, and a row stride of Q + 4 words, which spreads 16 lanes'
// 16-byte reads over all banks.  With one accumulation chain the kernel fits
// 128 registers and 35 KB of LDS at Q = 32, so four blocks share a CU.
// Epilogue as in k_conv.
// X3: the products as three bf16 pieces each (split8_bf16x3) on the bf16
// matrix cores, v_mfma_f32_32x32x16_bf16, six per 16 contraction indices
// against eight FP32 ones per 16: lane half lk holds chunk positions
// 32 lk + 8 s + e (e < 8) in product s of four, the same positions as above.
// The taps are split once, while staged: a tap row holds the three pieces of
// its Q taps one after the other, 3 Q / 2 + 4 words (16-byte reads of 8 lanes
// on distinct banks); a chunk of B is split once for all NTC tiles.
// nw waves (4 or 8) share a block's window; a block may have more waves than
// that (a work-list stage runs every problem with the same block size): the
// others help stage the taps and write the outputs.  Results do not depend on
// the block size, only on nw (the order of the waves' partial sums).
constexpr int kConvMaxWaves = 8;

template <int Q>
__host__ __device__ constexpr int conv_x3_row_words() { return 3 * Q / 2 + 4; }

template <int Q, int NTC = 1, bool X3 = false>
__device__ __forceinline__ void conv_mfma_body(int bx, int by, const float* __restrict__ fine,
                                                   const float* __restrict__ hq, int M, int Lh,
                                                   int PK, const float* base, float sign,
                                                   const float* __restrict__ g,
                                                   const float* __restrict__ dbasis, float* out, long tstride,
                                                   BinSkip bs, int nw) {
  constexpr int CK = 64;        // (n, t) positions per chunk
  constexpr int CN = CK / Q;    // rows n per chunk
  constexpr int TS = Q + 4;     // tap row stride
  extern __shared__ __align__(16) float sm[];
  float* taps = sm;  // [Lh + 1][TS]: tap rows 0 .. Lh - 1, then a zero row
  const int tr0 = bx * 32;
  const int m0 = by * 32 * NTC;  // NTC output tiles of 32 samples, m0 + 32 j
  const long MQ = long(M) * Q;
  constexpr int TS3 = conv_x3_row_words<Q>();
  if constexpr (X3) {
    // [Lh + 1][TS3] words: a row's three pieces of Q taps, padding, a zero row
    unsigned* t3 = reinterpret_cast<unsigned*>(sm);
    for (int i = threadIdx.x; i < (Lh + 1) * TS3; i += blockDim.x) {
      const int r = i / TS3, c = i - r * TS3;
      if (r >= Lh || c >= 3 * Q / 2) t3[i] = 0u;
    }
    constexpr int Q4 = Q / 4;
    const float4* h4 = reinterpret_cast<const float4*>(hq);
    const int n4 = Lh * Q4;
    constexpr int U = 8;
    for (int i0 = threadIdx.x; i0 < n4; i0 += U * blockDim.x) {
      float4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = h4[min(i0 + u * int(blockDim.x), n4 - 1)];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * blockDim.x;
        if (i < n4) {
          const int k = i / Q4, c = i - k * Q4;  // taps 4 c .. 4 c + 3 of row k
          uint2 p1, p2, p3;
          split_pair_bf16x3(v[u].x, v[u].y, p1.x, p2.x, p3.x);
          split_pair_bf16x3(v[u].z, v[u].w, p1.y, p2.y, p3.y);
          uint2* row = reinterpret_cast<uint2*>(t3 + k * TS3 + 2 * c);
          row[0] = p1;
          row[Q / 4] = p2;
          row[Q / 2] = p3;
        }
      }
    }
  } else {
    // zero rows and columns first, then the taps with 16-byte loads, several
    // in flight per thread (hq rows are Q floats, 16-byte aligned)
    constexpr int R4 = TS / 4, Q4 = Q / 4;
    float4* t4 = reinterpret_cast<float4*>(taps);
    for (int i = threadIdx.x; i < (Lh + 1) * R4; i += blockDim.x) {
      const int r = i / R4, c = i - r * R4;
      if (r >= Lh || c >= Q4) t4[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    const float4* h4 = reinterpret_cast<const float4*>(hq);
    const int n4 = Lh * Q4;
    constexpr int U = 8;
    for (int i0 = threadIdx.x; i0 < n4; i0 += U * blockDim.x) {
      float4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = h4[min(i0 + u * int(blockDim.x), n4 - 1)];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // past the end: a zero into the zero row (no branch, so the loads
        // above stay ahead of every store)
        const int i = i0 + u * blockDim.x;
        const bool in = i < n4;
        const int k = in ? i / Q4 : Lh, c = in ? i - k * Q4 : 0;
        t4[k * R4 + c] = in ? v[u] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 31, lk = lane >> 5;
  const int ro = (32 * lk) / Q, t0 = (32 * lk) % Q;  // this lane's row and first tap within a chunk
  // rows n that meet an output m in [m0, m0 + 32 NTC): m0 - Lh <= n <= m0 + 32 NTC - 2
  constexpr int EXT = 32 * (NTC - 1);
  const ChunkOrder co(m0 + EXT, Lh + EXT, CN);
  // a template pass whose template reaches none of the tile's input rows
  // multiplies nothing (the epilogue still runs)
  const bool reach = __syncthreads_or(threadIdx.x < 32 && tr0 + int(threadIdx.x) < PK &&
                                      bin_reaches(bs, tr0 + threadIdx.x, long(m0 - Lh) * Q,
                                                  long(m0 + 31 + EXT) * Q));
  const int rounds = reach && wave < nw ? (co.P + nw - 1) / nw : 0;
  floatx16 acc[NTC];
#pragma unroll
  for (int j = 0; j < NTC; ++j)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[j][i] = 0.0f;
  // B: trace tr0 + li (traces past the last read the last one: they only feed
  // output columns that are never written).  Loads are unconditional, from a
  // row clamped into [0, M); a row outside [0, M), or a step past the window,
  // takes the A row of zeros instead, so B needs no masking.
  const float* src = fine + size_t(min(tr0 + li, PK - 1)) * tstride + t0;
  // the chunk of step ch = rd nw + wave advances by nw per round, modulo P
  int jf = (wave + co.rot) % co.P, jm = jf;  // fetch and multiply positions
  int sf = wave, sm_ = wave;                  // their steps
  auto next_row = [&](int& j, int& step) {
    const int nc = step < co.P ? co.v_lo + j * CN : -(1 << 30);  // past the window: no row
    step += nw;
    j += nw;
    while (j >= co.P) j -= co.P;
    return nc;
  };
  auto fetch = [&](float4 (&b)[8]) {
    const int nc = next_row(jf, sf);
    const int n = min(max(nc + ro, 0), M - 1);
    const float4* p = reinterpret_cast<const float4*>(src + long(n) * Q);
#pragma unroll
    for (int u = 0; u < 8; ++u) b[u] = p[u];
  };
  const int m = m0 + li;
  auto multiply = [&](const float4 (&b)[8]) {
    const int nc = next_row(jm, sm_);
    const int n = nc + ro;
    if constexpr (X3) {
      Pieces8 bp[4];  // the chunk's B: positions 8 s .. 8 s + 7 of the lane's 32
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) bp[s4] = split8_bf16x3(b[2 * s4], b[2 * s4 + 1]);
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int j = 0; j < NTC; ++j) {
        if (NTC > 1 && (nc > m0 + 32 * j + 30 || nc + CN - 1 < m0 + 32 * j - Lh)) continue;
        int k = m + 32 * j - 1 - n;
        if (n < 0 || n >= M || unsigned(k) >= unsigned(Lh)) k = Lh;
        const uint4* arow = reinterpret_cast<const uint4*>(sm) + k * (TS3 / 4) + t0 / 8;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const uint4 a[3] = {arow[s4], arow[Q / 8 + s4], arow[Q / 4 + s4]};
          acc[j] = mfma_bf16x3(a, bp[s4].p, acc[j]);
        }
      }
      __builtin_amdgcn_s_setprio(0);
      return;
    }
    // a wave issuing its chunk's MFMAs takes precedence over waves issuing
    // loads and address arithmetic (measured: 2-4 % on this kernel; the
    // correlation, whose operands come from LDS, is slower with it)
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int j = 0; j < NTC; ++j) {
      // tile j needs rows [m0 + 32 j - Lh, m0 + 32 j + 30]: a chunk wholly
      // outside them is skipped (uniform over the wave)
      if (NTC > 1 && (nc > m0 + 32 * j + 30 || nc + CN - 1 < m0 + 32 * j - Lh)) continue;
      // tap row k = m - 1 - n; the zero row for rows outside [0, M) or the window
      int k = m + 32 * j - 1 - n;
      if (n < 0 || n >= M || unsigned(k) >= unsigned(Lh)) k = Lh;
      const float4* arow = reinterpret_cast<const float4*>(taps + k * TS + t0);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const float4 av = arow[u];
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, b[u].x, acc[j], 0, 0, 0);
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, b[u].y, acc[j], 0, 0, 0);
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, b[u].z, acc[j], 0, 0, 0);
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.w, b[u].w, acc[j], 0, 0, 0);
      }
    }
    __builtin_amdgcn_s_setprio(0);
  };
  // the epilogue's inputs for this thread's EPT NTC outputs, fetched now so
  // that they arrive while the window multiplies
  // (outputs per thread of one 32 x 32 tile: 1024 / blockDim.x, at most 4)
  const int ept = 1024 / int(blockDim.x);
  float pre_base[4 * NTC], pre_db[4 * NTC], pre_g[4 * NTC];
#pragma unroll
  for (int q = 0; q < 4 * NTC; ++q) {
    const int e = threadIdx.x + (q & 3) * blockDim.x;
    const int mm = min(m0 + 32 * (q >> 2) + (e & 31), M - 1), tr = min(tr0 + (e >> 5), PK - 1);
    const size_t idx = size_t(tr) * M + mm;
    const bool use = (q & 3) < ept;
    pre_base[q] = base && use ? base[idx] : 0.0f;
    pre_db[q] = g && use ? dbasis[idx] : 0.0f;
    pre_g[q] = g && use ? g[tr] : 0.0f;
  }
  __syncthreads();  // taps staged
  // two register sets in turn: the next chunk is in flight while one multiplies
  float4 b0[8], b1[8];
  if (wave < nw) {  // uniform over the wave
    fetch(b0);
    for (int rd = 0; rd < rounds; rd += 2) {
      fetch(b1);
      multiply(b0);
      fetch(b0);
      multiply(b1);
    }
  }
  __syncthreads();  // every wave is done with the taps: reuse them for the reduction
  // sum the waves' partial tiles of each output tile: red[j][wave][row][col]
  float* red = sm;
  if (wave < nw) {
#pragma unroll
    for (int j = 0; j < NTC; ++j)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int row = 8 * (i >> 2) + 4 * lk + (i & 3);
        red[((j * nw + wave) * 32 + row) * 33 + li] = acc[j][i];
      }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4 * NTC; ++q) {
    const int j = q >> 2;
    const int e = threadIdx.x + (q & 3) * blockDim.x;
    const int col = e >> 5, row = e & 31;  // consecutive threads: consecutive m of one trace
    const int mm = m0 + 32 * j + row, tr = tr0 + col;
    if ((q & 3) < ept && mm < M && tr < PK) {
      const float* rj = red + j * nw * 32 * 33;
      float v = rj[row * 33 + col];
      for (int w = 1; w < nw; ++w) v += rj[(w * 32 + row) * 33 + col];
      float val = sign * v;
      if (base) val += pre_base[q];
      if (g) val -= pre_g[q] * pre_db[q];
      out[size_t(tr) * M + mm] = val;
    }
  }
}

template <int Q, int NTC, bool X3>
__global__ __launch_bounds__(64 * kConvMaxWaves) void k_conv_mfma(const float* __restrict__ fine,
                                                   const float* __restrict__ hq, int M, int Lh,
                                                   int PK, const float* base, float sign,
                                                   const float* __restrict__ g,
                                                   const float* __restrict__ dbasis, float* out, long tstride,
                                                   BinSkip bs, int nw) {
  conv_mfma_body<Q, NTC, X3>(blockIdx.x, blockIdx.y, fine, hq, M, Lh, PK, base, sign, g, dbasis, out, tstride, bs, nw);
}

// The same with the grid's dimensions swapped (sample tiles fastest).
template <int Q, int NTC, bool X3>
__global__ __launch_bounds__(64 * kConvMaxWaves) void k_conv_mfma_t(const float* __restrict__ fine, const float* __restrict__ hq,
                                                     int M, int Lh, int PK, const float* base, float sign,
                                                     const float* __restrict__ g, const float* __restrict__ dbasis,
                                                     float* out, long tstride, BinSkip bs, int nw) {
  conv_mfma_body<Q, NTC, X3>(blockIdx.y, blockIdx.x, fine, hq, M, Lh, PK, base, sign, g, dbasis, out, tstride, bs, nw);
}

// C on the matrix cores with 16-bit storage (Q in {32, 64}): as k_conv_mfma,
// with v_mfma_f32_32x32x8 {f16, bf16}: each lane holds four consecutive
// (n, t) values of A (taps of one row, read as one 8-byte LDS word) and of B
// (one staged trace).  Taps are converted to the storage type while staged.
template <int Q, int ST>
__global__ __launch_bounds__(256) void k_conv_mfma16(const typename Store<ST>::T* __restrict__ fine,
                                                     const float* __restrict__ hq, int M, int Lh, int PK,
                                                     const typename Store<ST>::T* base, float sign,
                                                     const float* __restrict__ g,
                                                     const float* __restrict__ dbasis,
                                                     typename Store<ST>::T* out) {
  using T = typename Store<ST>::T;
  constexpr int CK = 64;       // (n, t) pairs per chunk
  constexpr int CN = CK / Q;   // rows n per chunk
  constexpr int TS = Q + 4;    // tap row stride (8-byte aligned rows)
  constexpr int SB = CK + 4;   // staged row stride
  extern __shared__ __align__(16) char smc[];
  T* taps = reinterpret_cast<T*>(smc);                               // [Lh][TS]
  T* stage = taps + ((Lh * TS + 7) & ~7);                            // [4 waves][32 traces][SB]
  float* red = reinterpret_cast<float*>(stage);                       // reused at the end
  const int tr0 = blockIdx.x * 32;
  const int m0 = blockIdx.y * 32;
  const long MQ = long(M) * Q;
  stage_block<float>(Lh * TS, [&](int i) { const int k = i / TS, t = i - k * TS; return hq[k * Q + min(t, Q - 1)]; },
                     [&](int i, float v) { taps[i] = Store<ST>::put(i % TS < Q ? v : 0.0f); });
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 31, lk = lane >> 5;
  T* st = stage + wave * 32 * SB;
  const ChunkOrder co(m0, Lh, CN);
  const int rounds = (co.P + 3) / 4;
  floatx16 acc[2];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[0][i] = acc[1][i] = 0.0f;
  // B chunk of one wave: 32 traces x 64 values = 32 x 128 bytes; 8 lanes x 16 bytes per
  // trace, 8 traces per load instruction, 4 instructions; prefetched one chunk ahead
  const int sub = lane & 7, tq = lane >> 3;
  uint4 pre[4];
  auto fetch = [&](int ch) {
    const int nc = ch < co.P ? co.row(ch) : -CN;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int tr = u * 8 + tq;
      const int kp = sub * 8;  // first of eight consecutive (n, t) values
      const int n = nc + kp / Q;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (n >= 0 && n < M && tr0 + tr < PK)
        v = *reinterpret_cast<const uint4*>(fine + size_t(tr0 + tr) * MQ + size_t(nc) * Q + kp);
      pre[u] = v;
    }
  };
  const int m = m0 + li;
  __syncthreads();  // taps staged
  fetch(wave);
  for (int rd = 0; rd < rounds; ++rd) {
    const int ch = rd * 4 + wave;
    const int nc = ch < co.P ? co.row(ch) : -CN;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      uint2* d = reinterpret_cast<uint2*>(st + (u * 8 + tq) * SB + sub * 8);
      d[0] = make_uint2(pre[u].x, pre[u].y);
      d[1] = make_uint2(pre[u].z, pre[u].w);
    }
    __builtin_amdgcn_wave_barrier();  // the staging buffer is private to this wave
    fetch(ch + 4);
    if (nc + CN > 0 && nc < M) {
      const T* trow[CN];
      bool tok[CN];
#pragma unroll
      for (int r = 0; r < CN; ++r) {
        const int k = m - 1 - nc - r;
        tok[r] = k >= 0 && k < Lh;
        trow[r] = taps + (tok[r] ? k : 0) * TS + 4 * lk - r * Q;
      }
      const T* srow = st + li * SB + 4 * lk;
#pragma unroll
      for (int kk = 0; kk < CK; kk += 8) {
        const int r = kk / Q;  // compile-time: kk + 4 lk + 3 stays in row kk / Q
        uint2 av = *reinterpret_cast<const uint2*>(trow[r] + kk);
        if (!tok[r]) av = make_uint2(0u, 0u);
        const uint2 bv = *reinterpret_cast<const uint2*>(srow + kk);
        acc[(kk >> 3) & 1] = Store<ST>::mfma(av, bv, acc[(kk >> 3) & 1]);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[0][i] += acc[1][i];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int row = 8 * (i >> 2) + 4 * lk + (i & 3);
    red[(wave * 32 + row) * 33 + li] = acc[0][i];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
    const int col = e >> 5, row = e & 31;
    const int mm = m0 + row, tr = tr0 + col;
    if (mm < M && tr < PK) {
      const float v = red[(0 * 32 + row) * 33 + col] + red[(1 * 32 + row) * 33 + col] +
                      red[(2 * 32 + row) * 33 + col] + red[(3 * 32 + row) * 33 + col];
      const size_t idx = size_t(tr) * M + mm;
      float val = sign * v;
      if (base) val += Store<ST>::get(base[idx]);
      if (g) val -= g[tr] * dbasis[idx];
      out[idx] = Store<ST>::put(val);
    }
  }
}

// C^T on the matrix cores with 16-bit storage: as k_corr_mfma with
// v_mfma_f32_32x32x8 {f16, bf16}.  A = Hankel rows: the trace segment is kept
// as overlapping quads q[j] = (r[j], r[j+1], r[j+2], r[j+3]) so every lane's
// four consecutive values are one aligned 8-byte LDS word; B = taps stored
// transposed [t][k] for the same reason.
template <int QT, int NT, int ST>
__global__ __launch_bounds__(256) void k_corr_mfma16(const typename Store<ST>::T* __restrict__ rt,
                                                     const float* __restrict__ hq, int M, int Lh,
                                                     typename Store<ST>::T* __restrict__ fine) {
  using T = typename Store<ST>::T;
  constexpr int Q = 32 * QT;
  constexpr int ROWS = 4 * NT * 32;
  extern __shared__ __align__(16) char smc[];
  const int L8 = (Lh + 7) & ~7;    // taps padded to a multiple of the K step
  const int KS = L8 + 4;           // transposed tap row stride
  T* tapsT = reinterpret_cast<T*>(smc);                                    // [Q][KS]
  uint2* quad = reinterpret_cast<uint2*>(tapsT + ((Q * KS + 3) & ~3));     // [ROWS + L8]
  const int ij = blockIdx.x;
  const int n_blk = blockIdx.y * ROWS;
  const T* r = rt + size_t(ij) * M;
  stage_block<float>(Q * KS, [&](int i) { const int t = i / KS, k = i - t * KS; return hq[min(k, Lh - 1) * Q + t]; },
                     [&](int i, float v) { tapsT[i] = Store<ST>::put(i % KS < Lh ? v : 0.0f); });
  for (int j = threadIdx.x; j < ROWS + L8; j += blockDim.x) {
    T v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int mm = n_blk + 1 + j + e;
      v[e] = mm < M ? r[mm] : Store<ST>::put(0.0f);
    }
    uint2 w;
    __builtin_memcpy(&w, v, 8);
    quad[j] = w;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 31, lk = lane >> 5;
  floatx16 acc[NT][QT];
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < QT; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;
  const int row0 = wave * NT * 32;
  for (int k0 = 0; k0 < L8; k0 += 8) {
    uint2 bv[QT];
#pragma unroll
    for (int b = 0; b < QT; ++b) bv[b] = *reinterpret_cast<const uint2*>(tapsT + (b * 32 + li) * KS + k0 + 4 * lk);
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const uint2 av = quad[row0 + a * 32 + li + k0 + 4 * lk];
#pragma unroll
      for (int b = 0; b < QT; ++b) acc[a][b] = Store<ST>::mfma(av, bv[b], acc[a][b]);
    }
  }
  T* c = fine + size_t(ij) * M * Q;
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int n = n_blk + row0 + a * 32 + 8 * (i >> 2) + 4 * lk + (i & 3);
      if (n < M) {
#pragma unroll
        for (int b = 0; b < QT; ++b) c[size_t(n) * Q + b * 32 + li] = Store<ST>::put(acc[a][b][i]);
      }
    }
}

template <int ST>
__global__ void k_direct(const float* __restrict__ g, const float* __restrict__ dbasis, int M,
                         size_t total, int accumulate, typename Store<ST>::T* __restrict__ y) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < total; k += stride) {
    const float v = g[k / M] * dbasis[k];
    y[k] = Store<ST>::put(accumulate ? Store<ST>::get(y[k]) + v : v);
  }
}

int grid_1d(size_t n) {
  size_t b = (n + 255) / 256;
  return int(b > 8192 ? 8192 : (b ? b : 1));
}

int lh_pad(int Lh) { return (Lh + kR - 1) / kR * kR; }

template <int Q>
void launch_conv_q(const umbir_geometry& G, const float* fine, const float* hq, const float* base,
                   float sign, const float* g, float* out, long tstride, hipStream_t s) {
  constexpr int per_block = 4 * (64 / Q) * kR;
  const int LhP = lh_pad(G.Lh);
  dim3 grid(G.traces(), (G.M + per_block - 1) / per_block);
  UMBIR_LAUNCH("conv", k_conv<Q>, grid, dim3(256), size_t(LhP) * Q * sizeof(float), s, fine, hq, G.M,
               G.Lh, LhP, base, sign, g, G.dbasis, out, tstride);
}

template <int Q>
void launch_corr_q(const umbir_geometry& G, const float* r, const float* hq, float* fine, long tstride,
                   hipStream_t s) {
  constexpr int per_block = 4 * (64 / Q) * kR;
  const int LhP = lh_pad(G.Lh);
  dim3 grid(G.traces(), (G.M + per_block - 1) / per_block);
  UMBIR_LAUNCH("corr", k_corr<Q>, grid, dim3(256), size_t(LhP) * Q * sizeof(float), s, r, hq, G.M,
               G.Lh, LhP, fine, tstride);
}

// Waves sharing a convolution block's window: eight with bf16-piece products
// when the grid leaves fewer than two blocks per CU (the waves of a block
// then hide each other's row loads; measured: 256x256, 97 against 111 us),
// else four.
int conv_waves(const umbir_geometry& G) {
  const long tt = (G.traces() + 31) / 32, mt = (G.M + 32 * G.conv_tiles - 1) / (32 * G.conv_tiles);
  return conv_split(G) && tt * mt < 512 ? 8 : 4;
}

// LDS of the matrix-core convolution: the padded taps, reused at the end for
// the nw waves' partial tiles of each of the NTC output tiles
size_t conv_mfma_lds(const umbir_geometry& G) {
  const size_t row = conv_split(G) ? size_t(3 * G.Q / 2 + 4) : size_t(G.Q + 4);  // words per tap row
  return std::max<size_t>(size_t(G.Lh + 1) * row, size_t(G.conv_tiles) * conv_waves(G) * 32 * 33) * sizeof(float);
}

template <int Q, int NTC, bool X3>
void launch_conv_mfma_x(const umbir_geometry& G, const float* fine, const float* hq, const float* base,
                        float sign, const float* g, float* out, long tstride, int gbin, hipStream_t s) {
  const size_t lds = conv_mfma_lds(G);
  const int nw = conv_waves(G);
  const unsigned tt = unsigned((G.traces() + 31) / 32), mt = unsigned((G.M + 32 * NTC - 1) / (32 * NTC));
  if (G.conv_grid == 2)
    UMBIR_LAUNCH("conv", (k_conv_mfma_t<Q, NTC, X3>), dim3(mt, tt), dim3(64 * nw), lds, s, fine, hq, G.M, G.Lh,
                 G.traces(),
                 base, sign, g, G.dbasis, out, tstride, bin_skip(G, gbin), nw);
  else
    UMBIR_LAUNCH("conv", (k_conv_mfma<Q, NTC, X3>), dim3(tt, mt), dim3(64 * nw), lds, s, fine, hq, G.M, G.Lh,
                 G.traces(),
                 base, sign, g, G.dbasis, out, tstride, bin_skip(G, gbin), nw);
}

template <int Q, int NTC>
void launch_conv_mfma_n(const umbir_geometry& G, const float* fine, const float* hq, const float* base,
                        float sign, const float* g, float* out, long tstride, int gbin, hipStream_t s) {
  if (conv_split(G)) launch_conv_mfma_x<Q, NTC, true>(G, fine, hq, base, sign, g, out, tstride, gbin, s);
  else launch_conv_mfma_x<Q, NTC, false>(G, fine, hq, base, sign, g, out, tstride, gbin, s);
}

template <int Q>
void launch_conv_mfma(const umbir_geometry& G, const float* fine, const float* hq, const float* base,
                      float sign, const float* g, float* out, long tstride, int gbin, hipStream_t s) {
  if (G.conv_tiles == 1) return launch_conv_mfma_n<Q, 1>(G, fine, hq, base, sign, g, out, tstride, gbin, s);
  if (G.conv_tiles == 4) return launch_conv_mfma_n<Q, 4>(G, fine, hq, base, sign, g, out, tstride, gbin, s);
  return launch_conv_mfma_n<Q, 2>(G, fine, hq, base, sign, g, out, tstride, gbin, s);
}

template <int Q, int ST>
void launch_conv_mfma16(const umbir_geometry& G, const void* fine, const float* hq, const void* base,
                        float sign, const float* g, void* out, hipStream_t s) {
  using T = typename Store<ST>::T;
  const size_t taps = (size_t(G.Lh) * (Q + 4) + 7) & ~size_t(7);
  const size_t stage = std::max<size_t>(4 * 32 * (64 + 4) * sizeof(T), 4 * 32 * 33 * sizeof(float));
  const size_t lds = taps * sizeof(T) + stage;
  dim3 grid((G.traces() + 31) / 32, (G.M + 31) / 32);
  UMBIR_LAUNCH("conv", (k_conv_mfma16<Q, ST>), grid, dim3(256), lds, s, static_cast<const T*>(fine), hq, G.M,
               G.Lh, G.traces(), static_cast<const T*>(base), sign, g, G.dbasis, static_cast<T*>(out));
}

// gbin >= 0: the pass of attenuation template gbin (output tiles its template
// never reaches skip their products).  FP32: trace t's fine-grid signal starts
// at fine + t * tstride elements (tstride = M Q when 0).
void launch_conv(const umbir_geometry& G, const void* fine_v, const float* hq, const void* base_v,
                 float sign, const float* g, void* out_v, int gbin, hipStream_t s, long tstride = 0) {
  if (G.storage == UMBIR_STORAGE_F16) {
    if (G.Q == 32) return launch_conv_mfma16<32, UMBIR_STORAGE_F16>(G, fine_v, hq, base_v, sign, g, out_v, s);
    return launch_conv_mfma16<64, UMBIR_STORAGE_F16>(G, fine_v, hq, base_v, sign, g, out_v, s);
  }
  if (G.storage == UMBIR_STORAGE_BF16) {
    if (G.Q == 32) return launch_conv_mfma16<32, UMBIR_STORAGE_BF16>(G, fine_v, hq, base_v, sign, g, out_v, s);
    return launch_conv_mfma16<64, UMBIR_STORAGE_BF16>(G, fine_v, hq, base_v, sign, g, out_v, s);
  }
  const float* fine = static_cast<const float*>(fine_v);
  const float* base = static_cast<const float*>(base_v);
  float* out = static_cast<float*>(out_v);
  const long ts = tstride > 0 ? tstride : long(G.fine_per_trace());
  if (G.Q == 32) return launch_conv_mfma<32>(G, fine, hq, base, sign, g, out, ts, gbin, s);
  if (G.Q == 64) return launch_conv_mfma<64>(G, fine, hq, base, sign, g, out, ts, gbin, s);
  switch (G.Q) {
    case 1: launch_conv_q<1>(G, fine, hq, base, sign, g, out, ts, s); break;
    case 2: launch_conv_q<2>(G, fine, hq, base, sign, g, out, ts, s); break;
    case 4: launch_conv_q<4>(G, fine, hq, base, sign, g, out, ts, s); break;
    case 8: launch_conv_q<8>(G, fine, hq, base, sign, g, out, ts, s); break;
    default: launch_conv_q<16>(G, fine, hq, base, sign, g, out, ts, s); break;
  }
}

template <int QT, int NT>
void launch_corr_mfma_nt(const umbir_geometry& G, const float* r, const float* hq, float* fine, long tstride,
                         int gbin, hipStream_t s) {
  constexpr int rows = 4 * NT * 32;
  const size_t lds = size_t(corr_lds_words(32 * QT, rows, corr_half(G.Lh))) * sizeof(float);
  // about corr_blocks blocks (four per CU by default), each walking several
  // row blocks of one trace with the taps staged once
  const int nrb = (G.M + rows - 1) / rows;
  const int per = std::max(1, int((long(G.traces()) * nrb) / std::max(1, G.corr_blocks)));
  dim3 grid(G.traces(), (nrb + per - 1) / per);
  UMBIR_LAUNCH("corr", (k_corr_mfma<QT, NT>), grid, dim3(256), lds, s, r, hq, G.M, G.Lh, per, fine, tstride,
               bin_skip(G, gbin));
}

template <int QT>
void launch_corr_x3(const umbir_geometry& G, const float* r, const float* hq, float* fine, long tstride, int gbin,
                    hipStream_t s) {
  const size_t lds = size_t(corr_x3_lds_words(32 * QT, corr_half(G.Lh))) * sizeof(float);
  const int nrb = (G.M + kCorrX3Rows - 1) / kCorrX3Rows;
  const int per = std::max(1, int((long(G.traces()) * nrb) / std::max(1, G.corr_blocks)));
  dim3 grid(G.traces(), (nrb + per - 1) / per);
  UMBIR_LAUNCH("corr", (k_corr_x3<QT>), grid, dim3(256), lds, s, r, hq, G.M, G.Lh, per, fine, tstride,
               bin_skip(G, gbin));
}

template <int QT>
void launch_corr_mfma(const umbir_geometry& G, const float* r, const float* hq, float* fine, long tstride,
                      int gbin, hipStream_t s) {
  if (corr_split(G)) return launch_corr_x3<QT>(G, r, hq, fine, tstride, gbin, s);
  if (G.corr_tiles == 1) return launch_corr_mfma_nt<QT, 1>(G, r, hq, fine, tstride, gbin, s);
  if (G.corr_tiles == 4) return launch_corr_mfma_nt<QT, 4>(G, r, hq, fine, tstride, gbin, s);
  return launch_corr_mfma_nt<QT, 2>(G, r, hq, fine, tstride, gbin, s);
}

template <int QT, int ST>
void launch_corr_mfma16(const umbir_geometry& G, const void* r, const float* hq, void* fine, hipStream_t s) {
  using T = typename Store<ST>::T;
  constexpr int NT = 2;
  constexpr int rows = 4 * NT * 32;
  const int L8 = (G.Lh + 7) & ~7;
  const size_t tapsT = (size_t(32 * QT) * (L8 + 4) + 3) & ~size_t(3);
  const size_t lds = tapsT * sizeof(T) + size_t(rows + L8) * 8;
  dim3 grid(G.traces(), (G.M + rows - 1) / rows);
  UMBIR_LAUNCH("corr", (k_corr_mfma16<QT, NT, ST>), grid, dim3(256), lds, s, static_cast<const T*>(r), hq, G.M,
               G.Lh, static_cast<T*>(fine));
}

// gbin >= 0: the pass of attenuation template gbin (rows its template never
// reaches are left unwritten).  FP32: trace t's output starts at fine +
// t * tstride elements (tstride = M Q when 0).
void launch_corr(const umbir_geometry& G, const void* r_v, const float* hq, void* fine_v, int gbin,
                 hipStream_t s, long tstride = 0) {
  if (G.storage == UMBIR_STORAGE_F16)
    return G.Q == 32 ? launch_corr_mfma16<1, UMBIR_STORAGE_F16>(G, r_v, hq, fine_v, s)
                     : launch_corr_mfma16<2, UMBIR_STORAGE_F16>(G, r_v, hq, fine_v, s);
  if (G.storage == UMBIR_STORAGE_BF16)
    return G.Q == 32 ? launch_corr_mfma16<1, UMBIR_STORAGE_BF16>(G, r_v, hq, fine_v, s)
                     : launch_corr_mfma16<2, UMBIR_STORAGE_BF16>(G, r_v, hq, fine_v, s);
  const float* r = static_cast<const float*>(r_v);
  float* fine = static_cast<float*>(fine_v);
  const long ts = tstride > 0 ? tstride : long(G.fine_per_trace());
  if (G.Q == 32) return launch_corr_mfma<1>(G, r, hq, fine, ts, gbin, s);
  if (G.Q == 64) return launch_corr_mfma<2>(G, r, hq, fine, ts, gbin, s);
  switch (G.Q) {
    case 1: launch_corr_q<1>(G, r, hq, fine, ts, s); break;
    case 2: launch_corr_q<2>(G, r, hq, fine, ts, s); break;
    case 4: launch_corr_q<4>(G, r, hq, fine, ts, s); break;
    case 8: launch_corr_q<8>(G, r, hq, fine, ts, s); break;
    default: launch_corr_q<16>(G, r, hq, fine, ts, s); break;
  }
}

size_t aligned(size_t b) { return (b + 255) & ~size_t(255); }

// Tile of the all-templates splat: one tile per template beside the row
// pointers in the workgroup's LDS, a multiple of 64 positions and at most the
// usual tile; 0 if not even 64 positions per template fit.
int splat_mt_tile(const umbir_geometry& G) {
  const long avail = kSplatLdsBytes - 1024 - long(G.n_seg + 1) * G.nx * long(sizeof(int2));
  const long per = (avail / long(sizeof(unsigned long long)) - 1) / G.n_gamma - 2;
  const long t = std::min<long>(G.tile_bins, per / 64 * 64);
  return t >= 64 ? int(t) : 0;
}

// Dynamic LDS of a splat workgroup: one alignment word, nt tiles of tile + 2
// slots, the row pointers and the column offsets.
size_t splat_lds_bytes(int nt, int tile, const umbir_geometry& G) {
  return (1 + size_t(nt) * (tile + 2)) * sizeof(unsigned long long) + size_t(G.n_seg + 1) * G.nx * sizeof(int2);
}

// blocks of k_prescale, one per 1024 voxels up to kPrescaleBlocks
int prescale_blocks(const umbir_geometry& G) {
  return int(std::min<size_t>(kPrescaleBlocks, (size_t(G.voxels()) + 1023) / 1024));
}

template <bool ABSW, bool WIDE, int ST, bool ATT, bool MT>
void launch_splat_k(const umbir_geometry& G, dim3 grid, const float* xt, int qs, int MQ, const Segments& seg,
                    const unsigned* xmax, int n_xmax, int gbin, void* fine, hipStream_t s, const CostFold& fold) {
  using T = typename Store<ST>::T;
  const int nt = MT ? G.n_gamma : 1;
  const int tile = MT ? splat_mt_tile(G) : G.tile_bins;
  // (with a cost to fold, at least the 256 doubles its sums use)
  const size_t lds = std::max<size_t>(fold.out ? 256 * sizeof(double) : 0, splat_lds_bytes(nt, tile, G));
  UMBIR_LAUNCH("splat", (k_splat<ABSW, WIDE, ST, ATT, MT>), grid, dim3(64 * kSplatWaves), lds, s, xt, G.nx,
               G.nzp, G.n_off, G.legs_t, G.gunit_t, G.base, G.P, G.K, qs, MQ, seg, int(G.chunk_bins), tile, xmax,
               n_xmax, gbin,
               G.n_gamma - 1,
               bin_skip(G, ATT && !MT ? gbin : -1), static_cast<T*>(fine), fold);
}

// ATT: the splat pass of template gbin (attenuation bins, FP32 storage only);
// MT (with ATT): one pass over every template's grid
template <int ST, bool ATT, bool MT = false>
void launch_splat(const umbir_geometry& G, bool abs_op, dim3 grid, const float* xt, int qs, int MQ,
                  const Segments& seg, const unsigned* xmax, int n_xmax, int gbin, void* fine, hipStream_t s,
                  const CostFold* fold = nullptr) {
  const CostFold f = fold ? *fold : CostFold{};
  const bool wide = G.nx * (seg.hi[seg.n - 1] - seg.lo[0]) < kSplatNarrowMin;
  if (abs_op) {
    if (wide) launch_splat_k<true, true, ST, ATT, MT>(G, grid, xt, qs, MQ, seg, xmax, n_xmax, gbin, fine, s, f);
    else launch_splat_k<true, false, ST, ATT, MT>(G, grid, xt, qs, MQ, seg, xmax, n_xmax, gbin, fine, s, f);
  } else {
    if (wide) launch_splat_k<false, true, ST, ATT, MT>(G, grid, xt, qs, MQ, seg, xmax, n_xmax, gbin, fine, s, f);
    else launch_splat_k<false, false, ST, ATT, MT>(G, grid, xt, qs, MQ, seg, xmax, n_xmax, gbin, fine, s, f);
  }
}

template <int ST, bool ATT, bool ONE, bool MULTI>
void launch_gather_k(const umbir_geometry& G, bool abs_op, dim3 grid, int qs, int MQ, int tpg, int t_off,
                     int batch, int vpb, int gbin, int accum, const void* fine, float* partial, hipStream_t s) {
  using T = typename Store<ST>::T;
  constexpr int VPT = 4;
  if (abs_op)
    UMBIR_LAUNCH("gather", (k_gather<true, VPT, ST, ATT, ONE, MULTI>), grid, dim3(256), 0, s,
                 static_cast<const T*>(fine), G.nx, G.nz, G.n_off, G.legs, G.gunit, G.tau, G.base, G.P, G.K, qs, MQ, tpg,
                 t_off, batch, vpb, gbin, G.n_gamma - 1, accum, partial);
  else
    UMBIR_LAUNCH("gather", (k_gather<false, VPT, ST, ATT, ONE, MULTI>), grid, dim3(256), 0, s,
                 static_cast<const T*>(fine), G.nx, G.nz, G.n_off, G.legs, G.gunit, G.tau, G.base, G.P, G.K, qs, MQ, tpg,
                 t_off, batch, vpb, gbin, G.n_gamma - 1, accum, partial);
}

// Does every trace group's range of this launch lie within one scan position?
bool gather_one_scan(const umbir_geometry& G, int tpg, int t_off, int batch) {
  const int PK = G.traces();
  for (int g = 0; g < G.trace_groups; ++g) {
    const int t0 = g * tpg + t_off;
    const int t1 = std::min(t0 + batch, std::min((g + 1) * tpg, PK));
    if (t0 < t1 && t0 / G.K != (t1 - 1) / G.K) return false;
  }
  return true;
}

// The windowed gather (one template, window table built).
template <int ST>
void launch_gather_lds(const umbir_geometry& G, bool abs_op, int qs, int MQ, int tpg, int t_off, int batch,
                       const void* fine, float* partial, hipStream_t s) {
  int tpb;
  const dim3 grid(G.trace_groups, gather_lds_blocks(G.nx, G.nz, G.trace_groups, &tpb));
  const size_t lds = size_t(kGatherWinBytes);
  const auto* f = static_cast<const typename Store<ST>::T*>(fine);
  const bool one = gather_one_scan(G, tpg, t_off, batch);
#define UMBIR_GATHER_LDS(A, O)                                                                                 \
  UMBIR_LAUNCH("gather", (k_gather_lds<A, O, ST>), grid, dim3(512), lds, s, f, G.nx, G.nz, G.n_off, G.legs, G.tau, \
               G.base, G.P, G.K, qs, MQ, tpg, t_off, batch, G.gwin, tpb, partial)
  if (abs_op) {
    if (one) UMBIR_GATHER_LDS(true, true);
    else UMBIR_GATHER_LDS(true, false);
  } else {
    if (one) UMBIR_GATHER_LDS(false, true);
    else UMBIR_GATHER_LDS(false, false);
  }
#undef UMBIR_GATHER_LDS
}

// MULTI: one pass over the resident grids of all templates (see k_gather)
template <int ST, bool ATT, bool MULTI = false>
void launch_gather(const umbir_geometry& G, bool abs_op, dim3 grid, int qs, int MQ, int tpg, int t_off,
                   int batch, int vpb, int gbin, int accum, const void* fine, float* partial, hipStream_t s) {
  if (gather_one_scan(G, tpg, t_off, batch))
    launch_gather_k<ST, ATT, true, MULTI>(G, abs_op, grid, qs, MQ, tpg, t_off, batch, vpb, gbin, accum, fine,
                                          partial, s);
  else
    launch_gather_k<ST, ATT, false, MULTI>(G, abs_op, grid, qs, MQ, tpg, t_off, batch, vpb, gbin, accum, fine,
                                           partial, s);
}


// ---- work-list forms of the sweeps for persistent batches: block b takes
// items b, b + gridDim.x, ...; an item (problem, x, y) runs the block (x, y)
// of that problem's own launch with the problem's arguments, so every problem
// gets bitwise the result of its own launches.  A barrier separates items (a
// block reuses its LDS).

__global__ __launch_bounds__(64 * kSplatWaves) void k_splat_list(const BatchProb* __restrict__ probs,
                                                                 const int* __restrict__ active,
                                                                 const int4* __restrict__ items, int n_items) {
  const BinSkip none{nullptr, 0, 0};
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    if (!active[w.x]) continue;
    const BatchProb& p = probs[w.x];
    if (p.wide)
      splat_body<false, true, UMBIR_STORAGE_F32, false, false>(
          w.y, w.z, p.xt, p.nx, p.nzp, p.n_off, p.legs_t, nullptr, p.base, p.P, p.K, p.qs, p.MQ, p.seg,
          p.chunk_bins, p.tile_bins, p.pmax, p.nblk, 0, 0, none, p.fine);
    else
      splat_body<false, false, UMBIR_STORAGE_F32, false, false>(
          w.y, w.z, p.xt, p.nx, p.nzp, p.n_off, p.legs_t, nullptr, p.base, p.P, p.K, p.qs, p.MQ, p.seg,
          p.chunk_bins, p.tile_bins, p.pmax, p.nblk, 0, 0, none, p.fine);
    __syncthreads();
  }
}

// residual e = y - A x - g D of the iteration
template <int Q>
__global__ __launch_bounds__(64 * kConvMaxWaves) void k_conv_list(const BatchProb* __restrict__ probs, const int* __restrict__ active,
                                                   const int4* __restrict__ items, int n_items) {
  const BinSkip none{nullptr, 0, 0};
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    if (!active[w.x]) continue;
    const BatchProb& p = probs[w.x];
    // the problem's own tile count and products (uniform over the block)
    auto body = [&](auto ntc, auto x3) {
      conv_mfma_body<Q, decltype(ntc)::value, decltype(x3)::value>(w.y, w.z, p.fine, p.h, p.M, p.Lh, p.P * p.K, p.y,
                                                                   -1.0f, p.g, p.dbasis, p.e, long(p.MQ), none,
                                                                   p.conv_waves);
    };
    using T = std::true_type;
    using F = std::false_type;
    if (p.conv_tiles == 1) {
      if (p.conv_split) body(std::integral_constant<int, 1>(), T()); else body(std::integral_constant<int, 1>(), F());
    } else if (p.conv_tiles == 4) {
      if (p.conv_split) body(std::integral_constant<int, 4>(), T()); else body(std::integral_constant<int, 4>(), F());
    } else {
      if (p.conv_split) body(std::integral_constant<int, 2>(), T()); else body(std::integral_constant<int, 2>(), F());
    }
    __syncthreads();
  }
}

template <int QT>
__global__ __launch_bounds__(256) void k_corr_list(const BatchProb* __restrict__ probs, const int* __restrict__ active,
                                                   const int4* __restrict__ items, int n_items) {
  const BinSkip none{nullptr, 0, 0};
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    if (!active[w.x]) continue;
    const BatchProb& p = probs[w.x];
    if (p.corr_split) corr_x3_body<QT>(w.y, w.z, p.e, p.h, p.M, p.Lh, p.corr_per, p.fine, long(p.MQ), none);
    else corr_mfma_body<QT, 2>(w.y, w.z, p.e, p.h, p.M, p.Lh, p.corr_per, p.fine, long(p.MQ), none);
    __syncthreads();
  }
}

// An item is (problem, trace group, voxel block, batch b): block (group,
// voxel block) of the plain path's gather launch b, which covers traces
// [b gbatch, (b + 1) gbatch) of each group and adds to the partial images of
// the launches before it.  Batches run as separate launches, in order.
__global__ __launch_bounds__(256) void k_gather_list(const BatchProb* __restrict__ probs,
                                                     const int* __restrict__ active,
                                                     const int4* __restrict__ items, int n_items) {
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    if (!active[w.x]) continue;
    const BatchProb& p = probs[w.x];
    const int PK = p.P * p.K;
    const int t_off = w.w * p.gbatch;
    const int t0 = w.y * p.tpg + t_off;
    const int t1 = min(t0 + p.gbatch, min((w.y + 1) * p.tpg, PK));
    // the transmit legs are shared when the batch's traces lie in one scan
    // position (the same values either way, so the same result)
    if (t0 < t1 && t0 / p.K == (t1 - 1) / p.K)
      gather_body<false, 4, UMBIR_STORAGE_F32, false, true, false>(
          w.y, w.z, p.fine, p.nx, p.nz, p.n_off, p.legs, nullptr, p.tau, p.base, p.P, p.K, p.qs, p.MQ, p.tpg,
          t_off, p.gbatch, p.vpb, 0, 0, 0, p.partial);
    else
      gather_body<false, 4, UMBIR_STORAGE_F32, false, false, false>(
          w.y, w.z, p.fine, p.nx, p.nz, p.n_off, p.legs, nullptr, p.tau, p.base, p.P, p.K, p.qs, p.MQ, p.tpg,
          t_off, p.gbatch, p.vpb, 0, 0, 0, p.partial);
  }
}

// The windowed gather over a work list: items (problem, trace group, block of
// voxel tiles, batch b) as the problem's own k_gather_lds launch b.
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_gather_lds_list(
    const BatchProb* __restrict__ probs, const int* __restrict__ active, const int4* __restrict__ items, int n_items) {
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    if (!active[w.x]) continue;
    const BatchProb& p = probs[w.x];
    const int PK = p.P * p.K;
    const int t_off = w.w * p.gbatch;
    const int t0 = w.y * p.tpg + t_off;
    const int t1 = min(t0 + p.gbatch, min((w.y + 1) * p.tpg, PK));
    if (t0 < t1 && t0 / p.K == (t1 - 1) / p.K)
      gather_lds_body<false, true>(w.y, w.z, p.fine, p.nx, p.nz, p.n_off, p.legs, p.tau, p.base, p.P, p.K, p.qs,
                                   p.MQ, p.tpg, t_off, p.gbatch, p.gwin, p.vpb, p.partial);
    else
      gather_lds_body<false, false>(w.y, w.z, p.fine, p.nx, p.nz, p.n_off, p.legs, p.tau, p.base, p.P, p.K, p.qs,
                                    p.MQ, p.tpg, t_off, p.gbatch, p.gwin, p.vpb, p.partial);
  }
}

}  // namespace

void plan_sweeps(const umbir_geometry& G, int pi, BatchProb& bp, std::vector<int4>* items, size_t* lds) {
  const int PK = G.traces(), N = G.voxels();
  bp.legs = G.legs;
  bp.legs_t = G.legs_t;
  bp.nzp = G.nzp;
  bp.base = G.base;
  bp.tau = G.tau;
  bp.h = G.h;
  bp.dbasis = G.dbasis;
  bp.dnorm = G.dnorm;
  bp.nx = G.nx;
  bp.nz = G.nz;
  bp.n_off = G.n_off;
  bp.P = G.P;
  bp.K = G.K;
  bp.M = G.M;
  bp.Q = G.Q;
  bp.qs = log2_int(G.Q);
  bp.Lh = G.Lh;
  bp.MQ = int(G.fine_per_trace());
  bp.seg.n = G.n_seg;
  for (int k = 0; k < kMaxLayers; ++k) {
    bp.seg.lo[k] = G.seg_lo[k];
    bp.seg.hi[k] = G.seg_hi[k];
  }
  // splat: as launch_splat_k without attenuation
  bp.chunk_bins = int(G.chunk_bins);
  bp.tile_bins = G.tile_bins;
  bp.wide = G.nx * (G.seg_hi[G.n_seg - 1] - G.seg_lo[0]) < kSplatNarrowMin;
  lds[kStSplat] = std::max(lds[kStSplat], splat_lds_bytes(1, G.tile_bins, G));
  for (int t = 0; t < PK; ++t)
    for (int c = 0; c < G.chunks; ++c) items[kStSplat].push_back(make_int4(pi, c, t, 0));
  // convolution: as launch_conv_mfma (the problem's tile count and order,
  // so its sums run in the order of its own launch)
  bp.conv_tiles = G.conv_tiles;
  bp.conv_split = conv_split(G);
  bp.conv_waves = conv_waves(G);
  bp.corr_split = corr_split(G);
  lds[kStConv] = std::max(lds[kStConv], conv_mfma_lds(G));
  const int mts = (G.M + 32 * G.conv_tiles - 1) / (32 * G.conv_tiles);
  if (G.conv_grid == 2) {
    for (int tx = 0; tx < (PK + 31) / 32; ++tx)
      for (int my = 0; my < mts; ++my) items[kStConv].push_back(make_int4(pi, tx, my, 0));
  } else {
    for (int my = 0; my < mts; ++my)
      for (int tx = 0; tx < (PK + 31) / 32; ++tx) items[kStConv].push_back(make_int4(pi, tx, my, 0));
  }
  // correlation: two 32-row tiles per wave whatever the tuning (the tile
  // shape does not change a result), row blocks per workgroup as tuned
  {
    constexpr int rows = 4 * 2 * 32;
    const int nrb = (G.M + rows - 1) / rows;
    bp.corr_per = std::max(1, int((long(PK) * nrb) / std::max(1, G.corr_blocks)));
    static_assert(rows == kCorrX3Rows, "the split correlation's row block");
    lds[kStCorr] = std::max(lds[kStCorr], size_t(bp.corr_split ? corr_x3_lds_words(G.Q, corr_half(G.Lh))
                                                         : corr_lds_words(G.Q, rows, corr_half(G.Lh))) *
                                              sizeof(float));
    for (int rg = 0; rg < (nrb + bp.corr_per - 1) / bp.corr_per; ++rg)
      for (int t = 0; t < PK; ++t) items[kStCorr].push_back(make_int4(pi, t, rg, 0));
  }
  // gather: as run_adjoint_partial without attenuation, in the problem's
  // gather form
  {
    bp.groups = G.trace_groups;
    bp.tpg = (PK + G.trace_groups - 1) / G.trace_groups;
    bp.gwin = G.gwin;
    const bool windowed = G.gather_form == 2 && G.gwin;
    int nb;
    if (windowed) {
      nb = gather_lds_blocks(G.nx, G.nz, G.trace_groups, &bp.vpb);
      lds[kStGatherW] = std::max(lds[kStGatherW], size_t(kGatherWinBytes));
    } else {
      nb = std::max(1, std::min((N + 1023) / 1024, 1024 / G.trace_groups));
      bp.vpb = (N + nb - 1) / nb;
    }
    const size_t trace_bytes = size_t(bp.MQ) * sizeof(float);
    bp.gbatch = int(std::max<size_t>(1, std::min<size_t>(bp.tpg, (size_t(G.gather_batch_kb) << 10) / trace_bytes)));
    const int batches = (bp.tpg + bp.gbatch - 1) / bp.gbatch;
    const int stage = windowed ? kStGatherW : kStGather;
    for (int b = 0; b < batches; ++b)
      for (int vb = 0; vb < nb; ++vb)
        for (int gr = 0; gr < G.trace_groups; ++gr) items[stage].push_back(make_int4(pi, gr, vb, b));
  }
}

int launch_sweep_stage(int stage, int Q, const BatchProb* probs, const int* active, const StageLaunch& L, int which,
                       hipStream_t s) {
  if (L.n_items == 0) return UMBIR_OK;
  const dim3 grid(unsigned(L.grid));
  switch (stage) {
    case kStSplat:
      UMBIR_LAUNCH("splat", k_splat_list, grid, dim3(64 * kSplatWaves), L.lds, s, probs, active, L.items, L.n_items);
      break;
    case kStConv:
      if (Q == 32)
        UMBIR_LAUNCH("conv", k_conv_list<32>, grid, dim3(64 * kConvMaxWaves), L.lds, s, probs, active, L.items,
                     L.n_items);
      else
        UMBIR_LAUNCH("conv", k_conv_list<64>, grid, dim3(64 * kConvMaxWaves), L.lds, s, probs, active, L.items,
                     L.n_items);
      break;
    case kStCorr:
      if (Q == 32) UMBIR_LAUNCH("corr", k_corr_list<1>, grid, dim3(256), L.lds, s, probs, active, L.items, L.n_items);
      else UMBIR_LAUNCH("corr", k_corr_list<2>, grid, dim3(256), L.lds, s, probs, active, L.items, L.n_items);
      break;
    case kStGather:
      UMBIR_LAUNCH("gather", k_gather_list, grid, dim3(256), L.lds, s, probs, active, L.items, L.n_items);
      break;
    case kStGatherW:
      UMBIR_LAUNCH("gather", k_gather_lds_list, grid, dim3(512), L.lds, s, probs, active, L.items, L.n_items);
      break;
    default: return fail(UMBIR_EINVAL, "not a sweep stage");
  }
  return check_hip(hipGetLastError(), "work-list sweep");
}

int launch_fill(float* p, size_t n, float v, hipStream_t s) {
  UMBIR_LAUNCH("fill", k_fill, dim3(grid_1d(n / 4 + 1)), dim3(256), 0, s, p, n, v);
  return check_hip(hipGetLastError(), "k_fill");
}

int launch_copy(float* dst, const float* src, size_t n, hipStream_t s) {
  UMBIR_LAUNCH("copy", k_copy, dim3(grid_1d(n)), dim3(256), 0, s, dst, src, n);
  return check_hip(hipGetLastError(), "k_copy");
}

size_t forward_work_bytes(const umbir_geometry& G) { return aligned(G.fine_bytes()) + 256; }

size_t adjoint_work_bytes(const umbir_geometry& G) {
  return forward_work_bytes(G) + aligned(size_t(G.trace_groups) * G.voxels() * sizeof(float)) + 256;
}

int log2_int(int q) {
  int k = 0;
  while ((1 << k) < q) ++k;
  return k;
}


bool direct_eligible(const umbir_geometry& G) {
  return G.storage == UMBIR_STORAGE_F32 && G.n_gamma == 1 && direct_fwd_lds(G) <= 65536;
}

int run_prescale_blocks(const umbir_geometry& G, const float* x, void* fine, unsigned* maxima, int blocks,
                        hipStream_t s) {
  float* xt = reinterpret_cast<float*>(static_cast<char*>(fine) + G.grids_bytes());
  UMBIR_LAUNCH("prescale", k_prescale, dim3(unsigned(blocks)), dim3(64), 0, s, x, G.tau, G.nx, G.nzp, G.voxels(),
               xt, maxima);
  return check_hip(hipGetLastError(), "k_prescale");
}

int run_forward(const umbir_geometry& G, const float* x, void* out, const void* base, float sign,
                const float* g, bool abs_op, void* fine, hipStream_t s, const unsigned* pre_max, int n_pre_max,
                const CostFold* fold) {
  // after the fine grid(s): the prescaled image tau x, then one 32-bit
  // scalar, the largest |tau x|
  float* xt = reinterpret_cast<float*>(static_cast<char*>(fine) + G.grids_bytes());
  unsigned* xmax = reinterpret_cast<unsigned*>(static_cast<char*>(fine) + G.fine_bytes() - 4 * kPrescaleBlocks);
  int n_xmax = prescale_blocks(G);
  const int MQ = int(G.fine_per_trace());
  const int qs = log2_int(G.Q);
  Segments seg;
  seg.n = G.n_seg;
  for (int k = 0; k < kMaxLayers; ++k) {
    seg.lo[k] = G.seg_lo[k];
    seg.hi[k] = G.seg_hi[k];
  }
  if (pre_max) {  // tau x is in place, its maxima given
    xmax = const_cast<unsigned*>(pre_max);
    n_xmax = n_pre_max;
  } else {
    UMBIR_LAUNCH("prescale", k_prescale, dim3(prescale_blocks(G)), dim3(1024), 0, s, x, G.tau, G.nx, G.nzp,
                 G.voxels(), xt, xmax);
  }
  dim3 grid(G.chunks, G.traces());
  if (G.form == 2) {  // the direct form (FP32, one template; see direct_eligible)
    if (fold) {
      UMBIR_LAUNCH("cost", k_fold_cost, dim3(1), dim3(256), 0, s, *fold);
      const int st = check_hip(hipGetLastError(), "k_fold_cost");
      if (st) return st;
    }
    const bool wide = G.voxels() < kSplatNarrowMin;
    const size_t lds = direct_fwd_lds(G);
    const float* yb = static_cast<const float*>(base);
    float* yo = static_cast<float*>(out);
    if (abs_op) {
      if (wide)
        UMBIR_LAUNCH("fwd_direct", (k_fwd_direct<true, true>), dim3(G.traces()), dim3(1024), lds, s, xt, G.nx, G.nz, G.nzp,
                     G.n_off, G.legs, G.base, G.P, G.K, qs, G.Lh, G.M, G.bank, xmax, n_xmax, yb, sign, g,
                     G.dbasis, yo);
      else
        UMBIR_LAUNCH("fwd_direct", (k_fwd_direct<true, false>), dim3(G.traces()), dim3(1024), lds, s, xt, G.nx, G.nz, G.nzp,
                     G.n_off, G.legs, G.base, G.P, G.K, qs, G.Lh, G.M, G.bank, xmax, n_xmax, yb, sign, g,
                     G.dbasis, yo);
    } else {
      if (wide)
        UMBIR_LAUNCH("fwd_direct", (k_fwd_direct<false, true>), dim3(G.traces()), dim3(1024), lds, s, xt, G.nx, G.nz, G.nzp,
                     G.n_off, G.legs, G.base, G.P, G.K, qs, G.Lh, G.M, G.bank, xmax, n_xmax, yb, sign, g,
                     G.dbasis, yo);
      else
        UMBIR_LAUNCH("fwd_direct", (k_fwd_direct<false, false>), dim3(G.traces()), dim3(1024), lds, s, xt, G.nx,
                     G.nz, G.nzp, G.n_off, G.legs, G.base, G.P, G.K, qs, G.Lh, G.M, G.bank, xmax, n_xmax, yb,
                     sign, g, G.dbasis, yo);
    }
    return check_hip(hipGetLastError(), "k_fwd_direct");
  }
  if (G.multi_grid() && splat_mt_tile(G) > 0) {
    // attenuation with every template's grid resident: one splat walk fills
    // them all ([template][trace][position]), then one convolution per
    // template; later ones add to the traces the first one wrote
    launch_splat<UMBIR_STORAGE_F32, true, true>(G, abs_op, grid, xt, qs, MQ, seg, xmax, n_xmax, 0, fine, s, fold);
    int st = check_hip(hipGetLastError(), "k_splat");
    if (st) return st;
    for (int gb = 0; gb < G.n_gamma; ++gb) {
      const float* taps = (abs_op ? G.habs : G.h) + size_t(gb) * G.taps_per_bin();
      launch_conv(G, static_cast<float*>(fine) + size_t(gb) * G.traces() * MQ, taps, gb == 0 ? base : out, sign,
                  gb == 0 ? g : nullptr, out, gb, s);
      if ((st = check_hip(hipGetLastError(), "k_conv"))) return st;
    }
    return UMBIR_OK;
  }
  // one splat + convolution per attenuation template (one without
  // attenuation); later passes add to the traces the first one wrote
  for (int gb = 0; gb < G.n_gamma; ++gb) {
    const CostFold* fold_here = gb == 0 ? fold : nullptr;
    switch (G.storage) {
      case UMBIR_STORAGE_F16:
        launch_splat<UMBIR_STORAGE_F16, false>(G, abs_op, grid, xt, qs, MQ, seg, xmax, n_xmax, 0, fine, s,
                                               fold_here);
        break;
      case UMBIR_STORAGE_BF16:
        launch_splat<UMBIR_STORAGE_BF16, false>(G, abs_op, grid, xt, qs, MQ, seg, xmax, n_xmax, 0, fine, s,
                                                fold_here);
        break;
      default:
        if (G.n_gamma > 1)
          launch_splat<UMBIR_STORAGE_F32, true>(G, abs_op, grid, xt, qs, MQ, seg, xmax, n_xmax, gb, fine, s,
                                                fold_here);
        else
          launch_splat<UMBIR_STORAGE_F32, false>(G, abs_op, grid, xt, qs, MQ, seg, xmax, n_xmax, 0, fine, s,
                                                 fold_here);
        break;
    }
    int st = check_hip(hipGetLastError(), "k_splat");
    if (st) return st;
    const float* taps = (abs_op ? G.habs : G.h) + size_t(gb) * G.taps_per_bin();
    launch_conv(G, fine, taps, gb == 0 ? base : out, sign, gb == 0 ? g : nullptr, out, G.n_gamma > 1 ? gb : -1, s);
    if ((st = check_hip(hipGetLastError(), "k_conv"))) return st;
  }
  return UMBIR_OK;
}

int run_adjoint_partial(const umbir_geometry& G, const void* r, bool abs_op, void* fine, float* partial,
                        hipStream_t s) {
  const int MQ = int(G.fine_per_trace());
  const int qs = log2_int(G.Q);
  const int tpg = (G.traces() + G.trace_groups - 1) / G.trace_groups;
  // one generation: at most 1024 blocks (four per CU), chunks of 256 * 4 voxels
  const int chunk = 256 * 4;
  int nb = (G.voxels() + chunk - 1) / chunk;
  nb = std::max(1, std::min(nb, 1024 / G.trace_groups));
  const int vpb = (G.voxels() + nb - 1) / nb;
  dim3 grid(G.trace_groups, nb);
  if (G.form == 2) {  // the direct form: every trace of a group in one pass
    const size_t lds = (size_t(G.Q) * G.Lh + 2) * sizeof(float);
    const float* rr = static_cast<const float*>(r);
    if (abs_op)
      UMBIR_LAUNCH("adj_direct", (k_adj_direct<true, 4>), grid, dim3(256), lds, s, rr, G.nx, G.nz, G.n_off, G.legs,
                   G.tau, G.base, G.P, G.K, qs, G.Lh, G.M, G.bank, tpg, vpb, partial);
    else
      UMBIR_LAUNCH("adj_direct", (k_adj_direct<false, 4>), grid, dim3(256), lds, s, rr, G.nx, G.nz, G.n_off, G.legs,
                   G.tau, G.base, G.P, G.K, qs, G.Lh, G.M, G.bank, tpg, vpb, partial);
    return check_hip(hipGetLastError(), "k_adj_direct");
  }
  // traces per launch: batches of gather_batch_kb of fine-grid data per group
  // (4 MiB by default, one XCD's L2: the autotuner's choice on the 256 x 256
  // and 512 x 512 workloads, 1-2 % faster per reconstruction than 8 MiB and
  // 3-5 % faster than 2 MiB)
  const bool multi = G.multi_grid();
  // (with every template's grid resident a pair still reads one grid: the
  // batch is sized by one grid per trace)
  const size_t trace_bytes = size_t(MQ) * G.elem();
  const int batch =
      int(std::max<size_t>(1, std::min<size_t>(tpg, (size_t(G.gather_batch_kb) << 10) / trace_bytes)));
  int st = UMBIR_OK;
  if (multi) {
    // attenuation with every template's grid resident: one correlation per
    // template into its own grid ([trace][template][position]), then one
    // gather in which every pair reads its own template's grid
    const long tstride = long(G.n_gamma) * MQ;
    for (int gb = 0; gb < G.n_gamma; ++gb) {
      launch_corr(G, r, (abs_op ? G.habs : G.h) + size_t(gb) * G.taps_per_bin(),
                  static_cast<float*>(fine) + size_t(gb) * MQ, gb, s, tstride);
      if ((st = check_hip(hipGetLastError(), "k_corr"))) return st;
    }
    for (int t_off = 0; t_off < tpg; t_off += batch)
      launch_gather<UMBIR_STORAGE_F32, true, true>(G, abs_op, grid, qs, MQ, tpg, t_off, batch, vpb, 0, 0, fine,
                                                   partial, s);
    return check_hip(hipGetLastError(), "k_gather");
  }
  // one correlation + gather per attenuation template (one without
  // attenuation); later passes add to the partial images
  for (int gb = 0; gb < G.n_gamma; ++gb) {
    launch_corr(G, r, (abs_op ? G.habs : G.h) + size_t(gb) * G.taps_per_bin(), fine, G.n_gamma > 1 ? gb : -1, s);
    if ((st = check_hip(hipGetLastError(), "k_corr"))) return st;
    const int accum = gb > 0;
    for (int t_off = 0; t_off < tpg; t_off += batch) {
      switch (G.storage) {
        case UMBIR_STORAGE_F16:
          if (G.gather_form == 2 && G.gwin)
            launch_gather_lds<UMBIR_STORAGE_F16>(G, abs_op, qs, MQ, tpg, t_off, batch, fine, partial, s);
          else
            launch_gather<UMBIR_STORAGE_F16, false>(G, abs_op, grid, qs, MQ, tpg, t_off, batch, vpb, 0, 0, fine,
                                                    partial, s);
          break;
        case UMBIR_STORAGE_BF16:
          if (G.gather_form == 2 && G.gwin)
            launch_gather_lds<UMBIR_STORAGE_BF16>(G, abs_op, qs, MQ, tpg, t_off, batch, fine, partial, s);
          else
            launch_gather<UMBIR_STORAGE_BF16, false>(G, abs_op, grid, qs, MQ, tpg, t_off, batch, vpb, 0, 0, fine,
                                                     partial, s);
          break;
        default:
          if (G.n_gamma > 1)
            launch_gather<UMBIR_STORAGE_F32, true>(G, abs_op, grid, qs, MQ, tpg, t_off, batch, vpb, gb, accum,
                                                   fine, partial, s);
          else if (G.gather_form == 2 && G.gwin)
            launch_gather_lds<UMBIR_STORAGE_F32>(G, abs_op, qs, MQ, tpg, t_off, batch, fine, partial, s);
          else
            launch_gather<UMBIR_STORAGE_F32, false>(G, abs_op, grid, qs, MQ, tpg, t_off, batch, vpb, 0, 0, fine,
                                                    partial, s);
          break;
      }
    }
    if ((st = check_hip(hipGetLastError(), "k_gather"))) return st;
  }
  return UMBIR_OK;
}

int run_adjoint(const umbir_geometry& G, const void* r, float* out, float scale, bool abs_op,
                void* fine, float* partial, hipStream_t s) {
  int st = run_adjoint_partial(G, r, abs_op, fine, partial, s);
  if (st) return st;
  UMBIR_LAUNCH("reduce_groups", k_reduce_groups, dim3((G.voxels() + 255) / 256), dim3(256), 0, s, partial,
               G.trace_groups, G.voxels(), scale, out);
  return check_hip(hipGetLastError(), "k_reduce_groups");
}

int launch_direct(const umbir_geometry& G, const float* g, void* y, int accumulate, hipStream_t s) {
  const size_t total = size_t(G.traces()) * G.M;
  switch (G.storage) {
    case UMBIR_STORAGE_F16:
      UMBIR_LAUNCH("direct", k_direct<UMBIR_STORAGE_F16>, dim3(grid_1d(total)), dim3(256), 0, s, g, G.dbasis, G.M,
                   total, accumulate, static_cast<Store<UMBIR_STORAGE_F16>::T*>(y));
      break;
    case UMBIR_STORAGE_BF16:
      UMBIR_LAUNCH("direct", k_direct<UMBIR_STORAGE_BF16>, dim3(grid_1d(total)), dim3(256), 0, s, g, G.dbasis,
                   G.M, total, accumulate, static_cast<Store<UMBIR_STORAGE_BF16>::T*>(y));
      break;
    default:
      UMBIR_LAUNCH("direct", k_direct<UMBIR_STORAGE_F32>, dim3(grid_1d(total)), dim3(256), 0, s, g, G.dbasis, G.M,
                   total, accumulate, static_cast<float*>(y));
      break;
  }
  return check_hip(hipGetLastError(), "k_direct");
}

}  // namespace umbir

using namespace umbir;

extern "C" {

size_t umbir_workspace_bytes(const umbir_geometry* G, int kind) {
  if (!G) return 0;
  switch (kind) {
    case UMBIR_WORK_FORWARD: return forward_work_bytes(*G);
    case UMBIR_WORK_ADJOINT: return adjoint_work_bytes(*G);
    case UMBIR_WORK_RECONSTRUCT: {
      // the iteration buffers (fine grid, partial images of A^T e, residual,
      // curvature, reductions) plus the two images of the ping-pong
      const size_t N = G->voxels(), PK = G->traces();
      const size_t nblk = (N + kPriorVox - 1) / kPriorVox + 1;
      // + the prior update's per-block image maxima and its arrival counter
      return adjoint_work_bytes(*G) + aligned(G->trace_bytes()) + 3 * aligned(N * sizeof(float)) +
             aligned(PK * sizeof(double)) + aligned(nblk * sizeof(double)) + aligned(nblk * sizeof(unsigned)) +
             256 + 16 * 256;
    }
    default: return 0;
  }
}

int umbir_forward(const umbir_geometry* G, const float* x, void* y, int accumulate, void* work,
                  size_t work_bytes, void* stream) {
  if (!G || !x || !y) return fail(UMBIR_EINVAL, "NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws;
  int st = ws.acquire(work, work_bytes, forward_work_bytes(*G), s);
  if (st) return st;
  Carve cv{static_cast<char*>(ws.ptr)};
  void* fine = cv.take<char>(G->fine_bytes());
  return run_forward(*G, x, y, accumulate ? y : nullptr, 1.0f, nullptr, false, fine, s);
}

int umbir_adjoint(const umbir_geometry* G, const void* r, float* x, void* work, size_t work_bytes,
                  void* stream) {
  if (!G || !r || !x) return fail(UMBIR_EINVAL, "NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws;
  int st = ws.acquire(work, work_bytes, adjoint_work_bytes(*G), s);
  if (st) return st;
  Carve cv{static_cast<char*>(ws.ptr)};
  void* fine = cv.take<char>(G->fine_bytes());
  float* partial = cv.take<float>(size_t(G->trace_groups) * G->voxels());
  return run_adjoint(*G, r, x, 1.0f, false, fine, partial, s);
}

int umbir_direct(const umbir_geometry* G, const float* g, void* y, int accumulate, void* stream) {
  if (!G || !g || !y) return fail(UMBIR_EINVAL, "NULL argument");
  return launch_direct(*G, g, y, accumulate, static_cast<hipStream_t>(stream));
}

int umbir_sqs_denominator(const umbir_geometry* G, double sigma, float* d, void* work,
                          size_t work_bytes, void* stream) {
  if (!G || !d) return fail(UMBIR_EINVAL, "NULL argument");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(UMBIR_EINVAL, "sigma must be > 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t need = adjoint_work_bytes(*G) + aligned(G->trace_bytes()) + 256;
  Workspace ws;
  int st = ws.acquire(work, work_bytes, need, s);
  if (st) return st;
  Carve cv{static_cast<char*>(ws.ptr)};
  void* fine = cv.take<char>(G->fine_bytes());
  float* partial = cv.take<float>(size_t(G->trace_groups) * G->voxels());
  void* col = cv.take<char>(G->trace_bytes());
  if ((st = run_forward(*G, nullptr, col, nullptr, 1.0f, nullptr, true, fine, s))) return st;
  return run_adjoint(*G, col, d, float(1.0 / (sigma * sigma)), true, fine, partial, s);
}

int umbir_autotune(umbir_geometry* G, void* stream, umbir_tuning* chosen) {
  if (!G) return fail(UMBIR_EINVAL, "NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t wb = adjoint_work_bytes(*G), tb = aligned(G->trace_bytes());
  Workspace ws;
  int st = ws.acquire(nullptr, 0, wb + tb + aligned(size_t(G->voxels()) * sizeof(float)), s);
  if (st) return st;
  Carve cv{static_cast<char*>(ws.ptr)};
  void* fine = cv.take<char>(G->fine_bytes());
  float* partial = cv.take<float>(size_t(G->trace_groups) * G->voxels());
  char* traces = static_cast<char*>(ws.ptr) + wb;
  float* img = reinterpret_cast<float*>(traces + tb);
  if ((st = check_hip(hipMemsetAsync(traces, 0, G->trace_bytes(), s), "hipMemsetAsync"))) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((st = check_hip(hipEventCreate(&e0), "hipEventCreate")) || (st = check_hip(hipEventCreate(&e1), "hipEventCreate"))) {
    if (e0) (void)hipEventDestroy(e0);
    return st;
  }
  // average of three runs after one warm-up; the image is all ones (x = NULL)
  auto time_ms = [&](auto&& run, float* ms) {
    int r = run();
    if (!r) r = check_hip(hipEventRecord(e0, s), "hipEventRecord");
    for (int k = 0; k < 3 && !r; ++k) r = run();
    if (!r) r = check_hip(hipEventRecord(e1, s), "hipEventRecord");
    if (!r) r = check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
    if (!r) r = check_hip(hipEventElapsedTime(ms, e0, e1), "hipEventElapsedTime");
    *ms /= 3.0f;
    return r;
  };
  auto forward = [&]() { return run_forward(*G, nullptr, traces, nullptr, 1.0f, nullptr, false, fine, s); };
  auto adjoint = [&]() { return run_adjoint(*G, traces, img, 1.0f, false, fine, partial, s); };
  // the operator's form: factored (splat + convolution, correlation +
  // gather) or direct, for an A + A^T pair with the current launch shapes
  if (direct_eligible(*G)) {
    int best_form = G->form;
    float best_pair = 3.4e38f;
    for (int f : {1, 2}) {
      G->form = f;
      float ms = 0.0f;
      if ((st = time_ms([&]() {
             int r = forward();
             return r ? r : adjoint();
           }, &ms)))
        break;
      if (ms < best_pair) { best_pair = ms; best_form = f; }
    }
    G->form = best_form;
  }
  // the splat: one to four chunks per trace, and fixed workgroup targets
  const long PK = G->traces();
  std::vector<long> cand = {PK, 2 * PK, 4 * PK, 1024, 2048, 4096};
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  long best_blocks = G->splat_blocks;
  float best = 3.4e38f;
  for (long c : cand) {
    apply_splat_blocks(G, c);
    float ms = 0.0f;
    if ((st = time_ms(forward, &ms))) break;
    if (ms < best) { best = ms; best_blocks = c; }
  }
  apply_splat_blocks(G, best_blocks);
  // the matrix-core convolution's output tiles per workgroup and tile order
  // (FP32, Q of 32 or 64)
  if (!st && G->storage == UMBIR_STORAGE_F32 && (G->Q == 32 || G->Q == 64)) {
    int best_grid = G->conv_grid, best_tiles = G->conv_tiles;
    best = 3.4e38f;
    for (int nt : {1, 2, 4}) {
      for (int cg : {1, 2}) {
        G->conv_tiles = nt;
        G->conv_grid = cg;
        float ms = 0.0f;
        if ((st = time_ms(forward, &ms))) break;
        if (ms < best) { best = ms; best_grid = cg; best_tiles = nt; }
      }
      if (st) break;
    }
    G->conv_grid = best_grid;
    G->conv_tiles = best_tiles;
  }
  // the matrix-core correlation's tile rows per wave (FP32 products only:
  // the bf16-piece form has one tile shape) and workgroup count
  if (!st && G->storage == UMBIR_STORAGE_F32 && (G->Q == 32 || G->Q == 64)) {
    int best_t = G->corr_tiles, best_b = G->corr_blocks;
    best = 3.4e38f;
    const bool one_shape = corr_split(*G);
    for (int t : {1, 2, 4}) {
      if (one_shape && t != best_t) continue;
      for (int nb : {512, 1024, 2048}) {
        G->corr_tiles = t;
        G->corr_blocks = nb;
        float ms = 0.0f;
        if ((st = time_ms(adjoint, &ms))) break;
        if (ms < best) { best = ms; best_t = t; best_b = nb; }
      }
      if (st) break;
    }
    G->corr_tiles = best_t;
    G->corr_blocks = best_b;
  }
  // the gather: its form (row-wise, or windowed where the table exists) and
  // fine-grid KiB per trace group and launch
  int best_kb = G->gather_batch_kb, best_gf = G->gather_form;
  best = 3.4e38f;
  for (int gf = 1; gf <= (G->gwin ? 2 : 1); ++gf)
    for (int kb : {2048, 4096, 8192, 16384, 32768}) {
      if (st) break;
      G->gather_form = gf;
      G->gather_batch_kb = kb;
      float ms = 0.0f;
      if ((st = time_ms(adjoint, &ms))) break;
      if (ms < best) { best = ms; best_kb = kb; best_gf = gf; }
    }
  G->gather_batch_kb = best_kb;
  G->gather_form = best_gf;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  if (chosen) {
    chosen->splat_blocks = G->splat_blocks;
    chosen->gather_batch_kb = G->gather_batch_kb;
    chosen->conv_grid = G->conv_grid;
    chosen->conv_tile_rows = 32 * G->conv_tiles;
    chosen->corr_tile_rows = 32 * G->corr_tiles;
    chosen->corr_blocks = G->corr_blocks;
    chosen->operator_form = G->form;
    chosen->products = G->split ? 2 : 1;
    chosen->gather_form = G->gather_form;
  }
  return UMBIR_OK;
}

}  // extern "C"
