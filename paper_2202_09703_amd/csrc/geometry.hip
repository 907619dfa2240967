// Geometry build: validation, FP64 Snell leg table, tabulated pulse and the
// direct-arrival basis, plus the handle, error and workspace plumbing.
//
// Legs (Sec. 2, Eqs. (4)-(6)).  A one-way path from a point on the array face
// to a voxel centre at depth z and lateral distance X crosses layer l over a
// vertical extent eta_l.  Snell's law keeps sin(theta_l)/c_l equal to one ray
// parameter kappa, and the lateral offset of Eq. (5),
//     X(kappa) = sum_l eta_l kappa c_l / sqrt(1 - kappa^2 c_l^2),
// increases with kappa, so kappa is found by binary search, as the paper does
// for the incidence angle.  The search runs on kappa in [0, 1/c_max) with c_max
// the fastest crossed layer: the paper's range theta_1 in [0, pi/2] reaches
// past the critical angle of any faster deeper layer, where Eq. (6) has no
// solution, whereas every X >= 0 has a kappa in [0, 1/c_max).
// The travel time is evaluated as T = kappa X + sum_l eta_l cos(theta_l)/c_l,
// which equals sum_l eta_l / (c_l cos theta_l) of Eq. (4) at the exact root and
// is stationary in kappa there, so the last-bit error of the search does not
// reach T to first order.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "internal.h"

namespace umbir {

namespace {
thread_local std::string g_last_error;

constexpr int kBisectSteps = 60;

// One leg per thread: the Snell ray parameter kappa = sin(theta_l) / c_l by
// bisection on the lateral offset it reaches (Eqs. (5)-(6)), then the travel
// time (Eq. (4)), cos^beta of the angle sum (Eq. (12)) and, when `gam` is not
// NULL, the path attenuation sum_l alpha_l eta_l / cos(theta_l) (gamma_l of
// Eq. (3) summed over the leg's layers).
__global__ void k_legs(Layers L, int nz, int n_off, double z0, double dz, double half_dx,
                       double fs, int beta, Leg* __restrict__ legs, int nzp, Leg* __restrict__ legs_t, int qs,
                       double* __restrict__ gam) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nz * n_off) return;
  const int row = idx / n_off;
  const int slot = idx - row * n_off;
  const int half = n_off / 2;
  const int o = slot < half ? 2 * slot : 2 * (slot - half) + 1;
  const double z = z0 + (row + 0.5) * dz;
  const double X = o * half_dx;
  double eta[kMaxLayers];
  double cmax = 0.0;
#pragma unroll
  for (int l = 0; l < kMaxLayers; ++l) {
    double e = 0.0;
    if (l < L.n) {
      e = fmin(z, L.bottom[l]) - L.top[l];
      e = e > 0.0 ? e : 0.0;
      if (e > 0.0) cmax = fmax(cmax, L.speed[l]);
    }
    eta[l] = e;
  }
  double kap = 0.0;
  if (X > 0.0) {
    double lo = 0.0, hi = 1.0 / cmax;
    for (int it = 0; it < kBisectSteps; ++it) {
      const double mid = 0.5 * (lo + hi);
      double xm = 0.0;
#pragma unroll
      for (int l = 0; l < kMaxLayers; ++l) {
        if (eta[l] > 0.0) {
          const double s = mid * L.speed[l];
          xm += eta[l] * s / sqrt((1.0 - s) * (1.0 + s));
        }
      }
      if (xm < X) lo = mid; else hi = mid;
    }
    kap = 0.5 * (lo + hi);
  }
  double T = kap * X;
  double theta = 0.0, att = 0.0;
#pragma unroll
  for (int l = 0; l < kMaxLayers; ++l) {
    if (eta[l] > 0.0) {
      const double s = kap * L.speed[l];
      const double cv = sqrt((1.0 - s) * (1.0 + s));
      T += eta[l] * cv / L.speed[l];
      theta += asin(s);
      att += L.atten[l] * eta[l] / cv;
    }
  }
  // cos^beta by repeated squaring (beta is a non-negative integer)
  double base = cos(theta), pw = 1.0;
  for (int b = beta; b > 0; b >>= 1) {
    if (b & 1) pw *= base;
    base *= base;
  }
  Leg rec;
  rec.delay = __double2ll_rn(fs * T * kTwo32);
  rec.apod = static_cast<float>(pw);
  rec.spare = 0;
  legs[idx] = rec;
  // the position-major copy (the splat's) holds the delay in fine positions:
  // times Q = 2^qs, exact (travel times stay far below 2^(31 - qs) samples)
  rec.delay = int64_t(uint64_t(rec.delay) << qs);
  legs_t[size_t(slot) * nzp + row] = rec;
  if (gam) gam[idx] = att;
}

// Leg attenuation in template bins: Gamma / dgamma (float64), in the legs'
// layout and in the transposed one of legs_t.
__global__ void k_leg_units(int n, int n_off, int nzp, const double* __restrict__ gam, double step,
                            double* __restrict__ gunit, double* __restrict__ gunit_t) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const double u = gam[idx] / step;
  const int row = idx / n_off, slot = idx - row * n_off;
  gunit[idx] = u;
  gunit_t[size_t(slot) * nzp + row] = u;
}

// Windowed pulse of Eq. (10) at fine-grid index n (time n / (Q fs)): the
// Gaussian-windowed sine, zero outside the open window 0 < n < Q L_h.
__device__ double pulse_at(long n, int QLh, double dt, double f_c, double inv2s2, double t_c) {
  if (n <= 0 || n >= QLh) return 0.0;
  const double u = n * dt - t_c;
  return sin(2.0 * M_PI * f_c * u) * exp(-u * u * inv2s2);
}

__global__ void k_bank(int Q, int Lh, double dt, double f_c, double inv2s2, double t_c,
                       float* __restrict__ bank, float* __restrict__ h,
                       float* __restrict__ habs) {
  const int QLh = Q * Lh;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < QLh + 2) bank[idx] = static_cast<float>(pulse_at(idx, QLh, dt, f_c, inv2s2, t_c));
  if (idx < QLh) {
    const int k = idx / Q, t = idx - k * Q;
    const float v = static_cast<float>(pulse_at(long(k + 1) * Q - t, QLh, dt, f_c, inv2s2, t_c));
    h[idx] = v;
    habs[idx] = fabsf(v);
  }
}

// Attenuated templates g = 1 .. n_gamma - 1 (Eqs. (9)-(10)): with S the
// spectrum of the Gaussian-windowed sine, h(gamma, t) = int_0^inf
// [G(f - f_c) - G(f + f_c)] e^{-gamma f} sin(2 pi f (t - t_c)) df, G the
// spectrum of the Gaussian.  `nodes` holds the quadrature: frequencies f_k,
// then amplitudes w_k [G(f_k - f_c) - G(f_k + f_c)].  Row g of the bank (stride
// Q L_h + 2) is written at the fine indices n = 0 .. Q L_h + 1, zero outside
// the open window.
__global__ void k_bank_att(int QLh, double dt, double t_c, double step, int n_nodes,
                           const double* __restrict__ nodes, float* __restrict__ bank) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = blockIdx.y + 1;
  if (n >= QLh + 2) return;
  double acc = 0.0;
  if (n > 0 && n < QLh) {
    const double gamma = g * step;
    const double w = 2.0 * M_PI * (n * dt - t_c);
    for (int k = 0; k < n_nodes; ++k) {
      const double f = nodes[k];
      acc += nodes[n_nodes + k] * exp(-gamma * f) * sin(w * f);
    }
  }
  bank[size_t(g) * (QLh + 2) + n] = static_cast<float>(acc);
}

// Polyphase taps of bank rows g0 .. G-1: h_t[k] = b[(k + 1) Q - t], and |h|.
__global__ void k_polyphase(int Q, int Lh, int g0, int G, const float* __restrict__ bank, float* __restrict__ h,
                            float* __restrict__ habs) {
  const int QLh = Q * Lh;
  const long idx = long(blockIdx.x) * blockDim.x + threadIdx.x + long(g0) * QLh;
  if (idx >= long(G) * QLh) return;
  const int g = int(idx / QLh), r = int(idx - long(g) * QLh);
  const int k = r / Q, t = r - k * Q;
  const float v = bank[size_t(g) * (QLh + 2) + size_t(k + 1) * Q - t];
  h[idx] = v;
  habs[idx] = fabsf(v);
}

// Template occupancy: for trace blockIdx.x and voxel v, the template of the
// pair marks the blocks of its fine positions J and J + 1 (the splat puts its
// weight on both).  A block ORs the marks of its voxels (every gridDim.y-th
// run of blockDim.x) into its own copy of the trace's mask row in LDS (nb
// words of dynamic LDS), then ORs the row's nonzero words into memory: one
// global atomic per word and block instead of one per pair.
__global__ void k_bin_mask(const Leg* __restrict__ legs, const double* __restrict__ gunit, int n_off,
                           const int* __restrict__ base, int P, int K, int nx, int N, int qs, long MQ, int last, int nb,
                           unsigned long long* __restrict__ mask) {
  extern __shared__ unsigned long long row_mask[];  // [nb]
  const int t = blockIdx.x;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) row_mask[i] = 0ull;
  __syncthreads();
  const int half = n_off / 2;
  const int bt = base[t / K], br = base[P + t];
  for (int v = blockIdx.y * blockDim.x + threadIdx.x; v < N; v += gridDim.y * blockDim.x) {
    const int row = v / nx, col = v - row * nx;
    const size_t ka = size_t(row) * n_off + leg_slot(abs(bt + 2 * col), half);
    const size_t kb = size_t(row) * n_off + leg_slot(abs(br + 2 * col), half);
    const uint64_t D = uint64_t(legs[ka].delay + legs[kb].delay);
    const long J = long(D >> (32 - qs));
    const unsigned long long bit = 1ull << gamma_bin(gunit[ka] + gunit[kb], last);
    if (J < MQ) atomicOr(&row_mask[J >> kMaskShift], bit);
    if (J + 1 < MQ && ((J + 1) >> kMaskShift) != (J >> kMaskShift)) atomicOr(&row_mask[(J + 1) >> kMaskShift], bit);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x)
    if (row_mask[i]) atomicOr(&mask[size_t(t) * nb + i], row_mask[i]);
}

// Column (i, j) of D: the tabulated pulse delayed by td[ij] samples, linearly
// interpolated on the fine grid; also its squared norm.
// The windowed gather's table: for trace blockIdx.x and voxel tile
// blockIdx.y (kGatherTileRows x kGatherTileCols, row-major over the grid), the
// fine positions J = floor(delay Q) of the tile's voxels that fall inside the
// record, as {first, count}: first a multiple of `align` (16 bytes of the
// fine grid) at or below the smallest J, first + count a multiple of `align`
// above the largest J + 1 (each voxel reads J and J + 1); {0, 0} when no
// voxel's J lies in the record.  J is the gather's
// own: the two legs' Q32.32 delays summed and shifted.
__global__ __launch_bounds__(512) void k_gather_windows(const Leg* __restrict__ legs, const int* __restrict__ base,
                                                        int P, int K, int nx, int nz, int n_off, int qs, int MQ,
                                                        int align, int2* __restrict__ gwin) {
  const int t = blockIdx.x, tile = blockIdx.y;
  const int tiles_x = (nx + kGatherTileCols - 1) / kGatherTileCols;
  const int tz = tile / tiles_x, tx = tile - tz * tiles_x;
  const int half = n_off / 2, sh = 32 - qs;
  const int bt = base[t / K], br = base[P + t];
  const int wave = int(threadIdx.x >> 6), lane = int(threadIdx.x & 63);
  unsigned lo = 0xffffffffu, hi = 0u;
  for (int row = tz * kGatherTileRows + wave; row < min(nz, (tz + 1) * kGatherTileRows); row += 8) {
    const int col = tx * kGatherTileCols + lane;
    if (col < nx) {
      const int64_t da = legs[size_t(row) * n_off + leg_slot(abs(bt + 2 * col), half)].delay;
      const int64_t db = legs[size_t(row) * n_off + leg_slot(abs(br + 2 * col), half)].delay;
      const unsigned J = unsigned(min(uint64_t(da + db) >> sh, uint64_t(MQ)));
      if (J < unsigned(MQ)) {
        lo = min(lo, J);
        hi = max(hi, J);
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, unsigned(__shfl_xor(int(lo), o)));
    hi = max(hi, unsigned(__shfl_xor(int(hi), o)));
  }
  __shared__ unsigned slo[8], shi[8];
  if (lane == 0) {
    slo[wave] = lo;
    shi[wave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < int(blockDim.x >> 6); ++w) {
      lo = min(lo, slo[w]);
      hi = max(hi, shi[w]);
    }
    int2 win = make_int2(0, 0);
    if (lo != 0xffffffffu) {
      const unsigned m = unsigned(align) - 1u;
      const unsigned first = lo & ~m;
      win = make_int2(int(first), int((hi + 2u - first + m) & ~m));
    }
    gwin[size_t(tile) * (P * K) + t] = win;
  }
}

__global__ void k_dbasis(const float* __restrict__ bank, const double* __restrict__ td, int M,
                         int Q, int Lh, float* __restrict__ d, float* __restrict__ dnorm) {
  const int ij = blockIdx.x;
  const double t0 = td[ij];
  const int QLh = Q * Lh;
  double acc = 0.0;
  for (int m = threadIdx.x; m < M; m += blockDim.x) {
    const double z = (m - t0) * Q;
    float v = 0.0f;
    if (z > 0.0 && z < QLh) {
      const double n = floor(z);
      const double f = z - n;
      const int ni = static_cast<int>(n);
      v = static_cast<float>((1.0 - f) * bank[ni] + f * bank[ni + 1]);
    }
    d[size_t(ij) * M + m] = v;
    acc += double(v) * double(v);
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) dnorm[ij] = static_cast<float>(red[0]);
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Lattice base of a transducer at x: 2 (x0 - x) / dx + 1 must be an integer.
bool lattice_base(double x0, double dx, double x, long* out) {
  const double b = 2.0 * (x0 - x) / dx + 1.0;
  const double r = std::nearbyint(b);
  if (std::fabs(b - r) > 1e-6) return false;
  *out = static_cast<long>(r);
  return true;
}

}  // namespace

// Fine-grid chunks and LDS tiles of the splat sweep for a target workgroup
// count: ceil(target / traces) chunks per trace of at least 1024 positions,
// swept in tiles of 64-bit positions as large as fit in the workgroup's LDS
// (kSplatLdsBytes) beside the row pointers (at least 4096 positions, a
// multiple of 64, at most a chunk): every tile costs a fixed walk over the
// (column, layer) pointers, three barriers and a partly used first row block
// per (column, layer), so fewer, larger tiles run faster.
void apply_splat_blocks(umbir_geometry* G, long target) {
  const long MQ = long(G->M) * G->Q;
  const long min_chunk = 1024;
  long chunks = (target + G->traces() - 1) / G->traces();
  const long max_chunks = (MQ + min_chunk - 1) / min_chunk;
  if (chunks > max_chunks) chunks = max_chunks;
  if (chunks < 1) chunks = 1;
  G->splat_blocks = int(std::min<long>(target, 1L << 30));
  G->chunks = int(chunks);
  G->chunk_bins = (MQ + chunks - 1) / chunks;
  const long pointers = long(G->n_seg + 1) * G->nx * 8;  // per (column, layer) pointers and column offsets
  long tile = (kSplatLdsBytes - 1024 - pointers) / 8 - 2;
  tile = std::max<long>(4096, tile / 64 * 64);
  G->tile_bins = int(std::min<long>(tile, G->chunk_bins));
}

namespace {

struct Derived {
  int Lh = 0, n_off = 0;
  long omax = 0;          // largest lattice offset any transducer uses
  int n_gamma = 1;        // attenuation templates asked for (1 without attenuation)
  std::vector<int> base;  // [P + P*K]
};

// Composite Gauss-Legendre rule on [0, fmax]: `panels` panels of kGaussNodes
// nodes each.  The nodes of one panel are the roots of the Legendre polynomial
// P_n, found by Newton's method from the asymptotic guesses
// cos(pi (i + 3/4) / (n + 1/2)); the weights are 2 / ((1 - x^2) P_n'(x)^2).
constexpr int kGaussNodes = 20;

void gauss_legendre(std::vector<double>* x, std::vector<double>* w) {
  const int n = kGaussNodes;
  x->assign(n, 0.0);
  w->assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;  // P_0, P_1, then the three-term recurrence
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    (*x)[i] = z;
    (*w)[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Frequencies and amplitudes of the attenuated-template quadrature, laid out
// as k_bank_att reads them.  The Gaussian factor of the spectrum is below
// e^-72 of its peak past f_c + 6 / (pi sigma_t); a panel spans at most 1/8 of
// a period of the sine at the window's largest |t - t_c| = t_0 / 2.
std::vector<double> spectrum_nodes(double f_c, double sigma_t, double t_win) {
  std::vector<double> gx, gw;
  gauss_legendre(&gx, &gw);
  const double fmax = f_c + 6.0 / (M_PI * sigma_t);
  const int panels = std::max(16, int(std::ceil(8.0 * fmax * 0.5 * t_win)));
  const int n = panels * kGaussNodes;
  std::vector<double> out(2 * size_t(n));
  const double c = sigma_t * std::sqrt(2.0 * M_PI);
  const double hw = 0.5 * fmax / panels;
  for (int p = 0; p < panels; ++p) {
    const double mid = (p + 0.5) * (fmax / panels);
    for (int i = 0; i < kGaussNodes; ++i) {
      const double f = mid + hw * gx[i];
      const double a = M_PI * sigma_t * (f - f_c), b = M_PI * sigma_t * (f + f_c);
      out[size_t(p) * kGaussNodes + i] = f;
      out[n + size_t(p) * kGaussNodes + i] = hw * gw[i] * c * (std::exp(-2.0 * a * a) - std::exp(-2.0 * b * b));
    }
  }
  return out;
}

int validate(const umbir_problem* pb, Derived* dv) {
  if (!pb) return fail(UMBIR_EINVAL, "problem is NULL");
  const umbir_medium& md = pb->medium;
  if (md.n_layers < 1 || md.n_layers > kMaxLayers)
    return fail(UMBIR_EINVAL, "n_layers must be in 1..8");
  if (!md.speed || !md.density) return fail(UMBIR_EINVAL, "medium speed/density is NULL");
  if (md.n_layers > 1 && !md.thickness) return fail(UMBIR_EINVAL, "medium thickness is NULL");
  for (int l = 0; l < md.n_layers; ++l) {
    if (!finite_pos(md.speed[l])) return fail(UMBIR_EINVAL, "layer speed must be finite and > 0");
    if (!finite_pos(md.density[l])) return fail(UMBIR_EINVAL, "layer density must be finite and > 0");
    if (l + 1 < md.n_layers && !finite_pos(md.thickness[l]))
      return fail(UMBIR_EINVAL, "layer thickness must be finite and > 0");
    if (md.atten) {
      if (!std::isfinite(md.atten[l]) || md.atten[l] < 0.0)
        return fail(UMBIR_EINVAL, "attenuation must be finite and >= 0");
      if (md.atten[l] != 0.0) dv->n_gamma = 0;  // decided below
    }
  }
  const umbir_grid& g = pb->grid;
  if (g.nx < 1 || g.nz < 1) return fail(UMBIR_EINVAL, "grid must have nx, nz >= 1");
  if (double(g.nx) * g.nz > double(1 << 26)) return fail(UMBIR_EINVAL, "grid too large");
  if (!finite_pos(g.dx) || !finite_pos(g.dz)) return fail(UMBIR_EINVAL, "dx, dz must be > 0");
  if (!std::isfinite(g.x0) || !std::isfinite(g.z0) || g.z0 < 0.0)
    return fail(UMBIR_EINVAL, "x0 must be finite and z0 finite and >= 0");
  const umbir_array& a = pb->array;
  if (a.n_scans < 1 || a.n_rx < 1) return fail(UMBIR_EINVAL, "need n_scans, n_rx >= 1");
  if (double(a.n_scans) * a.n_rx > double(1 << 20)) return fail(UMBIR_EINVAL, "too many traces");
  if (!a.tx_x || !a.rx_offset) return fail(UMBIR_EINVAL, "array positions are NULL");
  if (a.beta < 0 || a.beta > 64) return fail(UMBIR_EINVAL, "beta must be an integer in 0..64");
  const umbir_acq& q = pb->acq;
  if (q.n_samples < 1 || q.n_samples > (1 << 22)) return fail(UMBIR_EINVAL, "n_samples out of range");
  if (!finite_pos(q.fs) || !finite_pos(q.f_c) || !finite_pos(q.sigma_t) || !finite_pos(q.t_win))
    return fail(UMBIR_EINVAL, "fs, f_c, sigma_t, t_win must be finite and > 0");
  const double lh = q.t_win * q.fs;
  const long lhi = std::lround(lh);
  if (std::fabs(lh - double(lhi)) > 1e-9 * std::max(1.0, lh) || lhi < 2)
    return fail(UMBIR_EINVAL, "t_win * fs must be an integer >= 2");
  if (q.oversample < 1 || q.oversample > 64 || (q.oversample & (q.oversample - 1)))
    return fail(UMBIR_ENOTSUP, "oversample must be a power of two in 1..64");
  if (q.storage != UMBIR_STORAGE_F32 && q.storage != UMBIR_STORAGE_F16 && q.storage != UMBIR_STORAGE_BF16)
    return fail(UMBIR_EINVAL, "storage must be UMBIR_STORAGE_F32, _F16 or _BF16");
  if (q.storage != UMBIR_STORAGE_F32 && q.oversample != 32 && q.oversample != 64)
    return fail(UMBIR_ENOTSUP, "16-bit storage needs oversample 32 or 64");
  if (dv->n_gamma == 0) {  // some alpha > 0
    dv->n_gamma = q.n_gamma == 0 ? 16 : q.n_gamma;
    if (dv->n_gamma < 2 || dv->n_gamma > kMaxGamma)
      return fail(UMBIR_EINVAL, "n_gamma must be 0 (16) or in 2..64 when some alpha > 0");
    if (q.storage != UMBIR_STORAGE_F32)
      return fail(UMBIR_ENOTSUP, "attenuation (alpha > 0) needs FP32 storage");
  }
  // the dense kernels stage the taps, padded to a multiple of 16 rows, in 64 KiB of LDS
  if ((lhi + 15) / 16 * 16 * q.oversample > 16384)
    return fail(UMBIR_ENOTSUP, "window (rounded up to 16) * oversample must be <= 16384");
  // the splat keeps a row pointer and its fine position per (column, layer) in
  // LDS beside a 32 KiB tile
  if (long(g.nx) * md.n_layers > 4096)
    return fail(UMBIR_ENOTSUP, "nx * n_layers must be <= 4096");
  if (double(q.n_samples) * q.oversample > double(1 << 28))
    return fail(UMBIR_ENOTSUP, "n_samples * oversample too large");
  dv->Lh = int(lhi);
  dv->base.assign(size_t(a.n_scans) * (1 + a.n_rx), 0);
  long omax = 0;
  auto add = [&](size_t slot, double x) -> bool {
    if (!std::isfinite(x)) return false;
    long b;
    if (!lattice_base(g.x0, g.dx, x, &b)) return false;
    const long lo = std::labs(b), hi = std::labs(b + 2L * (g.nx - 1));
    omax = std::max(omax, std::max(lo, hi));
    dv->base[slot] = int(b);
    return true;
  };
  for (int i = 0; i < a.n_scans; ++i) {
    if (!add(i, a.tx_x[i]))
      return fail(UMBIR_ENOTSUP, "transmitter off the half-voxel lattice (2 (x0 - x) / dx not an integer)");
    for (int j = 0; j < a.n_rx; ++j)
      if (!add(a.n_scans + size_t(i) * a.n_rx + j, a.tx_x[i] + a.rx_offset[j]))
        return fail(UMBIR_ENOTSUP, "receiver off the half-voxel lattice (2 (x0 - x) / dx not an integer)");
  }
  if (omax + 1 > (1 << 24)) return fail(UMBIR_EINVAL, "lateral extent too large");
  dv->omax = omax;
  dv->n_off = int((omax + 2) & ~1L);  // even, for the parity split of each row
  // the splat addresses the leg table and the image with 32-bit byte offsets
  const double nzp = double(padded_rows(g.nz));
  if (nzp * dv->n_off * sizeof(Leg) >= double(1u << 31) || nzp * g.nx * 4 >= double(1u << 31))
    return fail(UMBIR_ENOTSUP, "leg table or image of 2 GiB or more");
  return UMBIR_OK;
}

// Trace groups of the adjoint's gather: the gather runs one generation of at
// most 1024 blocks (groups x voxel blocks of 1024 voxels), so the voxel block
// count fixes how many groups fit; groups are a multiple of the 8 XCDs when
// there are enough traces, because group g runs on XCD g mod 8 (it is the
// fastest-varying block index).
int choose_trace_groups(int n_vox, int n_traces) {
  const int vox_blocks = (n_vox + 1023) / 1024;
  int g = std::max(1, 1024 / vox_blocks);
  if (n_traces >= 8) g = std::max(8, g / 8 * 8);
  if (g > n_traces) g = n_traces;
  return std::max(g, 1);
}

size_t table_bytes(int nz, int n_off, int P, int K, int M, int Q, int Lh, int n_gamma) {
  const size_t legs = size_t(nz) * n_off;
  // with attenuation: the legs' attenuation in template bins and the
  // template occupancy masks
  const size_t legs_t = size_t(n_off) * padded_rows(nz);
  const size_t att = n_gamma > 1 ? (legs + legs_t) * sizeof(double) + size_t(P) * K *
                                       ((size_t(M) * Q + (size_t(1) << kMaskShift) - 1) >> kMaskShift) * 8
                                 : 0;
  return (legs + legs_t) * sizeof(Leg) + size_t(nz) * sizeof(float) +
         size_t(P) * (1 + K) * sizeof(int) + size_t(n_gamma) * (Q * Lh + 2) * sizeof(float) +
         2 * size_t(n_gamma) * Q * Lh * sizeof(float) + size_t(P) * K * M * sizeof(float) +
         size_t(P) * K * sizeof(float) + att;
}

}  // namespace

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return UMBIR_OK;
  return fail(e == hipErrorOutOfMemory ? UMBIR_ENOMEM : UMBIR_EDEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

int Workspace::acquire(void* user, size_t user_bytes, size_t need, hipStream_t s) {
  stream = s;
  if (user) {
    if (user_bytes < need)
      return fail(UMBIR_EINVAL, "workspace smaller than umbir_workspace_bytes()");
    ptr = user;
    return UMBIR_OK;
  }
  int st = check_hip(hipMallocAsync(&ptr, need ? need : 256, s), "hipMallocAsync(workspace)");
  if (st) {
    ptr = nullptr;
    return st;
  }
  owned = true;
  return UMBIR_OK;
}

Workspace::~Workspace() {
  if (owned && ptr) (void)hipFreeAsync(ptr, stream);
}

}  // namespace umbir

using namespace umbir;

extern "C" {

const char* umbir_strerror(int status) {
  switch (status) {
    case UMBIR_OK: return "success";
    case UMBIR_EINVAL: return "invalid argument";
    case UMBIR_ENOMEM: return "out of device memory";
    case UMBIR_EDEVICE: return "HIP device error";
    case UMBIR_ENOTSUP: return "not supported by the library";
    case UMBIR_EDIVERGED: return "MAP cost diverged";
    default: return "unknown status";
  }
}

const char* umbir_last_error(void) { return g_last_error.c_str(); }

size_t umbir_estimate_bytes(const umbir_problem* pb) {
  Derived dv;
  std::string keep = g_last_error;
  if (validate(pb, &dv) != UMBIR_OK) {
    g_last_error = keep;
    return 0;
  }
  return table_bytes(pb->grid.nz, dv.n_off, pb->array.n_scans, pb->array.n_rx,
                     pb->acq.n_samples, pb->acq.oversample, dv.Lh, dv.n_gamma) +
         (dv.n_gamma > 1 ? 0
                         : gather_window_bytes(pb->grid.nx, pb->grid.nz, long(pb->array.n_scans) * pb->array.n_rx,
                                               long(pb->acq.n_samples) * pb->acq.oversample, pb->acq.storage));
}

void umbir_geometry_free(umbir_geometry* G) {
  if (!G) return;
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (G->device >= 0) (void)hipSetDevice(G->device);
  void* ptrs[] = {G->legs, G->legs_t, G->tau, G->base, G->bank, G->h, G->habs, G->dbasis, G->dnorm, G->gmask,
                  G->gunit, G->gunit_t, G->gwin};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (cur >= 0) (void)hipSetDevice(cur);
  delete G;
}

int umbir_build_geometry(const umbir_problem* pb, void* stream, umbir_geometry** out) {
  if (!out) return fail(UMBIR_EINVAL, "out is NULL");
  *out = nullptr;
  Derived dv;
  int st = validate(pb, &dv);
  if (st) return st;

  int dev = -1;
  if ((st = check_hip(hipGetDevice(&dev), "hipGetDevice"))) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);

  auto* G = new umbir_geometry();
  G->device = dev;
  const umbir_medium& md = pb->medium;
  G->layers.n = md.n_layers;
  double top = 0.0;
  for (int l = 0; l < md.n_layers; ++l) {
    G->layers.speed[l] = md.speed[l];
    G->layers.atten[l] = md.atten ? md.atten[l] : 0.0;
    G->layers.top[l] = top;
    const double bot = (l + 1 < md.n_layers) ? top + md.thickness[l] : INFINITY;
    G->layers.bottom[l] = bot;
    G->density[l] = md.density[l];
    top = bot;
  }
  G->nx = pb->grid.nx;
  G->nz = pb->grid.nz;
  G->dx = pb->grid.dx;
  G->dz = pb->grid.dz;
  G->x0 = pb->grid.x0;
  G->z0 = pb->grid.z0;
  G->P = pb->array.n_scans;
  G->K = pb->array.n_rx;
  G->beta = pb->array.beta;
  G->tx_x.assign(pb->array.tx_x, pb->array.tx_x + G->P);
  G->rx_off.assign(pb->array.rx_offset, pb->array.rx_offset + G->K);
  G->M = pb->acq.n_samples;
  G->Q = pb->acq.oversample;
  G->storage = pb->acq.storage;
  G->Lh = dv.Lh;
  G->fs = pb->acq.fs;
  G->f_c = pb->acq.f_c;
  G->sigma_t = pb->acq.sigma_t;
  G->t_win = pb->acq.t_win;
  G->n_off = dv.n_off;
  G->trace_groups = choose_trace_groups(G->voxels(), G->traces());
  {
    // layer segments of the rows: a row belongs to the deepest layer whose top
    // lies above its centre (the legs' crossing extents use the same rule)
    int prev = -1;
    for (int r = 0; r < G->nz; ++r) {
      const double z = G->z0 + (r + 0.5) * G->dz;
      int l = 0;
      while (l + 1 < G->layers.n && z > G->layers.top[l + 1]) ++l;
      if (l != prev) {
        G->seg_lo[G->n_seg] = r;
        ++G->n_seg;
        prev = l;
      }
      G->seg_hi[G->n_seg - 1] = r + 1;
    }
    apply_splat_blocks(G, G->splat_blocks);
    // output tiles per convolution workgroup: with FP32 products two when
    // that still leaves at least two workgroups per CU; with bf16 pieces
    // (whose splitting of the fetched rows more tiles share) four when that
    // leaves one workgroup per CU, else two likewise (small problems keep the
    // wider grid)
    const long tt = (G->traces() + 31) / 32;
    if (G->split && tt * ((G->M + 127) / 128) >= 256) G->conv_tiles = 4;
    else if (G->split && tt * ((G->M + 63) / 64) >= 256) G->conv_tiles = 2;
    else G->conv_tiles = tt * ((G->M + 63) / 64) >= 512 ? 2 : 1;
    // correlation workgroups: the bf16-piece form's 72 KB of LDS leave two
    // per CU, so 512 make one generation (each stages its taps once)
    if (G->split) G->corr_blocks = 512;
  }

  const size_t legs = size_t(G->nz) * G->n_off;
  G->nzp = padded_rows(G->nz);
  const size_t legs_t = size_t(G->nzp) * G->n_off;
  const size_t PK = size_t(G->P) * G->K;
  const int QLh = G->Q * G->Lh;
  auto alloc = [&](void** p, size_t bytes) {
    G->bytes += bytes;
    return check_hip(hipMalloc(p, bytes ? bytes : 4), "hipMalloc(geometry)");
  };
  double* td_dev = nullptr;
  if ((st = alloc((void**)&G->legs, legs * sizeof(Leg))) ||
      (st = alloc((void**)&G->legs_t, legs_t * sizeof(Leg))) ||
      (st = alloc((void**)&G->tau, G->nz * sizeof(float))) ||
      (st = alloc((void**)&G->base, dv.base.size() * sizeof(int))) ||
      (st = alloc((void**)&G->dbasis, PK * G->M * sizeof(float))) ||
      (st = alloc((void**)&G->dnorm, PK * sizeof(float)))) {
    umbir_geometry_free(G);
    return st;
  }
  // transmittance product per row (Eqs. (3), (7)); reading: each interface
  // between layers a and b passes 4 Z_a Z_b / (Z_a + Z_b)^2 of the pressure
  // both ways at normal incidence, Z = rho c; layer 0 has tau = 1.
  std::vector<float> tau(G->nz);
  for (int r = 0; r < G->nz; ++r) {
    const double z = G->z0 + (r + 0.5) * G->dz;
    double t = 1.0;
    for (int l = 0; l + 1 < G->layers.n; ++l) {
      if (z > G->layers.bottom[l]) {
        const double za = G->density[l] * G->layers.speed[l];
        const double zb = G->density[l + 1] * G->layers.speed[l + 1];
        t *= 4.0 * za * zb / ((za + zb) * (za + zb));
      }
    }
    tau[r] = float(t);
  }
  // direct-arrival delay of each trace in samples: |x_rx - x_tx| / c_0
  std::vector<double> td(PK);
  for (int i = 0; i < G->P; ++i)
    for (int j = 0; j < G->K; ++j)
      td[size_t(i) * G->K + j] = G->fs * std::fabs(G->rx_off[j]) / G->layers.speed[0];

  if ((st = check_hip(hipMallocAsync((void**)&td_dev, PK * sizeof(double), s), "hipMallocAsync")) ||
      (st = check_hip(hipMemcpyAsync(td_dev, td.data(), PK * sizeof(double), hipMemcpyHostToDevice, s),
                      "hipMemcpyAsync")) ||
      (st = check_hip(hipMemcpyAsync(G->tau, tau.data(), G->nz * sizeof(float), hipMemcpyHostToDevice, s),
                      "hipMemcpyAsync")) ||
      (st = check_hip(hipMemcpyAsync(G->base, dv.base.data(), dv.base.size() * sizeof(int),
                                     hipMemcpyHostToDevice, s),
                      "hipMemcpyAsync"))) {
    if (td_dev) (void)hipFreeAsync(td_dev, s);
    (void)hipStreamSynchronize(s);
    umbir_geometry_free(G);
    return st;
  }
  // legs; with attenuation also each leg's path attenuation, from which the
  // template bins follow
  double* gam_dev = nullptr;
  double* nodes_dev = nullptr;
  auto bail = [&](int code) {
    if (td_dev) (void)hipFreeAsync(td_dev, s);
    if (gam_dev) (void)hipFreeAsync(gam_dev, s);
    if (nodes_dev) (void)hipFreeAsync(nodes_dev, s);
    (void)hipStreamSynchronize(s);
    umbir_geometry_free(G);
    return code;
  };
  if (dv.n_gamma > 1 &&
      (st = check_hip(hipMallocAsync((void**)&gam_dev, legs * sizeof(double), s), "hipMallocAsync")))
    return bail(st);
  // the padding rows of the transposed table stay zero
  if ((st = check_hip(hipMemsetAsync(G->legs_t, 0, legs_t * sizeof(Leg), s), "hipMemsetAsync(legs_t)")))
    return bail(st);
  const int n_legs = int(legs);
  UMBIR_LAUNCH("legs", k_legs, dim3((n_legs + 255) / 256), dim3(256), 0, s, G->layers, G->nz, G->n_off, G->z0,
               G->dz, 0.5 * G->dx, G->fs, G->beta, G->legs, G->nzp, G->legs_t, log2_int(G->Q), gam_dev);
  if ((st = check_hip(hipGetLastError(), "k_legs"))) return bail(st);
  if (dv.n_gamma > 1) {
    // Gamma_max: at a fixed depth a leg's attenuation grows with its lateral
    // offset, so every row's largest is at the largest offset in use
    std::vector<double> gam(legs);
    if ((st = check_hip(hipMemcpyAsync(gam.data(), gam_dev, legs * sizeof(double), hipMemcpyDeviceToHost, s),
                        "hipMemcpyAsync")) ||
        (st = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize")))
      return bail(st);
    const int slot = leg_slot(int(dv.omax), G->n_off / 2);
    double gmax = 0.0;
    for (int r = 0; r < G->nz; ++r) gmax = std::max(gmax, gam[size_t(r) * G->n_off + slot]);
    if (gmax > 0.0) {
      G->n_gamma = dv.n_gamma;
      G->gamma_step = 2.0 * gmax / (G->n_gamma - 1);
      if ((st = alloc((void**)&G->gunit, legs * sizeof(double))) ||
          (st = alloc((void**)&G->gunit_t, legs_t * sizeof(double))) ||
          (st = check_hip(hipMemsetAsync(G->gunit_t, 0, legs_t * sizeof(double), s), "hipMemsetAsync(gunit_t)")))
        return bail(st);
      UMBIR_LAUNCH("leg_units", k_leg_units, dim3((n_legs + 255) / 256), dim3(256), 0, s, n_legs, G->n_off, G->nzp,
                   gam_dev, G->gamma_step, G->gunit, G->gunit_t);
    }
  }
  // the windowed gather's table (where it applies: one template, no
  // attenuation asked for)
  const size_t wb =
      dv.n_gamma > 1 ? 0 : gather_window_bytes(G->nx, G->nz, long(PK), G->fine_per_trace(), G->storage);
  if (wb) {
    if ((st = alloc((void**)&G->gwin, wb))) return bail(st);
    UMBIR_LAUNCH("gather_windows", k_gather_windows, dim3(unsigned(PK), unsigned(gather_tiles(G->nx, G->nz))),
                 dim3(512), 0, s, G->legs, G->base, G->P, G->K, G->nx, G->nz, G->n_off, log2_int(G->Q),
                 int(G->fine_per_trace()), gather_window_align(G->storage), G->gwin);
    if ((st = check_hip(hipGetLastError(), "k_gather_windows"))) return bail(st);
    if (gather_windowed_default(G->nx, G->nz, G->trace_groups)) {
      G->gather_form = 2;
      // gather batches of 16 traces per voxel tile a block takes (measured at
      // 256 x 256: one tile per block, 4 MiB; at 512 x 512: two, 16 MiB
      // against 5.02 ms per operator pair at 4 MiB and 5.00 at 32 MiB)
      int tpb;
      (void)gather_lds_blocks(G->nx, G->nz, G->trace_groups, &tpb);
      const long kb = 16L * tpb * long(G->fine_per_trace()) * long(G->elem()) / 1024;
      G->gather_batch_kb = int(std::min(long(1) << 20, std::max(long(G->gather_batch_kb), kb)));
    }
  }
  const int NG = G->n_gamma;
  if ((st = alloc((void**)&G->bank, size_t(NG) * (QLh + 2) * sizeof(float))) ||
      (st = alloc((void**)&G->h, size_t(NG) * QLh * sizeof(float))) ||
      (st = alloc((void**)&G->habs, size_t(NG) * QLh * sizeof(float))))
    return bail(st);
  {
    const double dt = 1.0 / (double(G->Q) * G->fs);
    UMBIR_LAUNCH("bank", k_bank, dim3((QLh + 2 + 255) / 256), dim3(256), 0, s, G->Q, G->Lh, dt, G->f_c,
                       1.0 / (2.0 * G->sigma_t * G->sigma_t), 0.5 * G->t_win, G->bank, G->h, G->habs);
    if (NG > 1) {
      const std::vector<double> nodes = spectrum_nodes(G->f_c, G->sigma_t, G->t_win);
      const int n_nodes = int(nodes.size() / 2);
      if ((st = check_hip(hipMallocAsync((void**)&nodes_dev, nodes.size() * sizeof(double), s),
                          "hipMallocAsync")) ||
          (st = check_hip(hipMemcpyAsync(nodes_dev, nodes.data(), nodes.size() * sizeof(double),
                                         hipMemcpyHostToDevice, s), "hipMemcpyAsync")))
        return bail(st);
      UMBIR_LAUNCH("bank_att", k_bank_att, dim3((QLh + 2 + 255) / 256, NG - 1), dim3(256), 0, s, QLh, dt,
                   0.5 * G->t_win, G->gamma_step, n_nodes, nodes_dev, G->bank);
      const long rest = long(NG - 1) * QLh;
      UMBIR_LAUNCH("polyphase", k_polyphase, dim3(unsigned((rest + 255) / 256)), dim3(256), 0, s, G->Q, G->Lh, 1,
                   NG, G->bank, G->h, G->habs);
    }
    UMBIR_LAUNCH("dbasis", k_dbasis, dim3(unsigned(PK)), dim3(256), 0, s, G->bank, td_dev, G->M, G->Q,
                       G->Lh, G->dbasis, G->dnorm);
  }
  if (NG > 1) {
    const long MQ = long(G->M) * G->Q;
    G->mask_blocks = int((MQ + (1L << kMaskShift) - 1) >> kMaskShift);
    const size_t mb = PK * size_t(G->mask_blocks) * sizeof(unsigned long long);
    if ((st = alloc((void**)&G->gmask, mb)) ||
        (st = check_hip(hipMemsetAsync(G->gmask, 0, mb, s), "hipMemsetAsync(mask)")))
      return bail(st);
    int qs = 0;
    while ((1 << qs) < G->Q) ++qs;
    // eight blocks per trace, each with the trace's mask row in LDS
    const unsigned vblocks = unsigned(std::min<long>(8, (long(G->voxels()) + 255) / 256));
    UMBIR_LAUNCH("bin_mask", k_bin_mask, dim3(unsigned(PK), vblocks), dim3(256),
                 size_t(G->mask_blocks) * sizeof(unsigned long long), s, G->legs, G->gunit, G->n_off, G->base, G->P,
                 G->K, G->nx, G->voxels(), qs, MQ, NG - 1, G->mask_blocks, G->gmask);
  }
  if (gam_dev) (void)hipFreeAsync(gam_dev, s);
  if (nodes_dev) (void)hipFreeAsync(nodes_dev, s);
  st = check_hip(hipGetLastError(), "geometry kernels");
  (void)hipFreeAsync(td_dev, s);
  const int st2 = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize(build_geometry)");
  if (!st) st = st2;
  if (st) {
    umbir_geometry_free(G);
    return st;
  }
  *out = G;
  return UMBIR_OK;
}

size_t umbir_geometry_bytes(const umbir_geometry* G) { return G ? G->bytes : 0; }

int umbir_get_tuning(const umbir_geometry* G, umbir_tuning* out) {
  if (!G || !out) return fail(UMBIR_EINVAL, "NULL argument");
  out->splat_blocks = G->splat_blocks;
  out->gather_batch_kb = G->gather_batch_kb;
  out->conv_grid = G->conv_grid;
  out->conv_tile_rows = 32 * G->conv_tiles;
  out->corr_tile_rows = 32 * G->corr_tiles;
  out->corr_blocks = G->corr_blocks;
  out->operator_form = G->form;
  out->products = G->split ? 2 : 1;
  out->gather_form = G->gather_form;
  return UMBIR_OK;
}

int umbir_set_tuning(umbir_geometry* G, const umbir_tuning* t) {
  if (!G || !t) return fail(UMBIR_EINVAL, "NULL argument");
  if (t->conv_grid > 2) return fail(UMBIR_EINVAL, "conv_grid must be 1 or 2");
  if (t->operator_form > 2) return fail(UMBIR_EINVAL, "operator_form must be 1 or 2");
  if (t->products > 2) return fail(UMBIR_EINVAL, "products must be 1 or 2");
  if (t->gather_form > 2) return fail(UMBIR_EINVAL, "gather_form must be 1 or 2");
  if (t->gather_form == 2 && !G->gwin)
    return fail(UMBIR_ENOTSUP, "the windowed gather needs no attenuation and M * Q a multiple of 16 bytes");
  if (t->operator_form == 2 && !direct_eligible(*G))
    return fail(UMBIR_ENOTSUP, "the direct form needs FP32 storage, one template and 8 M + 4 (Q L_h + 2) <= 65536");
  if (t->corr_tile_rows > 0 && t->corr_tile_rows != 32 && t->corr_tile_rows != 64 && t->corr_tile_rows != 128)
    return fail(UMBIR_EINVAL, "corr_tile_rows must be 32, 64 or 128");
  if (t->conv_tile_rows > 0 && t->conv_tile_rows != 32 && t->conv_tile_rows != 64 && t->conv_tile_rows != 128)
    return fail(UMBIR_EINVAL, "conv_tile_rows must be 32, 64 or 128");
  if (t->splat_blocks > 0) apply_splat_blocks(G, t->splat_blocks);
  if (t->gather_batch_kb > 0) G->gather_batch_kb = t->gather_batch_kb;
  if (t->conv_grid > 0) G->conv_grid = t->conv_grid;
  if (t->conv_tile_rows > 0) G->conv_tiles = t->conv_tile_rows / 32;
  if (t->corr_tile_rows > 0) G->corr_tiles = t->corr_tile_rows / 32;
  if (t->corr_blocks > 0) G->corr_blocks = t->corr_blocks;
  if (t->operator_form > 0) G->form = t->operator_form;
  if (t->products > 0) G->split = t->products == 2;
  if (t->gather_form > 0) G->gather_form = t->gather_form;
  return UMBIR_OK;
}

int umbir_get_dims(const umbir_geometry* G, umbir_dims* d) {
  if (!G || !d) return fail(UMBIR_EINVAL, "NULL argument");
  d->nx = G->nx;
  d->nz = G->nz;
  d->n_scans = G->P;
  d->n_rx = G->K;
  d->n_samples = G->M;
  d->n_off = G->n_off;
  d->window = G->Lh;
  d->oversample = G->Q;
  d->n_layers = G->layers.n;
  d->trace_groups = G->trace_groups;
  d->storage = G->storage;
  d->n_gamma = G->n_gamma;
  d->gamma_step = G->gamma_step;
  return UMBIR_OK;
}

int umbir_copy_table(const umbir_geometry* G, int which, void* dst, size_t bytes) {
  if (!G || !dst) return fail(UMBIR_EINVAL, "NULL argument");
  const void* src = nullptr;
  size_t need = 0;
  const size_t legs = size_t(G->nz) * G->n_off;
  switch (which) {
    case UMBIR_TABLE_DELAY: need = legs * sizeof(int64_t); break;
    case UMBIR_TABLE_APOD: need = legs * sizeof(float); break;
    case UMBIR_TABLE_TAU: src = G->tau; need = G->nz * sizeof(float); break;
    case UMBIR_TABLE_BANK: src = G->bank; need = size_t(G->n_gamma) * (G->Q * G->Lh + 2) * sizeof(float); break;
    case UMBIR_TABLE_DBASIS: src = G->dbasis; need = size_t(G->traces()) * G->M * sizeof(float); break;
    case UMBIR_TABLE_OFFSET: src = G->base; need = size_t(G->P) * (1 + G->K) * sizeof(int); break;
    case UMBIR_TABLE_ATTEN: need = legs * sizeof(double); break;
    default: return fail(UMBIR_EINVAL, "unknown table");
  }
  if (bytes != need) return fail(UMBIR_EINVAL, "bytes does not match the table size");
  if (src) return check_hip(hipMemcpy(dst, src, need, hipMemcpyDeviceToHost), "hipMemcpy(table)");
  const int half = G->n_off / 2;
  if (which == UMBIR_TABLE_ATTEN) {  // zero with a single template
    std::vector<double> gu(legs, 0.0);
    if (G->gunit) {
      int st = check_hip(hipMemcpy(gu.data(), G->gunit, legs * sizeof(double), hipMemcpyDeviceToHost),
                         "hipMemcpy(attenuation)");
      if (st) return st;
    }
    for (int r = 0; r < G->nz; ++r)
      for (int o = 0; o < G->n_off; ++o)
        static_cast<double*>(dst)[size_t(r) * G->n_off + o] = gu[size_t(r) * G->n_off + leg_slot(o, half)];
    return UMBIR_OK;
  }
  // leg tables: one field of the packed records
  std::vector<Leg> rec(legs);
  int st = check_hip(hipMemcpy(rec.data(), G->legs, legs * sizeof(Leg), hipMemcpyDeviceToHost),
                     "hipMemcpy(legs)");
  if (st) return st;
  for (int r = 0; r < G->nz; ++r)
    for (int o = 0; o < G->n_off; ++o) {
      const Leg& L = rec[size_t(r) * G->n_off + leg_slot(o, half)];
      const size_t k = size_t(r) * G->n_off + o;
      if (which == UMBIR_TABLE_DELAY) static_cast<int64_t*>(dst)[k] = L.delay;
      else static_cast<float*>(dst)[k] = L.apod;
    }
  return UMBIR_OK;
}

}  // extern "C"
