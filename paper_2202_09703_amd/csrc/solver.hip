// MAP reconstruction of Eq. (18) with the QGGMRF prior of Eqs. (14)-(17).
//
// The paper minimises the cost with ICD.  Here every voxel is updated at once
// from one A x and one A^T e per iteration, by a separable surrogate of the
// cost (data term: curvature d = |A|^T |A| 1 / sigma^2, which bounds A^T A /
// sigma^2 because |A| >= |entries of A| and all its entries are >= 0; prior
// term: each pair potential bounded by the quadratic through rho at the
// current difference with the same slope, split evenly between the two
// voxels).  Each step lowers the cost, and the cost being strictly convex
// (Sec. 2, "Optimization") the iteration shares ICD's minimiser.
//
// Iteration n (from x^n, g^n):
//   1. e = y - A x - D g                        (k_conv epilogue)
//   2. record C(x^n, g^n); if estimating g: g += <d_ij, e_ij> / |d_ij|^2 per
//      trace and e -= d_ij * dg (the columns of D have disjoint rows)
//   3. u = A^T e
//   4. for every voxel s, over its 8 neighbours r (Eq. (14) cliques):
//        B = b_sr rho'(x_s - x_r) / (2 (x_s - x_r))
//        x_s -= (-u_s / sigma^2 + sum_r 2 B (x_s - x_r)) / (d_s + sum_r 4 B)
// Reading of the clique weights (not given in the paper): the 8-neighbourhood
// with weights proportional to inverse centre distance, normalised so an
// interior voxel's eight weights sum to one; missing neighbours at the border
// are dropped.  The scale of Eq. (16) uses m_s of Eq. (17) with depth = the
// voxel-centre depth and maximum depth = the deepest centre.

#include <algorithm>
#include <cmath>

#include <cstdio>
#include <mutex>
#include <vector>

#include "internal.h"
#include "storage.h"

namespace umbir {
namespace {

__device__ __forceinline__ float depth_mod(int row, int nz, const PriorConst& pc) {
  const double depth = pc.z0 + (row + 0.5) * pc.dz;
  const double dmax = pc.z0 + (nz - 0.5) * pc.dz;
  return float(1.0 + (pc.m - 1.0) * pow(depth / dmax, pc.a));
}

// Half curvature rho'(D) / (2 D) and rho(D) of Eq. (15) with q = 2, u = |D| / (T sg):
//   rho'(D) / (2 D) = (T sg)^(p-2) / (2 sg^p) * (2/p + u^(2-p)) / (1 + u^(2-p))^2
//                   = T^(p-2) / (2 sg^2) * (2/p + u^(2-p)) / (1 + u^(2-p))^2,
//   rho(D) = |D|^p / (p sg^p) * u^(2-p) / (1 + u^(2-p))
//          = D^2 T^(p-2) / (p sg^2 (1 + u^(2-p)))
// (|D|^p u^(2-p) = D^2 (T sg)^(p-2)): one power per pair, finite at D = 0.
__device__ __forceinline__ void qggmrf(float delta, float sg, const PriorConst& pc, float* half_curv,
                                       float* rho) {
  const float a = fabsf(delta);
  const float inv_sg2 = 1.0f / (sg * sg);
  const float uq = powf(a / (pc.T * sg), 2.0f - pc.p);
  const float den = 1.0f + uq;
  const float c = pc.T_pm2 * inv_sg2;
  *half_curv = 0.5f * c * (2.0f / pc.p + uq) / (den * den);
  *rho = a * a * c / (pc.p * den);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Sums a and b over a block of four waves: a shuffle tree within each wave,
// then the four wave sums in order (the same order on every call).  Every
// thread receives both totals.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh /* [8] */) {
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[w] = a;
    sh[4 + w] = b;
  }
  __syncthreads();
  a = ((sh[0] + sh[1]) + sh[2]) + sh[3];
  b = ((sh[4] + sh[5]) + sh[6]) + sh[7];
}

// Per trace: |e|^2 before the g step, then the exact g step (e in the storage type).
template <int ST>
__device__ __forceinline__ void gstep_body(int bx, int by, typename Store<ST>::T* __restrict__ e, const float* __restrict__ d,
                                               const float* __restrict__ dnorm, float* __restrict__ g,
                                               int M, int estimate, double* __restrict__ ess) {
  __shared__ double sh[8];
  __shared__ float dg_sh;
  const int ij = bx;
  typename Store<ST>::T* et = e + size_t(ij) * M;
  const float* dt = d + size_t(ij) * M;
  // traces of up to R blockDim samples stay in registers between the two
  // passes, their loads all in flight together; the sums run in the same
  // order either way
  constexpr int R = 8;
  const bool held = M <= R * int(blockDim.x);
  float ec[R], dc[R];
  double ee = 0.0, de = 0.0;
  if (held) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int m = min(int(threadIdx.x) + u * int(blockDim.x), M - 1);
      ec[u] = Store<ST>::get(et[m]);
      dc[u] = dt[m];
    }
#pragma unroll
    for (int u = 0; u < R; ++u)
      if (int(threadIdx.x) + u * int(blockDim.x) < M) {
        const double ev = ec[u];
        ee += ev * ev;
        de += double(dc[u]) * ev;
      }
  } else {
    for (int m = threadIdx.x; m < M; m += blockDim.x) {
      const double ev = Store<ST>::get(et[m]);
      ee += ev * ev;
      de += double(dt[m]) * ev;
    }
  }
  block_sum2(ee, de, sh);  // four waves: launched with 256 threads
  if (threadIdx.x == 0) {
    ess[ij] = ee;
    float dg = 0.0f;
    if (estimate && dnorm[ij] > 0.0f) {
      dg = float(de / double(dnorm[ij]));
      g[ij] += dg;
    }
    dg_sh = dg;
  }
  __syncthreads();
  const float dg = dg_sh;
  if (dg == 0.0f) return;
  if (held) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int m = int(threadIdx.x) + u * int(blockDim.x);
      if (m < M) et[m] = Store<ST>::put(fmaf(-dg, dc[u], ec[u]));
    }
  } else {
    for (int m = threadIdx.x; m < M; m += blockDim.x) et[m] = Store<ST>::put(fmaf(-dg, dt[m], Store<ST>::get(et[m])));
  }
}

template <int ST>
__global__ __launch_bounds__(256) void k_gstep(typename Store<ST>::T* __restrict__ e, const float* __restrict__ d,
                                               const float* __restrict__ dnorm, float* __restrict__ g,
                                               int M, int estimate, double* __restrict__ ess) {
  gstep_body<ST>(blockIdx.x, blockIdx.y, e, d, dnorm, g, M, estimate, ess);
}

// Prior cost of x (pairs counted once) into pcost[block]; with UPDATE also the
// surrogate step into xout, with A^T e the sum of the adjoint's `groups`
// partial images (lane q of the voxel sums groups q, q + 4, ..., then a fixed
// butterfly over the four lanes).  Four lanes per voxel, two of its eight
// neighbours each (then summed across the four lanes); the depth modulation
// of the rows the block touches is tabulated once per block.
// With xt set, the prior update also prepares the next forward: xt = tau
// x_out by column (xt[col * nzp + row], the splat's layout), and per block
// the largest |tau x_out| of its voxels into pmax[block] (as float bits),
// from which the forward's splat takes the largest.
struct PriorFuse {
  const float* tau;
  float* xt;
  unsigned* pmax;
  int nzp;
};

template <bool UPDATE>
__device__ __forceinline__ void prior_body(int bx, int by, const float* __restrict__ x,
                                                         const float* __restrict__ part, int groups,
                                                         const float* __restrict__ den, int nx, int nz,
                                                         PriorConst pc, float* __restrict__ xout,
                                                         double* __restrict__ pcost, const PriorFuse& fz) {
  __shared__ double sh[4];
  __shared__ float ms_tab[kPriorVox + 4];  // rows r_lo ..: the block's rows and one on each side
  const float b_edge = float(1.0 / (4.0 + 2.0 * M_SQRT2));
  const float b_diag = float(1.0 / (4.0 + 2.0 * M_SQRT2) / M_SQRT2);
  const int N = nx * nz;
  const int q = threadIdx.x & 3;
  const int v0 = bx * kPriorVox;
  const int v = v0 + (threadIdx.x >> 2);
  const int r_lo = max(v0 / nx - 1, 0);
  const int r_hi = min((min(v0 + kPriorVox, N) - 1) / nx + 1, nz - 1);
  for (int i = threadIdx.x; i <= r_hi - r_lo; i += blockDim.x) ms_tab[i] = depth_mod(r_lo + i, nz, pc);
  __syncthreads();
  double cost = 0.0;
  float slope = 0.0f, curv = 0.0f, xs = 0.0f;
  // the adjoint's group partials of the voxel, every fourth group per lane,
  // loaded first so that they arrive while the prior terms are computed
  float u = 0.0f, dv = 0.0f;
  if (UPDATE && v < N) {
    for (int g = q; g < groups; g += 4) u += part[size_t(g) * N + v];
    if (q == 0) dv = den[v];
  }
  int row = 0, col = 0;
  if (v < N) {
    row = v / nx;
    col = v - row * nx;
    xs = x[v];
    const float ms = ms_tab[row - r_lo];
#pragma unroll
    for (int k = 2 * q; k < 2 * q + 2; ++k) {
      const int idx = k < 4 ? k : k + 1;  // the 3 x 3 neighbourhood without its centre
      const int dr = idx / 3 - 1, dc = idx % 3 - 1;
      const int r2 = row + dr, c2 = col + dc;
      if (r2 < 0 || r2 >= nz || c2 < 0 || c2 >= nx) continue;
      const float sg = pc.sigma0 * sqrtf(ms * ms_tab[r2 - r_lo]);
      const float bw = (dr == 0 || dc == 0) ? b_edge : b_diag;
      const float delta = xs - x[r2 * nx + c2];
      float hc, rho;
      qggmrf(delta, sg, pc, &hc, &rho);
      const float B = bw * hc;
      slope = fmaf(2.0f * B, delta, slope);
      curv = fmaf(4.0f, B, curv);
      // each unordered pair once: the neighbour to the right or below
      if (dr == 1 || (dr == 0 && dc == 1)) cost += double(bw) * double(rho);
    }
  }
  // the voxel's four lanes are adjacent: a butterfly gives each the same sums
  slope += __shfl_xor(slope, 1, 64);
  slope += __shfl_xor(slope, 2, 64);
  curv += __shfl_xor(curv, 1, 64);
  curv += __shfl_xor(curv, 2, 64);
  if (UPDATE) {
    u += __shfl_xor(u, 1, 64);
    u += __shfl_xor(u, 2, 64);
  }
  unsigned mbits = 0;  // |tau x_out| as float bits (non-negative floats order like their bits)
  if (UPDATE && v < N && q == 0) {
    const float grad = fmaf(-u, pc.inv_sigma2, slope);
    const float xn = xs - grad / (dv + curv);
    xout[v] = xn;
    if (fz.xt) {
      const float t = fz.tau[row] * xn;
      fz.xt[size_t(col) * fz.nzp + row] = t;
      mbits = __float_as_uint(fabsf(t));
    }
  }
  for (int off = 32; off > 0; off >>= 1) cost += __shfl_down(cost, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = cost;
  __shared__ unsigned wmax[4];
  if (UPDATE && fz.xt) {
    for (int off = 32; off >= 1; off >>= 1) mbits = max(mbits, unsigned(__shfl_xor(int(mbits), off)));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mbits;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    pcost[bx] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    if (UPDATE && fz.xt) fz.pmax[bx] = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
  }
}

template <bool UPDATE>
__global__ __launch_bounds__(4 * kPriorVox) void k_prior(const float* __restrict__ x,
                                                         const float* __restrict__ part, int groups,
                                                         const float* __restrict__ den, int nx, int nz,
                                                         PriorConst pc, float* __restrict__ xout,
                                                         double* __restrict__ pcost) {
  prior_body<UPDATE>(blockIdx.x, blockIdx.y, x, part, groups, den, nx, nz, pc, xout, pcost, PriorFuse{});
}

// The prior update with the cost (and, updating, the forward's prescale of
// x_out) folded in: see PriorFuse.
template <bool UPDATE>
__global__ __launch_bounds__(4 * kPriorVox) void k_prior_fused(const float* __restrict__ x,
                                                               const float* __restrict__ part, int groups,
                                                               const float* __restrict__ den, int nx, int nz,
                                                               PriorConst pc, float* __restrict__ xout,
                                                               double* __restrict__ pcost, PriorFuse fz) {
  prior_body<UPDATE>(blockIdx.x, blockIdx.y, x, part, groups, den, nx, nz, pc, xout, pcost, fz);
}

// Cost = data term + prior term, written to out[*counter] (then the counter
// advances) or to out[0] when counter is NULL.  The device-side counter lets a
// captured iteration graph append to the history wherever it is replayed.
__device__ __forceinline__ void cost_body(int bx, int by, const double* __restrict__ ess, int n_ess,
                                              const double* __restrict__ pcost, int n_p,
                                              double inv_2sigma2, double* __restrict__ out,
                                              int* __restrict__ counter) {
  __shared__ double sh[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n_ess; i += blockDim.x) a += ess[i];
  for (int i = threadIdx.x; i < n_p; i += blockDim.x) b += pcost[i];
  a = block_sum(a, sh);
  b = block_sum(b, sh);
  if (threadIdx.x == 0) {
    if (counter) {
      out[*counter] = a * inv_2sigma2 + b;
      *counter += 1;
    } else {
      *out = a * inv_2sigma2 + b;
    }
  }
}

__global__ __launch_bounds__(256) void k_cost(const double* __restrict__ ess, int n_ess,
                                              const double* __restrict__ pcost, int n_p,
                                              double inv_2sigma2, double* __restrict__ out,
                                              int* __restrict__ counter) {
  cost_body(blockIdx.x, blockIdx.y, ess, n_ess, pcost, n_p, inv_2sigma2, out, counter);
}

// Work-list forms for persistent batches (see the sweeps' in operator.hip):
// item (problem, x, 0) runs block x of that problem's own launch.
__global__ __launch_bounds__(256) void k_gstep_list(const BatchProb* __restrict__ probs,
                                                    const int* __restrict__ active,
                                                    const int4* __restrict__ items, int n_items) {
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    if (!active[w.x]) continue;  // uniform: the problem left the batch
    const BatchProb& p = probs[w.x];
    gstep_body<UMBIR_STORAGE_F32>(w.y, 0, p.e, p.dbasis, p.dnorm, p.g, p.M, p.est, p.ess);
    __syncthreads();
  }
}

__global__ __launch_bounds__(4 * kPriorVox) void k_prior_list(const BatchProb* __restrict__ probs,
                                                             const int* __restrict__ active,
                                                             const int4* __restrict__ items, int n_items,
                                                             int which) {
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    if (!active[w.x]) continue;
    const BatchProb& p = probs[w.x];
    const PriorFuse fz{p.tau, p.xt, p.pmax, p.nzp};
    prior_body<true>(w.y, 0, p.x[which], p.partial, p.groups, p.den, p.nx, p.nz, p.pc, p.x[which ^ 1], p.pcost, fz);
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_cost_list(const BatchProb* __restrict__ probs, const int* __restrict__ active,
                                                   const int4* __restrict__ items, int n_items) {
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    if (!active[w.x]) continue;
    const BatchProb& p = probs[w.x];
    cost_body(0, 0, p.ess, p.P * p.K, p.pcost, p.nblk, p.inv_2s2, p.cost, p.counter);
    __syncthreads();
  }
}

__global__ void k_zero_int(int* p) { *p = 0; }

int validate_prior(const umbir_prior* pr) {
  if (!pr) return fail(UMBIR_EINVAL, "prior is NULL");
  auto fin = [](double v) { return std::isfinite(v); };
  if (!fin(pr->sigma) || pr->sigma <= 0.0) return fail(UMBIR_EINVAL, "sigma must be > 0");
  if (!fin(pr->q) || pr->q != 2.0) return fail(UMBIR_EINVAL, "q must equal 2 (Sec. 2: 1 < p < q = 2)");
  if (!fin(pr->p) || !(pr->p > 1.0) || pr->p > pr->q)
    return fail(UMBIR_EINVAL, "p must satisfy 1 < p <= q");
  if (!fin(pr->T) || pr->T <= 0.0) return fail(UMBIR_EINVAL, "T must be > 0");
  if (!fin(pr->sigma0) || pr->sigma0 <= 0.0) return fail(UMBIR_EINVAL, "sigma0 must be > 0");
  if (!fin(pr->m) || pr->m <= 0.0) return fail(UMBIR_EINVAL, "m must be > 0");
  if (!fin(pr->a) || pr->a < 0.0) return fail(UMBIR_EINVAL, "a must be >= 0");
  return UMBIR_OK;
}

size_t aligned(size_t b) { return (b + 255) & ~size_t(255); }

PriorConst prior_const(const umbir_geometry& G, const umbir_prior& pr) {
  PriorConst pc;
  pc.inv_sigma2 = float(1.0 / (pr.sigma * pr.sigma));
  pc.p = float(pr.p);
  pc.T = float(pr.T);
  pc.T_pm2 = float(std::pow(pr.T, pr.p - 2.0));
  pc.sigma0 = float(pr.sigma0);
  pc.m = pr.m;
  pc.a = pr.a;
  pc.z0 = G.z0;
  pc.dz = G.dz;
  return pc;
}

// Buffers of one MAP iteration (workspace or resident session state).
struct IterBuffers {
  void* fine;
  float* partial;
  void* e;  // residual, in the storage type
  float* den;
  double* ess;
  double* pcost;
  unsigned* pmax;  // the prior update's per-block maxima of |tau x|
  int nblk;
};

IterBuffers carve_iter(Carve& cv, const umbir_geometry& G) {
  const size_t N = G.voxels(), PK = G.traces();
  IterBuffers b;
  b.nblk = int((N + kPriorVox - 1) / kPriorVox);
  b.fine = cv.take<char>(G.fine_bytes());
  b.partial = cv.take<float>(size_t(G.trace_groups) * N);
  b.e = cv.take<char>(G.trace_bytes());
  b.den = cv.take<float>(N);
  b.ess = cv.take<double>(PK);
  b.pcost = cv.take<double>(b.nblk);
  b.pmax = cv.take<unsigned>(b.nblk);
  return b;
}

size_t iter_bytes(const umbir_geometry& G) {
  const size_t N = G.voxels(), PK = G.traces();
  const size_t nblk = (N + kPriorVox - 1) / kPriorVox + 1;
  return adjoint_work_bytes(G) + aligned(G.trace_bytes()) + aligned(N * sizeof(float)) +
         aligned(PK * sizeof(double)) + aligned(nblk * sizeof(double)) + aligned(nblk * sizeof(unsigned)) + 8 * 256;
}

int enqueue_curvature(const umbir_geometry& G, const IterBuffers& b, const PriorConst& pc, hipStream_t s) {
  int st = run_forward(G, nullptr, b.e, nullptr, 1.0f, nullptr, true, b.fine, s);
  if (st) return st;
  return run_adjoint(G, b.e, b.den, pc.inv_sigma2, true, b.fine, b.partial, s);
}

// One surrogate iteration from x_in to x_out (or, with last, only the cost of
// x_in); the cost goes to cost_out[*counter] (counter != NULL) or cost_out[0]
// (none with cost_out NULL).  With prev_cost, the cost of the iteration
// before (whose sums the buffers still hold) goes to *prev_cost, computed by
// the forward's first kernel.
int enqueue_iteration(const umbir_geometry& G, const IterBuffers& b, const PriorConst& pc, double inv_2s2,
                      int est, const void* y, const float* x_in, float* x_out, float* g, bool last,
                      double* cost_out, int* counter, hipStream_t s, double* prev_cost = nullptr) {
  const int PK = G.traces();
  // the workspace holds tau x_in and its block maxima (from
  // run_prescale_blocks before the first iteration, from the previous
  // iteration's prior update after that)
  const CostFold fold{b.ess, PK, b.pcost, b.nblk, inv_2s2, prev_cost};
  int st = run_forward(G, x_in, b.e, y, -1.0f, g, false, b.fine, s, b.pmax, b.nblk, prev_cost ? &fold : nullptr);
  if (st) return st;
  switch (G.storage) {
    case UMBIR_STORAGE_F16:
      UMBIR_LAUNCH("gstep", k_gstep<UMBIR_STORAGE_F16>, dim3(unsigned(PK)), dim3(256), 0, s,
                   static_cast<Store<UMBIR_STORAGE_F16>::T*>(b.e), G.dbasis, G.dnorm, g, G.M, last ? 0 : est, b.ess);
      break;
    case UMBIR_STORAGE_BF16:
      UMBIR_LAUNCH("gstep", k_gstep<UMBIR_STORAGE_BF16>, dim3(unsigned(PK)), dim3(256), 0, s,
                   static_cast<Store<UMBIR_STORAGE_BF16>::T*>(b.e), G.dbasis, G.dnorm, g, G.M, last ? 0 : est, b.ess);
      break;
    default:
      UMBIR_LAUNCH("gstep", k_gstep<UMBIR_STORAGE_F32>, dim3(unsigned(PK)), dim3(256), 0, s, static_cast<float*>(b.e),
                   G.dbasis, G.dnorm, g, G.M, last ? 0 : est, b.ess);
      break;
  }
  if ((st = check_hip(hipGetLastError(), "k_gstep"))) return st;
  if (last) {
    UMBIR_LAUNCH("prior", k_prior<false>, dim3(b.nblk), dim3(4 * kPriorVox), 0, s, x_in, nullptr, 0, nullptr, G.nx,
                 G.nz, pc, nullptr, b.pcost);
  } else {
    // the update also puts tau x_out and its block maxima in place for the
    // next iteration's forward
    if ((st = run_adjoint_partial(G, b.e, false, b.fine, b.partial, s))) return st;
    const PriorFuse fz{G.tau, reinterpret_cast<float*>(static_cast<char*>(b.fine) + G.grids_bytes()), b.pmax, G.nzp};
    UMBIR_LAUNCH("prior", k_prior_fused<true>, dim3(b.nblk), dim3(4 * kPriorVox), 0, s, x_in, b.partial,
                 G.trace_groups, b.den, G.nx, G.nz, pc, x_out, b.pcost, fz);
  }
  if ((st = check_hip(hipGetLastError(), "k_prior"))) return st;
  if (cost_out) {
    UMBIR_LAUNCH("cost", k_cost, dim3(1), dim3(256), 0, s, b.ess, PK, b.pcost, b.nblk, inv_2s2, cost_out,
                 counter);
    if ((st = check_hip(hipGetLastError(), "k_cost"))) return st;
  }
  return UMBIR_OK;
}

// Before the first iteration from x: tau x and its block maxima into place
// for the forward (the iterations' prior updates keep them in place after).
int enqueue_start(const umbir_geometry& G, const IterBuffers& b, const float* x, hipStream_t s) {
  return run_prescale_blocks(G, x, b.fine, b.pmax, b.nblk, s);
}

// ---------------------------------------------------------------------------
// Grouped ICD (Sec. 2, "Optimization").  The paper's ICD moves one voxel at a
// time.  Here the voxels are split into the lattice groups (row % R, col % S)
// (R, S >= 2: no two members are 8-neighbours) and a group moves at once:
// member v takes its one-voxel step
//   x_v -= (-(A_v^T e) / sigma^2 + slope_v) / (dG_v / sigma^2 + curv_v)
// with the prior's neighbours held fixed (slope, curvature sum_r 2 B_sr
// (x_v - x_r) and sum_r 2 B_sr) and dG = (Abar^T Abar 1_G)_v, which bounds
// the group's block of A^T A, so every group step lowers the cost.  Then
// e -= A (step on the group).  Per group three kernels: window dot products
// per trace, the step per member (trace sums in a fixed order), and the
// residual update per trace (integer LDS accumulation: bitwise reproducible).
// A member's column in trace t is W * I_b(m Q - D Q): with J = floor(D Q) and
// phi = D Q - J, sample m holds W (phi b[k - 1] + (1 - phi) b[k]), k = m Q - J,
// nonzero for 1 <= k <= Q L_h.
struct IcdGroup {
  int r0, c0;  // first row and column of the class
  int gr;      // rows in the group
  int size;    // members
};

// Member i of a group, rows fastest: neighbouring lanes take members of one
// column Sr rows apart, whose delays differ by far more than those of
// neighbouring columns, so their windows meet fewer common samples at once.
__device__ __forceinline__ void icd_member(const IcdGroup& gp, int Sr, int Sc, int i, int* row, int* col) {
  const int cc = i / gp.gr;
  *row = gp.r0 + (i - cc * gp.gr) * Sr;
  *col = gp.c0 + cc * Sc;
}

// delay (Q32.32 samples) and weight of voxel (row, col) in trace t
__device__ __forceinline__ void icd_pair(const Leg* __restrict__ legs, int n_off, const int* __restrict__ base, int P,
                                         int K, const float* __restrict__ tau, int t, int row, int col, int64_t* D,
                                         float* W) {
  const int half = n_off / 2;
  const Leg a = legs[size_t(row) * n_off + leg_slot(abs(base[t / K] + 2 * col), half)];
  const Leg b = legs[size_t(row) * n_off + leg_slot(abs(base[P + t] + 2 * col), half)];
  *D = a.delay + b.delay;
  *W = tau[row] * (a.apod * b.apod);
}

struct IcdWindow {
  long J;
  float phi;
  int m_lo, m_hi;  // inclusive, empty when m_lo > m_hi
};

__device__ __forceinline__ IcdWindow icd_window(int64_t D, int qs, int Q, int QLh, int M) {
  IcdWindow w;
  w.J = long(uint64_t(D) >> (32 - qs));
  w.phi = float(uint32_t(uint64_t(D)) << qs) * 2.3283064365386963e-10f;
  const long lo = (w.J + Q) / Q;  // ceil((J + 1) / Q)
  const long hi = (w.J + QLh) / Q;
  w.m_lo = int(lo < 0 ? 0 : (lo > M ? M : lo));
  w.m_hi = int(hi >= M ? M - 1 : hi);
  return w;
}

constexpr int kIcdThreads = 1024;

// Window of member i in trace t: its samples lo, lo + 1, ... read the
// template at bk[d Q - 1] and bk[d Q] (k = lo Q - J + d Q), and its weight.
struct IcdSpan {
  const float* bk;
  int lo, n;  // first sample and count (0: no sample)
  float phi, W;
};

template <bool ABS>
__device__ __forceinline__ IcdSpan icd_span(const float* sb, int Q, int qs, int QLh, int M,
                                            const Leg* __restrict__ legs, int n_off, const int* __restrict__ base,
                                            int P, int K, const float* __restrict__ tau, int t, int row, int col) {
  int64_t D;
  IcdSpan o;
  icd_pair(legs, n_off, base, P, K, tau, t, row, col, &D, &o.W);
  if (ABS) o.W = fabsf(o.W);
  const IcdWindow w = icd_window(D, qs, Q, QLh, M);
  o.lo = w.m_lo;
  o.n = w.m_hi >= w.m_lo ? w.m_hi - w.m_lo + 1 : 0;
  o.phi = w.phi;
  o.bk = o.n ? sb + (long(w.m_lo) * Q - w.J) : sb + 1;  // lo Q - J >= 1: delays are non-negative
  return o;
}

// partial[i][t] = A_{t, v_i}^T e_t for the members i of the group (ABS: the
// operator of |W| and |b|): one thread per member over its window, with the
// trace and the template in LDS.
template <bool ABS>
__global__ __launch_bounds__(kIcdThreads) void k_icd_dots(const float* __restrict__ e, int M,
                                                          const float* __restrict__ bank, int Q, int qs, int QLh,
                                                          const Leg* __restrict__ legs, int n_off,
                                                          const int* __restrict__ base, int P, int K,
                                                          const float* __restrict__ tau, IcdGroup gp, int Sr, int Sc,
                                                          float* __restrict__ partial) {
  extern __shared__ float sm[];
  float* se = sm;      // [M]
  float* sb = sm + M;  // [QLh + 2]
  const int t = blockIdx.x;
  const float* et = e + size_t(t) * M;
  stage_block<float>(M, [&](int m) { return et[m]; }, [&](int m, float v) { se[m] = v; });
  stage_block<float>(QLh + 2, [&](int n) { return bank[n]; }, [&](int n, float v) { sb[n] = ABS ? fabsf(v) : v; });
  __syncthreads();
  for (int i = blockIdx.y * blockDim.x + threadIdx.x; i < gp.size; i += gridDim.y * blockDim.x) {
    int row, col;
    icd_member(gp, Sr, Sc, i, &row, &col);
    const IcdSpan w = icd_span<ABS>(sb, Q, qs, QLh, M, legs, n_off, base, P, K, tau, t, row, col);
    const float* ev = se + w.lo;
    float acc = 0.0f;
#pragma unroll 4
    for (int d = 0; d < w.n; ++d) {
      const float* b = w.bk + d * Q;
      acc = fmaf(ev[d], fmaf(w.phi, b[-1] - b[0], b[0]), acc);
    }
    partial[size_t(i) * gridDim.x + t] = w.W * acc;  // member-major: the step reads a member's traces together
  }
}

// One wave per member: the trace sum of its partials (lane strides, then a
// fixed shuffle tree).  CURV: den[v] = that sum.  Otherwise the member step
// x_v += step_i, delta[i] = step_i; the prior's eight neighbour terms are
// taken by lanes 0..7 and summed in a fixed tree.
template <bool CURV>
__global__ __launch_bounds__(256) void k_icd_step(const float* __restrict__ partial, int PK, IcdGroup gp, int Sr,
                                                  int Sc, int nx, int nz, PriorConst pc,
                                                  const float* __restrict__ ms_row, float* __restrict__ den,
                                                  float* __restrict__ x, float* __restrict__ delta) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (i >= gp.size) return;  // uniform over the wave
  int row, col;
  icd_member(gp, Sr, Sc, i, &row, &col);
  const int v = row * nx + col;
  double acc = 0.0;
  for (int t = lane; t < PK; t += 64) acc += partial[size_t(i) * PK + t];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (CURV) {
    if (lane == 0) den[v] = float(acc);
    return;
  }
  const float xs = x[v];
  float slope = 0.0f, curv = 0.0f;
  if (lane < 8) {
    const int q = lane < 4 ? lane : lane + 1;  // the 3 x 3 neighbourhood without its centre
    const int dr = q / 3 - 1, dc = q % 3 - 1;
    const int r2 = row + dr, c2 = col + dc;
    if (r2 >= 0 && r2 < nz && c2 >= 0 && c2 < nx) {
      const float b_edge = float(1.0 / (4.0 + 2.0 * M_SQRT2));
      const float b_diag = float(1.0 / (4.0 + 2.0 * M_SQRT2) / M_SQRT2);
      const float sg = pc.sigma0 * sqrtf(ms_row[row] * ms_row[r2]);
      const float bw = (dr == 0 || dc == 0) ? b_edge : b_diag;
      const float d = xs - x[r2 * nx + c2];
      float hc, rho;
      qggmrf(d, sg, pc, &hc, &rho);
      const float B = bw * hc;
      slope = 2.0f * B * d;
      curv = 2.0f * B;
    }
  }
  for (int off = 4; off > 0; off >>= 1) {
    slope += __shfl_down(slope, off, 64);
    curv += __shfl_down(curv, off, 64);
  }
  if (lane != 0) return;
  const float theta1 = -float(acc) * pc.inv_sigma2;
  const float theta2 = den[v] * pc.inv_sigma2;
  const float h = theta2 + curv;
  const float step = h > 0.0f ? -(theta1 + slope) / h : 0.0f;
  x[v] = xs + step;
  delta[i] = step;
}

// e_t -= sum_i delta_i A_{t, v_i} (ABS: the operator of |W| and |b|), summed
// in 64-bit fixed point in LDS.  Every term is at most dmax = max_i |delta_i|
// (weights, template and interpolation are <= 1) and at most `size` terms
// meet at a sample, so the scale 2^kx keeps every sum below 2^62.
template <bool ABS>
__global__ __launch_bounds__(kIcdThreads) void k_icd_scatter(float* __restrict__ e, int M,
                                                             const float* __restrict__ bank, int Q, int qs, int QLh,
                                                             const Leg* __restrict__ legs, int n_off,
                                                             const int* __restrict__ base, int P, int K,
                                                             const float* __restrict__ tau, IcdGroup gp, int Sr,
                                                             int Sc, const float* __restrict__ delta) {
  extern __shared__ unsigned long long acc[];  // [M], then the template as floats
  float* sb = reinterpret_cast<float*>(acc + M);
  __shared__ float wmax[kIcdThreads / 64];
  const int t = blockIdx.x;
  const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  float mx = 0.0f;
  for (int i = threadIdx.x; i < gp.size; i += blockDim.x) mx = fmaxf(mx, fabsf(delta[i]));
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) wmax[threadIdx.x >> 6] = mx;
  for (int m = threadIdx.x; m < M; m += blockDim.x) acc[m] = 0ull;
  stage_block<float>(QLh + 2, [&](int n) { return bank[n]; }, [&](int n, float v) { sb[n] = ABS ? fabsf(v) : v; });
  __syncthreads();
  float dmax = 0.0f;
  for (int k = 0; k < nw; ++k) dmax = fmaxf(dmax, wmax[k]);
  if (!(dmax > 0.0f)) return;  // uniform: nothing moved
  int lg = 0;
  while ((1 << lg) < gp.size) ++lg;
  const int kx = 61 - lg - ilogbf(dmax);
  const double scale = ldexp(1.0, kx);
  for (int i = threadIdx.x; i < gp.size; i += blockDim.x) {
    const float dl = delta[i];
    if (dl == 0.0f) continue;
    int row, col;
    icd_member(gp, Sr, Sc, i, &row, &col);
    const IcdSpan w = icd_span<ABS>(sb, Q, qs, QLh, M, legs, n_off, base, P, K, tau, t, row, col);
    const float s = dl * w.W;
    unsigned long long* av = acc + w.lo;
#pragma unroll 4
    for (int d = 0; d < w.n; ++d) {
      const float* b = w.bk + d * Q;
      const float v = s * fmaf(w.phi, b[-1] - b[0], b[0]);
      atomicAdd(&av[d], static_cast<unsigned long long>(__double2ll_rn(double(v) * scale)));
    }
  }
  __syncthreads();
  for (int m = threadIdx.x; m < M; m += blockDim.x) {
    const long long a = static_cast<long long>(acc[m]);
    if (a != 0) e[size_t(t) * M + m] -= float(ldexp(double(a), -kx));
  }
}

// m_s of Eq. (17) per row
__global__ void k_depth_rows(int nz, PriorConst pc, float* __restrict__ ms_row) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nz) ms_row[r] = depth_mod(r, nz, pc);
}

// delta[i] = -1 for every member: a scatter then adds the group's columns
// (e -= -1 * column)
__global__ void k_icd_unit(int n, float* __restrict__ delta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) delta[i] = -1.0f;
}

IcdGroup icd_group(const umbir_geometry& G, int Sr, int Sc, int k) {
  IcdGroup gp;
  gp.r0 = k / Sc;
  gp.c0 = k % Sc;
  gp.gr = gp.r0 < G.nz ? (G.nz - gp.r0 + Sr - 1) / Sr : 0;
  const int gc = gp.c0 < G.nx ? (G.nx - gp.c0 + Sc - 1) / Sc : 0;
  gp.size = gp.gr * gc;
  return gp;
}

int icd_max_group(const umbir_geometry& G, int Sr, int Sc) {
  return ((G.nz + Sr - 1) / Sr) * ((G.nx + Sc - 1) / Sc);
}

size_t icd_bytes(const umbir_geometry& G, int Sr, int Sc) {
  const size_t N = G.voxels(), PK = G.traces();
  const size_t gmax = size_t(icd_max_group(G, Sr, Sc));
  const size_t nblk = (N + kPriorVox - 1) / kPriorVox + 1;
  return forward_work_bytes(G) + 2 * aligned(G.trace_bytes()) + aligned(N * sizeof(float)) +
         aligned(size_t(G.nz) * sizeof(float)) +
         aligned(PK * gmax * sizeof(float)) + aligned(gmax * sizeof(float)) + aligned(PK * sizeof(double)) +
         aligned(nblk * sizeof(double)) + 16 * 256;
}

}  // namespace
}  // namespace umbir

using namespace umbir;

struct umbir_solver {
  const umbir_geometry* G = nullptr;
  umbir_prior prior{};
  PriorConst pc{};
  double inv_2s2 = 0.0;
  int est = 0;
  int device = -1;
  int max_iter = 0;
  int done = 0;     // iterations run so far
  int parity = 0;   // 0: the current image is xa, 1: xb
  void* mem = nullptr;
  size_t bytes = 0;
  IterBuffers b{};
  void* y = nullptr;  // copy of the data, storage type
  float *xa = nullptr, *xb = nullptr, *g = nullptr;
  double* cost = nullptr;  // [max_iter + 1]
  int* counter = nullptr;
  hipStream_t cap = nullptr;       // private stream used to capture the graphs
  hipGraph_t graph[2] = {nullptr, nullptr};     // xa -> xb and xb -> xa (kept for batches)
  hipGraphExec_t step[2] = {nullptr, nullptr};  // their instances
  hipEvent_t idle = nullptr;  // recorded after the last launch of an iteration graph
};

// A batch of sessions run side by side on kBatchStreams internal streams:
// session i belongs to stream i mod kBatchStreams.  UMBIR_BATCH_STREAMS
// launches each session's own iteration graphs there; UMBIR_BATCH_GRAPH
// replays one graph per image direction, captured once across the same
// streams (fork from the first, one chain of sessions per stream, join).
constexpr int kBatchStreams = 4;

struct umbir_batch {
  int device = -1;
  int mode = UMBIR_BATCH_STREAMS;
  // UMBIR_BATCH_WORKLIST: the problems split into lanes (one per batch
  // stream); per lane its problems' arguments (BatchProb[m]), their active
  // flags (int[m]) and every launch's work list in one device buffer, and its
  // launches.  A session whose max_iter is reached leaves the batch (its flag
  // is cleared and its items are skipped).
  struct Lane {
    std::vector<int> members;  // batch indices of the lane's sessions
    void* plan = nullptr;
    int* active = nullptr;
    std::vector<StageLaunch> launches;
    std::vector<int> kinds;  // BatchStage of each launch
  };
  std::vector<Lane> lanes;
  std::vector<int> lane_of, slot_of;  // per session: its lane and index there
  std::vector<char> live;
  int Q = 0;
  std::vector<umbir_solver*> s;
  std::vector<int> done;  // each session's iteration count as the batch left it
  int parity = 0;         // exec[parity] advances every session by one (graph mode)
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipStream_t st[kBatchStreams] = {};
  hipEvent_t fork = nullptr, join[kBatchStreams] = {};
  hipEvent_t idle = nullptr;  // recorded after the last batch launch
};

namespace {

size_t solver_bytes(const umbir_geometry& G, int max_iter) {
  const size_t N = G.voxels(), PK = G.traces();
  return iter_bytes(G) + aligned(G.trace_bytes()) + 2 * aligned(N * sizeof(float)) +
         aligned(PK * sizeof(float)) + aligned((size_t(max_iter) + 1) * sizeof(double)) + aligned(sizeof(int)) +
         8 * 256;
}

void solver_release(umbir_solver* S) {
  if (!S) return;
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (S->device >= 0) (void)hipSetDevice(S->device);
  // launches are asynchronous: no graph is destroyed before its last launch ended
  if (S->idle) {
    (void)hipEventSynchronize(S->idle);
    (void)hipEventDestroy(S->idle);
  }
  for (hipGraphExec_t& ge : S->step)
    if (ge) (void)hipGraphExecDestroy(ge);
  for (hipGraph_t& g : S->graph)
    if (g) (void)hipGraphDestroy(g);
  if (S->cap) (void)hipStreamDestroy(S->cap);
  if (S->mem) (void)hipFree(S->mem);
  if (cur >= 0) (void)hipSetDevice(cur);
  delete S;
}

int capture_step(umbir_solver* S, const float* x_in, float* x_out, hipGraph_t* graph, hipGraphExec_t* out) {
  int st = check_hip(hipStreamBeginCapture(S->cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  if (st) return st;
  const int st_enq = enqueue_iteration(*S->G, S->b, S->pc, S->inv_2s2, S->est, S->y, x_in, x_out, S->g, false,
                                       S->cost, S->counter, S->cap);
  st = check_hip(hipStreamEndCapture(S->cap, graph), "hipStreamEndCapture");
  if (st_enq) st = st_enq;
  if (!st) st = check_hip(hipGraphInstantiate(out, *graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  return st;
}

void batch_release(umbir_batch* B) {
  if (!B) return;
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (B->device >= 0) (void)hipSetDevice(B->device);
  if (B->idle) {
    (void)hipEventSynchronize(B->idle);
    (void)hipEventDestroy(B->idle);
  }
  for (hipGraphExec_t& ge : B->exec)
    if (ge) (void)hipGraphExecDestroy(ge);
  for (auto& L : B->lanes)
    if (L.plan) (void)hipFree(L.plan);
  if (B->fork) (void)hipEventDestroy(B->fork);
  for (int k = 0; k < kBatchStreams; ++k) {
    if (B->join[k]) (void)hipEventDestroy(B->join[k]);
    if (B->st[k]) (void)hipStreamDestroy(B->st[k]);
  }
  if (cur >= 0) (void)hipSetDevice(cur);
  delete B;
}

// Makes the batch's streams wait for `from`, and `to` wait for all of them.
int batch_fork(umbir_batch* B, hipStream_t from) {
  int st = check_hip(hipEventRecord(B->fork, from), "hipEventRecord");
  for (int k = 0; k < kBatchStreams && !st; ++k)
    st = check_hip(hipStreamWaitEvent(B->st[k], B->fork, 0), "hipStreamWaitEvent");
  return st;
}
int batch_join(umbir_batch* B, hipStream_t to) {
  int st = UMBIR_OK;
  for (int k = 0; k < kBatchStreams && !st; ++k) {
    st = check_hip(hipEventRecord(B->join[k], B->st[k]), "hipEventRecord");
    if (!st) st = check_hip(hipStreamWaitEvent(to, B->join[k], 0), "hipStreamWaitEvent");
  }
  return st;
}

// exec[which] runs one iteration of every session, in the image direction it
// will be in after `which` batch steps from now: captured from the first
// batch stream, forked to all of them, one chain of sessions per stream.
int batch_graph(umbir_batch* B, int which, hipGraphExec_t* out) {
  hipStream_t s0 = B->st[0];
  int st = check_hip(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  if (st) return st;
  int st_enq = check_hip(hipEventRecord(B->fork, s0), "hipEventRecord");
  for (int k = 1; k < kBatchStreams && !st_enq; ++k)
    st_enq = check_hip(hipStreamWaitEvent(B->st[k], B->fork, 0), "hipStreamWaitEvent");
  for (size_t i = 0; i < B->s.size() && !st_enq; ++i) {
    umbir_solver* S = B->s[i];
    const bool a_to_b = (S->parity ^ which) == 0;
    st_enq = enqueue_iteration(*S->G, S->b, S->pc, S->inv_2s2, S->est, S->y, a_to_b ? S->xa : S->xb,
                               a_to_b ? S->xb : S->xa, S->g, false, S->cost, S->counter,
                               B->st[i % kBatchStreams]);
  }
  for (int k = 1; k < kBatchStreams && !st_enq; ++k) {
    st_enq = check_hip(hipEventRecord(B->join[k], B->st[k]), "hipEventRecord");
    if (!st_enq) st_enq = check_hip(hipStreamWaitEvent(s0, B->join[k], 0), "hipStreamWaitEvent");
  }
  hipGraph_t g = nullptr;
  st = check_hip(hipStreamEndCapture(s0, &g), "hipStreamEndCapture");
  if (st_enq) st = st_enq;
  if (!st) st = check_hip(hipGraphInstantiate(out, g, nullptr, nullptr, 0), "hipGraphInstantiate");
  if (g) (void)hipGraphDestroy(g);
  return st;
}

// One iteration of one lane of a work-list batch: its launches in order,
// each over the lane's problems' work items; `which` selects each problem's
// input image (x[which]; the update writes x[which ^ 1]).
int enqueue_lane(const umbir_batch::Lane& L, int Q, int which, hipStream_t s) {
  const BatchProb* probs = static_cast<const BatchProb*>(L.plan);
  const int* active = L.active;
  int st = UMBIR_OK;
  for (size_t k = 0; k < L.launches.size() && !st; ++k) {
    const StageLaunch& SL = L.launches[k];
    if (SL.n_items == 0) continue;
    const dim3 grid(unsigned(SL.grid));
    switch (L.kinds[k]) {
      case kStGstep:
        UMBIR_LAUNCH("gstep", k_gstep_list, grid, dim3(256), 0, s, probs, active, SL.items, SL.n_items);
        st = check_hip(hipGetLastError(), "k_gstep_list");
        break;
      case kStPrior:
        UMBIR_LAUNCH("prior", k_prior_list, grid, dim3(4 * kPriorVox), 0, s, probs, active, SL.items, SL.n_items,
                     which);
        st = check_hip(hipGetLastError(), "k_prior_list");
        break;
      case kStCost:
        UMBIR_LAUNCH("cost", k_cost_list, grid, dim3(256), 0, s, probs, active, SL.items, SL.n_items);
        st = check_hip(hipGetLastError(), "k_cost_list");
        break;
      default: st = launch_sweep_stage(L.kinds[k], Q, probs, active, SL, which, s); break;
    }
  }
  return st;
}

// One graph per image direction: fork from the first batch stream to one
// stream per lane, each lane's launches, join.
int worklist_graph(umbir_batch* B, int which, hipGraphExec_t* out) {
  hipStream_t s0 = B->st[0];
  const int nl = int(B->lanes.size());
  int st = check_hip(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  if (st) return st;
  int st_enq = check_hip(hipEventRecord(B->fork, s0), "hipEventRecord");
  for (int k = 1; k < nl && !st_enq; ++k)
    st_enq = check_hip(hipStreamWaitEvent(B->st[k], B->fork, 0), "hipStreamWaitEvent");
  for (int k = 0; k < nl && !st_enq; ++k) st_enq = enqueue_lane(B->lanes[k], B->Q, which, B->st[k]);
  for (int k = 1; k < nl && !st_enq; ++k) {
    st_enq = check_hip(hipEventRecord(B->join[k], B->st[k]), "hipEventRecord");
    if (!st_enq) st_enq = check_hip(hipStreamWaitEvent(s0, B->join[k], 0), "hipStreamWaitEvent");
  }
  hipGraph_t g = nullptr;
  st = check_hip(hipStreamEndCapture(s0, &g), "hipStreamEndCapture");
  if (st_enq) st = st_enq;
  if (!st) st = check_hip(hipGraphInstantiate(out, g, nullptr, nullptr, 0), "hipGraphInstantiate");
  if (g) (void)hipGraphDestroy(g);
  return st;
}

// Builds one lane: its problems' arguments, active flags and work lists (the
// launch shapes of each problem's own iteration, so every problem gets
// bitwise the result of stepping it alone), uploaded to one device buffer,
// and its launches: splat, convolution, g step, correlation, one gather
// launch per batch of traces, prior update (with the next prescale), cost.  Each launch has a
// block per item, so the lanes' launches interleave on the device.
int worklist_lane(umbir_batch* B, umbir_batch::Lane& L) {
  const int n = int(L.members.size());
  std::vector<BatchProb> probs(n);
  std::vector<int4> items[kStages];
  size_t lds[kStages] = {};
  for (int i = 0; i < n; ++i) {
    umbir_solver* S = B->s[L.members[i]];
    const umbir_geometry& G = *S->G;
    BatchProb& bp = probs[i];
    plan_sweeps(G, i, bp, items, lds);
    bp.y = static_cast<const float*>(S->y);
    bp.e = static_cast<float*>(S->b.e);
    bp.fine = static_cast<float*>(S->b.fine);
    bp.xt = reinterpret_cast<float*>(static_cast<char*>(S->b.fine) + G.grids_bytes());
    bp.partial = S->b.partial;
    bp.den = S->b.den;
    bp.ess = S->b.ess;
    bp.pcost = S->b.pcost;
    bp.pmax = S->b.pmax;
    bp.nblk = S->b.nblk;
    bp.x[0] = S->parity ? S->xb : S->xa;  // the current image
    bp.x[1] = S->parity ? S->xa : S->xb;
    bp.g = S->g;
    bp.cost = S->cost;
    bp.counter = S->counter;
    bp.pc = S->pc;
    bp.inv_2s2 = S->inv_2s2;
    bp.est = S->est;
    for (int t = 0; t < G.traces(); ++t) items[kStGstep].push_back(make_int4(i, t, 0, 0));
    for (int b = 0; b < S->b.nblk; ++b) items[kStPrior].push_back(make_int4(i, b, 0, 0));
    items[kStCost].push_back(make_int4(i, 0, 0, 0));
  }
  // (no prescale launch: the prior update keeps each session's tau x of its
  // current image and the block maxima in place)
  // the gather's items by launch (batch index), in problem order within one
  for (int k : {int(kStGather), int(kStGatherW)})
    std::stable_sort(items[k].begin(), items[k].end(), [](const int4& a, const int4& b) { return a.w < b.w; });
  size_t bytes = aligned(size_t(n) * sizeof(BatchProb)) + aligned(size_t(n) * sizeof(int));
  for (int k = 0; k < kStages; ++k) bytes += aligned(items[k].size() * sizeof(int4));
  int st = check_hip(hipMalloc(&L.plan, bytes), "hipMalloc(batch plan)");
  if (st) return st;
  char* p = static_cast<char*>(L.plan);
  if ((st = check_hip(hipMemcpy(p, probs.data(), n * sizeof(BatchProb), hipMemcpyHostToDevice), "hipMemcpy")))
    return st;
  size_t off = aligned(size_t(n) * sizeof(BatchProb));
  L.active = reinterpret_cast<int*>(p + off);
  std::vector<int> flags(n);
  for (int i = 0; i < n; ++i) flags[i] = B->live[L.members[i]];
  if ((st = check_hip(hipMemcpy(L.active, flags.data(), n * sizeof(int), hipMemcpyHostToDevice), "hipMemcpy")))
    return st;
  off += aligned(size_t(n) * sizeof(int));
  const int4* dev_items[kStages];
  for (int k = 0; k < kStages; ++k) {
    dev_items[k] = reinterpret_cast<const int4*>(p + off);
    if (!items[k].empty() &&
        (st = check_hip(hipMemcpy(p + off, items[k].data(), items[k].size() * sizeof(int4), hipMemcpyHostToDevice),
                        "hipMemcpy")))
      return st;
    off += aligned(items[k].size() * sizeof(int4));
  }
  auto add = [&](int kind, const int4* first, int count) {
    StageLaunch SL;
    SL.items = first;
    SL.n_items = count;
    SL.grid = count;  // a block per item
    SL.lds = lds[kind];
    L.launches.push_back(SL);
    L.kinds.push_back(kind);
  };
  for (int k = 0; k < kStages; ++k) {
    if (k == kStGather || k == kStGatherW) {  // one launch per batch index
      size_t a = 0;
      while (a < items[k].size()) {
        size_t b = a;
        while (b < items[k].size() && items[k][b].w == items[k][a].w) ++b;
        add(k, dev_items[k] + a, int(b - a));
        a = b;
      }
    } else if (!items[k].empty()) {
      add(k, dev_items[k], int(items[k].size()));
    }
  }
  return UMBIR_OK;
}

// Splits the batch's problems into lanes of about equal work (largest first,
// each to the lane with the least so far) and builds every lane.
int worklist_plan(umbir_batch* B) {
  const int n = int(B->s.size());
  B->live.assign(n, 1);
  for (int i = 0; i < n; ++i) B->live[i] = B->s[i]->done < B->s[i]->max_iter;
  const int nl = std::min(n, kBatchStreams);
  B->lanes.resize(nl);
  std::vector<int> order(n);
  std::vector<double> work(n), load(nl, 0.0);
  for (int i = 0; i < n; ++i) {
    const umbir_solver* S = B->s[i];
    order[i] = i;
    work[i] = double(S->max_iter - S->done) * S->G->traces() * S->G->voxels();
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  B->lane_of.assign(n, 0);
  B->slot_of.assign(n, 0);
  for (int i : order) {
    const int l = int(std::min_element(load.begin(), load.end()) - load.begin());
    load[l] += work[i];
    B->lane_of[i] = l;
    B->slot_of[i] = int(B->lanes[l].members.size());
    B->lanes[l].members.push_back(i);
  }
  for (auto& L : B->lanes) {
    const int st = worklist_lane(B, L);
    if (st) return st;
  }
  return UMBIR_OK;
}

// Scratch of umbir_reconstruct_noalloc: a static device array, one copy per
// GPU, held from the library's load on that GPU until the process ends.  Host
// code never names it except to look up its address: on the host the name is
// only a stand-in, so kernels and copies take the per-device address below.
constexpr size_t kNoallocBytes = size_t(UMBIR_NOALLOC_SCRATCH_MIB) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};  // device address of `scratch` per device

// The current device's copy of the scratch, looked up once per device (with
// that device current) and kept.
int noalloc_scratch(void** out) {
  int dev = -1;
  int st = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (st) return st;
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(UMBIR_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if ((st = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"))) return st;
    if (!p) return fail(UMBIR_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return UMBIR_OK;
}

}  // namespace

extern "C" {

int umbir_reconstruct_noalloc(const umbir_geometry* G, const umbir_prior* pr, const void* y, int n_iter,
                              float* x_io, float* g_io, double* cost, void* stream) {
  if (!G || !y || !x_io || !g_io) return fail(UMBIR_EINVAL, "NULL argument");
  if (n_iter < 0) return fail(UMBIR_EINVAL, "n_iter must be >= 0");
  int st = validate_prior(pr);
  if (st) return st;
  const size_t need = umbir_workspace_bytes(G, UMBIR_WORK_RECONSTRUCT);
  if (need > kNoallocBytes) {
    char msg[200];
    std::snprintf(msg, sizeof msg,
                  "umbir_reconstruct_noalloc: the problem needs %zu bytes of scratch, the static scratch holds %zu",
                  need, kNoallocBytes);
    return fail(UMBIR_ENOTSUP, msg);
  }
  int dev = -1;
  if ((st = check_hip(hipGetDevice(&dev), "hipGetDevice"))) return st;
  if (dev != G->device) return fail(UMBIR_EINVAL, "the geometry's device must be current");
  void* work = nullptr;
  if ((st = noalloc_scratch(&work))) return st;
  // the iteration needs nothing of the scratch to start at zero: every
  // buffer carved from it is written before it is read
  return umbir_reconstruct(G, pr, y, n_iter, x_io, g_io, cost, work, kNoallocBytes, stream);
}

int umbir_reconstruct(const umbir_geometry* G, const umbir_prior* pr, const void* y, int n_iter,
                      float* x_io, float* g_io, double* cost, void* work, size_t work_bytes, void* stream) {
  if (!G || !y || !x_io || !g_io) return fail(UMBIR_EINVAL, "NULL argument");
  if (n_iter < 0) return fail(UMBIR_EINVAL, "n_iter must be >= 0");
  int st = validate_prior(pr);
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws;
  if ((st = ws.acquire(work, work_bytes, umbir_workspace_bytes(G, UMBIR_WORK_RECONSTRUCT), s))) return st;
  const size_t N = G->voxels();
  Carve cv{static_cast<char*>(ws.ptr)};
  const IterBuffers b = carve_iter(cv, *G);
  float* xa = cv.take<float>(N);
  float* xb = cv.take<float>(N);
  const PriorConst pc = prior_const(*G, *pr);
  const double inv_2s2 = 0.5 / (pr->sigma * pr->sigma);
  const int est = pr->estimate_direct ? 1 : 0;

  if ((st = enqueue_curvature(*G, b, pc, s))) return st;
  if ((st = launch_copy(xa, x_io, N, s))) return st;
  if ((st = enqueue_start(*G, b, xa, s))) return st;
  // the cost of iteration it - 1 is computed by iteration it's first kernel
  // (no launch of its own); the last iteration's by the cost kernel
  for (int it = 0; it <= n_iter; ++it) {
    const bool last = it == n_iter;
    if ((st = enqueue_iteration(*G, b, pc, inv_2s2, est, y, xa, xb, g_io, last,
                                cost && last ? cost + it : nullptr, nullptr, s,
                                cost && it > 0 ? cost + it - 1 : nullptr)))
      return st;
    if (!last) std::swap(xa, xb);
  }
  return launch_copy(x_io, xa, N, s);
}

size_t umbir_icd_workspace_bytes(const umbir_geometry* G, int group_rows, int group_cols) {
  if (!G || group_rows < 2 || group_cols < 2) return 0;
  return icd_bytes(*G, group_rows, group_cols);
}

int umbir_reconstruct_icd(const umbir_geometry* G, const umbir_prior* pr, const void* y, int n_sweeps,
                          int group_rows, int group_cols, float* x_io, float* g_io, double* cost, void* work,
                          size_t work_bytes, void* stream) {
  if (!G || !y || !x_io || !g_io) return fail(UMBIR_EINVAL, "NULL argument");
  if (n_sweeps < 0) return fail(UMBIR_EINVAL, "n_sweeps must be >= 0");
  if (group_rows < 2 || group_cols < 2 || group_rows > 4096 || group_cols > 4096)
    return fail(UMBIR_EINVAL, "group_rows and group_cols must be in 2..4096");
  int st = validate_prior(pr);
  if (st) return st;
  if (G->storage != UMBIR_STORAGE_F32) return fail(UMBIR_ENOTSUP, "ICD needs FP32 storage");
  if (G->n_gamma != 1) return fail(UMBIR_ENOTSUP, "ICD does not take attenuation templates");
  // a trace's residual (64-bit sums in the update) and the template stay in 64 KiB of LDS
  if (size_t(G->M) * 8 + (G->taps_per_bin() + 2) * 4 + 1024 > 65536)
    return fail(UMBIR_ENOTSUP, "ICD needs 8 n_samples + 4 (window * oversample + 2) <= 64512 bytes");
  const int Sr = group_rows, Sc = group_cols;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws;
  if ((st = ws.acquire(work, work_bytes, icd_bytes(*G, Sr, Sc), s))) return st;
  const size_t N = G->voxels();
  const int PK = G->traces(), M = G->M, Q = G->Q, QLh = int(G->taps_per_bin());
  const int qs = log2_int(Q);
  const int nblk = int((N + kPriorVox - 1) / kPriorVox);
  const int gmax = icd_max_group(*G, Sr, Sc);
  Carve cv{static_cast<char*>(ws.ptr)};
  void* fine = cv.take<char>(G->fine_bytes());
  float* e = cv.take<float>(size_t(PK) * M);
  float* etmp = cv.take<float>(size_t(PK) * M);
  float* den = cv.take<float>(N);
  float* ms_row = cv.take<float>(G->nz);
  float* part = cv.take<float>(size_t(PK) * gmax);
  float* delta = cv.take<float>(size_t(gmax));
  double* ess = cv.take<double>(PK);
  double* pcost = cv.take<double>(nblk);
  const PriorConst pc = prior_const(*G, *pr);
  const double inv_2s2 = 0.5 / (pr->sigma * pr->sigma);
  const int est = pr->estimate_direct ? 1 : 0;
  const int n_groups = Sr * Sc;

  const size_t lds_dots = (size_t(M) + QLh + 2) * sizeof(float);
  const size_t lds_scatter = size_t(M) * sizeof(unsigned long long) + (size_t(QLh) + 2) * sizeof(float);
  auto dots = [&](bool abs_op, const IcdGroup& gp, const float* ev) {
    // spread a trace's members over a few blocks when there are few traces
    const int ych = std::max(1, std::min((gp.size + kIcdThreads - 1) / kIcdThreads, 512 / std::max(PK, 1)));
    const dim3 grid{unsigned(PK), unsigned(ych), 1u};
    if (abs_op)
      UMBIR_LAUNCH("icd_dots", k_icd_dots<true>, grid, dim3(kIcdThreads), lds_dots, s, ev, M, G->bank, Q, qs, QLh,
                   G->legs, G->n_off, G->base, G->P, G->K, G->tau, gp, Sr, Sc, part);
    else
      UMBIR_LAUNCH("icd_dots", k_icd_dots<false>, grid, dim3(kIcdThreads), lds_dots, s, ev, M, G->bank, Q, qs, QLh,
                   G->legs, G->n_off, G->base, G->P, G->K, G->tau, gp, Sr, Sc, part);
  };
  auto scatter = [&](bool abs_op, const IcdGroup& gp, float* ev) {
    if (abs_op)
      UMBIR_LAUNCH("icd_scatter", k_icd_scatter<true>, dim3(unsigned(PK)), dim3(kIcdThreads), lds_scatter, s, ev, M,
                   G->bank, Q, qs, QLh, G->legs, G->n_off, G->base, G->P, G->K, G->tau, gp, Sr, Sc, delta);
    else
      UMBIR_LAUNCH("icd_scatter", k_icd_scatter<false>, dim3(unsigned(PK)), dim3(kIcdThreads), lds_scatter, s, ev,
                   M, G->bank, Q, qs, QLh, G->legs, G->n_off, G->base, G->P, G->K, G->tau, gp, Sr, Sc, delta);
  };
  const dim3 sblk(256);
  auto sgrid = [](const IcdGroup& gp) { return dim3(unsigned((gp.size + 3) / 4)); };

  UMBIR_LAUNCH("depth_rows", k_depth_rows, dim3(unsigned((G->nz + 255) / 256)), dim3(256), 0, s, G->nz, pc, ms_row);
  // group curvatures dG = (Abar^T Abar 1_G) on each group's members: the
  // group's |A| columns summed into a cleared trace buffer, then |A|^T of it
  for (int k = 0; k < n_groups; ++k) {
    const IcdGroup gp = icd_group(*G, Sr, Sc, k);
    if (gp.size == 0) continue;
    if ((st = launch_fill(etmp, size_t(PK) * M, 0.0f, s))) return st;
    UMBIR_LAUNCH("icd_unit", k_icd_unit, dim3(unsigned((gp.size + 255) / 256)), dim3(256), 0, s, gp.size, delta);
    scatter(true, gp, etmp);
    dots(true, gp, etmp);
    UMBIR_LAUNCH("icd_step", k_icd_step<true>, sgrid(gp), sblk, 0, s, part, PK, gp, Sr, Sc, G->nx, G->nz, pc,
                 ms_row, den, nullptr, nullptr);
  }
  if ((st = check_hip(hipGetLastError(), "icd curvature"))) return st;
  // e = y - A x - D g
  if ((st = run_forward(*G, x_io, e, y, -1.0f, g_io, false, fine, s))) return st;
  for (int sw = 0; sw <= n_sweeps; ++sw) {
    const bool last = sw == n_sweeps;
    UMBIR_LAUNCH("gstep", k_gstep<UMBIR_STORAGE_F32>, dim3(unsigned(PK)), dim3(256), 0, s, e, G->dbasis, G->dnorm,
                 g_io, M, last ? 0 : est, ess);
    UMBIR_LAUNCH("prior", k_prior<false>, dim3(nblk), dim3(4 * kPriorVox), 0, s, x_io, nullptr, 0, nullptr, G->nx, G->nz, pc,
                 nullptr, pcost);
    if (cost)
      UMBIR_LAUNCH("cost", k_cost, dim3(1), dim3(256), 0, s, ess, PK, pcost, nblk, inv_2s2, cost + sw, nullptr);
    if ((st = check_hip(hipGetLastError(), "icd cost"))) return st;
    if (last) break;
    for (int k = 0; k < n_groups; ++k) {
      const IcdGroup gp = icd_group(*G, Sr, Sc, k);
      if (gp.size == 0) continue;
      dots(false, gp, e);
      UMBIR_LAUNCH("icd_step", k_icd_step<false>, sgrid(gp), sblk, 0, s, part, PK, gp, Sr, Sc, G->nx, G->nz, pc,
                   ms_row, den, x_io, delta);
      scatter(false, gp, e);
    }
    if ((st = check_hip(hipGetLastError(), "icd sweep"))) return st;
  }
  return UMBIR_OK;
}

size_t umbir_solver_bytes(const umbir_geometry* G, int max_iter) {
  if (!G || max_iter < 0) return 0;
  return solver_bytes(*G, max_iter);
}

int umbir_solver_create(const umbir_geometry* G, const umbir_prior* pr, const void* y_dev,
                        const float* x0_dev, const float* g0_dev, int max_iter, void* stream,
                        umbir_solver** out) {
  if (!out) return fail(UMBIR_EINVAL, "out is NULL");
  *out = nullptr;
  if (!G || !y_dev) return fail(UMBIR_EINVAL, "NULL argument");
  if (max_iter < 0 || max_iter > (1 << 24)) return fail(UMBIR_EINVAL, "max_iter out of range");
  int st = validate_prior(pr);
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* S = new umbir_solver();
  S->G = G;
  S->prior = *pr;
  S->pc = prior_const(*G, *pr);
  S->inv_2s2 = 0.5 / (pr->sigma * pr->sigma);
  S->est = pr->estimate_direct ? 1 : 0;
  S->max_iter = max_iter;
  (void)hipGetDevice(&S->device);
  S->bytes = solver_bytes(*G, max_iter);
  if ((st = check_hip(hipMalloc(&S->mem, S->bytes), "hipMalloc(solver)"))) {
    S->mem = nullptr;
    solver_release(S);
    return st;
  }
  const size_t N = G->voxels(), PK = G->traces();
  Carve cv{static_cast<char*>(S->mem)};
  S->b = carve_iter(cv, *G);
  S->y = cv.take<char>(G->trace_bytes());
  S->xa = cv.take<float>(N);
  S->xb = cv.take<float>(N);
  S->g = cv.take<float>(PK);
  S->cost = cv.take<double>(size_t(max_iter) + 1);
  S->counter = cv.take<int>(1);
  if ((st = check_hip(hipStreamCreateWithFlags(&S->cap, hipStreamNonBlocking), "hipStreamCreate"))) {
    S->cap = nullptr;
    solver_release(S);
    return st;
  }
  if ((st = check_hip(hipEventCreateWithFlags(&S->idle, hipEventDisableTiming), "hipEventCreate"))) {
    S->idle = nullptr;
    solver_release(S);
    return st;
  }
  // state: copy of y, warm start (or zeros), curvature, cost counter at 0
  if ((st = check_hip(hipMemcpyAsync(S->y, y_dev, G->trace_bytes(), hipMemcpyDeviceToDevice, s),
                      "hipMemcpyAsync(y)")) ||
      (st = x0_dev ? launch_copy(S->xa, x0_dev, N, s) : launch_fill(S->xa, N, 0.0f, s)) ||
      (st = g0_dev ? launch_copy(S->g, g0_dev, PK, s) : launch_fill(S->g, PK, 0.0f, s)) ||
      (st = enqueue_curvature(*G, S->b, S->pc, s)) || (st = enqueue_start(*G, S->b, S->xa, s))) {
    (void)hipStreamSynchronize(s);
    solver_release(S);
    return st;
  }
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, S->counter);
  if ((st = check_hip(hipGetLastError(), "k_zero_int")) ||
      (st = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize(solver_create)"))) {
    solver_release(S);
    return st;
  }
  // one iteration graph per direction of the image ping-pong
  st = capture_step(S, S->xa, S->xb, &S->graph[0], &S->step[0]);
  if (!st) st = capture_step(S, S->xb, S->xa, &S->graph[1], &S->step[1]);
  if (st) {
    solver_release(S);
    return st;
  }
  *out = S;
  return UMBIR_OK;
}

int umbir_solver_step(umbir_solver* S, int n_iter, void* stream) {
  if (!S) return fail(UMBIR_EINVAL, "solver is NULL");
  if (n_iter < 0 || S->done + n_iter > S->max_iter)
    return fail(UMBIR_EINVAL, "n_iter would exceed the solver's max_iter");
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int k = 0; k < n_iter; ++k) {
    const int st = check_hip(hipGraphLaunch(S->step[S->parity], s), "hipGraphLaunch");
    if (st) return st;
    S->parity ^= 1;
    S->done += 1;
  }
  return n_iter > 0 ? check_hip(hipEventRecord(S->idle, s), "hipEventRecord") : UMBIR_OK;
}

int umbir_solver_iterations(const umbir_solver* S) { return S ? S->done : -1; }

int umbir_solver_read(umbir_solver* S, float* x_dev, float* g_dev, double* cost_dev, void* stream) {
  if (!S) return fail(UMBIR_EINVAL, "solver is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const umbir_geometry& G = *S->G;
  float* x = S->parity ? S->xb : S->xa;
  int st;
  if (cost_dev) {
    // cost of the current (x, g) into the slot after the history, then copy out
    if ((st = enqueue_iteration(G, S->b, S->pc, S->inv_2s2, S->est, S->y, x, nullptr, S->g, true,
                                S->cost + S->done, nullptr, s)))
      return st;
    if ((st = check_hip(hipMemcpyAsync(cost_dev, S->cost, (size_t(S->done) + 1) * sizeof(double),
                                       hipMemcpyDeviceToDevice, s),
                        "hipMemcpyAsync(cost)")))
      return st;
  }
  if (x_dev && (st = launch_copy(x_dev, x, G.voxels(), s))) return st;
  if (g_dev && (st = launch_copy(g_dev, S->g, G.traces(), s))) return st;
  return UMBIR_OK;
}

size_t umbir_solver_state_bytes(const umbir_solver* S) { return S ? S->bytes : 0; }

void umbir_solver_free(umbir_solver* S) { solver_release(S); }

int umbir_batch_create(umbir_solver* const* sessions, int n, int mode, umbir_batch** out) {
  if (!out) return fail(UMBIR_EINVAL, "out is NULL");
  *out = nullptr;
  if (!sessions || n <= 0) return fail(UMBIR_EINVAL, "need at least one session");
  if (mode != UMBIR_BATCH_STREAMS && mode != UMBIR_BATCH_GRAPH && mode != UMBIR_BATCH_WORKLIST)
    return fail(UMBIR_EINVAL, "unknown batch mode");
  for (int i = 0; i < n; ++i) {
    if (!sessions[i]) return fail(UMBIR_EINVAL, "NULL session");
    for (int j = 0; j < i; ++j)
      if (sessions[j] == sessions[i]) return fail(UMBIR_EINVAL, "session listed twice");
  }
  int dev = -1;
  int st = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (st) return st;
  for (int i = 0; i < n; ++i)
    if (sessions[i]->device != dev) return fail(UMBIR_EINVAL, "session on another device");
  if (mode == UMBIR_BATCH_WORKLIST) {
    const int q = sessions[0]->G->Q;
    for (int i = 0; i < n; ++i) {
      const umbir_geometry& G = *sessions[i]->G;
      if (G.storage != UMBIR_STORAGE_F32 || G.n_gamma != 1 || (G.Q != 32 && G.Q != 64) || G.Q != q || G.form != 1)
        return fail(UMBIR_ENOTSUP,
                    "work-list batches need FP32 storage, one template, the factored operator and one "
                    "oversampling factor of 32 or 64");
    }
  }
  auto* B = new umbir_batch();
  B->device = dev;
  B->mode = mode;
  B->s.assign(sessions, sessions + n);
  for (umbir_solver* S : B->s) B->done.push_back(S->done);
  auto event = [](hipEvent_t* e) {
    const int r = check_hip(hipEventCreateWithFlags(e, hipEventDisableTiming), "hipEventCreate");
    if (r) *e = nullptr;
    return r;
  };
  st = event(&B->idle);
  if (!st) st = event(&B->fork);
  for (int k = 0; k < kBatchStreams && !st; ++k) {
    st = event(&B->join[k]);
    if (!st) st = check_hip(hipStreamCreateWithFlags(&B->st[k], hipStreamNonBlocking), "hipStreamCreate");
    if (st) B->st[k] = nullptr;
  }
  if (!st && mode == UMBIR_BATCH_GRAPH) st = batch_graph(B, 0, &B->exec[0]);
  if (!st && mode == UMBIR_BATCH_GRAPH) st = batch_graph(B, 1, &B->exec[1]);
  if (!st && mode == UMBIR_BATCH_WORKLIST) {
    B->Q = sessions[0]->G->Q;
    st = worklist_plan(B);
    if (!st) st = worklist_graph(B, 0, &B->exec[0]);
    if (!st) st = worklist_graph(B, 1, &B->exec[1]);
  }
  if (st) {
    batch_release(B);
    return st;
  }
  *out = B;
  return UMBIR_OK;
}

int umbir_batch_step(umbir_batch* B, int n_iter, void* stream) {
  if (!B) return fail(UMBIR_EINVAL, "batch is NULL");
  if (n_iter < 0) return fail(UMBIR_EINVAL, "n_iter must be >= 0");
  for (size_t i = 0; i < B->s.size(); ++i) {
    const umbir_solver* S = B->s[i];
    if (S->done != B->done[i]) return fail(UMBIR_EINVAL, "a session was stepped outside its batch");
    if (S->done + n_iter > S->max_iter && B->mode != UMBIR_BATCH_WORKLIST)
      return fail(UMBIR_EINVAL, "n_iter would exceed a session's max_iter");
  }
  if (n_iter == 0) return UMBIR_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int st = UMBIR_OK;
  if (B->mode == UMBIR_BATCH_WORKLIST) {
    // sessions at their max_iter leave the batch before each iteration
    for (int k = 0; k < n_iter && !st; ++k) {
      bool any = false;
      for (size_t i = 0; i < B->s.size() && !st; ++i) {
        umbir_solver* S = B->s[i];
        if (B->live[i] && S->done >= S->max_iter) {
          B->live[i] = 0;
          UMBIR_LAUNCH("zero_int", k_zero_int, dim3(1), dim3(1), 0, s,
                       B->lanes[B->lane_of[i]].active + B->slot_of[i]);
          st = check_hip(hipGetLastError(), "k_zero_int");
        }
        any = any || B->live[i];
      }
      if (st || !any) break;
      st = check_hip(hipGraphLaunch(B->exec[B->parity], s), "hipGraphLaunch");
      if (st) break;
      B->parity ^= 1;
      for (size_t i = 0; i < B->s.size(); ++i)
        if (B->live[i]) {
          B->s[i]->parity ^= 1;
          B->s[i]->done += 1;
        }
    }
  } else if (B->mode == UMBIR_BATCH_GRAPH) {
    for (int k = 0; k < n_iter && !st; ++k) {
      st = check_hip(hipGraphLaunch(B->exec[B->parity], s), "hipGraphLaunch");
      if (st) break;
      B->parity ^= 1;
      for (umbir_solver* S : B->s) {
        S->parity ^= 1;
        S->done += 1;
      }
    }
  } else {
    // each session's n_iter iterations in a row on its stream, between one
    // fork from and one join to the caller's stream
    st = batch_fork(B, s);
    for (size_t i = 0; i < B->s.size() && !st; ++i) {
      umbir_solver* S = B->s[i];
      for (int k = 0; k < n_iter && !st; ++k) {
        st = check_hip(hipGraphLaunch(S->step[S->parity], B->st[i % kBatchStreams]), "hipGraphLaunch");
        if (st) break;
        S->parity ^= 1;
        S->done += 1;
      }
    }
    if (!st) st = batch_join(B, s);
  }
  for (size_t i = 0; i < B->s.size(); ++i) B->done[i] = B->s[i]->done;
  if (st) return st;
  // the batch and every session it ran wait for these launches before freeing
  st = check_hip(hipEventRecord(B->idle, s), "hipEventRecord");
  for (umbir_solver* S : B->s)
    if (!st) st = check_hip(hipEventRecord(S->idle, s), "hipEventRecord");
  return st;
}

void umbir_batch_free(umbir_batch* B) { batch_release(B); }

}  // extern "C"
