// stats.hpp -- statistics of a lattice state for bubble swarms (the
// curvature and equivalent-diameter PDFs of the swarm section): the
// histogram of the interfacial mean curvature kappa = div n (Eq.
// kappa_radius) and the cell counts of the dispersed components.  These
// evaluate a state between steps; they are not part of the coupled step.
#pragma once

#include "kernels.hpp"

namespace lbm {

constexpr int STATS_MAX_BINS = 4096;

// Outward unit normal of the dispersed phase, n = sgn grad phi / (|grad phi| +
// eps_n) with the isotropic gradient of the hydrodynamic lattice (sgn = +1 for
// bubbles, phi < 1/2 inside; -1 for droplets), written to n[a * S + idx].
template <int DIM, int QH, typename T>
__global__ __launch_bounds__(NT) void k_normal(const T* __restrict__ phi, T* __restrict__ n, Geo geo, T sgn,
                                               T eps_n) {
  using H = HydroQ<QH>;
  int x, y, z;
  block_cell(swizzled_block(), geo, x, y, z);
  if (x >= geo.nx || y >= geo.ny) return;
  const Nbr nb(x, y, z, geo);
  const int idx = nb(0, 0, 0);
  T gr[3], lap;
  grad_lap<QH, T>([&](int i) { return phi[nb(H::cx[i], H::cy[i], H::cz[i])]; }, gr, lap);
  T g2 = gr[0] * gr[0] + gr[1] * gr[1];
  if (DIM == 3) g2 += gr[2] * gr[2];
  const T den = sqrt(g2) + eps_n;
#pragma unroll
  for (int a = 0; a < DIM; ++a) n[a * geo.S + idx] = sgn * (gr[a] / den);
}

// Histogram of kappa = (1/cs^2) sum_i w_i c_i . n(x + c_i) over the interface
// cells, those with q = phi^ (1 - phi^) >= q_band (phi^ = phi clamped to
// [0, 1]).  Bin 0 counts kappa < kmin, bin nbins + 1 kappa >= kmax, bin
// 1 + floor((kappa - kmin) / (kmax - kmin) nbins) the rest, the bin taken in
// FP64 from kappa.  Counts gather in LDS per block, then in counts[].
template <int DIM, int QH, typename T>
__global__ __launch_bounds__(NT) void k_curv_hist(const T* __restrict__ phi, const T* __restrict__ n, Geo geo,
                                                  T q_band, double kmin, double kmax, int nbins,
                                                  unsigned long long* __restrict__ counts) {
  using H = HydroQ<QH>;
  __shared__ unsigned hist[STATS_MAX_BINS + 2];
  for (int b = threadIdx.x; b < nbins + 2; b += NT) hist[b] = 0u;
  __syncthreads();
  int x, y, z;
  block_cell(swizzled_block(), geo, x, y, z);
  if (x < geo.nx && y < geo.ny) {
    const Nbr nb(x, y, z, geo);
    const int idx = nb(0, 0, 0);
    const T p = phi[idx];
    const T ph = p < (T)0 ? (T)0 : (p > (T)1 ? (T)1 : p);
    if (ph * ((T)1 - ph) >= q_band) {
      T dv = 0;
#pragma unroll
      for (int i = 1; i < H::Q; i += 2) {
        const int c[3] = {H::cx[i], H::cy[i], H::cz[i]};
        const int yp = nb(c[0], c[1], c[2]), ym = nb(-c[0], -c[1], -c[2]);
        T d = 0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          if (!c[a]) continue;
          const T t = n[a * geo.S + yp] - n[a * geo.S + ym];
          d += c[a] > 0 ? t : -t;
        }
        dv += wt<H, T>(i) * d;
      }
      const double k = (double)((T)3 * dv);
      int b;
      if (k < kmin) b = 0;
      else if (k >= kmax) b = nbins + 1;
      else b = 1 + min(nbins - 1, (int)floor((k - kmin) / (kmax - kmin) * nbins));
      atomicAdd(&hist[b], 1u);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins + 2; b += NT)
    if (hist[b]) atomicAdd(&counts[b], (unsigned long long)hist[b]);
}

// Cells per component: every cell of the dispersed set (labels of k_cc_init /
// k_cc_merge, complete) adds one to the count of its root.
__global__ __launch_bounds__(NT) void k_cc_volume(Geo geo, const unsigned* __restrict__ L,
                                                  unsigned* __restrict__ vol) {
  int x, y, z;
  block_cell(swizzled_block(), geo, x, y, z);
  if (x >= geo.nx || y >= geo.ny) return;
  const unsigned idx = (unsigned)Nbr(x, y, z, geo)(0, 0, 0);
  unsigned r = L[idx];
  if (r == CC_NONE) return;
  for (unsigned up = L[r]; up != r; up = L[r]) r = up;
  atomicAdd(&vol[r], 1u);
}

// The roots' cell counts, in no particular order: out[k] for k < *count (at
// most max are written; *count is the number of components).
__global__ __launch_bounds__(NT) void k_cc_list(Geo geo, const unsigned* __restrict__ L,
                                                const unsigned* __restrict__ vol, unsigned* __restrict__ out,
                                                unsigned max, unsigned* __restrict__ count) {
  int x, y, z;
  block_cell(swizzled_block(), geo, x, y, z);
  if (x >= geo.nx || y >= geo.ny) return;
  const unsigned idx = (unsigned)Nbr(x, y, z, geo)(0, 0, 0);
  if (L[idx] != idx) return;
  const unsigned s = atomicAdd(count, 1u);
  if (s < max) out[s] = vol[idx];
}

}  // namespace lbm
