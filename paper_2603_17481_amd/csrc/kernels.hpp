// kernels.hpp -- HIP kernels of the coupled lattice step for gfx950.
//
// Per step (AA pattern, parity p = step mod 2, one population array per lattice):
//   k_phi      phi = sum_k g_k gathered with the AA parity; flags the near-contact
//              tiles that hold an interfacial cell (q >= q_th) and lists them.
//   k_nci      for listed tiles only: LDS phi tile with a halo of 4, normals and
//              indicator on tile + 3, partner search in the (2w+1)^d window and
//              the repulsive flux J (Sec. 2.3) written for every cell of the tile.
//   k_collide  fused hydrodynamic + phase-field collide and stream, in place,
//              structure-of-arrays; reads J only in flagged tiles.
//   k_diag     FP64 sums of phi and the droplet count (k_cc_init / k_cc_merge:
//              union-find labels of the dispersed set).
// Grids are 1-D; the block-to-tile mapping is XCD-aware (slab_block).
//
// Floating-point contraction is off for all of this code: every kernel that
// runs the per-cell update (single lattice, batch of lattices, with or without
// diagnostics) then evaluates exactly the operations written here in the same
// order, so a lattice's state does not depend on which kernel advanced it.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lattice.hpp"

#pragma clang fp contract(off)

namespace lbm {

constexpr int NT = 256;   // threads of the cell-wise kernels: a block covers NT cells of one
                          // z plane, 2^bxs along x (Geo::bxs) by NT >> bxs rows
constexpr int NT_NCI = 512;   // near-contact kernel: two blocks of 512 per CU fit its LDS
constexpr int PHI_HALO = 4;   // window radius 3 + 1 for the normals
constexpr int NQ_HALO = 3;    // window radius
constexpr int NPART = 16;     // doubles per block in the reduction scratch

// Reduction slots of the collide pass (k_diag uses 0 phi, 1 droplet roots,
// 6 non-finite): 0 p*, 1-3 rho u, 4 kinetic energy, 5 max |u|, 6 non-finite,
// 7 near-contact cells, 8 film cells, 9 |F_rep.n|, 10 |F_cap.n|, 11 |F_rep|
// (sums over the film), 12 max |F_rep|.  Slots 5 and 12 reduce by maximum.
__host__ __device__ constexpr bool max_slot(int k) { return k == 5 || k == 12; }

struct Geo {
  int nx, ny, nz;
  int nbx, nby;          // blocks along x and y (BX x BY cells each)
  long long S;           // plane stride of the structure-of-arrays fields (phi, J)
  int ntx, nty, ntz;     // near-contact tiles along x, y, z
  int rs;                // population chunks hold R = 2^rs rows ...
  int qc;                // ... i.e. qc = R nx cells per population
  int bxs;               // cell-wise blocks are 2^bxs cells wide (6, 7 or 8)
};

struct Phys {
  double rho_g, drho;    // rho = rho_g + drho phi
  double mu_a, mu_b;     // dynamic viscosity rho nu = mu_a + mu_b phi
  double beta4, kappa;   // mu_phi = beta4 phi (phi-1)(phi-1/2) - kappa lap phi
  double rho_mean;       // box mean of rho (for the buoyancy force)
  double g[3];
  double kc;             // M 4 / W (0 when the counter-gradient flux is off)
  double inv_tau_phi;    // 1 / (1/2 + M / cs_phi^2)
  double pstar_ref;      // reference p* of the 16-bit population encoding
  double eps_n;          // regularisation of the normal n = grad phi / (|grad phi| + eps_n)
};

struct NciP {
  double a_rep, q_th, eta, cos_opp, h0, p_exp, eps_n, eps_q, width, tie_eps;
  int w, orient;
};

// Near-contact tile of each (dimension, precision); the FP64 tile is thinner so
// that its LDS footprint stays below 96 KB.
template <int DIM, typename T>
struct NciTile;
template <typename T>
struct NciTile<2, T> {
  static constexpr int TX = 16, TY = 16, TZ = 1;
};
template <>
struct NciTile<3, float> {
  static constexpr int TX = 8, TY = 8, TZ = 8;
};
template <>
struct NciTile<3, double> {
  static constexpr int TX = 8, TY = 8, TZ = 4;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// XCD k (blocks b = k mod 8) takes the k-th eighth of the grid: the mapping of
// the multi-lattice launches and of the kernels whose atomics (tile flags and
// lists, component labels) should stay within one XCD's L2.
__device__ __forceinline__ int swizzled_block() {
  const int b = blockIdx.x, n = gridDim.x;
  const int full = n & ~7;
  return b < full ? (b & 7) * (n >> 3) + (b >> 3) : b;
}

__device__ __forceinline__ int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Populations are touched once per step: their aligned loads and stores carry
// the nontemporal hint (streamed past the caches), which takes the even AA
// parity from about 5.5 to 4.6 ms at 512^3 FP32 and the FP16-storage collide
// from 3.64 to 3.45 ms (hinted loads alone slow it down).  Store<S>::ldh / sth
// are the hinted forms, ld / st the plain ones.
template <typename E>
__device__ __forceinline__ E ld_nt(const E* p) { return __builtin_nontemporal_load(p); }
template <typename E>
__device__ __forceinline__ void st_nt(E* p, E v) { __builtin_nontemporal_store(v, p); }

template <typename S>
struct Store;
template <>
struct Store<double> {
  __device__ static double ld(const double* p, double) { return *p; }
  __device__ static void st(double* p, double v, double) { *p = v; }
  __device__ static double ldh(const double* p, double) { return ld_nt(p); }
  __device__ static void sth(double* p, double v, double) { st_nt(p, v); }
};
template <>
struct Store<float> {
  __device__ static float ld(const float* p, float) { return *p; }
  __device__ static void st(float* p, float v, float) { *p = v; }
  __device__ static float ldh(const float* p, float) { return ld_nt(p); }
  __device__ static void sth(float* p, float v, float) { st_nt(p, v); }
};
template <>
struct Store<__half> {
  __device__ static float ld(const __half* p, float off) { return __half2float(*p) + off; }
  __device__ static void st(__half* p, float v, float off) { *p = __float2half_rn(v - off); }
  __device__ static float ldh(const __half* p, float off) {
    return __half2float(__ushort_as_half(ld_nt((const unsigned short*)p))) + off;
  }
  __device__ static void sth(__half* p, float v, float off) {
    st_nt((unsigned short*)p, __half_as_ushort(__float2half_rn(v - off)));
  }
};
template <>
struct Store<__hip_bfloat16> {
  __device__ static float ld(const __hip_bfloat16* p, float off) { return __bfloat162float(*p) + off; }
  __device__ static void st(__hip_bfloat16* p, float v, float off) { *p = __float2bfloat16(v - off); }
  __device__ static float ldh(const __hip_bfloat16* p, float off) {
    return __bfloat162float(__ushort_as_bfloat16(ld_nt((const unsigned short*)p))) + off;
  }
  __device__ static void sth(__hip_bfloat16* p, float v, float off) {
    st_nt((unsigned short*)p, __bfloat16_as_ushort(__float2bfloat16(v - off)));
  }
};

// Element e of a population plane.  With OFF32 the byte offset is formed in 32
// bits (valid while every plane is below 4 GiB), so the access can use the
// uniform plane base in scalar registers plus a 32-bit per-lane offset.
template <bool OFF32, typename E>
__device__ __forceinline__ E* plane_at(E* base, unsigned e) {
  if constexpr (OFF32)
    return (E*)((char*)base + (unsigned)(e * (unsigned)sizeof(E)));
  else
    return base + e;
}

__device__ __forceinline__ float m_sqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ double m_sqrt(double a) { return sqrt(a); }
__device__ __forceinline__ float m_acosh(float a) { return acoshf(a); }
__device__ __forceinline__ double m_acosh(double a) { return acosh(a); }
__device__ __forceinline__ float m_pow(float a, float b) { return powf(a, b); }
__device__ __forceinline__ double m_pow(double a, double b) { return pow(a, b); }
__device__ __forceinline__ float m_abs(float a) { return fabsf(a); }
__device__ __forceinline__ float m_max(float a, float b) { return a > b ? a : b; }
__device__ __forceinline__ double m_max(double a, double b) { return a > b ? a : b; }
__device__ __forceinline__ double m_abs(double a) { return fabs(a); }

// Periodic neighbours of a cell: index of x + (dx, dy, dz), |d| <= 1.
struct Nbr {
  int xs[3];
  int ys[3];      // nx * y'
  long long zs[3];  // nx * ny * z'  (kept 64-bit to be safe; converted on use)
  __device__ Nbr(int x, int y, int z, const Geo& g) {
    xs[0] = x == 0 ? g.nx - 1 : x - 1;
    xs[1] = x;
    xs[2] = x == g.nx - 1 ? 0 : x + 1;
    ys[0] = g.nx * (y == 0 ? g.ny - 1 : y - 1);
    ys[1] = g.nx * y;
    ys[2] = g.nx * (y == g.ny - 1 ? 0 : y + 1);
    const long long pl = (long long)g.nx * g.ny;
    zs[0] = pl * (z == 0 ? g.nz - 1 : z - 1);
    zs[1] = pl * z;
    zs[2] = pl * (z == g.nz - 1 ? 0 : z + 1);
  }
  __device__ __forceinline__ int operator()(int dx, int dy, int dz) const {
    return xs[dx + 1] + ys[dy + 1] + (int)zs[dz + 1];
  }
};

// Population layout.  Within each z plane the rows are grouped in chunks of
// R = 2^rs rows, and a chunk stores the Q population planes of its qc = R nx
// cells one after the other.  Element (q; x, y, z) of an array of Q populations:
//   z nx ny Q + (y >> rs) Q qc + q qc + (y mod R) nx + x.
// A block covers cells of one z plane, so the z term is uniform over it and
// goes into the (scalar) base pointer; the rest, below nx ny Q, is the lane's
// offset.  The 26 streams of a block then fall into a few contiguous regions
// of a z plane instead of 26 planes gigabytes apart.
template <typename E>
__device__ __forceinline__ E* pop_zplane(E* base, int z, const Geo& g, int Q) {
  return base + (size_t)z * ((size_t)g.nx * g.ny * Q);
}
__device__ __forceinline__ unsigned pop_row(int y, const Geo& g, int Q) {
  return (unsigned)(y >> g.rs) * (unsigned)(Q * g.qc) + (unsigned)(y & ((1 << g.rs) - 1)) * (unsigned)g.nx;
}
__device__ __forceinline__ size_t pop_elem(int q, int x, int y, int z, const Geo& g, int Q) {
  return (size_t)z * ((size_t)g.nx * g.ny * Q) + pop_row(y, g, Q) + (unsigned)x + (unsigned)(q * g.qc);
}

// Periodic neighbourhood of a cell in the population layout of an array of Q
// populations: x' and the row part of the offset for y' = y - 1, y, y + 1, and
// the z plane bases for z - 1, z, z + 1.
template <typename E>
struct PopNbr {
  unsigned xs[3], ys[3];
  E* zp[3];
  unsigned qc;
  __device__ PopNbr(E* base, int x, int y, int z, const Geo& g, int Q) : qc((unsigned)g.qc) {
    xs[0] = (unsigned)(x == 0 ? g.nx - 1 : x - 1);
    xs[1] = (unsigned)x;
    xs[2] = (unsigned)(x == g.nx - 1 ? 0 : x + 1);
    ys[0] = pop_row(y == 0 ? g.ny - 1 : y - 1, g, Q);
    ys[1] = pop_row(y, g, Q);
    ys[2] = pop_row(y == g.ny - 1 ? 0 : y + 1, g, Q);
    zp[0] = pop_zplane(base, z == 0 ? g.nz - 1 : z - 1, g, Q);
    zp[1] = pop_zplane(base, z, g, Q);
    zp[2] = pop_zplane(base, z == g.nz - 1 ? 0 : z + 1, g, Q);
  }
  // population q of the cell at offset (dx, dy, dz)
  template <bool OFF32>
  __device__ __forceinline__ E* at(int q, int dx, int dy, int dz) const {
    return plane_at<OFF32>(zp[dz + 1], ys[dy + 1] + xs[dx + 1] + (unsigned)q * qc);
  }
};

// s . v for a lattice vector s whose components are -1, 0 or 1 and known at
// compile time once the direction loops are unrolled: the nonzero terms are
// added with their signs, so no product by 0 or +-1 is evaluated.
template <typename T>
__device__ __forceinline__ T sdot(int sx, int sy, int sz, T vx, T vy, T vz) {
  T acc = (T)0;
  bool any = false;
  auto add = [&](int sg, T v) {
    if (!sg) return;
    acc = any ? (sg > 0 ? acc + v : acc - v) : (sg > 0 ? v : -v);
    any = true;
  };
  add(sx, vx);
  add(sy, vy);
  add(sz, vz);
  return acc;
}

// a * b + c with one rounding (an explicit fused multiply-add; nothing is fused
// implicitly in this code).
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// c c : A for a symmetric tensor stored as (xx yy zz xy xz yz).
template <typename T>
__device__ __forceinline__ T ccdot(int cx, int cy, int cz, const T A[6]) {
  const T d = sdot(cx * cx, cy * cy, cz * cz, A[0], A[1], A[2]);
  if (cx * cy == 0 && cx * cz == 0 && cy * cz == 0) return d;
  return d + (T)2 * sdot(cx * cy, cx * cz, cy * cz, A[3], A[4], A[5]);
}

// Isotropic gradient and Laplacian with the weights of the hydrodynamic lattice
// of QH velocities (Eqs. grad_iso, lap_iso; 1/cs^2 = 3).  get(i) returns
// psi(x + c_i).
template <int QH, typename T, typename G>
__device__ __forceinline__ void grad_lap(const G& get, T gr[3], T& lap) {
  using L = HydroQ<QH>;
  constexpr int DIM = L::D;
  T g0 = 0, g1 = 0, g2 = 0, sn = 0;
#pragma unroll
  for (int i = 1; i < L::Q; i += 2) {
    const T a = get(i), b = get(i + 1);
    const T w = wt<L, T>(i);
    const T d = w * (a - b);
    if (L::cx[i]) g0 += L::cx[i] > 0 ? d : -d;
    if (L::cy[i]) g1 += L::cy[i] > 0 ? d : -d;
    if (DIM == 3 && L::cz[i]) g2 += L::cz[i] > 0 ? d : -d;
    sn += w * (a + b);
  }
  gr[0] = (T)3 * g0;
  gr[1] = (T)3 * g1;
  gr[2] = DIM == 3 ? (T)3 * g2 : (T)0;
  lap = (T)6 * (sn - ((T)1 - wt<L, T>(0)) * get(0));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T u = __shfl_xor(v, o, 64);
    v = u > v ? u : v;
  }
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T u = __shfl_xor(v, o, 64);
    v = u < v ? u : v;
  }
  return v;
}

// ---------------------------------------------------------------------------
// (a1) phi moment of the phase-field populations
// ---------------------------------------------------------------------------

// phi of one cell from its incoming phase-field populations (AA parity PAR),
// accumulated in FP64 (exact for FP32 populations) and rounded once.
template <int DIM, int PAR, typename T, typename GS>
__device__ __forceinline__ T phi_moment(const GS* __restrict__ g, const Geo& geo, int x, int y, int z) {
  using P = Phase<DIM>;
  double acc = 0.0;
  const PopNbr<const GS> pn(g, x, y, z, geo, P::Q);
  if constexpr (PAR == 0) {
#pragma unroll
    for (int i = 0; i < P::Q; ++i) acc += (double)ld_nt(pn.template at<false>(i, 0, 0, 0));
  } else {
#pragma unroll
    for (int i = 0; i < P::Q; ++i)
      acc += (double)ld_nt(pn.template at<false>(opp(i), -P::cx[i], -P::cy[i], -P::cz[i]));
  }
  return (T)acc;
}

// An interfacial cell (q = phi(1 - phi) at or above q_th, phi clamped to [0, 1])
// flags its near-contact tile and lists it once.
template <int DIM, typename T>
__device__ __forceinline__ void phi_mark(T s, const Geo& geo, unsigned* __restrict__ flags,
                                         unsigned* __restrict__ list, unsigned* __restrict__ cnt, T q_th,
                                         int x, int y, int z) {
  using TL = NciTile<DIM, T>;
  const T pc = s < (T)0 ? (T)0 : (s > (T)1 ? (T)1 : s);
  const T q = pc * ((T)1 - pc);
  if (q >= q_th) {
    const unsigned tile = (unsigned)(x / TL::TX + geo.ntx * (y / TL::TY + geo.nty * (z / TL::TZ)));
    if (flags[tile] == 0u && atomicExch(&flags[tile], 1u) == 0u) list[atomicAdd(cnt, 1u)] = tile;
  }
}

// phi of one cell (the moment, or the stored field of the finite-difference
// phase field), and its near-contact tile mark.
template <int DIM, int PAR, typename T, typename GS, bool GIVEN = false>
__device__ __forceinline__ void phi_cell(const GS* __restrict__ g, T* __restrict__ phi, const Geo& geo,
                                         unsigned* __restrict__ flags, unsigned* __restrict__ list,
                                         unsigned* __restrict__ cnt, int nci_on, T q_th, int x, int y,
                                         int z) {
  const int idx = x + geo.nx * (y + geo.ny * z);
  T s;
  if constexpr (GIVEN) {
    s = phi[idx];
  } else {
    s = phi_moment<DIM, PAR, T, GS>(g, geo, x, y, z);
    st_nt(phi + idx, s);   // read again by other kernels only
  }
  if (nci_on) phi_mark<DIM, T>(s, geo, flags, list, cnt, q_th, x, y, z);
}

// Tile of block for the fused collide + stream.  The hardware deals blocks to
// the 8 XCDs round-robin (block b to XCD b mod 8); here XCD k takes the slabs
// k, k + 8, k + 16, ... of the domain in order, a slab being a z plane in 3D
// and a row of blocks in 2D.  The XCDs thus stream through neighbouring slabs
// together, which keeps the HBM traffic of the moment within a few planes
// (2 % faster than giving each XCD one contiguous eighth); slabs beyond the
// last multiple of 8 keep their own order.
__device__ __forceinline__ int slab_block(const Geo& g) {
  const int b = blockIdx.x;
  const int per = g.nz > 1 ? g.nbx * g.nby : g.nbx;   // blocks per slab
  const int nslab = g.nz > 1 ? g.nz : g.nby;
  const int full = (nslab & ~7) * per;
  if (b >= full) return b;
  const int k = b & 7, i = b >> 3;
  return (k + 8 * (i / per)) * per + i % per;
}

// Cell of thread: block t of a domain covers 2^bxs x (NT >> bxs) cells of one
// z plane.  Rows of 256 cells (1 KB per population in FP32) stream 4.5 % faster
// through the collide than 64 x 4 blocks at 512^3; narrow boxes use 64-wide
// blocks so that few lanes idle.
__device__ __forceinline__ void block_cell(int t, const Geo& geo, int& x, int& y, int& z) {
  const int bx = t % geo.nbx, r = t / geo.nbx, by = r % geo.nby;
  z = r / geo.nby;
  x = (bx << geo.bxs) + (int)(threadIdx.x & ((1u << geo.bxs) - 1u));
  y = by * (NT >> geo.bxs) + (int)(threadIdx.x >> geo.bxs);
}

template <int DIM, int PAR, typename T, typename GS, bool GIVEN>
__global__ __launch_bounds__(NT) void k_phi(const GS* __restrict__ g, T* __restrict__ phi, Geo geo,
                                            unsigned* __restrict__ flags,
                                            unsigned* __restrict__ list,
                                            unsigned* __restrict__ cnt,
                                            unsigned* __restrict__ nci_count, int nci_on, T q_th) {
  if (nci_on && blockIdx.x == 0 && threadIdx.x == 0) {
    nci_count[0] = 0u;                 // cells with a partner
    nci_count[4] = nci_count[1];       // tiles the previous near-contact pass took
    nci_count[1] = 0u;                 // tiles selected for this one
  }
  int x, y, z;
  block_cell(swizzled_block(), geo, x, y, z);
  if (x >= geo.nx || y >= geo.ny) return;
  phi_cell<DIM, PAR, T, GS, GIVEN>(g, phi, geo, flags, list, cnt, nci_on, q_th, x, y, z);
}

// ---------------------------------------------------------------------------
// (a2) near-contact detection, pairing and repulsive flux (Sec. 2.3)
// ---------------------------------------------------------------------------

// Wrapped coordinate for offsets within one tile + halo of the box.
__device__ __forceinline__ int wrap_near(int v, int n) {
  if (n >= 32) return v < 0 ? v + n : (v >= n ? v - n : v);
  return wrapi(v, n);
}

// Lexicographic minimum of (d2, dot) over the lanes of an 8-lane group.
template <typename T>
__device__ __forceinline__ void group_min(int& d2, T& dot) {
#pragma unroll
  for (int o = 1; o < 8; o <<= 1) {
    const int d2o = __shfl_xor(d2, o, 64);
    const T doto = __shfl_xor(dot, o, 64);
    if (d2o < d2 || (d2o == d2 && doto < dot)) {
      d2 = d2o;
      dot = doto;
    }
  }
}

// Normal and indicator of one cell of the near-contact region, read as one
// 16-byte (FP32) / 32-byte (FP64) LDS access.
template <typename T>
struct alignas(4 * sizeof(T)) NQ {
  T n0, n1, n2, q;
};

template <int DIM, typename T>
struct NciShared {
  using TL = NciTile<DIM, T>;
  static constexpr int TX = TL::TX, TY = TL::TY, TZ = TL::TZ, TC = TX * TY * TZ;
  static constexpr int PX = TX + 2 * PHI_HALO, PY = TY + 2 * PHI_HALO, PZ = DIM == 3 ? TZ + 2 * PHI_HALO : 1;
  static constexpr int NX = TX + 2 * NQ_HALO, NY = TY + 2 * NQ_HALO, NZ = DIM == 3 ? TZ + 2 * NQ_HALO : 1;
  static constexpr int NPH = PX * PY * PZ, NNQ = NX * NY * NZ;
  struct Out {
    T gJ[TC][DIM];   // result per gated cell
    int gpart[TC];   // packed partner offset + 1 (0: no partner)
  };
  // normal ranges of step 2b: per x row and x half (A), then per z plane and
  // x, y half (B); 6 values each (lo[3], hi[3])
  struct Ranges {
    T A[NY * NZ * 2][6];
    T B[NZ * 4][6];
  };
  union {
    T phs[NPH];      // phi tile with halo (steps 1-2)
    Ranges rg;       // step 2b
    Out out;         // results (steps 4-6)
  };
  NQ<T> nq[NNQ];
  short glist[TC];   // gated tile cells
  short gslot[TC];   // tile cell -> index in glist, or -1
  T box[8][2][3];    // per sub-tile: smallest and largest normal components
  int ng;
};

// Clears the tile flags of the other AA parity (set by the previous step) so
// that the next step's phi pass starts from empty flags.
__device__ __forceinline__ void nci_clear_other(unsigned* __restrict__ flags_other,
                                                const unsigned* __restrict__ list_other,
                                                const unsigned* __restrict__ cnt_other) {
  const unsigned nother = *cnt_other;
  for (unsigned k = blockIdx.x * NT_NCI + threadIdx.x; k < nother; k += gridDim.x * NT_NCI)
    flags_other[list_other[k]] = 0u;
}

// The phi values of step 1 for one tile, held in registers: lanes along x, one
// row of PX cells per PX lanes, a compile-time number of passes.  load() is
// issued for the next tile while the current one is processed, so that its
// latency is hidden; store() puts the values into the LDS tile.
template <int DIM, typename T>
struct NciHalo {
  using S = NciShared<DIM, T>;
  using TL = NciTile<DIM, T>;
  static constexpr int RPI = NT_NCI / S::PX;      // rows per pass
  static constexpr int NROW = S::NPH / S::PX;
  static constexpr int NPASS = (NROW + RPI - 1) / RPI;
  T v[NPASS];
  __device__ __forceinline__ void load(unsigned t, const T* __restrict__ phi, const Geo& geo) {
    const int tx = (int)(t % (unsigned)geo.ntx);
    const int ty = (int)((t / (unsigned)geo.ntx) % (unsigned)geo.nty);
    const int tz = (int)(t / ((unsigned)geo.ntx * (unsigned)geo.nty));
    const int ex = (int)threadIdx.x % S::PX, rr = (int)threadIdx.x / S::PX;
    const int gx = wrap_near(tx * TL::TX + ex - PHI_HALO, geo.nx);
    if (rr >= RPI) return;
#pragma unroll
    for (int it = 0; it < NPASS; ++it) {
      const int r = rr + it * RPI;
      if (NROW % RPI != 0 && r >= NROW) break;
      const int ey = r % S::PY, ez = r / S::PY;
      const int gy = wrap_near(ty * TL::TY + ey - PHI_HALO, geo.ny);
      const int gz = DIM == 3 ? wrap_near(tz * TL::TZ + ez - PHI_HALO, geo.nz) : 0;
      v[it] = phi[gx + geo.nx * (gy + geo.ny * gz)];
    }
  }
  __device__ __forceinline__ void store(S& sm) const {
    const int ex = (int)threadIdx.x % S::PX, rr = (int)threadIdx.x / S::PX;
    if (rr >= RPI) return;
#pragma unroll
    for (int it = 0; it < NPASS; ++it) {
      const int r = rr + it * RPI;
      if (NROW % RPI != 0 && r >= NROW) break;
      sm.phs[ex + S::PX * r] = v[it];
    }
  }
};

// Per listed tile: (1) phi with a halo of 4 into LDS; (2) q on tile + 3 and
// n where q >= q_th, packed with q; (3) the gated cells of the tile are listed;
// (4) each gated cell gets an 8-lane group whose lanes scan one window plane
// each (dz in 3D, dy in 2D), the window radius WR being a compile-time
// constant so that the scan is unrolled and its LDS reads use immediate
// offsets: pass 0 finds the smallest |r|^2 and the smallest n(x).n(y) at it,
// pass 1 (only where a partner exists) the first candidate in scan order
// within tie_eps of that dot; the planes are combined with wave shuffles;
// (5) the group leader builds J (Sec. 2.3.3) and the tile's J is written from
// LDS, zero for cells without a partner.
template <int DIM, int QH, typename T, bool DEBUG, int WR>
__device__ __forceinline__ void nci_tile(NciShared<DIM, T>& sm, unsigned t, NciHalo<DIM, T>& halo, bool next,
                                         unsigned tn, const T* __restrict__ phi,
                                         T* __restrict__ J, int* __restrict__ chi_out,
                                         int* __restrict__ part_out, const Geo& geo, const NciP& np,
                                         unsigned& my_active) {
  using TL = NciTile<DIM, T>;
  using L = HydroQ<QH>;
  constexpr int TX = TL::TX, TY = TL::TY, TZ = TL::TZ;
  constexpr int TC = TX * TY * TZ;
  constexpr int PX = NciShared<DIM, T>::PX, PY = NciShared<DIM, T>::PY;
  constexpr int NX = NciShared<DIM, T>::NX, NY = NciShared<DIM, T>::NY;
  constexpr int NNQ = NciShared<DIM, T>::NNQ;
  static_assert(WR >= 1 && WR <= NQ_HALO, "window radius");
  const T q_th = (T)np.q_th, eta = (T)np.eta, cos_opp = (T)np.cos_opp, eps_n = (T)np.eps_n,
          eps_q = (T)np.eps_q, tie = (T)np.tie_eps;
  const int lane8 = threadIdx.x & 7, grp = threadIdx.x >> 3;
  constexpr int NGRP = NT_NCI / 8;
  const int tx = (int)(t % (unsigned)geo.ntx);
  const int ty = (int)((t / (unsigned)geo.ntx) % (unsigned)geo.nty);
  const int tz = (int)(t / ((unsigned)geo.ntx * (unsigned)geo.nty));
  const int ox = tx * TX, oy = ty * TY, oz = tz * TZ;
  if (threadIdx.x == 0) sm.ng = 0;
  // (1) phi tile with halo (loaded into registers before: for the first tile by
  // the caller, for the others during the previous tile), then the next
  // tile's loads are issued
  halo.store(sm);
  __syncthreads();
  if (next) halo.load(tn, phi, geo);
  // (2) indicator everywhere on tile + 3, normal where the indicator passes the gate
  {
    constexpr int RPI = NT_NCI / NX;
    constexpr int NROW = NNQ / NX;
    const int ex = (int)threadIdx.x % NX, rr = (int)threadIdx.x / NX;
    if (rr < RPI)
      for (int r = rr; r < NROW; r += RPI) {
        const int ey = r % NY, ez = r / NY;
        const int c = (ex + 1) + PX * ((ey + 1) + PY * (DIM == 3 ? ez + 1 : 0));
        const T ph = sm.phs[c];
        const T pc = ph < (T)0 ? (T)0 : (ph > (T)1 ? (T)1 : ph);
        NQ<T> v{(T)0, (T)0, (T)0, pc * ((T)1 - pc)};
        if (v.q >= q_th) {
          T gr[3], lap;
          grad_lap<QH, T>([&](int i) { return sm.phs[c + L::cx[i] + PX * (L::cy[i] + PY * L::cz[i])]; },
                           gr, lap);
          T mag = gr[0] * gr[0] + gr[1] * gr[1];
          if (DIM == 3) mag += gr[2] * gr[2];
          const T inv = (T)1 / (m_sqrt(mag) + eps_n);
          v.n0 = gr[0] * inv;
          v.n1 = gr[1] * inv;
          if (DIM == 3) v.n2 = gr[2] * inv;
        }
        sm.nq[ex + NX * r] = v;
      }
  }
  __syncthreads();
  // (2b) per sub-tile (the tile halved along each axis) the range [lo, hi] of
  // each normal component over the gated cells of the region that the windows
  // of its cells cover.  Minima and maxima are separable: each thread reduces
  // a run along x (one x row, one x half), then along y, then along z, with
  // a barrier between the passes and no cross-lane reductions.
  constexpr int SX = TX / 2, SY = TY / 2, SZ = DIM == 3 ? TZ / 2 : 1;
  {
    constexpr int RX = SX + 2 * NQ_HALO, RY = SY + 2 * NQ_HALO, RZ = DIM == 3 ? SZ + 2 * NQ_HALO : 1;
    constexpr int NSUB = DIM == 3 ? 8 : 4;
    constexpr int NZ = NciShared<DIM, T>::NZ;
    static_assert(NY * NZ * 2 <= NT_NCI, "one x run per thread");
    auto merge = [](T r[6], const T* v) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        r[a] = v[a] < r[a] ? v[a] : r[a];
        r[3 + a] = v[3 + a] > r[3 + a] ? v[3 + a] : r[3 + a];
      }
    };
    const int t = threadIdx.x;
    if (t < NY * NZ * 2) {   // t = 2 (row) + x half
      const int row = t >> 1, bx = (t & 1) * SX;
      T r[6] = {(T)1, (T)1, (T)1, (T)-1, (T)-1, (T)-1};
#pragma unroll
      for (int i = 0; i < RX; ++i) {
        const NQ<T> v = sm.nq[bx + i + NX * row];
        if (v.q >= q_th) {
          const T n[6] = {v.n0, v.n1, v.n2, v.n0, v.n1, v.n2};
          merge(r, n);
        }
      }
#pragma unroll
      for (int a = 0; a < 6; ++a) sm.rg.A[t][a] = r[a];
    }
    __syncthreads();
    if (t < NZ * 4) {   // t = 4 z + 2 (y half) + x half
      const int ez = t >> 2, by = ((t >> 1) & 1) * SY, sx = t & 1;
      T r[6] = {(T)1, (T)1, (T)1, (T)-1, (T)-1, (T)-1};
#pragma unroll
      for (int j = 0; j < RY; ++j) merge(r, sm.rg.A[2 * (by + j + NY * ez) + sx]);
#pragma unroll
      for (int a = 0; a < 6; ++a) sm.rg.B[t][a] = r[a];
    }
    __syncthreads();
    if (t < NSUB) {   // t = 4 (z half) + 2 (y half) + x half
      const int bz = (t >> 2) * SZ;
      T r[6] = {(T)1, (T)1, (T)1, (T)-1, (T)-1, (T)-1};
#pragma unroll
      for (int k = 0; k < RZ; ++k) merge(r, sm.rg.B[4 * (bz + k) + (t & 3)]);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sm.box[t][0][a] = r[a];
        sm.box[t][1][a] = r[3 + a];
      }
    }
    __syncthreads();
  }
  // (3) list the gated cells of the tile that may have a partner.  Every
  // candidate y of cell x in sub-tile s has n(y) in the box of s, so
  // n(x).n(y) >= sum_a min(n_a(x) lo_a, n_a(x) hi_a); when that bound exceeds
  // cos_opp (margin 1e-3 for rounding) x has no partner and its flux is zero.
  for (int e = threadIdx.x; e < TC; e += NT_NCI) {
    const int lx = e % TX, ly = (e / TX) % TY, lz = e / (TX * TY);
    const bool inside = ox + lx < geo.nx && oy + ly < geo.ny && oz + lz < geo.nz;
    const int cc = (lx + NQ_HALO) + NX * ((ly + NQ_HALO) + NY * (DIM == 3 ? lz + NQ_HALO : 0));
    short slot = -1;
    const NQ<T> v = sm.nq[cc];
    bool open = inside && v.q >= q_th;
    if (open) {
      const int sub = (lx >= SX ? 1 : 0) + (ly >= SY ? 2 : 0) + (DIM == 3 && lz >= SZ ? 4 : 0);
      const T n[3] = {v.n0, v.n1, v.n2};
      T bound = (T)0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const T p = n[a] * sm.box[sub][0][a], q = n[a] * sm.box[sub][1][a];
        bound += p < q ? p : q;
      }
      open = !(bound > cos_opp + (T)1e-3);
    }
    if (open) {
      slot = (short)atomicAdd(&sm.ng, 1);
      sm.glist[slot] = (short)e;
    }
    sm.gslot[e] = slot;
  }
  __syncthreads();
  const int ng = sm.ng;
  // (4) partner search, one 8-lane group per gated cell, one plane per lane
  constexpr int ROWS = DIM == 3 ? 2 * WR + 1 : 1;   // window rows scanned per lane
  for (int base = 0; base < ng; base += NGRP) {
    const int gi = base + grp;
    const bool cell_ok = gi < ng;
    const int e = cell_ok ? sm.glist[gi] : 0;
    const int lx = e % TX, ly = (e / TX) % TY, lz = e / (TX * TY);
    const int cc = (lx + NQ_HALO) + NX * ((ly + NQ_HALO) + NY * (DIM == 3 ? lz + NQ_HALO : 0));
    const NQ<T> vx = sm.nq[cc];
    const T qx = vx.q;
    const T tol = eta * (qx > eps_q ? qx : eps_q);
    const int plane = lane8 - WR;                  // dz (3D) or dy (2D)
    const bool lane_ok = cell_ok && lane8 <= 2 * WR;
    // first window cell of this lane: (dx, dy) = (-WR, -WR) in plane dz (3D), (-WR, dy) (2D)
    const int row0 = lane_ok ? cc - WR + (DIM == 3 ? NX * (-WR + NY * plane) : NX * plane) : cc;
    const int p2 = plane * plane;
    auto accept = [&](const NQ<T>& v, T& dot) -> bool {
      dot = vx.n0 * v.n0;
      dot += vx.n1 * v.n1;
      if (DIM == 3) dot += vx.n2 * v.n2;
      return v.q >= q_th && m_abs(v.q - qx) <= tol && dot <= cos_opp;
    };
    // pass 0
    int bd2 = 1 << 30;
    T bdot = (T)0;
    if (lane_ok) {
#pragma unroll 1
      for (int r = 0; r < ROWS; ++r) {
        // the row's cells are read first, then tested without branches
        NQ<T> v[2 * WR + 1];
#pragma unroll
        for (int i = 0; i < 2 * WR + 1; ++i) v[i] = sm.nq[row0 + i + NX * r];
        const int dyr = DIM == 3 ? r - WR : 0;
#pragma unroll
        for (int i = 0; i < 2 * WR + 1; ++i) {
          const int dx = i - WR;
          T dot;
          const bool ok = accept(v[i], dot);
          const int d2 = dx * dx + dyr * dyr + p2;
          const bool self = dx == 0 && dyr == 0 && plane == 0;
          const bool better = ok && !self && (d2 < bd2 || (d2 == bd2 && dot < bdot));
          bd2 = better ? d2 : bd2;
          bdot = better ? dot : bdot;
        }
      }
    }
    group_min(bd2, bdot);
    const bool found = bd2 < (1 << 30);
    // pass 1: first candidate in scan order at distance bd2 within tie_eps of bdot
    int key = 1 << 30;
    if (lane_ok && found) {
#pragma unroll 1
      for (int r = ROWS - 1; r >= 0; --r)
#pragma unroll
        for (int i = 2 * WR; i >= 0; --i) {
          const int dx = i - WR, dyr = DIM == 3 ? r - WR : 0;
          const int d2 = dx * dx + dyr * dyr + p2;
          if (d2 != bd2) continue;
          const NQ<T> v = sm.nq[row0 + i + NX * r];
          T dot;
          if (accept(v, dot) && dot <= bdot + tie) {
            const int dy = DIM == 3 ? dyr : plane;
            // scan-order key: plane index, then row, then column (scanning
            // backwards, the last match is the first in scan order)
            key = ((lane8 * 16) + (dy + 8)) * 16 + (dx + 8);
          }
        }
    }
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
      const int ko = __shfl_xor(key, o, 64);
      key = ko < key ? ko : key;
    }
    // (5) the group leader builds the repulsive flux of its cell
    if (cell_ok && lane8 == 0) {
      T Jv[3] = {0, 0, 0};
      int packed = 0;
      if (found && key < (1 << 30)) {
        const int kdx = (key & 15) - 8, kdy = ((key >> 4) & 15) - 8, kpl = (key >> 8) - WR;
        const int bdx = kdx, bdy = DIM == 3 ? kdy : kpl, bdz = DIM == 3 ? kpl : 0;
        const NQ<T> vy = sm.nq[cc + bdx + NX * (bdy + NY * bdz)];
        const T nyv[3] = {vy.n0, vy.n1, vy.n2};
        const T nxv[3] = {vx.n0, vx.n1, vx.n2};
        T dot = nxv[0] * nyv[0];
        dot += nxv[1] * nyv[1];
        if (DIM == 3) dot += nxv[2] * nyv[2];
        T qcl = (T)0.5 * (qx + vy.q);
        if (qcl < eps_q) qcl = eps_q;
        if (qcl > (T)0.25 - eps_q) qcl = (T)0.25 - eps_q;
        const T ff = -dot > (T)0 ? -dot : (T)0;
        packed = 1 + ((bdx + 8) | ((bdy + 8) << 5) | ((bdz + 8) << 10));
        if (ff != (T)0) {
          const T rn = m_sqrt((T)(bdx * bdx + bdy * bdy + bdz * bdz));
          const T rh[3] = {(T)bdx / rn, (T)bdy / rn, (T)bdz / rn};
          T nt[3] = {0, 0, 0}, nn = 0;
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            nt[a] = nxv[a] - nyv[a];
            nn += nt[a] * nt[a];
          }
          nn = m_sqrt(nn);
          T ns[3] = {0, 0, 0};
          if (nn < (T)1e-6) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) ns[a] = rh[a];
          } else {
#pragma unroll
            for (int a = 0; a < DIM; ++a) ns[a] = nt[a] / (nn + eps_n);
          }
          T ref = 0;
          if (np.orient == 0) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) ref += nxv[a] * ns[a];
          } else {
#pragma unroll
            for (int a = 0; a < DIM; ++a) ref += rh[a] * ns[a];
            ref *= (T)np.orient;
          }
          if (ref < (T)0) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) ns[a] = -ns[a];
          }
          const T h = (T)np.width * m_acosh((T)1 / ((T)2 * m_sqrt(qcl)));
          const T wh = (T)1 / ((T)1 + m_pow(h / (T)np.h0, (T)np.p_exp));
          const T amp = (T)np.a_rep * qcl * wh * ff;
#pragma unroll
          for (int a = 0; a < DIM; ++a) Jv[a] = amp * ns[a];
        }
        my_active += 1u;
      }
#pragma unroll
      for (int a = 0; a < DIM; ++a) sm.out.gJ[gi][a] = Jv[a];
      sm.out.gpart[gi] = packed;
    }
  }
  __syncthreads();
  // (6) the tile's flux (zero where there is no partner)
  for (int e = threadIdx.x; e < TC; e += NT_NCI) {
    const int lx = e % TX, ly = (e / TX) % TY, lz = e / (TX * TY);
    const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
    if (gx >= geo.nx || gy >= geo.ny || gz >= geo.nz) continue;
    const int idx = gx + geo.nx * (gy + geo.ny * gz);
    const int sl = sm.gslot[e];
#pragma unroll
    for (int a = 0; a < DIM; ++a) J[a * geo.S + idx] = sl >= 0 ? sm.out.gJ[sl][a] : (T)0;
    if constexpr (DEBUG) {
      const long long N = (long long)geo.nx * geo.ny * geo.nz;
      const int pk = sl >= 0 ? sm.out.gpart[sl] : 0;
      chi_out[idx] = pk != 0;
      part_out[idx] = pk ? ((pk - 1) & 31) - 8 : 0;
      part_out[N + idx] = pk ? (((pk - 1) >> 5) & 31) - 8 : 0;
      part_out[2 * N + idx] = pk ? (((pk - 1) >> 10) & 31) - 8 : 0;
    }
  }
  __syncthreads();
}

// The tile routine with the window radius as a compile-time constant.
template <int DIM, int QH, typename T, bool DEBUG>
__device__ __forceinline__ void nci_tile_w(NciShared<DIM, T>& sm, unsigned t, NciHalo<DIM, T>& halo,
                                           bool next, unsigned tn, const T* __restrict__ phi,
                                           T* __restrict__ J, int* __restrict__ chi_out,
                                           int* __restrict__ part_out, const Geo& geo, const NciP& np,
                                           unsigned& my_active) {
  if (np.w == 3)
    nci_tile<DIM, QH, T, DEBUG, 3>(sm, t, halo, next, tn, phi, J, chi_out, part_out, geo, np, my_active);
  else if (np.w == 2)
    nci_tile<DIM, QH, T, DEBUG, 2>(sm, t, halo, next, tn, phi, J, chi_out, part_out, geo, np, my_active);
  else
    nci_tile<DIM, QH, T, DEBUG, 1>(sm, t, halo, next, tn, phi, J, chi_out, part_out, geo, np, my_active);
}

// The tiles list[first], list[first + stride], ... of one lattice, each
// tile's phi loads issued during the previous tile.
template <int DIM, int QH, typename T, bool DEBUG>
__device__ __forceinline__ void nci_tiles(NciShared<DIM, T>& sm, const unsigned* __restrict__ list,
                                          unsigned ntiles, unsigned first, unsigned stride,
                                          const T* __restrict__ phi, T* __restrict__ J,
                                          int* __restrict__ chi_out, int* __restrict__ part_out,
                                          const Geo& geo, const NciP& np, unsigned& my_active) {
  NciHalo<DIM, T> halo;
  if (first < ntiles) halo.load(list[first], phi, geo);
  for (unsigned k = first; k < ntiles; k += stride) {
    const unsigned kn = k + stride;
    const bool next = kn < ntiles;
    nci_tile_w<DIM, QH, T, DEBUG>(sm, list[k], halo, next, next ? list[kn] : 0u, phi, J, chi_out, part_out,
                                  geo, np, my_active);
  }
}

template <int DIM, int QH, typename T, bool DEBUG>
__global__ __launch_bounds__(NT_NCI) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) void k_nci(const T* __restrict__ phi, T* __restrict__ J,
                                                int* __restrict__ chi_out, int* __restrict__ part_out,
                                                const unsigned* __restrict__ list,
                                                const unsigned* __restrict__ cnt,
                                                unsigned* __restrict__ flags_other,
                                                const unsigned* __restrict__ list_other,
                                                const unsigned* __restrict__ cnt_other,
                                                unsigned* __restrict__ nci_count, Geo geo, NciP np) {
  __shared__ NciShared<DIM, T> sm;
  nci_clear_other(flags_other, list_other, cnt_other);
  const unsigned ntiles = *cnt;
  unsigned my_active = 0;
  nci_tiles<DIM, QH, T, DEBUG>(sm, list, ntiles, blockIdx.x, gridDim.x, phi, J, chi_out, part_out, geo, np,
                               my_active);
  my_active = wave_sum(my_active);
  if ((threadIdx.x & 63) == 0 && my_active) atomicAdd(nci_count, my_active);
}

// Tiles that cannot hold a partner, found before the near-contact pass.  A
// gated cell can only pair with a gated cell of its window whose normal faces
// its own (n(x).n(y) <= cos_opp).  k_nci_ranges gives each listed tile, per
// sub-tile (the tile halved along each axis), the range [lo, hi] of each normal
// component over its gated cells, from the operations k_nci uses for them;
// k_nci_select bounds n(x).n(y) from below over the gated cells x of a tile
// and the gated cells y of every sub-tile that the windows of its cells reach,
// and lists the tile for k_nci unless the bound exceeds cos_opp by the margin
// of k_nci's own sub-tile pruning.  A tile left out is flagged NCI_SKIPPED: no
// cell of it has a partner, and the collide reads no J there.  Where most tiles
// face another interface (dense swarms) the selection costs more than it saves:
// it runs when the previous pass took at most half of its listed tiles, and on
// probe steps; otherwise k_nci takes the whole list.  Either way the results
// are the same.
constexpr unsigned NCI_SKIPPED = 2u;

// Whether this pass selects tiles: prev_listed and prev_taken are the tile
// counts of the previous pass (its list, and the tiles it processed).
__device__ __forceinline__ bool nci_selecting(unsigned prev_listed, unsigned prev_taken, int probe) {
  return probe || prev_listed == 0u || 2u * prev_taken <= prev_listed;
}

template <int DIM, typename T>
struct NciSub {
  using TL = NciTile<DIM, T>;
  static constexpr int SX = TL::TX / 2, SY = TL::TY / 2, SZ = DIM == 3 ? TL::TZ / 2 : 1;
  static constexpr int NSUB = DIM == 3 ? 8 : 4, CPS = SX * SY * SZ;   // sub-tiles, cells per sub-tile
  static_assert(CPS <= 64 && 64 % CPS == 0 && NSUB * CPS <= NT_NCI, "sub-tile lanes");
};

// Empty range: lo above hi (normal components lie in [-1, 1]).
template <typename T>
__device__ __forceinline__ void rng_empty(T r[6]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[a] = (T)2;
    r[3 + a] = (T)-2;
  }
}
template <typename T>
__device__ __forceinline__ void rng_merge(T r[6], const T* v) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[a] = v[a] < r[a] ? v[a] : r[a];
    r[3 + a] = v[3 + a] > r[3 + a] ? v[3 + a] : r[3 + a];
  }
}
// Minimum and maximum over groups of W consecutive lanes (W a power of two).
template <int W, typename T>
__device__ __forceinline__ void rng_lanes(T r[6]) {
#pragma unroll
  for (int o = 1; o < W; o <<= 1) {
    T v[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) v[a] = __shfl_xor(r[a], o, 64);
    rng_merge(r, v);
  }
}

// One block per listed tile (grid-stride): lane group sid of CPS lanes takes
// sub-tile sid, one cell per lane; the ranges go to srng[(tile NSUB + sid) 6].
template <int DIM, int QH, typename T>
__global__ __launch_bounds__(NT_NCI) void k_nci_ranges(const T* __restrict__ phi, Geo geo,
                                                       const unsigned* __restrict__ list,
                                                       const unsigned* __restrict__ cnt, T* __restrict__ srng,
                                                       T q_th, T eps_n, const unsigned* __restrict__ prev_listed,
                                                       const unsigned* __restrict__ prev_taken, int probe) {
  using TL = NciTile<DIM, T>;
  using SB = NciSub<DIM, T>;
  using L = HydroQ<QH>;
  if (!nci_selecting(*prev_listed, *prev_taken, probe)) return;
  const unsigned ntiles = *cnt;
  const int sid = (int)threadIdx.x / SB::CPS, l = (int)threadIdx.x % SB::CPS;
  for (unsigned k = blockIdx.x; k < ntiles; k += gridDim.x) {
    const unsigned tile = list[k];
    const int tx = (int)(tile % (unsigned)geo.ntx), ty = (int)((tile / (unsigned)geo.ntx) % (unsigned)geo.nty);
    const int tz = (int)(tile / ((unsigned)geo.ntx * (unsigned)geo.nty));
    T r[6];
    rng_empty(r);
    if (sid < SB::NSUB) {
      const int x = tx * TL::TX + (sid & 1) * SB::SX + l % SB::SX;
      const int y = ty * TL::TY + ((sid >> 1) & 1) * SB::SY + (l / SB::SX) % SB::SY;
      const int z = DIM == 3 ? tz * TL::TZ + (sid >> 2) * SB::SZ + l / (SB::SX * SB::SY) : 0;
      if (x < geo.nx && y < geo.ny && z < geo.nz) {
        const Nbr nb(x, y, z, geo);
        const T ph = phi[nb(0, 0, 0)];
        const T pc = ph < (T)0 ? (T)0 : (ph > (T)1 ? (T)1 : ph);
        if (pc * ((T)1 - pc) >= q_th) {
          T gr[3], lap;
          grad_lap<QH, T>([&](int i) { return phi[nb(L::cx[i], L::cy[i], L::cz[i])]; }, gr, lap);
          T mag = gr[0] * gr[0] + gr[1] * gr[1];
          if (DIM == 3) mag += gr[2] * gr[2];
          const T inv = (T)1 / (m_sqrt(mag) + eps_n);
          const T n[3] = {gr[0] * inv, gr[1] * inv, DIM == 3 ? gr[2] * inv : (T)0};
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            r[a] = n[a];
            r[3 + a] = n[a];
          }
        }
      }
    }
    rng_lanes<SB::CPS>(r);
    if (sid < SB::NSUB && l == 0) {
#pragma unroll
      for (int a = 0; a < 6; ++a) srng[((size_t)tile * SB::NSUB + sid) * 6 + a] = r[a];
    }
  }
}

// One wave per listed tile (grid-stride over waves).  Along each axis the
// distinct sub-tiles holding the cells within w of the tile (periodic) are
// listed; the lanes share their product, merging the ranges of the sub-tiles
// of listed tiles (flags of this parity, set by the phi pass).
template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_nci_select(Geo geo, unsigned* __restrict__ flags,
                                                    const unsigned* __restrict__ list,
                                                    const unsigned* __restrict__ cnt, const T* __restrict__ srng,
                                                    unsigned* __restrict__ alist, unsigned* __restrict__ acnt,
                                                    int w, T cos_opp, const unsigned* __restrict__ prev_listed,
                                                    const unsigned* __restrict__ prev_taken, int probe) {
  using TL = NciTile<DIM, T>;
  using SB = NciSub<DIM, T>;
  constexpr int MAXS = 8;   // distinct sub-tiles per axis: at most (T + 2 w) / S + 1 with w <= 3, S >= 2
  const unsigned ntiles = *cnt;
  if (!nci_selecting(*prev_listed, *prev_taken, probe)) {
    // the whole list
    for (unsigned k = blockIdx.x * blockDim.x + threadIdx.x; k < ntiles; k += gridDim.x * blockDim.x)
      alist[k] = list[k];
    if (blockIdx.x == 0 && threadIdx.x == 0) *acnt = ntiles;
    return;
  }
  const int lane = (int)(threadIdx.x & 63);
  const unsigned nw = gridDim.x * (blockDim.x >> 6);
  for (unsigned k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); k < ntiles; k += nw) {
    const unsigned tile = list[k];
    const int tc[3] = {(int)(tile % (unsigned)geo.ntx), (int)((tile / (unsigned)geo.ntx) % (unsigned)geo.nty),
                       (int)(tile / ((unsigned)geo.ntx * (unsigned)geo.nty))};
    const int nn[3] = {geo.nx, geo.ny, geo.nz}, tt[3] = {TL::TX, TL::TY, TL::TZ}, ss[3] = {SB::SX, SB::SY, SB::SZ};
    int sl[3][MAXS], ns[3];
    bool over = false;   // more distinct sub-tiles than listed: select the tile
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ns[a] = 0;
      if (a >= DIM) {
        sl[a][0] = 0;
        ns[a] = 1;
        continue;
      }
      const int lo = tc[a] * tt[a] - w, hi = min(tc[a] * tt[a] + tt[a], nn[a]) - 1 + w;
      int prev = -1;
      for (int c = lo; c <= hi; ++c) {
        const int s = wrapi(c, nn[a]) / ss[a];
        if (s != prev) {   // a repeat after a wrap only merges twice
          if (ns[a] < MAXS)
            sl[a][ns[a]++] = s;
          else
            over = true;
        }
        prev = s;
      }
    }
    T u[6], own[6];
    rng_empty(u);
    rng_empty(own);
    const int total = ns[0] * ns[1] * ns[2];
    for (int q = lane; q < total; q += 64) {
      const int sx = sl[0][q % ns[0]], sy = sl[1][(q / ns[0]) % ns[1]], sz = sl[2][q / (ns[0] * ns[1])];
      const unsigned nt = (unsigned)(sx / 2 + geo.ntx * (sy / 2 + geo.nty * (sz / 2)));
      if (flags[nt]) rng_merge(u, srng + ((size_t)nt * SB::NSUB + (sx & 1) + 2 * (sy & 1) + 4 * (sz & 1)) * 6);
    }
    if (lane < SB::NSUB) rng_merge(own, srng + ((size_t)tile * SB::NSUB + lane) * 6);
    rng_lanes<64>(u);
    rng_lanes<64>(own);
    // lower bound of n(x).n(y): per component the least product of the two intervals
    T bound = (T)0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const T p0 = own[a] * u[a], p1 = own[a] * u[3 + a], p2 = own[3 + a] * u[a], p3 = own[3 + a] * u[3 + a];
      const T m0 = p0 < p1 ? p0 : p1, m1 = p2 < p3 ? p2 : p3;
      bound += m0 < m1 ? m0 : m1;
    }
    if (lane == 0) {
      if (!over && bound > cos_opp + (T)1e-3)
        flags[tile] = NCI_SKIPPED;
      else
        alist[atomicAdd(acnt, 1u)] = tile;
    }
  }
}

// ---------------------------------------------------------------------------
// (b) fused collide + stream of both lattices (AA, in place)
// ---------------------------------------------------------------------------

enum { MODE_STEP = 0, MODE_STEP_DIAG = 1, MODE_DRY = 2 };

// Block reduction of the NPART per-thread values (sums, or maxima in the
// max_slot slots).
__device__ __forceinline__ void block_partials(double v[NPART], double* __restrict__ out) {
  __shared__ double red[NT / 64][NPART];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NPART; ++k) v[k] = max_slot(k) ? wave_max(v[k]) : wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NPART; ++k) red[wv][k] = v[k];
  __syncthreads();
  if (threadIdx.x < NPART) {
    const int k = threadIdx.x;
    double a = red[0][k];
    for (int j = 1; j < NT / 64; ++j) a = max_slot(k) ? (red[j][k] > a ? red[j][k] : a) : a + red[j][k];
    out[blockIdx.x * NPART + k] = a;
  }
}

// Base pointers of the two population arrays (kernel arguments).
template <typename FS, typename GS>
struct Planes {
  FS* f;   // hydrodynamic populations
  GS* g;   // phase-field populations
};

// Mixture and forcing constants in the arithmetic type of the kernel.
template <typename T>
struct PhysT {
  T rho_g, drho, mu_a, mu_b, beta4, kappa, rho_mean, g[3], kc, inv_tau_phi, eps_n;
  T fref[27];   // w_i pstar_ref: offset of the 16-bit population encoding
};

__device__ __forceinline__ float m_rcp(float a) { return __builtin_amdgcn_rcpf(a); }
__device__ __forceinline__ double m_rcp(double a) { return 1.0 / a; }

// ---------------------------------------------------------------------------
// Moment storage of the hydrodynamic populations (the paper's "thread-safe"
// update, Sec. 2.1): instead of its Q post-collision populations a cell keeps
// the NMOM coefficients they are built from (below), in one of two buffers, and
// the next step rebuilds each incoming population f_i(x) = f*_i(x - c_i) from the
// coefficients of the cell it streams from.  Coefficient order:
//   p*, u (3), h = F / (2 rho) (3), Ah = (1 - omega) A2 (xx yy zz xy xz yz).
// ---------------------------------------------------------------------------
constexpr int NMOM = 13;

// f*_i of a cell with coefficients m (c = c_i, w = w_i): the expansion of the
// collision below, f*_i = w_i [p* - 1.5 tr B + 4.5 c.B.c + 3 c.A1 + t3] with
// A1 = u + h, B = uu + Ah + u h + h u and
// t3 = (c.u) (13.5 c.Ah.c + 4.5 ((c.u)^2 - u.u) - 4.5 tr Ah) - 9 c.Ah.u.
template <typename T>
__device__ __forceinline__ T post_population(int cx, int cy, int cz, T w, const T m[NMOM]) {
  const T* u = m + 1;
  const T* h = m + 4;
  const T* A = m + 7;
  const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const T trA = A[0] + A[1] + A[2];
  const T uh = u[0] * h[0] + u[1] * h[1] + u[2] * h[2];
  const T trB = uu + trA + (T)2 * uh;
  if (cx == 0 && cy == 0 && cz == 0) return w * (m[0] - (T)1.5 * trB);
  const T cu = sdot(cx, cy, cz, u[0], u[1], u[2]);
  const T ch = sdot(cx, cy, cz, h[0], h[1], h[2]);
  const T cAc = ccdot(cx, cy, cz, A);
  const T Au[3] = {A[0] * u[0] + A[3] * u[1] + A[4] * u[2], A[3] * u[0] + A[1] * u[1] + A[5] * u[2],
                   A[4] * u[0] + A[5] * u[1] + A[2] * u[2]};
  const T cAu = sdot(cx, cy, cz, Au[0], Au[1], Au[2]);
  const T cBc = cu * cu + cAc + (T)2 * cu * ch;
  const T t3 = cu * ((T)13.5 * cAc + (T)4.5 * (cu * cu - uu) - (T)4.5 * trA) - (T)9 * cAu;
  return w * (m[0] - (T)1.5 * trB + (T)4.5 * cBc + (T)3 * (cu + ch) + t3);
}

// Incoming populations of the cell at nb(0, 0, 0) from the coefficients of the
// cells they stream from (planes of stride S).
template <int QH, typename T>
__device__ __forceinline__ void pull_populations(const T* __restrict__ mom, long long S, const Nbr& nb,
                                                 T fi[HydroQ<QH>::Q]) {
  using H = HydroQ<QH>;
#pragma unroll
  for (int i = 0; i < H::Q; ++i) {
    const long long j = (long long)nb(-H::cx[i], -H::cy[i], -H::cz[i]);
    T m[NMOM];
#pragma unroll
    for (int k = 0; k < NMOM; ++k) m[k] = mom[k * S + j];
    fi[i] = post_population(H::cx[i], H::cy[i], H::cz[i], wt<H, T>(i), m);
  }
}

// The moments p* = sum f_i, m = sum f_i c_i and M2 = sum f_i c_i c_i (xx yy zz xy
// xz yz) of the incoming populations, each population rebuilt from the
// coefficients of the cell it streams from and added at once.  The loads of
// direction i + 2 are made to wait for the population of direction i (an empty
// asm statement that takes that population and passes the load offset through),
// so about two directions' coefficients are in flight; issued all at once, the
// 13 Q loads held 270 registers and left one wave per SIMD.
template <int QH, typename T, bool OFF32>
__device__ __forceinline__ void pull_moments(const T* __restrict__ mom, long long S, const Nbr& nb, T& ps,
                                             T m[3], T M2[6]) {
  using H = HydroQ<QH>;
  ps = (T)0;
  for (int a = 0; a < 3; ++a) m[a] = (T)0;
  for (int a = 0; a < 6; ++a) M2[a] = (T)0;
  unsigned jd[H::Q];
#pragma unroll
  for (int i = 0; i < H::Q; ++i) jd[i] = (unsigned)nb(-H::cx[i], -H::cy[i], -H::cz[i]);
#pragma unroll
  for (int i = 0; i < H::Q; ++i) {
    const int cx = H::cx[i], cy = H::cy[i], cz = H::cz[i];
    T c[NMOM];
#pragma unroll
    for (int k = 0; k < NMOM; ++k) c[k] = *plane_at<OFF32>(mom + k * S, jd[i]);
    const T f = post_population(cx, cy, cz, wt<H, T>(i), c);
    ps += f;
    if (cx) m[0] += cx > 0 ? f : -f;
    if (cy) m[1] += cy > 0 ? f : -f;
    if (cz) m[2] += cz > 0 ? f : -f;
    if (cx) M2[0] += f;
    if (cy) M2[1] += f;
    if (cz) M2[2] += f;
    if (cx && cy) M2[3] += cx * cy > 0 ? f : -f;
    if (cx && cz) M2[4] += cx * cz > 0 ? f : -f;
    if (cy && cz) M2[5] += cy * cz > 0 ? f : -f;
    if (i + 2 < H::Q) asm volatile("" : "+v"(jd[i + 2]) : "v"(f));
  }
}

// Post-collision populations, written as Hermite coefficients.  f^eq, the
// regularised non-equilibrium part and S/2 all lie in the span of the Hermite
// polynomials up to third order (the Guo term has no third-order part), so
//   f*_i = w_i [ p* + c_i.A1/cs^2 + H2_i:B2/(2cs^4) + H3_i...B3/(6cs^6) ]
// with A1 = u + F/(2 rho), B2 = uu + (1-omega) A2 + (uF + Fu)/(2 rho) and
// B3 = uuu + (1-omega) S(u (x) A2); on these lattices the contractions reduce to
//   H2:B2/(2cs^4) = 4.5 c.B2.c - 1.5 tr B2,
//   H3...B3/(6cs^6) = 4.5 cu (cu^2 - u^2) + (1-omega)(13.5 cu c.A2.c - 4.5 cu trA2 - 9 c.A2.u).
// Each opposite pair (c, -c) shares the even part and flips the odd part.
// One cell of the fused collide + stream (AA parity PAR).  MODE_STEP updates
// the populations in place; MODE_STEP_DIAG also fills acc with the cell's
// contributions to the FP64 diagnostics; MODE_DRY leaves the populations and
// writes p*, rho, u, F to macro (when given).
template <int DIM, int QH, int PAR, int MODE, typename T, typename FS, typename GS, bool OFF32,
          bool XCH = false, bool PRE = false, bool MOM = false>
__device__ __forceinline__ void collide_cell(const Planes<FS, GS>& pl, const T* __restrict__ phi,
                                             const T* __restrict__ J,
                                             const unsigned* __restrict__ flags, const Geo& geo,
                                             const PhysT<T>& pp, int nci_on, T* __restrict__ macro,
                                             T* __restrict__ uout, int x, int y, int z,
                                             double acc[NPART], FS* xf = nullptr,
                                             GS* xg = nullptr, const T* fpre = nullptr,
                                             const T* gpre = nullptr, const T* __restrict__ min = nullptr,
                                             T* __restrict__ mout = nullptr) {
  using H = HydroQ<QH>;
  using P = Phase<DIM>;
  using TL = NciTile<DIM, T>;
  constexpr int Q = H::Q, QG = P::Q;
  static_assert(!XCH || PAR == 1, "the row exchange serves the odd parity");
  static_assert(!MOM || (!XCH && !PRE && DIM == 3), "moment storage: 3D, cell-wise kernel");
  // MOM: the hydrodynamic populations are rebuilt from the coefficients in min
  // (moment storage, see post_population) and the new coefficients go to mout;
  // the phase-field populations keep the AA pattern of parity PAR.
  const Nbr nb(x, y, z, geo);
  const unsigned idx = (unsigned)nb(0, 0, 0);
  // XCH (k_collide_row): the odd parity's x-shifted populations of this cell's
  // row are staged in LDS, xf / xg holding for x-shifted pair j (odd direction
  // i) the row of slot i at (y + c_y, z + c_z) at 2 j nx and the row of slot
  // i + 1 at (y - c_y, z - c_z) at (2 j + 1) nx.  PRE: the populations of the
  // directions with c_x = 0 were loaded by the caller (fpre, gpre, indexed by
  // direction), before its staging barrier.
  const int xl = x == 0 ? geo.nx - 1 : x - 1, xr = x == geo.nx - 1 ? 0 : x + 1;
  // Population accesses stream past the caches (nontemporal) where they are
  // aligned: every access of the even parity, and the odd parity's accesses of
  // directions with c_x = 0.  The odd parity's accesses with c_x != 0 are
  // shifted by one cell, so two blocks write parts of one line; kept cached, L2
  // merges them (hinted, the odd collide wrote 7 % more bytes: 5.34 ms instead
  // of 5.19 ms at 512^3 FP32; 5.15 ms with the aligned ones hinted).

  const long long S = geo.S;
  // ---- phase field around the cell: grad, lap, mu_phi
  T gr[3], lap;
  grad_lap<QH, T>([&](int i) { return *plane_at<OFF32>(phi, (unsigned)nb(H::cx[i], H::cy[i], H::cz[i])); },
                   gr, lap);
  const T ph = *plane_at<OFF32>(phi, idx);
  T gmag = gr[0] * gr[0] + gr[1] * gr[1];
  if (DIM == 3) gmag += gr[2] * gr[2];
  gmag = m_sqrt(gmag);
  const T inv_g = m_rcp(gmag + pp.eps_n);
  const T mu = pp.beta4 * ph * (ph - (T)1) * (ph - (T)0.5) - pp.kappa * lap;
  // ---- mixture (linear rho, linear dynamic viscosity)
  const T rho = pp.rho_g + pp.drho * ph;
  const T inv_rho = m_rcp(rho);
  const T nu = (pp.mu_a + pp.mu_b * ph) * inv_rho;
  const T omega = m_rcp((T)0.5 + (T)3 * nu);
  // ---- hydrodynamic populations and their moments
  const PopNbr<FS> pf(pl.f, x, y, z, geo, Q);
  T fi[Q];
  // hinted loads where the access is aligned, plain ones (a separate loop, so
  // that the two kinds are not merged) where it is shifted along x
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (MOM || (PAR == 1 && H::cx[i] != 0)) continue;
    if constexpr (PRE)
      fi[i] = fpre[i];
    else
      fi[i] = Store<FS>::ldh(PAR == 0 ? pf.template at<OFF32>(i, 0, 0, 0)
                                      : pf.template at<OFF32>(opp(i), 0, -H::cy[i], -H::cz[i]),
                             pp.fref[i]);
  }
  if constexpr (XCH) {
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
      if (H::cx[i] == 0) continue;
      const int j = xpair<H>(i), xm = H::cx[i] > 0 ? xl : xr, xp = H::cx[i] > 0 ? xr : xl;
      fi[i] = Store<FS>::ld(xf + (2 * j + 1) * geo.nx + xm, pp.fref[i]);
      fi[i + 1] = Store<FS>::ld(xf + 2 * j * geo.nx + xp, pp.fref[i]);
    }
  } else if constexpr (!MOM) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (PAR == 0 || H::cx[i] == 0) continue;
      fi[i] = Store<FS>::ld(pf.template at<OFF32>(opp(i), -H::cx[i], -H::cy[i], -H::cz[i]), pp.fref[i]);
    }
  }
  T ps, m[3] = {0, 0, 0}, M2[6] = {0, 0, 0, 0, 0, 0};  // xx yy zz xy xz yz
  if constexpr (MOM)
    pull_moments<QH, T, OFF32>(min, S, nb, ps, m, M2);
  else
    ps = fi[0];
#pragma unroll
  for (int i = 1; i < (MOM ? 0 : Q); i += 2) {
    const T s = fi[i] + fi[i + 1], d = fi[i] - fi[i + 1];
    ps += s;
    const int cx = H::cx[i], cy = H::cy[i], cz = H::cz[i];
    if (cx) m[0] += cx > 0 ? d : -d;
    if (cy) m[1] += cy > 0 ? d : -d;
    if (cz) m[2] += cz > 0 ? d : -d;
    if (cx) M2[0] += s;
    if (cy) M2[1] += s;
    if (cz) M2[2] += s;
    if (cx && cy) M2[3] += cx * cy > 0 ? s : -s;
    if (cx && cz) M2[4] += cx * cz > 0 ? s : -s;
    if (cy && cz) M2[5] += cy * cz > 0 ? s : -s;
  }
  // ---- forces (Eq. Fsplit): capillary, pressure correction, repulsion, buoyancy
  T Jv[3] = {0, 0, 0};
  if (nci_on) {
    const unsigned tile = (unsigned)(x / TL::TX + geo.ntx * (y / TL::TY + geo.nty * (z / TL::TZ)));
    if (flags[tile] == 1u) {   // listed and not skipped (NCI_SKIPPED: no partner in the tile)
#pragma unroll
      for (int a = 0; a < DIM; ++a) Jv[a] = *plane_at<OFF32>(J + a * S, idx);
    }
  }
  const T cs2 = (T)(1.0 / 3.0);
  const T inv2rho = (T)0.5 * inv_rho;
  const T pc = ps * cs2;
  const T prho = pc * pp.drho;
  const T dens = rho - pp.rho_mean;
  T Fp[3], up[3], F[3], u[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Fp[a] = a < DIM ? (mu - prho) * gr[a] + rho * Jv[a] + dens * pp.g[a] : (T)0;
    up[a] = m[a] + Fp[a] * inv2rho;
  }
  // viscous correction (Eq. Fnu) from the second moment of f - feq(p*, u')
  {
    const T Pxx = M2[0] - pc - up[0] * up[0], Pyy = M2[1] - pc - up[1] * up[1];
    const T Pzz = M2[2] - pc - up[2] * up[2];
    const T Pxy = M2[3] - up[0] * up[1], Pxz = M2[4] - up[0] * up[2], Pyz = M2[5] - up[1] * up[2];
    const T kf = -(T)3 * nu * omega * pp.drho;
    F[0] = Fp[0] + kf * (Pxx * gr[0] + Pxy * gr[1] + Pxz * gr[2]);
    F[1] = Fp[1] + kf * (Pxy * gr[0] + Pyy * gr[1] + Pyz * gr[2]);
    F[2] = DIM == 3 ? Fp[2] + kf * (Pxz * gr[0] + Pyz * gr[1] + Pzz * gr[2]) : (T)0;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = m[a] + F[a] * inv2rho;
  if constexpr (MODE != MODE_DRY) {
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const T om1 = (T)1 - omega;
    // second-order Hermite coefficient of f - feq + S/2, and the post-collision ones
    T A[6], B[6];
    {
      const T gxx = u[0] * F[0] * inv2rho, gyy = u[1] * F[1] * inv2rho, gzz = u[2] * F[2] * inv2rho;
      const T gxy = (u[0] * F[1] + u[1] * F[0]) * inv2rho;
      const T gxz = (u[0] * F[2] + u[2] * F[0]) * inv2rho;
      const T gyz = (u[1] * F[2] + u[2] * F[1]) * inv2rho;
      const T uxx = u[0] * u[0], uyy = u[1] * u[1], uzz = u[2] * u[2];
      const T uxy = u[0] * u[1], uxz = u[0] * u[2], uyz = u[1] * u[2];
      A[0] = M2[0] - pc - uxx + (T)2 * gxx;
      A[1] = M2[1] - pc - uyy + (T)2 * gyy;
      A[2] = DIM == 3 ? M2[2] - pc - uzz + (T)2 * gzz : (T)0;
      A[3] = M2[3] - uxy + gxy;
      A[4] = DIM == 3 ? M2[4] - uxz + gxz : (T)0;
      A[5] = DIM == 3 ? M2[5] - uyz + gyz : (T)0;
      B[0] = uxx + om1 * A[0] + (T)2 * gxx;
      B[1] = uyy + om1 * A[1] + (T)2 * gyy;
      B[2] = DIM == 3 ? uzz + om1 * A[2] + (T)2 * gzz : (T)0;
      B[3] = uxy + om1 * A[3] + gxy;
      B[4] = DIM == 3 ? uxz + om1 * A[4] + gxz : (T)0;
      B[5] = DIM == 3 ? uyz + om1 * A[5] + gyz : (T)0;
    }
    const T trA = A[0] + A[1] + A[2];
    const T trB = B[0] + B[1] + B[2];
    const T Au[3] = {A[0] * u[0] + A[3] * u[1] + A[4] * u[2], A[3] * u[0] + A[1] * u[1] + A[5] * u[2],
                     A[4] * u[0] + A[5] * u[1] + A[2] * u[2]};
    const T A1[3] = {u[0] + F[0] * inv2rho, u[1] + F[1] * inv2rho, u[2] + F[2] * inv2rho};
    const T base = ps - (T)1.5 * trB;
    const T k3 = (T)13.5 * om1, k3t = (T)4.5 * om1 * trA, k3u = (T)9 * om1;
    if constexpr (MOM) {
      // the coefficients of f* (post_population rebuilds it where it streams to)
      st_nt(mout + idx, ps);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        st_nt(mout + (1 + a) * S + idx, u[a]);
        st_nt(mout + (4 + a) * S + idx, F[a] * inv2rho);
      }
#pragma unroll
      for (int k = 0; k < 6; ++k) st_nt(mout + (7 + k) * S + idx, om1 * A[k]);
    } else {
    Store<FS>::sth(pf.template at<OFF32>(0, 0, 0, 0), wt<H, T>(0) * base, pp.fref[0]);
    T fsx[Q];   // odd parity, c_x != 0: stored plain after the loop
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
      const int cx = H::cx[i], cy = H::cy[i], cz = H::cz[i];
      const T w = wt<H, T>(i);
      const T cu = sdot(cx, cy, cz, u[0], u[1], u[2]);
      const T cA1 = sdot(cx, cy, cz, A1[0], A1[1], A1[2]);
      const T cAu = sdot(cx, cy, cz, Au[0], Au[1], Au[2]);
      const T cAc = ccdot(cx, cy, cz, A);
      const T cBc = ccdot(cx, cy, cz, B);
      const T ev = w * fmad((T)4.5, cBc, base);
      const T t3 = fmad(cu, fmad(k3, cAc, fmad((T)4.5, fmad(cu, cu, -uu), -k3t)), -(k3u * cAu));
      const T od = w * fmad((T)3, cA1, t3);
      const T fa = ev + od, fb = ev - od;   // directions i and opp(i)
      if constexpr (PAR == 0) {
        Store<FS>::sth(pf.template at<OFF32>(i + 1, 0, 0, 0), fa, pp.fref[i]);
        Store<FS>::sth(pf.template at<OFF32>(i, 0, 0, 0), fb, pp.fref[i]);
      } else if (cx == 0) {
        Store<FS>::sth(pf.template at<OFF32>(i, 0, cy, cz), fa, pp.fref[i]);
        Store<FS>::sth(pf.template at<OFF32>(i + 1, 0, -cy, -cz), fb, pp.fref[i]);
      } else {
        fsx[i] = fa;
        fsx[i + 1] = fb;
      }
    }
    if constexpr (PAR == 1) {
#pragma unroll
      for (int i = 1; i < Q; i += 2) {
        const int cx = H::cx[i], cy = H::cy[i], cz = H::cz[i];
        if (cx == 0) continue;
        if constexpr (XCH) {
          const int j = xpair<H>(i), xm = cx > 0 ? xl : xr, xp = cx > 0 ? xr : xl;
          Store<FS>::st(xf + 2 * j * geo.nx + xp, fsx[i], pp.fref[i]);
          Store<FS>::st(xf + (2 * j + 1) * geo.nx + xm, fsx[i + 1], pp.fref[i]);
        } else {
          Store<FS>::st(pf.template at<OFF32>(i, cx, cy, cz), fsx[i], pp.fref[i]);
          Store<FS>::st(pf.template at<OFF32>(i + 1, -cx, -cy, -cz), fsx[i + 1], pp.fref[i]);
        }
      }
    }
    }
    if (uout) {
      // finite-difference phase field: the velocity of this collision feeds
      // the explicit update (which forms a = phi (1 - phi) n itself)
#pragma unroll
      for (int a = 0; a < DIM; ++a) st_nt(uout + a * S + idx, u[a]);
    } else {
    // ---- conservative Allen-Cahn populations: BGK towards
    //      geq_k = w_k (phi + c_k . j / cs_phi^2), j = phi u + M (4/W) phi (1-phi) n
    const T kc = pp.kc * ph * ((T)1 - ph) * inv_g;
    const T jv[3] = {ph * u[0] + kc * gr[0], ph * u[1] + kc * gr[1], ph * u[2] + kc * gr[2]};
    const T itp = pp.inv_tau_phi;
    const PopNbr<GS> pg(pl.g, x, y, z, geo, QG);
    T gi[QG];
#pragma unroll
    for (int k = 0; k < QG; ++k) {
      if (PAR == 1 && P::cx[k] != 0) continue;
      if constexpr (PRE)
        gi[k] = gpre[k];
      else
        gi[k] = (T)ld_nt(PAR == 0 ? pg.template at<OFF32>(k, 0, 0, 0)
                                  : pg.template at<OFF32>(opp(k), 0, -P::cy[k], -P::cz[k]));
    }
    if constexpr (XCH) {
#pragma unroll
      for (int k = 1; k < QG; k += 2) {
        if (P::cx[k] == 0) continue;
        const int j = xpair<P>(k), xm = P::cx[k] > 0 ? xl : xr, xp = P::cx[k] > 0 ? xr : xl;
        gi[k] = (T)xg[(2 * j + 1) * geo.nx + xm];
        gi[k + 1] = (T)xg[2 * j * geo.nx + xp];
      }
    } else {
#pragma unroll
      for (int k = 0; k < QG; ++k) {
        if (PAR == 0 || P::cx[k] == 0) continue;
        gi[k] = (T)*pg.template at<OFF32>(opp(k), -P::cx[k], -P::cy[k], -P::cz[k]);
      }
    }
    // geq - g is formed with the product unrounded: a rounded w_k (phi + c.j/cs^2)
    // (the D2Q9 weights are not powers of two) would bias the phase-field mass
    // of every step, like weights that do not sum to one.
    st_nt(pg.template at<OFF32>(0, 0, 0, 0), (GS)fmad(fmad(wt<P, T>(0), ph, -gi[0]), itp, gi[0]));
    GS gsx[QG];   // odd parity, c_x != 0: stored plain after the loop
#pragma unroll
    for (int k = 1; k < QG; k += 2) {
      const int cx = P::cx[k], cy = P::cy[k], cz = P::cz[k];
      const T cj = sdot(cx, cy, cz, jv[0], jv[1], jv[2]) * (T)P::inv_cs2;
      const T wk = wt<P, T>(k);
      const T ga = fmad(fmad(wk, ph + cj, -gi[k]), itp, gi[k]);
      const T gb = fmad(fmad(wk, ph - cj, -gi[k + 1]), itp, gi[k + 1]);
      if constexpr (PAR == 0) {
        st_nt(pg.template at<OFF32>(k + 1, 0, 0, 0), (GS)ga);
        st_nt(pg.template at<OFF32>(k, 0, 0, 0), (GS)gb);
      } else if (cx == 0) {
        st_nt(pg.template at<OFF32>(k, 0, cy, cz), (GS)ga);
        st_nt(pg.template at<OFF32>(k + 1, 0, -cy, -cz), (GS)gb);
      } else {
        gsx[k] = (GS)ga;
        gsx[k + 1] = (GS)gb;
      }
    }
    if constexpr (PAR == 1) {
#pragma unroll
      for (int k = 1; k < QG; k += 2) {
        const int cx = P::cx[k], cy = P::cy[k], cz = P::cz[k];
        if (cx == 0) continue;
        if constexpr (XCH) {
          const int j = xpair<P>(k), xm = cx > 0 ? xl : xr, xp = cx > 0 ? xr : xl;
          xg[2 * j * geo.nx + xp] = gsx[k];
          xg[(2 * j + 1) * geo.nx + xm] = gsx[k + 1];
        } else {
          *pg.template at<OFF32>(k, cx, cy, cz) = gsx[k];
          *pg.template at<OFF32>(k + 1, -cx, -cy, -cz) = gsx[k + 1];
        }
      }
    }
    }
  } else if (macro) {
    // dry evaluation: macroscopic fields of the current state
    macro[idx] = ps;
    macro[S + idx] = rho;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      macro[(2 + a) * S + idx] = u[a];
      macro[(2 + DIM + a) * S + idx] = F[a];
    }
  }
  if constexpr (MODE != MODE_STEP) {
    const double dr = (double)rho;
    acc[0] = (double)ps;
    acc[1] = dr * (double)u[0];
    acc[2] = dr * (double)u[1];
    acc[3] = dr * (double)u[2];
    const double sp2 = (double)u[0] * (double)u[0] + (double)u[1] * (double)u[1] + (double)u[2] * (double)u[2];
    acc[4] = 0.5 * dr * sp2;
    acc[5] = sqrt(sp2);
    const bool fin = isfinite((double)ps) && isfinite(sp2);
    acc[6] = fin ? 0.0 : 1.0;
    if (!fin) acc[5] = 0.0;
    // film region of the near-contact force (J != 0 exactly where a partner was
    // found): Sec. 3.3 sums of |F_rep.n|, |F_cap.n|, |F_rep| (Eq. RnAbs) with
    // F_rep = rho J, F_cap = mu grad phi and n the unit normal of the step
    if (Jv[0] != (T)0 || Jv[1] != (T)0 || Jv[2] != (T)0) {
      double fr2 = 0.0, frn = 0.0, fcn = 0.0;
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const double fr = dr * (double)Jv[a];
        const double fc = (double)mu * (double)gr[a];
        const double na = (double)(gr[a] * inv_g);
        fr2 += fr * fr;
        frn += fr * na;
        fcn += fc * na;
      }
      acc[8] = 1.0;
      acc[9] = fabs(frn);
      acc[10] = fabs(fcn);
      acc[11] = sqrt(fr2);
      acc[12] = acc[11];
    }
  }
}

template <int DIM, int QH, int PAR, int MODE, typename T, typename FS, typename GS, bool OFF32>
__global__ __launch_bounds__(NT) void k_collide(Planes<FS, GS> pl, const T* __restrict__ phi,
                                                const T* __restrict__ J,
                                                const unsigned* __restrict__ flags,
                                                unsigned* __restrict__ cnt_other, Geo geo,
                                                PhysT<T> pp, int nci_on, T* __restrict__ macro,
                                                T* __restrict__ uout, double* __restrict__ partials) {
  if (nci_on && blockIdx.x == 0 && threadIdx.x == 0) *cnt_other = 0u;
  int x, y, z;
  block_cell(slab_block(geo), geo, x, y, z);
  const bool valid = x < geo.nx && y < geo.ny;
  double acc[NPART] = {};
  if (MODE == MODE_STEP && !valid) return;
  if (valid)
    collide_cell<DIM, QH, PAR, MODE, T, FS, GS, OFF32>(pl, phi, J, flags, geo, pp, nci_on, macro, uout, x, y, z,
                                                       acc);
  if constexpr (MODE != MODE_STEP) block_partials(acc, partials);
}

// Fused collide + stream with the hydrodynamic populations in moment storage
// (3D): reads the coefficients of min, writes those of mout; the phase-field
// populations stay in AA parity PAR.
template <int QH, int PAR, int MODE, typename T, bool OFF32>
__global__ __launch_bounds__(NT) void k_collide_mom(Planes<T, T> pl, const T* __restrict__ min,
                                                    T* __restrict__ mout, const T* __restrict__ phi,
                                                    const T* __restrict__ J, const unsigned* __restrict__ flags,
                                                    unsigned* __restrict__ cnt_other, Geo geo, PhysT<T> pp,
                                                    int nci_on, T* __restrict__ macro,
                                                    double* __restrict__ partials) {
  if (nci_on && blockIdx.x == 0 && threadIdx.x == 0) *cnt_other = 0u;
  int x, y, z;
  block_cell(slab_block(geo), geo, x, y, z);
  const bool valid = x < geo.nx && y < geo.ny;
  double acc[NPART] = {};
  if (MODE == MODE_STEP && !valid) return;
  if (valid)
    collide_cell<3, QH, PAR, MODE, T, T, T, OFF32, false, false, true>(
        pl, phi, J, flags, geo, pp, nci_on, macro, nullptr, x, y, z, acc, nullptr, nullptr, nullptr, nullptr, min,
        mout);
  if constexpr (MODE != MODE_STEP) block_partials(acc, partials);
}

// Raw bits of a stored population (what the staging copies move).
template <typename E>
struct Bits {
  using type = E;
};
template <>
struct Bits<__half> {
  using type = unsigned short;
};
template <>
struct Bits<__hip_bfloat16> {
  using type = unsigned short;
};

// LDS bytes of k_collide_row for rows of nx cells: the x-shifted hydrodynamic
// pairs, then (at a 16-byte boundary) the x-shifted phase-field pairs.
template <int QH, typename FS>
__host__ __device__ constexpr unsigned xrow_f_bytes(int nx) {
  return (unsigned)((2 * xpair<HydroQ<QH>>(QH) * nx * (int)sizeof(FS) + 15) & ~15);
}
template <int DIM, int QH, typename FS, typename GS>
__host__ __device__ constexpr unsigned xrow_bytes(int nx) {
  return xrow_f_bytes<QH, FS>(nx) + (unsigned)(2 * xpair<Phase<DIM>>(Phase<DIM>::Q) * nx * (int)sizeof(GS));
}

// Fused collide + stream of the odd AA parity (3D), one block per x row.  In
// the odd parity a cell reads and writes its neighbours' slots, so the accesses
// of directions with c_x != 0 sit one cell off the row's alignment and the
// lines at block edges are shared by two blocks.  Here the block owns whole
// rows of those slots: it reads them aligned and streaming into LDS, the cells
// exchange their values there, and the rows go back aligned.  Each staged
// element is read and then written by exactly one cell (AA streaming swaps
// values in place), so the cells need no barrier among themselves; a row
// (y', z') of slot i is staged only by the block of row (y' - c_y, z' - c_z).
// Rows map to XCDs as the planes of slab_block: XCD k takes the planes k,
// k + 8, ... .  Blocks have NTR threads, each taking the cells x, x + NTR, ...
// With ONE (nx = NTR, one cell per thread) each thread also issues its cell's
// loads of the directions with c_x = 0 before the staging barrier, so that all
// of the cell's population loads are in flight together.
template <int QH, typename T, typename FS, typename GS, bool OFF32, int NTR, bool ONE = false>
__global__ __launch_bounds__(NTR) void k_collide_row(Planes<FS, GS> pl, const T* __restrict__ phi,
                                                    const T* __restrict__ J,
                                                    const unsigned* __restrict__ flags,
                                                    unsigned* __restrict__ cnt_other, Geo geo,
                                                    PhysT<T> pp, int nci_on, T* __restrict__ uout) {
  using H = HydroQ<QH>;
  using P = Phase<3>;
  using BF = typename Bits<FS>::type;
  using BG = typename Bits<GS>::type;
  extern __shared__ __align__(16) unsigned char xlds[];
  const int nx = geo.nx;
  FS* xf = (FS*)xlds;
  GS* xg = (GS*)(xlds + xrow_f_bytes<QH, FS>(nx));
  BF* bf = (BF*)xf;
  BG* bg = (BG*)xg;
  if (nci_on && blockIdx.x == 0 && threadIdx.x == 0) *cnt_other = 0u;
  int r = blockIdx.x;
  {
    const int per = geo.ny, full = (geo.nz & ~7) * per;
    if (r < full) {
      const int k = r & 7, i = r >> 3;
      r = (k + 8 * (i / per)) * per + i % per;
    }
  }
  const int y = r % geo.ny, z = r / geo.ny;
  const bool phase = uout == nullptr;   // LBM phase field (the FD one has no g)
  T fpre[H::Q], gpre[P::Q];
  if constexpr (ONE) {
    const PopNbr<const FS> pc(pl.f, (int)threadIdx.x, y, z, geo, H::Q);
#pragma unroll
    for (int i = 0; i < H::Q; ++i) {
      if (H::cx[i] != 0) continue;
      fpre[i] = Store<FS>::ldh(pc.template at<OFF32>(opp(i), 0, -H::cy[i], -H::cz[i]), pp.fref[i]);
    }
    if (phase) {
      const PopNbr<const GS> pgc(pl.g, (int)threadIdx.x, y, z, geo, P::Q);
#pragma unroll
      for (int k = 0; k < P::Q; ++k) {
        if (P::cx[k] != 0) continue;
        gpre[k] = (T)ld_nt(pgc.template at<OFF32>(opp(k), 0, -P::cy[k], -P::cz[k]));
      }
    }
  }
  for (int p = (int)threadIdx.x; p < nx; p += NTR) {
    const PopNbr<const FS> pf(pl.f, p, y, z, geo, H::Q);
#pragma unroll
    for (int i = 1; i < H::Q; i += 2) {
      if (H::cx[i] == 0) continue;
      const int j = xpair<H>(i);
      bf[2 * j * nx + p] = ld_nt((const BF*)pf.template at<OFF32>(i, 0, H::cy[i], H::cz[i]));
      bf[(2 * j + 1) * nx + p] = ld_nt((const BF*)pf.template at<OFF32>(i + 1, 0, -H::cy[i], -H::cz[i]));
    }
    if (phase) {
      const PopNbr<const GS> pg(pl.g, p, y, z, geo, P::Q);
#pragma unroll
      for (int k = 1; k < P::Q; k += 2) {
        if (P::cx[k] == 0) continue;
        const int j = xpair<P>(k);
        bg[2 * j * nx + p] = ld_nt((const BG*)pg.template at<OFF32>(k, 0, P::cy[k], P::cz[k]));
        bg[(2 * j + 1) * nx + p] = ld_nt((const BG*)pg.template at<OFF32>(k + 1, 0, -P::cy[k], -P::cz[k]));
      }
    }
  }
  __syncthreads();
  double acc[NPART];   // not used by the plain step
  if constexpr (ONE) {
    collide_cell<3, QH, 1, MODE_STEP, T, FS, GS, OFF32, true, true>(
        pl, phi, J, flags, geo, pp, nci_on, nullptr, uout, (int)threadIdx.x, y, z, acc, xf, xg, fpre, gpre);
  } else {
    for (int x = (int)threadIdx.x; x < nx; x += NTR)
      collide_cell<3, QH, 1, MODE_STEP, T, FS, GS, OFF32, true>(pl, phi, J, flags, geo, pp, nci_on, nullptr,
                                                               uout, x, y, z, acc, xf, xg);
  }
  __syncthreads();
  for (int p = (int)threadIdx.x; p < nx; p += NTR) {
    const PopNbr<FS> pf(pl.f, p, y, z, geo, H::Q);
#pragma unroll
    for (int i = 1; i < H::Q; i += 2) {
      if (H::cx[i] == 0) continue;
      const int j = xpair<H>(i);
      st_nt((BF*)pf.template at<OFF32>(i, 0, H::cy[i], H::cz[i]), bf[2 * j * nx + p]);
      st_nt((BF*)pf.template at<OFF32>(i + 1, 0, -H::cy[i], -H::cz[i]), bf[(2 * j + 1) * nx + p]);
    }
    if (phase) {
      const PopNbr<GS> pg(pl.g, p, y, z, geo, P::Q);
#pragma unroll
      for (int k = 1; k < P::Q; k += 2) {
        if (P::cx[k] == 0) continue;
        const int j = xpair<P>(k);
        st_nt((BG*)pg.template at<OFF32>(k, 0, P::cy[k], P::cz[k]), bg[2 * j * nx + p]);
        st_nt((BG*)pg.template at<OFF32>(k + 1, 0, -P::cy[k], -P::cz[k]), bg[(2 * j + 1) * nx + p]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// (b2) finite-difference phase field (Sec. 2.1.1): one explicit step of the
//      conservative Allen-Cahn equation, Eq. phi_update_muscl
// ---------------------------------------------------------------------------

// Periodic coordinate for offsets of at most two cells (any n >= 1).
__device__ __forceinline__ int wrap2(int v, int n) {
  if (v < 0) v += n;
  if (v < 0) v += n;
  if (v >= n) v -= n;
  if (v >= n) v -= n;
  return v;
}

// Eq. minmod: the smaller slope when both have the same sign, else zero, i.e.
// the median of (0, a, b) (one v_med3 in FP32).
__device__ __forceinline__ float minmod(float a, float b) { return __builtin_amdgcn_fmed3f(0.0f, a, b); }
__device__ __forceinline__ double minmod(double a, double b) { return fmax(fmin(a, b), fmin(fmax(a, b), 0.0)); }

// Advective flux through the face between cells 0 and 1 (Eqs. face_flux_def,
// slope_minmod_x, recon_lr_x, upwind_select_x): phi reconstructed linearly
// with limited slopes on each side (pm and p2 are the outer neighbours of
// cells 0 and 1) and taken from the upwind side of the face velocity uf.
template <typename T>
__device__ __forceinline__ T face_flux(T pm, T p0, T p1, T p2, T uf) {
  const T d = p1 - p0;
  const T phL = fmad((T)0.5, minmod(p0 - pm, d), p0);
  const T phR = fmad((T)-0.5, minmod(d, p2 - p1), p1);
  return uf * (uf >= (T)0 ? phL : phR);
}

// F(x + e_ax / 2) - F(x - e_ax / 2) of the advective flux along axis ax.
// Accessors: ph(dx, dy, dz) phi at an offset of up to two cells along ax,
// uv(ax, d) velocity component ax at offset d along ax.
template <typename T, typename PH, typename UV>
__device__ __forceinline__ T flux_difference(const PH& ph, const UV& uv, int ax) {
  T p[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) p[k] = ph(ax == 0 ? k - 2 : 0, ax == 1 ? k - 2 : 0, ax == 2 ? k - 2 : 0);
  const T um = uv(ax, -1), u0 = uv(ax, 0), up = uv(ax, 1);
  const T fp = face_flux(p[1], p[2], p[3], p[4], (T)0.5 * (u0 + up));
  const T fm = face_flux(p[0], p[1], p[2], p[3], (T)0.5 * (um + u0));
  return fp - fm;
}

// Increment phi' - phi = -div_h(u phi) + M lap_h phi - kappa div_iso(a), every
// term from the state before the step (div = div_h(u phi), the sum of the
// flux differences over the axes): u the velocity of that state's collision,
// the face velocity the mean of the two cells', lap_h the isotropic Laplacian
// (Eq. lap_iso), a = phi (1 - phi) n written by the collision, div_iso(a) =
// (1/cs^2) sum_i w_i c_i . a(x + c_i) on the hydrodynamic lattice and kappa =
// 4 M / W (Eqs. source_sharp, kappa_delta).  Accessors: ph(dx, dy, dz) phi at
// a lattice offset, av(comp, dx, dy, dz) component comp of a at one.
// Both stencils are summed per weight class (|c|^2 = 1, 2) before the weight
// is applied.  The Laplacian is summed over (phi(x + c) + phi(x - c)) - 2 phi(x),
// each exactly zero on a uniform field (the rounded weights sum to one only
// approximately, and that residue would add mass every step), and the
// increment is formed before it is added to phi (added term by term, parts
// smaller than half an ulp of phi would each be rounded away).
template <int DIM, int QH, typename T, typename PH, typename AV>
__device__ __forceinline__ T muscl_increment(const PH& ph, const AV& av, T div, T mob, T kap) {
  using H = HydroQ<QH>;
  const T p2 = ph(0, 0, 0) + ph(0, 0, 0);
  // the sums start at -0, which the first addition folds away
  T sl[3] = {(T)-0.0, (T)-0.0, (T)-0.0}, dc[3] = {(T)-0.0, (T)-0.0, (T)-0.0};
#pragma unroll
  for (int i = 1; i < H::Q; i += 2) {
    const int c[3] = {H::cx[i], H::cy[i], H::cz[i]};
    const int cl = c[0] * c[0] + c[1] * c[1] + c[2] * c[2] - 1;
    sl[cl] += (ph(c[0], c[1], c[2]) + ph(-c[0], -c[1], -c[2])) - p2;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      if (!c[a]) continue;
      const T d = av(a, c[0], c[1], c[2]) - av(a, -c[0], -c[1], -c[2]);
      dc[cl] += c[a] > 0 ? d : -d;
    }
  }
  // one weight per speed class |c|^2 = 1, 2 (and 3 on D3Q27): directions 1, 7, 19
  const T w1 = wt<H, T>(1), w2 = wt<H, T>(DIM == 2 ? 5 : 7);
  T lap = w1 * sl[0] + w2 * sl[1], dvi = w1 * dc[0] + w2 * dc[1];
  if constexpr (QH == 27) {
    lap += wt<H, T>(19) * sl[2];
    dvi += wt<H, T>(19) * dc[2];
  }
  lap = (T)6 * lap;
  dvi = (T)3 * dvi;
  return (mob * lap - div) - kap * dvi;
}

// Square root for the interface normal of the finite-difference update: the
// hardware instruction in FP32 (within 1 ulp, against about fifteen
// instructions for the correctly rounded one), the correctly rounded one in FP64.
__device__ __forceinline__ float fast_sqrt(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ __forceinline__ double fast_sqrt(double a) { return sqrt(a); }

// The sharpening flux a = phi (1 - phi) n of the finite-difference update at
// one cell (Eq. source_sharp), with the interface normal n = grad phi /
// (|grad phi| + eps_n) of the isotropic gradient on the hydrodynamic lattice
// (Eq. grad_iso).  get(i) is phi at the neighbour along direction i, get(0) the cell's own.
template <int QH, typename T, typename G>
__device__ __forceinline__ void sharpening_flux(const G& get, T eps_n, T a[3]) {
  using H = HydroQ<QH>;
  constexpr int DIM = H::D;
  // differences across the cell summed per speed class |c|^2 = 1, 2, 3 and
  // weighted once per class; the sums start at -0, which the first addition
  // folds away
  T s[3][3];
#pragma unroll
  for (int cl = 0; cl < 3; ++cl)
#pragma unroll
    for (int k = 0; k < 3; ++k) s[cl][k] = (T)-0.0;
#pragma unroll
  for (int i = 1; i < H::Q; i += 2) {
    const int c[3] = {H::cx[i], H::cy[i], H::cz[i]};
    const int cl = c[0] * c[0] + c[1] * c[1] + c[2] * c[2] - 1;
    const T d = get(i) - get(i + 1);
#pragma unroll
    for (int k = 0; k < DIM; ++k)
      if (c[k]) s[cl][k] += c[k] > 0 ? d : -d;
  }
  constexpr double w1 = 3 * H::w[1], w2 = 3 * H::w[DIM == 2 ? 5 : 7];
  constexpr double w3 = QH == 27 ? 3 * H::w[QH == 27 ? 19 : 0] : 0.0;
  T gr[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    gr[k] = (T)w1 * s[0][k] + (T)w2 * s[1][k];
    if constexpr (QH == 27) gr[k] += (T)w3 * s[2][k];
  }
  T gmag = gr[0] * gr[0] + gr[1] * gr[1];
  if (DIM == 3) gmag += gr[2] * gr[2];
  gmag = fast_sqrt(gmag);
  const T ph = get(0);
  const T kn = ph * ((T)1 - ph) * m_rcp(gmag + eps_n);
#pragma unroll
  for (int k = 0; k < 3; ++k) a[k] = k < DIM ? kn * gr[k] : (T)0;
}

// One cell per thread, neighbours read from global memory (2D boxes).  uv holds
// the velocity (DIM planes, plane stride S); a at the eight neighbours is formed
// here from phi up to two cells away.  out must not alias phi.
template <int DIM, int QH, typename T>
__global__ __launch_bounds__(NT) void k_muscl(const T* __restrict__ phi, T* __restrict__ out,
                                              const T* __restrict__ uvel, Geo geo, T mob, T kap, T eps_n) {
  static_assert(DIM == 2, "3D boxes take k_muscl3");
  using H = HydroQ<QH>;
  int x, y, z;
  block_cell(swizzled_block(), geo, x, y, z);
  if (x >= geo.nx || y >= geo.ny) return;
  const long long S = geo.S;
  const int cc[2] = {x, y};
  const int nn[2] = {geo.nx, geo.ny};
  const int st[2] = {1, geo.nx};
  const int idx = x + geo.nx * y;
  // offset of the cell d cells along axis ax (|d| <= 2, periodic)
  auto at = [&](int ax, int d) { return (wrap2(cc[ax] + d, nn[ax]) - cc[ax]) * st[ax]; };
  auto off = [&](int dx, int dy) {
    int o = idx;
    if (dx) o += at(0, dx);
    if (dy) o += at(1, dy);
    return o;
  };
  auto ph = [&](int dx, int dy, int) { return phi[off(dx, dy)]; };
  auto uv = [&](int ax, int d) { return uvel[ax * S + (d ? idx + at(ax, d) : idx)]; };
  T an[3][3][3];
#pragma unroll
  for (int i = 1; i < H::Q; ++i) {
    const int dx = H::cx[i], dy = H::cy[i];
    sharpening_flux<QH, T>([&](int k) { return phi[off(dx + H::cx[k], dy + H::cy[k])]; }, eps_n,
                           an[dy + 1][dx + 1]);
  }
  T div = 0;
#pragma unroll
  for (int ax = 0; ax < DIM; ++ax) div += flux_difference<T>(ph, uv, ax);
  const T inc = muscl_increment<DIM, QH, T>(
      ph, [&](int a, int dx, int dy, int) { return an[dy + 1][dx + 1][a]; }, div, mob, kap);
  out[idx] = phi[idx] + inc;
}

// 3D: a block owns a 64 x TY column of cells and marches along z through
// MUSCL_ZRUN planes.  Every plane of phi (halo 2 in x and y) is fetched from HBM
// once per block into an LDS ring of six planes; a = phi (1 - phi) n of the
// plane above the one being updated is then formed from the ring (halo 1) into
// a ring of three planes, so that a costs no HBM traffic.  u_x (halo 1 along x)
// and u_y (halo 1 along y) of the updated plane are staged in LDS too, double
// buffered; the cell's own u_z stays in registers.  The loads of the next plane
// are issued before the work on this one, so that their latency hides behind
// it.  Two barriers per plane: after the staging stores and after a.  Unrolled
// by the period of the rings (6 planes), every ring slot of the march is a
// compile-time constant and each LDS access one instruction with an immediate
// offset from a loop-invariant lane address.
constexpr int MUSCL_ZRUN = 64;   // planes a block marches through
constexpr int MZ_TX = 64;        // cells per block row
constexpr int MZ_RING = 6;       // phi planes in LDS (z - 1 .. z + 3 in use)
template <typename T>
struct MuslTile {
  static constexpr int TY = 8;   // rows per block: a is formed on 1.29 cells per cell (1.55 with 4 rows)
  static constexpr int NT = MZ_TX * TY;
  static constexpr int PW = MZ_TX + 4, PN = PW * (TY + 4);   // phi planes, halo 2
  static constexpr int AW = MZ_TX + 2, AN = AW * (TY + 2);   // a planes, halo 1
  static constexpr int XN = (MZ_TX + 2) * TY;                // u_x: halo 1 along x
  static constexpr int YN = MZ_TX * (TY + 2);                // u_y: halo 1 along y
  static constexpr int KP = (PN + NT - 1) / NT, KA = (AN + NT - 1) / NT;   // staged cells per thread
  static constexpr int KX = (XN + NT - 1) / NT, KY = (YN + NT - 1) / NT;
};

template <int V>
using Const = std::integral_constant<int, V>;

// D3Q19 in FP32: the march unrolled, registers capped at 128 (four waves per
// SIMD): 1.12 ms at 512^3, against 1.69 ms uncapped (131 registers, two waves)
// and 1.32 ms rolled.  D3Q27 stays rolled: its unrolled body is six times the
// larger stencil (2.1 ms unrolled, 1.70 ms rolled).
template <int QH, typename T>
constexpr bool muscl_unrolled() { return QH == 19 && std::is_same<T, float>::value; }

template <int QH, typename T>
__global__ __launch_bounds__(MuslTile<T>::NT, (muscl_unrolled<QH, T>() ? 4 : 1)) void k_muscl3(const T* __restrict__ phi, T* __restrict__ out,
                                                            const T* __restrict__ uvel, Geo geo, T mob, T kap,
                                                            T eps_n, int ntx, int nty) {
  using M = MuslTile<T>;
  using H = HydroQ<QH>;
  constexpr int KP = M::KP, KA = M::KA, KX = M::KX, KY = M::KY;
  __shared__ T sp[MZ_RING][M::PN];
  __shared__ T sa[3][3][M::AN];
  __shared__ T sx[2][M::XN];
  __shared__ T sy[2][M::YN];
  const int t = swizzled_block();
  const int tx = t % ntx, r = t / ntx, ty = r % nty, zc = r / nty;
  const int x0 = tx * MZ_TX, y0 = ty * M::TY;
  const int z0 = zc * MUSCL_ZRUN, z1 = min(z0 + MUSCL_ZRUN, geo.nz);
  const int tid = threadIdx.x, lx = tid & (MZ_TX - 1), ly = tid / MZ_TX;
  const int nx = geo.nx, ny = geo.ny, nz = geo.nz;
  const bool valid = x0 + lx < nx && y0 + ly < ny;
  const int plane = nx * ny;
  const int own = valid ? (x0 + lx) + nx * (y0 + ly) : 0;
  const long long S = geo.S;
  // in-plane byte offsets of the staged cells, the same on every plane; the
  // slots k below NT-multiples of a tile's size are always in use
  auto used = [&](int k, int n) { return (k + 1) * M::NT <= n || tid + k * M::NT < n; };
  auto inplane = [&](int ex, int ey) { return (unsigned)(wrapi(ex, nx) + nx * wrapi(ey, ny)) * sizeof(T); };
  unsigned po[KP], xo[KX], yo[KY];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int s = tid + k * M::NT;
    po[k] = used(k, M::PN) ? inplane(x0 - 2 + s % M::PW, y0 - 2 + s / M::PW) : 0u;
  }
#pragma unroll
  for (int k = 0; k < KX; ++k) {
    const int s = tid + k * M::NT;
    xo[k] = used(k, M::XN) ? inplane(x0 - 1 + s % (MZ_TX + 2), y0 + s / (MZ_TX + 2)) : 0u;
  }
#pragma unroll
  for (int k = 0; k < KY; ++k) {
    const int s = tid + k * M::NT;
    yo[k] = used(k, M::YN) ? inplane(x0 + s % MZ_TX, y0 - 1 + s / MZ_TX) : 0u;
  }
  int pa[KA];   // the staged a cells in a phi plane
#pragma unroll
  for (int k = 0; k < KA; ++k) {
    const int s = tid + k * M::NT;
    pa[k] = (s / M::AW + 1) * M::PW + s % M::AW + 1;
  }
  const unsigned owno = (unsigned)own * sizeof(T);
  // a plane of a field as a uniform base; cells are read at 32-bit byte offsets
  auto zbase = [&](const T* f, int z) { return (const char*)(f + (long long)wrapi(z, nz) * plane); };
  auto ld = [](const char* b, unsigned o) { return *(const T*)(b + o); };
  // registers in flight: phi of one plane, u_x and u_y of one plane, own u_z
  T rp[KP], rx[KX], ry[KY], rv = 0;
  auto fetch_phi = [&](int zp) {
    const char* bp = zbase(phi, zp);
#pragma unroll
    for (int k = 0; k < KP; ++k) rp[k] = used(k, M::PN) ? ld(bp, po[k]) : (T)0;
  };
  auto fetch_u = [&](int zu) {
    const char* bx = zbase(uvel, zu);
    const char* by = zbase(uvel + S, zu);
#pragma unroll
    for (int k = 0; k < KX; ++k) rx[k] = used(k, M::XN) ? ld(bx, xo[k]) : (T)0;
#pragma unroll
    for (int k = 0; k < KY; ++k) ry[k] = used(k, M::YN) ? ld(by, yo[k]) : (T)0;
    if (valid) rv = ld(zbase(uvel + 2 * S, zu + 1), owno);
  };
  auto put_phi = [&](T* dst) {
#pragma unroll
    for (int k = 0; k < KP; ++k)
      if (used(k, M::PN)) dst[tid + k * M::NT] = rp[k];
  };
  // a over the tile and its halo of one cell into a slot, from three
  // consecutive phi planes of the ring
  auto make_a = [&](T (*dst)[M::AN], const T* Pl, const T* Pc, const T* Pu) {
    const T* P[3] = {Pl, Pc, Pu};
#pragma unroll
    for (int k = 0; k < KA; ++k) {
      if (!used(k, M::AN)) continue;
      const int s = tid + k * M::NT, c = pa[k];
      T av[3];
      sharpening_flux<QH, T>([&](int i) { return P[1 + H::cz[i]][c + H::cy[i] * M::PW + H::cx[i]]; }, eps_n,
                             av);
#pragma unroll
      for (int a = 0; a < 3; ++a) dst[a][s] = av[a];
    }
  };
  // Ring slots, with j = (z - z0) mod 6 for the plane z being updated: phi of
  // plane z + d in sp[(j + d + 2) mod 6], a of plane z + d in sa[(j + d + 1) mod 3],
  // u_x and u_y of plane z in buffer j mod 2.
  // prologue: phi planes z0 - 2 .. z0 + 1, a of planes z0 - 1 and z0, the
  // flux through the face z0 - 1/2, then the loads of the first plane
#pragma unroll
  for (int d = -2; d <= 1; ++d) {
    fetch_phi(z0 + d);
    put_phi(sp[d + 2]);
  }
  T v0 = 0, v1 = 0;
  if (valid) {
    v0 = ld(zbase(uvel + 2 * S, z0 - 1), owno);
    v1 = ld(zbase(uvel + 2 * S, z0), owno);
  }
  fetch_phi(z0 + 2);
  fetch_u(z0);
  __syncthreads();
  make_a(sa[0], sp[0], sp[1], sp[2]);
  make_a(sa[1], sp[1], sp[2], sp[3]);
  const int cp = (ly + 2) * M::PW + lx + 2;   // the cell in a phi plane
  const int ca = (ly + 1) * M::AW + lx + 1;   // the cell in an a plane
  T fzm = face_flux(sp[0][cp], sp[1][cp], sp[2][cp], sp[3][cp], (T)0.5 * (v0 + v1));   // face z0 - 1/2
  // one plane z, ring phase J = (z - z0) mod 6 (a compile-time constant when
  // the march is unrolled)
  auto plane_step = [&](int z, auto J) {
    const int j = J;
    T* const Pm = sp[(j + 1) % MZ_RING];
    T* const P0 = sp[(j + 2) % MZ_RING];
    T* const Pp = sp[(j + 3) % MZ_RING];
    T* const Pq = sp[(j + 4) % MZ_RING];
    put_phi(Pq);
#pragma unroll
    for (int k = 0; k < KX; ++k)
      if (used(k, M::XN)) sx[j & 1][tid + k * M::NT] = rx[k];
#pragma unroll
    for (int k = 0; k < KY; ++k)
      if (used(k, M::YN)) sy[j & 1][tid + k * M::NT] = ry[k];
    const T v2 = rv;
    __syncthreads();
    if (z + 1 < z1) {
      fetch_phi(z + 3);
      fetch_u(z + 1);
    }
    make_a(sa[(j + 2) % 3], P0, Pp, Pq);
    __syncthreads();
    if (valid) {
      const T* Ux = sx[j & 1];
      const T* Uy = sy[j & 1];
      const T q1 = Pm[cp], q2 = P0[cp], q3 = Pp[cp], q4 = Pq[cp];
      auto ph = [&](int dx, int dy, int dz) -> T {
        const T* P = dz < 0 ? Pm : (dz > 0 ? Pp : P0);
        return P[cp + dy * M::PW + dx];
      };
      auto uv = [&](int ax, int d) -> T {
        if (ax == 2) return d < 0 ? v0 : (d > 0 ? v2 : v1);
        return ax == 0 ? Ux[ly * (MZ_TX + 2) + lx + 1 + d] : Uy[(ly + 1 + d) * MZ_TX + lx];
      };
      auto av = [&](int a, int dx, int dy, int dz) -> T {
        return sa[(j + 1 + dz + 3) % 3][a][ca + dy * M::AW + dx];
      };
      // the face below this cell is the face above the previous one
      const T fzp = face_flux(q1, q2, q3, q4, (T)0.5 * (v1 + v2));
      const T div = (flux_difference<T>(ph, uv, 0) + flux_difference<T>(ph, uv, 1)) + (fzp - fzm);
      fzm = fzp;
      const T inc = muscl_increment<3, QH, T>(ph, av, div, mob, kap);
      st_nt((T*)((char*)(out + (long long)z * plane) + owno), q2 + inc);
    }
    v0 = v1;
    v1 = v2;
  };
  if constexpr (!muscl_unrolled<QH, T>()) {
#pragma unroll 1
    for (int z = z0, j = 0; z < z1; ++z, j = j == MZ_RING - 1 ? 0 : j + 1) plane_step(z, j);
    return;
  }
#pragma unroll 1
  for (int z = z0; z < z1; z += MZ_RING) {
    plane_step(z, Const<0>{});
    if (z + 1 >= z1) break;
    plane_step(z + 1, Const<1>{});
    if (z + 2 >= z1) break;
    plane_step(z + 2, Const<2>{});
    if (z + 3 >= z1) break;
    plane_step(z + 3, Const<3>{});
    if (z + 4 >= z1) break;
    plane_step(z + 4, Const<4>{});
    if (z + 5 >= z1) break;
    plane_step(z + 5, Const<5>{});
  }
}

// ---------------------------------------------------------------------------
// (c) diagnostics: sum phi and the number of droplets, i.e. the connected
//     components of the dispersed set (8- / 26-connectivity, periodic)
// ---------------------------------------------------------------------------

constexpr unsigned CC_NONE = 0xffffffffu;   // label of a cell outside the dispersed set

// Labels are read with device-scope atomic loads: other workgroups, on other
// XCDs, lower them while the merge kernel runs.
__device__ __forceinline__ unsigned cc_load(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of the tree of x.  Every label is at most its own index and a root is
// its own label, so the walk visits strictly decreasing indices and ends.  x is
// then pointed at the root (an atomic minimum keeps labels monotone).
__device__ __forceinline__ unsigned cc_find(unsigned* L, unsigned x) {
  unsigned r = x, y;
  while ((y = cc_load(L + r)) != r) r = y;
  if (r != x) atomicMin(L + x, r);
  return r;
}

// Joins the trees of cells a and b: the larger root is hung under the smaller
// one by an atomic minimum.  If that root had meanwhile been hung elsewhere the
// minimum returns its new parent and the join is retried from there; the larger
// of the two roots strictly decreases on every retry.
__device__ __forceinline__ void cc_unite(unsigned* L, unsigned a, unsigned b) {
  while (true) {
    a = cc_find(L, a);
    b = cc_find(L, b);
    if (a == b) return;
    if (a > b) {
      const unsigned t = a;
      a = b;
      b = t;
    }
    const unsigned old = atomicMin(L + b, a);
    if (old == b) return;
    b = old;
  }
}

// L[idx] = idx for cells of the dispersed set, CC_NONE elsewhere.
template <int DIM, typename T>
__global__ __launch_bounds__(NT) void k_cc_init(const T* __restrict__ phi, Geo geo, int dispersed,
                                                unsigned* __restrict__ L) {
  int x, y, z;
  block_cell(swizzled_block(), geo, x, y, z);
  if (x >= geo.nx || y >= geo.ny) return;
  const unsigned idx = (unsigned)Nbr(x, y, z, geo)(0, 0, 0);
  const T v = phi[idx];
  const bool in = dispersed ? (v > (T)0.5) : (v < (T)0.5);
  L[idx] = in ? idx : CC_NONE;
}

// Every cell of the set joins its neighbours of the set at the 4 (2D) / 13 (3D)
// offsets that precede it in (z, y, x) order; with the periodic wrap this
// covers each adjacent pair once.  Membership is read from phi (the test of
// k_cc_init), with plain cached loads: only the label walks need the
// device-scope atomic loads.
template <int DIM, typename T>
__global__ __launch_bounds__(NT) void k_cc_merge(const T* __restrict__ phi, Geo geo, int dispersed,
                                                 unsigned* __restrict__ L) {
  int x, y, z;
  block_cell(swizzled_block(), geo, x, y, z);
  if (x >= geo.nx || y >= geo.ny) return;
  const Nbr nb(x, y, z, geo);
  const unsigned idx = (unsigned)nb(0, 0, 0);
  auto in = [&](unsigned j) { return dispersed ? (phi[j] > (T)0.5) : (phi[j] < (T)0.5); };
  if (!in(idx)) return;
  const int dz0 = DIM == 3 ? -1 : 0;
  for (int dz = dz0; dz <= 0; ++dz)
    for (int dy = -1; dy <= (dz < 0 ? 1 : 0); ++dy)
      for (int dx = -1; dx <= ((dz < 0 || dy < 0) ? 1 : -1); ++dx) {
        const unsigned j = (unsigned)nb(dx, dy, dz);
        if (in(j)) cc_unite(L, idx, j);
      }
}

// Per-block partials of the diagnostics: [0] sum phi, [1] roots of the
// component labels (one per droplet), [6] non-finite phi.  A block covers
// DIAG_PER row blocks of the cell-wise grid (nblk of them in all), so that its
// FP64 block reduction is paid once per DIAG_PER x NT cells.
constexpr int DIAG_PER = 8;
template <int DIM, typename T>
__global__ __launch_bounds__(NT) void k_diag(const T* __restrict__ phi, Geo geo,
                                             const unsigned* __restrict__ L, int nblk,
                                             double* __restrict__ partials) {
  const int t = swizzled_block();
  double a0 = 0.0, a1 = 0.0, a6 = 0.0;
#pragma unroll
  for (int r = 0; r < DIAG_PER; ++r) {
    const int lb = t * DIAG_PER + r;
    if (lb >= nblk) break;
    int x, y, z;
    block_cell(lb, geo, x, y, z);
    if (x < geo.nx && y < geo.ny) {
      const unsigned idx = (unsigned)Nbr(x, y, z, geo)(0, 0, 0);
      const T p0 = phi[idx];
      a0 += (double)p0;
      a6 += isfinite((double)p0) ? 0.0 : 1.0;
      a1 += L[idx] == idx ? 1.0 : 0.0;
    }
  }
  // the three used slots only (the other slots are zero)
  __shared__ double red[NT / 64][3];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a6 = wave_sum(a6);
  if (lane == 0) {
    red[wv][0] = a0;
    red[wv][1] = a1;
    red[wv][2] = a6;
  }
  __syncthreads();
  if (threadIdx.x < NPART) {
    const int k = threadIdx.x, r = k == 0 ? 0 : (k == 1 ? 1 : (k == 6 ? 2 : -1));
    double a = r < 0 ? 0.0 : red[0][r];
    for (int j = 1; j < NT / 64; ++j) a = r < 0 ? a : a + red[j][r];
    partials[blockIdx.x * NPART + k] = a;
  }
}

// First stage of the reduction: block b reduces partials [b*chunk, (b+1)*chunk)
// into out[b] (fixed order, deterministic).
__global__ __launch_bounds__(NT) void k_reduce_stage(const double* __restrict__ p, int n, int chunk,
                                                     double* __restrict__ out) {
  __shared__ double red[NT][NPART];
  const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  double v[NPART] = {};
  for (int b = lo + (int)threadIdx.x; b < hi; b += NT)
    for (int k = 0; k < NPART; ++k) v[k] = max_slot(k) ? fmax(v[k], p[b * NPART + k]) : v[k] + p[b * NPART + k];
  for (int k = 0; k < NPART; ++k) red[threadIdx.x][k] = v[k];
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < NPART; ++k)
        red[threadIdx.x][k] = max_slot(k) ? fmax(red[threadIdx.x][k], red[threadIdx.x + s][k])
                                       : red[threadIdx.x][k] + red[threadIdx.x + s][k];
    __syncthreads();
  }
  if (threadIdx.x < NPART) out[blockIdx.x * NPART + threadIdx.x] = red[0][threadIdx.x];
}

// Deterministic final reduction of per-block partials: out[0..7] for the
// collide partials, out[8..15] for the diag partials.
__global__ __launch_bounds__(NT) void k_reduce(const double* __restrict__ pa, int na,
                                               const double* __restrict__ pb, int nb_,
                                               const unsigned* __restrict__ nci_count,
                                               double* __restrict__ out) {
  __shared__ double red[NT][NPART];
  for (int pass = 0; pass < 2; ++pass) {
    const double* p = pass ? pb : pa;
    const int n = pass ? nb_ : na;
    double v[NPART] = {};
    for (int b = threadIdx.x; b < n; b += NT)
      for (int k = 0; k < NPART; ++k) v[k] = max_slot(k) ? fmax(v[k], p[b * NPART + k]) : v[k] + p[b * NPART + k];
    for (int k = 0; k < NPART; ++k) red[threadIdx.x][k] = v[k];
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s)
        for (int k = 0; k < NPART; ++k)
          red[threadIdx.x][k] = max_slot(k) ? fmax(red[threadIdx.x][k], red[threadIdx.x + s][k])
                                         : red[threadIdx.x][k] + red[threadIdx.x + s][k];
      __syncthreads();
    }
    if (threadIdx.x < NPART) out[pass * NPART + threadIdx.x] = red[0][threadIdx.x];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[7] = nci_count ? (double)*nci_count : 0.0;
}

// ---------------------------------------------------------------------------
// initial populations, population I/O
// ---------------------------------------------------------------------------

// f = feq(p*, u) (Eq. feq3), g = geq(phi, u, n) in natural layout (parity 0).
template <int DIM, int QH, typename T, typename FS, typename GS>
__global__ __launch_bounds__(NT) void k_init(FS* __restrict__ f, GS* __restrict__ g,
                                             const T* __restrict__ phi, const T* __restrict__ uin,
                                             const T* __restrict__ psin, Geo geo, PhysT<T> pp) {
  using H = HydroQ<QH>;
  using P = Phase<DIM>;
  int x, y, z;
  block_cell(swizzled_block(), geo, x, y, z);
  if (x >= geo.nx || y >= geo.ny) return;
  const Nbr nb(x, y, z, geo);
  const int idx = nb(0, 0, 0);
  const long long S = geo.S;
  T u[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) u[a] = uin[a * S + idx];
  const T ps = psin[idx];
  const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
  for (int i = 0; i < H::Q; ++i) {
    const T cu = i == 0 ? (T)0 : sdot(H::cx[i], H::cy[i], H::cz[i], u[0], u[1], u[2]);
    const T fe = wt<H, T>(i) * (ps + (T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * uu + (T)4.5 * cu * cu * cu -
                               (T)4.5 * cu * uu);
    Store<FS>::st(f + pop_elem(i, x, y, z, geo, H::Q), fe, pp.fref[i]);
  }
  T gr[3], lap;
  grad_lap<QH, T>([&](int i) { return phi[nb(H::cx[i], H::cy[i], H::cz[i])]; }, gr, lap);
  const T ph = phi[idx];
  T gmag = m_sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
  const T kc = pp.kc * ph * ((T)1 - ph) / (gmag + pp.eps_n);
  const T jv[3] = {ph * u[0] + kc * gr[0], ph * u[1] + kc * gr[1], ph * u[2] + kc * gr[2]};
#pragma unroll
  for (int k = 0; k < P::Q; ++k) {
    const T cj = k == 0 ? (T)0 : sdot(P::cx[k], P::cy[k], P::cz[k], jv[0], jv[1], jv[2]);
    g[pop_elem(k, x, y, z, geo, P::Q)] = (GS)(wt<P, T>(k) * (ph + cj * (T)P::inv_cs2));
  }
}

// Moment storage, initial state: the coefficients (p*, u, 0, 0), whose
// populations are feq(p*, u) (Eq. feq3), so that the first incoming populations
// of a cell are the equilibria of the cells they stream from; g = geq(phi, u, n)
// in natural layout (parity 0).
template <int QH, typename T>
__global__ __launch_bounds__(NT) void k_init_mom(T* __restrict__ mom, T* __restrict__ g,
                                                 const T* __restrict__ phi, const T* __restrict__ uin,
                                                 const T* __restrict__ psin, Geo geo, PhysT<T> pp) {
  using H = HydroQ<QH>;
  using P = Phase<3>;
  int x, y, z;
  block_cell(swizzled_block(), geo, x, y, z);
  if (x >= geo.nx || y >= geo.ny) return;
  const Nbr nb(x, y, z, geo);
  const int idx = nb(0, 0, 0);
  const long long S = geo.S;
  const T u[3] = {uin[idx], uin[S + idx], uin[2 * S + idx]};
  mom[idx] = psin[idx];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    mom[(1 + a) * S + idx] = u[a];
    mom[(4 + a) * S + idx] = (T)0;
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) mom[(7 + k) * S + idx] = (T)0;
  T gr[3], lap;
  grad_lap<QH, T>([&](int i) { return phi[nb(H::cx[i], H::cy[i], H::cz[i])]; }, gr, lap);
  const T ph = phi[idx];
  T gmag = m_sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
  const T kc = pp.kc * ph * ((T)1 - ph) / (gmag + pp.eps_n);
  const T jv[3] = {ph * u[0] + kc * gr[0], ph * u[1] + kc * gr[1], ph * u[2] + kc * gr[2]};
#pragma unroll
  for (int k = 0; k < P::Q; ++k) {
    const T cj = k == 0 ? (T)0 : sdot(P::cx[k], P::cy[k], P::cz[k], jv[0], jv[1], jv[2]);
    g[pop_elem(k, x, y, z, geo, P::Q)] = (T)(wt<P, T>(k) * (ph + cj * (T)P::inv_cs2));
  }
}

// Moment storage: incoming populations on a wrapped box, rebuilt from the
// coefficients, as doubles, SoA [q][box]; g as k_getpop.
template <int QH, int PAR, typename T>
__global__ __launch_bounds__(NT) void k_getpop_mom(const T* __restrict__ mom, const T* __restrict__ g, Geo geo,
                                                   int x0, int y0, int z0, int bxn, int byn, int bzn,
                                                   double* __restrict__ fo, double* __restrict__ go) {
  using H = HydroQ<QH>;
  using P = Phase<3>;
  const long long B = (long long)bxn * byn * bzn;
  const long long e = (long long)blockIdx.x * NT + threadIdx.x;
  if (e >= B) return;
  const int lx = (int)(e % bxn), ly = (int)((e / bxn) % byn), lz = (int)(e / ((long long)bxn * byn));
  const int x = wrapi(x0 + lx, geo.nx), y = wrapi(y0 + ly, geo.ny), z = wrapi(z0 + lz, geo.nz);
  const Nbr nb(x, y, z, geo);
  T fi[H::Q];
  pull_populations<QH, T>(mom, geo.S, nb, fi);
  for (int i = 0; i < H::Q; ++i) fo[i * B + e] = (double)fi[i];
  const PopNbr<const T> pg(g, x, y, z, geo, P::Q);
  for (int k = 0; k < P::Q; ++k) {
    const T* src = PAR == 0 ? pg.template at<false>(k, 0, 0, 0)
                            : pg.template at<false>(opp(k), -P::cx[k], -P::cy[k], -P::cz[k]);
    go[k * B + e] = (double)*src;
  }
}

// Incoming populations on a wrapped box, as doubles, SoA [q][box].
template <int DIM, int QH, int PAR, typename T, typename FS, typename GS>
__global__ __launch_bounds__(NT) void k_getpop(const FS* __restrict__ f, const GS* __restrict__ g,
                                               Geo geo, PhysT<T> pp, int x0, int y0, int z0, int bxn,
                                               int byn, int bzn, double* __restrict__ fo,
                                               double* __restrict__ go) {
  using H = HydroQ<QH>;
  using P = Phase<DIM>;
  const long long B = (long long)bxn * byn * bzn;
  const long long e = (long long)blockIdx.x * NT + threadIdx.x;
  if (e >= B) return;
  const int lx = (int)(e % bxn), ly = (int)((e / bxn) % byn), lz = (int)(e / ((long long)bxn * byn));
  const int x = wrapi(x0 + lx, geo.nx), y = wrapi(y0 + ly, geo.ny), z = wrapi(z0 + lz, geo.nz);
  const PopNbr<const FS> pf(f, x, y, z, geo, H::Q);
  const PopNbr<const GS> pg(g, x, y, z, geo, P::Q);
  for (int i = 0; i < H::Q; ++i) {
    const FS* src = PAR == 0 ? pf.template at<false>(i, 0, 0, 0)
                             : pf.template at<false>(opp(i), -H::cx[i], -H::cy[i], -H::cz[i]);
    fo[i * B + e] = (double)Store<FS>::ld(src, pp.fref[i]);
  }
  for (int k = 0; k < P::Q; ++k) {
    const GS* src = PAR == 0 ? pg.template at<false>(k, 0, 0, 0)
                             : pg.template at<false>(opp(k), -P::cx[k], -P::cy[k], -P::cz[k]);
    go[k * B + e] = (double)*src;
  }
}

// Whole-field populations (doubles, SoA [q][N]) into natural layout.
template <int DIM, int QH, typename T, typename FS, typename GS>
__global__ __launch_bounds__(NT) void k_setpop(FS* __restrict__ f, GS* __restrict__ g, Geo geo,
                                               PhysT<T> pp, const double* __restrict__ fi,
                                               const double* __restrict__ gi) {
  using H = HydroQ<QH>;
  using P = Phase<DIM>;
  const long long N = (long long)geo.nx * geo.ny * geo.nz;
  const long long e = (long long)blockIdx.x * NT + threadIdx.x;
  if (e >= N) return;
  const int x = (int)(e % geo.nx), y = (int)((e / geo.nx) % geo.ny), z = (int)(e / ((long long)geo.nx * geo.ny));
  for (int i = 0; i < H::Q; ++i)
    Store<FS>::st(f + pop_elem(i, x, y, z, geo, H::Q), (T)fi[i * N + e], pp.fref[i]);
  for (int k = 0; k < P::Q; ++k) g[pop_elem(k, x, y, z, geo, P::Q)] = (GS)gi[k * N + e];
}

// ---------------------------------------------------------------------------
// multi-domain launches (serving): one grid covers every lattice of a batch
// ---------------------------------------------------------------------------

// One resident lattice in a batch.  The table lives in device memory; blocks
// find their lattice by its first block index, and each lattice keeps its own
// AA parity (step + s) so that lattices admitted at different times can share
// one launch.  The per-cell code is the single-domain code, so every lattice
// evolves bit for bit as it would alone.
template <typename T, typename FS, typename GS>
struct Job {
  Planes<FS, GS> pl;
  T* phi;
  T* J;
  unsigned* flags[2];
  unsigned* list[2];
  unsigned* cnt;      // [0], [1]: tile-list lengths per parity; [2]: cells with chi = 1
  Geo geo;
  PhysT<T> pp;
  NciP np;
  int nci_on;
  T q_th;
  int blk0, nblk;     // first block of this lattice in the batch grid, and its block count
  int pblk0, pnblk;   // the same in the grid of the phi pass, whose blocks take PHI_PER row blocks each
  long long step;     // completed steps of this lattice when the launch sequence starts
};

// Row blocks per block of the multi-lattice phi pass: its per-cell work is a few
// loads, so each block amortises its job-table lookup over several row blocks,
// and issues the loads of all of them before its first store.
constexpr int PHI_PER = 8;
// Lattices of a batch whose near-contact work is spread as one list (more fall
// back to a loop over the lattices).
constexpr int NCI_FLAT_JOBS = 64;

template <typename JT>
__device__ __forceinline__ int find_job(const JT* __restrict__ jobs, int njobs, int t) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].blk0 <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename JT>
__device__ __forceinline__ int find_job_phi(const JT* __restrict__ jobs, int njobs, int t) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].pblk0 <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The PHI_PER row blocks of phi-pass block t: the cells past the lattice's end
// load the clamped cell (in bounds) and store nothing.
template <int DIM, int PAR, typename T, typename FS, typename GS>
__device__ __forceinline__ void phi_rows(const Job<T, FS, GS>& jb, int t) {
  T sv[PHI_PER];
  int cx[PHI_PER], cy[PHI_PER], cz[PHI_PER];
  bool ok[PHI_PER];
#pragma unroll
  for (int r = 0; r < PHI_PER; ++r) {
    const int lb = (t - jb.pblk0) * PHI_PER + r;
    int x, y, z;
    block_cell(lb, jb.geo, x, y, z);
    ok[r] = lb < jb.nblk && x < jb.geo.nx && y < jb.geo.ny;
    cx[r] = min(x, jb.geo.nx - 1);
    cy[r] = min(y, jb.geo.ny - 1);
    cz[r] = min(z, jb.geo.nz - 1);
  }
#pragma unroll
  for (int r = 0; r < PHI_PER; ++r) sv[r] = phi_moment<DIM, PAR, T, GS>(jb.pl.g, jb.geo, cx[r], cy[r], cz[r]);
#pragma unroll
  for (int r = 0; r < PHI_PER; ++r) {
    if (!ok[r]) continue;
    st_nt(jb.phi + (cx[r] + jb.geo.nx * (cy[r] + jb.geo.ny * cz[r])), sv[r]);
    if (jb.nci_on)
      phi_mark<DIM, T>(sv[r], jb.geo, jb.flags[PAR], jb.list[PAR], jb.cnt + PAR, jb.q_th, cx[r], cy[r], cz[r]);
  }
}

template <int DIM, typename T, typename FS, typename GS>
__global__ __launch_bounds__(NT) void k_phi_multi(const Job<T, FS, GS>* __restrict__ jobs, int njobs,
                                                  int s) {
  const int t = swizzled_block();
  const Job<T, FS, GS>& jb = jobs[find_job_phi(jobs, njobs, t)];
  const int par = (int)((jb.step + s) & 1);
  if (jb.nci_on && t == jb.pblk0 && threadIdx.x == 0) jb.cnt[2] = 0u;
  if (par == 0) phi_rows<DIM, 0>(jb, t);
  else phi_rows<DIM, 1>(jb, t);
}

// Near-contact pass of a batch.  Up to NCI_FLAT_JOBS lattices: the listed tiles
// of all lattices form one list (prefix sums over the lattices' tile counts), so
// that the blocks share the work whatever its split between lattices, and each
// block reads the job table once per tile instead of looping over every
// lattice.  A tile's phi halo is prefetched during the previous tile, also
// across lattices.  More lattices: a loop over them, each spread over all blocks.
template <int DIM, int QH, typename T, typename FS, typename GS>
__global__ __launch_bounds__(NT_NCI) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) void k_nci_multi(const Job<T, FS, GS>* __restrict__ jobs,
                                                      int njobs, int s) {
  __shared__ NciShared<DIM, T> sm;
  __shared__ unsigned pre[NCI_FLAT_JOBS + 1], preo[NCI_FLAT_JOBS + 1];
  if (njobs <= NCI_FLAT_JOBS) {
    if (threadIdx.x < 64) {
      const int j = (int)threadIdx.x;
      unsigned a = 0u, b = 0u;
      if (j < njobs && jobs[j].nci_on) {
        const int par = (int)((jobs[j].step + s) & 1);
        a = jobs[j].cnt[par];
        b = jobs[j].cnt[1 - par];
      }
      // inclusive scan over the wave
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const unsigned va = __shfl_up(a, d), vb = __shfl_up(b, d);
        if (j >= d) {
          a += va;
          b += vb;
        }
      }
      pre[j + 1] = a;
      preo[j + 1] = b;
      if (j == 0) pre[0] = preo[0] = 0u;
    }
    __syncthreads();
    auto owner = [&](const unsigned* p, unsigned k) {   // the lattice whose range holds k
      int lo = 0, hi = njobs - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p[mid] <= k) lo = mid;
        else hi = mid - 1;
      }
      return lo;
    };
    // the other parity's flags, cleared for the next step's tile lists
    const unsigned totalo = preo[njobs];
    for (unsigned k = blockIdx.x * NT_NCI + threadIdx.x; k < totalo; k += gridDim.x * NT_NCI) {
      const int j = owner(preo, k);
      const Job<T, FS, GS>& jb = jobs[j];
      const int par = (int)((jb.step + s) & 1);
      jb.flags[1 - par][jb.list[1 - par][k - preo[j]]] = 0u;
    }
    const unsigned total = pre[njobs];
    unsigned k = blockIdx.x;
    if (k >= total) return;
    int j = owner(pre, k);
    NciHalo<DIM, T> halo;
    {
      const Job<T, FS, GS>& jb = jobs[j];
      const int par = (int)((jb.step + s) & 1);
      halo.load(jb.list[par][k - pre[j]], jb.phi, jb.geo);
    }
    unsigned act = 0;
    while (k < total) {
      const Job<T, FS, GS>& jb = jobs[j];
      const int par = (int)((jb.step + s) & 1);
      const unsigned kn = k + gridDim.x;
      const int jn = kn < total ? owner(pre, kn) : j;
      const bool same = kn < total && jn == j;
      nci_tile_w<DIM, QH, T, false>(sm, jb.list[par][k - pre[j]], halo, same,
                                    same ? jb.list[par][kn - pre[j]] : 0u, jb.phi, jb.J, nullptr, nullptr,
                                    jb.geo, jb.np, act);
      if (!same) {
        // leaving this lattice: count its near-contact cells, and prefetch the next one's halo
        act = wave_sum(act);
        if ((threadIdx.x & 63) == 0 && act) atomicAdd(jb.cnt + 2, act);
        act = 0;
        if (kn < total) {
          const Job<T, FS, GS>& jn_ = jobs[jn];
          const int parn = (int)((jn_.step + s) & 1);
          halo.load(jn_.list[parn][kn - pre[jn]], jn_.phi, jn_.geo);
        }
      }
      k = kn;
      j = jn;
    }
    return;
  }
  for (int j = 0; j < njobs; ++j) {
    const Job<T, FS, GS>& jb = jobs[j];
    if (!jb.nci_on) continue;
    const int par = (int)((jb.step + s) & 1);
    nci_clear_other(jb.flags[1 - par], jb.list[1 - par], jb.cnt + (1 - par));
    const unsigned ntiles = jb.cnt[par];
    unsigned act = 0;
    nci_tiles<DIM, QH, T, false>(sm, jb.list[par], ntiles, blockIdx.x, gridDim.x, jb.phi, jb.J, nullptr, nullptr,
                                 jb.geo, jb.np, act);
    act = wave_sum(act);
    if ((threadIdx.x & 63) == 0 && act) atomicAdd(jb.cnt + 2, act);
  }
}

template <int DIM, int QH, typename T, typename FS, typename GS, bool OFF32>
__global__ __launch_bounds__(NT) void k_collide_multi(const Job<T, FS, GS>* __restrict__ jobs,
                                                      int njobs, int s) {
  const int t = swizzled_block();
  const Job<T, FS, GS>& jb = jobs[find_job(jobs, njobs, t)];
  const int lb = t - jb.blk0;
  const int par = (int)((jb.step + s) & 1);
  if (jb.nci_on && lb == 0 && threadIdx.x == 0) jb.cnt[1 - par] = 0u;
  int x, y, z;
  block_cell(lb, jb.geo, x, y, z);
  if (x >= jb.geo.nx || y >= jb.geo.ny) return;
  double acc[NPART];
  if (par == 0)
    collide_cell<DIM, QH, 0, MODE_STEP, T, FS, GS, OFF32>(jb.pl, jb.phi, jb.J, jb.flags[0], jb.geo, jb.pp,
                                                      jb.nci_on, nullptr, nullptr, x, y, z, acc);
  else
    collide_cell<DIM, QH, 1, MODE_STEP, T, FS, GS, OFF32>(jb.pl, jb.phi, jb.J, jb.flags[1], jb.geo, jb.pp,
                                                      jb.nci_on, nullptr, nullptr, x, y, z, acc);
}

// Advances the step counter of every lattice of the table (end of a replay).
template <typename T, typename FS, typename GS>
__global__ void k_advance(Job<T, FS, GS>* __restrict__ jobs, int njobs, int r) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < njobs) jobs[j].step += r;
}

}  // namespace lbm
