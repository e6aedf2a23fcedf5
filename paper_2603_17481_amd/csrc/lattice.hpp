// lattice.hpp -- velocity sets of the coupled step (device side).
//
// Hydrodynamics: D2Q9 / D3Q19 / D3Q27 with cs^2 = 1/3.  Phase field: D2Q9 (cs^2 = 1/3)
// in 2D and D3Q7 (w0 = 1/4, axis 1/8, cs^2 = 1/4) in 3D.  Velocities are ordered
// rest first, then opposite pairs (2k-1, 2k), so that the collision can evaluate
// the even and odd parts of each pair once (c_{2k} = -c_{2k-1}).
#pragma once

#include <type_traits>

namespace lbm {

// Each lattice also carries FP32 weights wf[] whose exact real sum is 1 (the
// nearest floats, with one weight moved by one ulp where needed).  With the
// plain rounded weights the D2Q9 sum is 1 + 7.45e-9, which makes every FP32
// step scale the phase-field mass by (1 + 7.45e-9 / tau_phi).

// Hydrodynamic lattices by velocity count: 9 (D2Q9), 19 (D3Q19), 27 (D3Q27).
template <int QH>
struct HydroQ;

template <>
struct HydroQ<9> {
  static constexpr int D = 2;
  static constexpr int Q = 9;
  static constexpr int cx[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
  static constexpr int cy[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
  static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                  1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  static constexpr float wf[9] = {0x1.c71c72p-2f, 0x1.c71c72p-4f, 0x1.c71c72p-4f, 0x1.c71c72p-4f,
                                  0x1.c71c72p-4f, 0x1.c71c70p-6f, 0x1.c71c70p-6f, 0x1.c71c70p-6f,
                                  0x1.c71c70p-6f};
};

template <>
struct HydroQ<19> {
  static constexpr int D = 3;
  static constexpr int Q = 19;
  static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                   1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  static constexpr float wf[19] = {0x1.555558p-2f, 0x1.c71c70p-5f, 0x1.c71c70p-5f, 0x1.c71c70p-5f,
                                   0x1.c71c70p-5f, 0x1.c71c70p-5f, 0x1.c71c70p-5f, 0x1.c71c70p-6f,
                                   0x1.c71c70p-6f, 0x1.c71c70p-6f, 0x1.c71c70p-6f, 0x1.c71c70p-6f,
                                   0x1.c71c70p-6f, 0x1.c71c70p-6f, 0x1.c71c70p-6f, 0x1.c71c70p-6f,
                                   0x1.c71c70p-6f, 0x1.c71c70p-6f, 0x1.c71c70p-6f};
};

// D3Q27, the tensor product of the D1Q3 weights (2/3, 1/6, 1/6): rest 8/27,
// axis 2/27, face diagonal 1/54, body diagonal 1/216.  FP32: the rest weight is
// one ulp below its nearest float and the face-diagonal ones one ulp above.
template <>
struct HydroQ<27> {
  static constexpr int D = 3;
  static constexpr int Q = 27;
  static constexpr int cx[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                                 1, -1, 1, -1, 1, -1, -1, 1};
  static constexpr int cy[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                                 1, -1, 1, -1, -1, 1, 1, -1};
  static constexpr int cz[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                                 1, -1, -1, 1, 1, -1, 1, -1};
  static constexpr double w[27] = {8.0 / 27,  2.0 / 27,  2.0 / 27,  2.0 / 27,  2.0 / 27,  2.0 / 27,
                                   2.0 / 27,  1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,
                                   1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,
                                   1.0 / 54,  1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216,
                                   1.0 / 216, 1.0 / 216, 1.0 / 216};
  static constexpr float wf[27] = {
      0x1.2f684ap-2f, 0x1.2f684cp-4f, 0x1.2f684cp-4f, 0x1.2f684cp-4f, 0x1.2f684cp-4f, 0x1.2f684cp-4f,
      0x1.2f684cp-4f, 0x1.2f684ep-6f, 0x1.2f684ep-6f, 0x1.2f684ep-6f, 0x1.2f684ep-6f, 0x1.2f684ep-6f,
      0x1.2f684ep-6f, 0x1.2f684ep-6f, 0x1.2f684ep-6f, 0x1.2f684ep-6f, 0x1.2f684ep-6f, 0x1.2f684ep-6f,
      0x1.2f684ep-6f, 0x1.2f684cp-8f, 0x1.2f684cp-8f, 0x1.2f684cp-8f, 0x1.2f684cp-8f, 0x1.2f684cp-8f,
      0x1.2f684cp-8f, 0x1.2f684cp-8f, 0x1.2f684cp-8f};
};

// The default hydrodynamic lattice of each dimension.
template <int DIM>
using Hydro = HydroQ<DIM == 2 ? 9 : 19>;

template <int DIM>
struct Phase;

template <>
struct Phase<2> {
  static constexpr int Q = 9;
  static constexpr double cs2 = 1.0 / 3.0;
  static constexpr double inv_cs2 = 3.0;
  static constexpr int cx[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
  static constexpr int cy[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
  static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                  1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  static constexpr float wf[9] = {0x1.c71c72p-2f, 0x1.c71c72p-4f, 0x1.c71c72p-4f, 0x1.c71c72p-4f,
                                  0x1.c71c72p-4f, 0x1.c71c70p-6f, 0x1.c71c70p-6f, 0x1.c71c70p-6f,
                                  0x1.c71c70p-6f};
};

template <>
struct Phase<3> {
  static constexpr int Q = 7;
  static constexpr double cs2 = 0.25;
  static constexpr double inv_cs2 = 4.0;
  static constexpr int cx[7] = {0, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[7] = {0, 0, 0, 1, -1, 0, 0};
  static constexpr int cz[7] = {0, 0, 0, 0, 0, 1, -1};
  static constexpr double w[7] = {0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125};
  static constexpr float wf[7] = {0.25f, 0.125f, 0.125f, 0.125f, 0.125f, 0.125f, 0.125f};
};

// Weight i of lattice L in the arithmetic type T.
template <typename L, typename T>
__host__ __device__ constexpr T wt(int i) {
  if constexpr (std::is_same<T, float>::value) return L::wf[i];
  else return (T)L::w[i];
}

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Rank of the odd direction i among the odd directions of lattice L with
// c_x != 0 (the pairs whose streaming shifts along x); xpair<L>(L::Q) counts them.
template <typename L>
__host__ __device__ constexpr int xpair(int i) {
  int r = 0;
  for (int j = 1; j < i; j += 2) r += L::cx[j] != 0 ? 1 : 0;
  return r;
}

}  // namespace lbm
