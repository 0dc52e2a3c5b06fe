// The other schemes of GAMER-2's fluid solver (Sec. 2.2) on padded patch
// groups: MHM or CTU (6 Riemann solves per cell), PLM or PPM on primitive or
// characteristic variables, generalized minmod / van Leer / van Albada /
// hybrid limiters, HLLC / Roe / HLLE solvers.  The default scheme (MHM, PLM
// on primitive variables, generalized minmod, HLLC) has its own fused
// kernels (mhm_fwd.hip); this path trades their on-chip staging for a
// general form: a chain of kernels, one thread per cell or face, passing
// primitive states, face states and fluxes through a caller-owned workspace
// in HBM, in the order the step defines them:
//   1. ext_prim:    cons -> prim on the padded block                 W [5][P^3]
//   2. ext_states:  face values and half step of every cell of
//                   [-1, 16]^3 (MHM: Hancock with the three axes'
//                   flux differences; CTU: the own axis' only)       S [6][5][18^3]
//   3. ext_flux1:   CTU only: first Riemann solves on every face
//                   between two cells of [-1, 16]^3                  F1 [3][5][17 18 18]
//   4. ext_correct: CTU only: transverse correction of the states
//                   with the other axes' first-solve fluxes         S in place
//   5. ext_flux:    Riemann solves at the faces of the interior      F [3][5][17 16 16]
//   6. ext_update:  U^{n+1} = U^n - dt/dx sum of flux differences (x, y, z)
// With dual energy every array carries a sixth field, the entropy per unit
// volume s = p / rho^(gamma-1), advected as a passive scalar (its specific
// value s/rho reconstructed like a primitive variable, the mass flux times
// the upwind s/rho as its Riemann flux), and the update takes E from s where
// E_th < xi E_kin and resets s from E elsewhere.
// Per-group arrays are indexed (group, field, cell); face arrays by (axis,
// field, face), the face of axis D at cell (x, y, z) being the one between
// that cell - e_D and it, laid out x fastest for every axis (face_idx,
// face1_idx), so that the threads of a wave, which take consecutive x,
// touch consecutive elements whatever the axis.

#include "ext_device.h"
#include "kernels.h"

namespace gh {

namespace {

constexpr int kS = 18;              // state cells per axis: -1 .. 16
constexpr int kS3 = kS * kS * kS;   // 5832
constexpr int kF1 = 17 * 18 * 18;   // first-solve faces per axis (transverse -1 .. 16)
constexpr int kF = 17 * 16 * 16;    // interior faces per axis

__device__ __forceinline__ int64_t cell_p(int P, int gh, int x, int y, int z) {
  return (int64_t(z + gh) * P + (y + gh)) * P + (x + gh);
}
__device__ __forceinline__ int cell_s(int x, int y, int z) { return ((z + 1) * kS + (y + 1)) * kS + (x + 1); }

// Face arrays, x fastest: interior faces of axis D (normal coordinate 0..16,
// transverse 0..15) and first-solve faces (normal 0..16, transverse -1..16).
__device__ __forceinline__ int face_idx(int D, int x, int y, int z) {
  const int nx = D == 0 ? 17 : 16, ny = D == 1 ? 17 : 16;
  return (z * ny + y) * nx + x;
}
__device__ __forceinline__ int face1_idx(int D, int x, int y, int z) {
  const int nx = D == 0 ? 17 : 18, ny = D == 1 ? 17 : 18;
  return ((z + (D == 2 ? 0 : 1)) * ny + (y + (D == 1 ? 0 : 1))) * nx + (x + (D == 0 ? 0 : 1));
}
// Cell coordinates of entry f of a box of cells, x fastest: extent m along
// axis D and t across it, starting at lo (along D) and tlo (across).
__device__ __forceinline__ void box_cell(int D, int f, int m, int lo, int t, int tlo, int& x, int& y, int& z) {
  const int nx = D == 0 ? m : t, ny = D == 1 ? m : t;
  x = f % nx + (D == 0 ? lo : tlo);
  y = (f / nx) % ny + (D == 1 ? lo : tlo);
  z = f / (nx * ny) + (D == 2 ? lo : tlo);
}

// Sum over the wave (the caller adds it to the counter once per wave).
__device__ __forceinline__ int wave_sum(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// dt from the device double if given (dt_dev), as the fused kernels do.
template <typename T>
__device__ __forceinline__ void ext_set_dt(Gas<T>& gas, const double* dt_dev, double dx) {
  if (dt_dev != nullptr) {
    const double dt = *dt_dev;
    gas.dtdx = T(dt / dx);
    gas.half_dtdx = T(0.5 * (dt / dx));
  }
}

template <typename T, int NF>
__global__ __launch_bounds__(256) void ext_prim_kernel(const T* __restrict__ Upad, T* __restrict__ W, int64_t G,
                                                       int P, Gas<T> gas) {
  const int64_t P3 = int64_t(P) * P * P;
  for (int64_t g = blockIdx.y; g < G; g += gridDim.y) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= P3) continue;
    const T* u = Upad + g * NF * P3 + i;
    T U[NF], Wc[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) U[q] = u[q * P3];
    cons_to_prim(U, gas, Wc);
    if constexpr (NF == 6) Wc[5] = Fp<T>::div(U[5], U[0]);  // entropy per unit mass
    T* w = W + g * NF * P3 + i;
#pragma unroll
    for (int q = 0; q < NF; ++q) w[q * P3] = Wc[q];
  }
}

// The stencil (cells -2..+2 along axis D; those beyond the reconstruction
// radius R repeat the centre and are not used) of the cell (x, y, z), read
// from the primitive block: the five Euler variables and, with NF = 6, the
// entropy per unit mass.
template <int D, int NF, typename T>
__device__ __forceinline__ void load_stencil(const T* __restrict__ Wg, int64_t P3, int P, int gh, int x, int y, int z,
                                             int R, T st[5][5], T ph[5]) {
#pragma unroll
  for (int j = -2; j <= 2; ++j) {
    const int o = (j < -R || j > R) ? 0 : j;
    const int xx = x + (D == 0 ? o : 0), yy = y + (D == 1 ? o : 0), zz = z + (D == 2 ? o : 0);
    const int64_t c = cell_p(P, gh, xx, yy, zz);
#pragma unroll
    for (int q = 0; q < 5; ++q) st[j + 2][q] = Wg[q * P3 + c];
    if constexpr (NF == 6) ph[j + 2] = Wg[5 * P3 + c];
  }
}

template <int D, int NF, typename T>
__device__ __forceinline__ void axis_states(const T* __restrict__ Wg, int64_t P3, int P, int gh, int x, int y, int z,
                                            const Gas<T>& gas, const ExtOpts& o, T Ut[2][NF], T Ff[2][NF]) {
  T st[5][5], ph[5], Wf[2][5];
  load_stencil<D, NF>(Wg, P3, P, gh, x, y, z, o.radius(), st, ph);
  ext_face_values<D>(st, gas, o, Wf);
  ext_cons_flux<D>(Wf[0], gas, Ut[0], Ff[0]);
  ext_cons_flux<D>(Wf[1], gas, Ut[1], Ff[1]);
  if constexpr (NF == 6) {
    // the entropy field: s = rho (s/rho) at the face, flux s u_n
    T pf[2];
    passive_face_values(ph, gas, o, pf);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      Ut[side][5] = Wf[side][0] * pf[side];
      Ff[side][5] = Ut[side][5] * Wf[side][1 + D];
    }
  }
}

template <typename T, int NF>
__global__ __launch_bounds__(256) void ext_states_kernel(const T* __restrict__ W, T* __restrict__ S, int64_t G, int P,
                                                         int gh, Gas<T> gas, const double* __restrict__ dt_dev,
                                                         double dx, ExtOpts o) {
  ext_set_dt(gas, dt_dev, dx);
  const int64_t P3 = int64_t(P) * P * P;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kS3) return;
  const int x = i % kS - 1, y = (i / kS) % kS - 1, z = i / (kS * kS) - 1;
  for (int64_t g = blockIdx.y; g < G; g += gridDim.y) {
    const T* Wg = W + g * NF * P3;
    T Ut[3][2][NF], Ff[3][2][NF];
    axis_states<0, NF>(Wg, P3, P, gh, x, y, z, gas, o, Ut[0], Ff[0]);
    axis_states<1, NF>(Wg, P3, P, gh, x, y, z, gas, o, Ut[1], Ff[1]);
    axis_states<2, NF>(Wg, P3, P, gh, x, y, z, gas, o, Ut[2], Ff[2]);
    if (o.ctu) {
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < NF; ++q) {
          const T dU = gas.half_dtdx * (Ff[d][0][q] - Ff[d][1][q]);
          Ut[d][0][q] = Ut[d][0][q] + dU;
          Ut[d][1][q] = Ut[d][1][q] + dU;
        }
    } else {
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        T s = Ff[0][0][q] - Ff[0][1][q];
        s = s + (Ff[1][0][q] - Ff[1][1][q]);
        s = s + (Ff[2][0][q] - Ff[2][1][q]);
        const T dU = gas.half_dtdx * s;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          Ut[d][0][q] = Ut[d][0][q] + dU;
          Ut[d][1][q] = Ut[d][1][q] + dU;
        }
      }
    }
    T* Sg = S + g * 6 * NF * int64_t(kS3) + i;
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int q = 0; q < NF; ++q) Sg[((d * 2 + s) * NF + q) * int64_t(kS3)] = Ut[d][s][q];
  }
}

template <int D, int NF, typename T>
__device__ __forceinline__ void load_state(const T* __restrict__ Sg, int x, int y, int z, int side, T U[NF]) {
  const int c = cell_s(x, y, z);
#pragma unroll
  for (int q = 0; q < NF; ++q) U[q] = Sg[((D * 2 + side) * NF + q) * int64_t(kS3) + c];
}

// Riemann solve of the face of axis D at cell (x, y, z), between cell - e_D
// (its high state) and the cell (its low state); returns the unphysical flag.
template <int D, int NF, typename T>
__device__ __forceinline__ int solve_face(const T* __restrict__ Sg, int x, int y, int z, const Gas<T>& gas,
                                          const ExtOpts& o, T F[NF]) {
  T L[NF], R[NF];
  load_state<D, NF>(Sg, x - (D == 0), y - (D == 1), z - (D == 2), 1, L);
  load_state<D, NF>(Sg, x, y, z, 0, R);
  return riemann_nf<D, NF>(L, R, gas, o, F) ? 1 : 0;
}

template <typename T, int NF>
__global__ __launch_bounds__(256) void ext_flux1_kernel(const T* __restrict__ S, T* __restrict__ F1, int64_t G,
                                                        Gas<T> gas, ExtOpts o) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * kF1) return;
  const int d = i / kF1, f = i % kF1;  // f = face1_idx(d, x, y, z)
  int x, y, z;
  box_cell(d, f, 17, 0, 18, -1, x, y, z);
  for (int64_t g = blockIdx.y; g < G; g += gridDim.y) {
    const T* Sg = S + g * 6 * NF * int64_t(kS3);
    T F[NF];
    if (d == 0) solve_face<0, NF>(Sg, x, y, z, gas, o, F);
    else if (d == 1) solve_face<1, NF>(Sg, x, y, z, gas, o, F);
    else solve_face<2, NF>(Sg, x, y, z, gas, o, F);
    T* out = F1 + g * 3 * NF * int64_t(kF1) + d * NF * int64_t(kF1) + f;
#pragma unroll
    for (int q = 0; q < NF; ++q) out[q * int64_t(kF1)] = F[q];
  }
}

// First-solve flux of the face of axis E at cell coordinates (x, y, z) (the
// face between (x, y, z) - e_E and (x, y, z)).
template <int NF, typename T>
__device__ __forceinline__ const T* f1_at(const T* __restrict__ F1g, int E, int x, int y, int z) {
  return F1g + E * NF * int64_t(kF1) + face1_idx(E, x, y, z);
}

template <typename T, int NF>
__global__ __launch_bounds__(256) void ext_correct_kernel(T* __restrict__ S, const T* __restrict__ F1, int64_t G,
                                                          Gas<T> gas, const double* __restrict__ dt_dev, double dx) {
  ext_set_dt(gas, dt_dev, dx);
  constexpr int kPer = 18 * 16 * 16;  // normal -1..16, transverse 0..15
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * kPer) return;
  const int d = i / kPer, f = i % kPer;
  int x, y, z;
  box_cell(d, f, 18, -1, 16, 0, x, y, z);
  for (int64_t g = blockIdx.y; g < G; g += gridDim.y) {
    const T* F1g = F1 + g * 3 * NF * int64_t(kF1);
    T corr[NF];
    bool first = true;
    for (int e = 0; e < 3; ++e) {
      if (e == d) continue;
      const T* Fp = f1_at<NF>(F1g, e, x + (e == 0), y + (e == 1), z + (e == 2));
      const T* Fm = f1_at<NF>(F1g, e, x, y, z);
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        const T dq = Fp[q * int64_t(kF1)] - Fm[q * int64_t(kF1)];
        corr[q] = first ? dq : corr[q] + dq;
      }
      first = false;
    }
    T* Sg = S + g * 6 * NF * int64_t(kS3) + cell_s(x, y, z);
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        T& v = Sg[((d * 2 + s) * NF + q) * int64_t(kS3)];
        v = v - gas.half_dtdx * corr[q];
      }
  }
}

template <typename T, int NF>
__global__ __launch_bounds__(256) void ext_flux_kernel(const T* __restrict__ S, T* __restrict__ F, int64_t G,
                                                       Gas<T> gas, ExtOpts o, int* __restrict__ n_bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < 3 * kF;
  const int d = live ? i / kF : 0, f = live ? i % kF : 0;  // f = face_idx(d, x, y, z)
  int x, y, z;
  box_cell(d, f, 17, 0, 16, 0, x, y, z);
  int bad = 0;
  for (int64_t g = blockIdx.y; g < G; g += gridDim.y) {
    if (!live) continue;
    const T* Sg = S + g * 6 * NF * int64_t(kS3);
    T Fv[NF];
    if (d == 0) bad += solve_face<0, NF>(Sg, x, y, z, gas, o, Fv);
    else if (d == 1) bad += solve_face<1, NF>(Sg, x, y, z, gas, o, Fv);
    else bad += solve_face<2, NF>(Sg, x, y, z, gas, o, Fv);
    T* out = F + g * 3 * NF * int64_t(kF) + d * NF * int64_t(kF) + f;
#pragma unroll
    for (int q = 0; q < NF; ++q) out[q * int64_t(kF)] = Fv[q];
  }
  bad = wave_sum(bad);
  if (n_bad != nullptr && (threadIdx.x & 63) == 0 && bad != 0) atomicAdd(n_bad, bad);
}

// x^e for the dual-energy relation p = s rho^(gamma-1)
__device__ __forceinline__ double pow_(double x, double e) { return ::pow(x, e); }
__device__ __forceinline__ float pow_(float x, float e) { return ::powf(x, e); }

template <typename T, int NF>
__global__ __launch_bounds__(256) void ext_update_kernel(const T* __restrict__ Upad, const T* __restrict__ F,
                                                         T* __restrict__ Uout, int64_t G, int P, int gh, Gas<T> gas,
                                                         const double* __restrict__ dt_dev, double dx, T xi,
                                                         int* __restrict__ n_bad) {
  ext_set_dt(gas, dt_dev, dx);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // < 4096 (grid sized exactly)
  const int x = i & 15, y = (i >> 4) & 15, z = i >> 8;
  const int64_t P3 = int64_t(P) * P * P;
  int bad = 0;
  for (int64_t g = blockIdx.y; g < G; g += gridDim.y) {
    const T* Fg = F + g * 3 * NF * int64_t(kF);
    // the low face of this cell along each axis; the high one is the next
    // entry along that axis (strides 1, 16, 256)
    const int fx = face_idx(0, x, y, z), fy = face_idx(1, x, y, z), fz = face_idx(2, x, y, z);
    T Un[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      const T* Fx = Fg + (0 * NF + q) * int64_t(kF);
      const T* Fy = Fg + (1 * NF + q) * int64_t(kF);
      const T* Fz = Fg + (2 * NF + q) * int64_t(kF);
      T acc = Fx[fx + 1] - Fx[fx];
      acc = acc + (Fy[fy + 16] - Fy[fy]);
      acc = acc + (Fz[fz + 256] - Fz[fz]);
      Un[q] = Upad[g * NF * P3 + q * P3 + cell_p(P, gh, x, y, z)] - gas.dtdx * acc;
    }
    if constexpr (NF == 6) {
      // dual energy: E from the entropy where E_th < xi E_kin, else the
      // entropy from E
      const T ekin = T(0.5) * (Un[1] * Un[1] + Un[2] * Un[2] + Un[3] * Un[3]) * Fp<T>::rcp(Un[0]);
      const T eth = Un[4] - ekin;
      const T rg = pow_(Un[0], gas.gm1);
      if (eth < xi * ekin) Un[4] = Un[5] * rg * gas.inv_gm1 + ekin;
      else Un[5] = Fp<T>::div(gas.gm1 * eth, rg);
    }
#pragma unroll
    for (int q = 0; q < NF; ++q) Uout[g * NF * 4096 + q * 4096 + i] = Un[q];
    bad += unphysical(Un, gas) ? 1 : 0;
  }
  bad = wave_sum(bad);
  if (n_bad != nullptr && (threadIdx.x & 63) == 0 && bad != 0) atomicAdd(n_bad, bad);
}

// Fluxes of the faces on the patch boundaries of every group, [G][9][5][256]:
// plane p = 3 axis + k holds the axis' faces at normal coordinate 8 k, entry
// [p][q][b * 16 + a] (a, b transverse in cyclic order) -- the coarse side of
// a coarse-fine interface (k = 0, 1, 2) and the fine side (k = 0, 2).
template <typename T>
__global__ __launch_bounds__(256) void ext_face_flux_kernel(const T* __restrict__ F, T* __restrict__ out, int64_t G) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // < 9 * 256
  const int p = i >> 8, ab = i & 255, d = p / 3, k = p % 3;
  const int a = ab & 15, b = ab >> 4;
  // the face at normal coordinate 8 k, transverse (a, b) in cyclic order
  const int f = d == 0 ? face_idx(0, 8 * k, a, b) : d == 1 ? face_idx(1, b, 8 * k, a) : face_idx(2, a, b, 8 * k);
  for (int64_t g = blockIdx.y; g < G; g += gridDim.y) {
#pragma unroll
    for (int q = 0; q < 5; ++q)
      out[((g * 9 + p) * 5 + q) * 256 + ab] = F[g * 15 * int64_t(kF) + (d * 5 + q) * int64_t(kF) + f];
  }
}

unsigned grid_y(int64_t G) { return unsigned(G < 65535 ? G : 65535); }

}  // namespace

int64_t ext_workspace_elems(int64_t n_groups, int ghost, const ExtOpts& o) {
  const int64_t P = 16 + 2 * ghost;
  const int64_t nf = o.de ? 6 : 5;
  auto up = [](int64_t v) { return (v + 63) / 64 * 64; };
  return n_groups * (up(nf * P * P * P) + up(6 * nf * int64_t(kS3)) + (o.ctu ? up(3 * nf * int64_t(kF1)) : 0) +
                     up(3 * nf * int64_t(kF)));
}

template <typename T, int NF>
hipError_t ext_step_nf(const T* U_pad, T* U_out, int64_t G, int ghost, const Gas<T>& gas, const double* dt_dev,
                       double dx, const ExtOpts& o, int* n_bad, T* work, T* face_flux, hipStream_t stream) {
  const int P = 16 + 2 * ghost;
  const int64_t P3 = int64_t(P) * P * P;
  auto up = [](int64_t v) { return (v + 63) / 64 * 64; };
  T* W = work;
  T* S = W + G * up(NF * P3);
  T* F1 = S + G * up(6 * NF * int64_t(kS3));
  T* F = F1 + (o.ctu ? G * up(3 * NF * int64_t(kF1)) : 0);
  // per-group strides of the arrays are the unpadded sizes; the padded sizes
  // above only separate the arrays
  const unsigned gy = grid_y(G);
  hipLaunchKernelGGL((ext_prim_kernel<T, NF>), dim3(unsigned((P3 + 255) / 256), gy), dim3(256), 0, stream, U_pad, W, G,
                     P, gas);
  hipLaunchKernelGGL((ext_states_kernel<T, NF>), dim3(unsigned((kS3 + 255) / 256), gy), dim3(256), 0, stream, W, S, G,
                     P, ghost, gas, dt_dev, dx, o);
  if (o.ctu) {
    hipLaunchKernelGGL((ext_flux1_kernel<T, NF>), dim3(unsigned((3 * kF1 + 255) / 256), gy), dim3(256), 0, stream, S,
                       F1, G, gas, o);
    hipLaunchKernelGGL((ext_correct_kernel<T, NF>), dim3(unsigned((3 * 18 * 256 + 255) / 256), gy), dim3(256), 0,
                       stream, S, F1, G, gas, dt_dev, dx);
  }
  hipLaunchKernelGGL((ext_flux_kernel<T, NF>), dim3(unsigned((3 * kF + 255) / 256), gy), dim3(256), 0, stream, S, F,
                     G, gas, o, n_bad);
  hipLaunchKernelGGL((ext_update_kernel<T, NF>), dim3(16u, gy), dim3(256), 0, stream, U_pad, F, U_out, G, P, ghost,
                     gas, dt_dev, dx, T(o.xi), n_bad);
  if (NF == 5 && face_flux != nullptr)
    hipLaunchKernelGGL(ext_face_flux_kernel<T>, dim3(9u, gy), dim3(256), 0, stream, F, face_flux, G);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ext_step(const T* U_pad, T* U_out, int64_t G, int ghost, const Gas<T>& gas, const double* dt_dev,
                           double dx, const ExtOpts& o, int* n_bad, T* work, T* face_flux, hipStream_t stream) {
  if (G == 0) return hipSuccess;
  if (o.de) return ext_step_nf<T, 6>(U_pad, U_out, G, ghost, gas, dt_dev, dx, o, n_bad, work, nullptr, stream);
  return ext_step_nf<T, 5>(U_pad, U_out, G, ghost, gas, dt_dev, dx, o, n_bad, work, face_flux, stream);
}

template hipError_t launch_ext_step<double>(const double*, double*, int64_t, int, const Gas<double>&, const double*,
                                            double, const ExtOpts&, int*, double*, double*, hipStream_t);
template hipError_t launch_ext_step<float>(const float*, float*, int64_t, int, const Gas<float>&, const double*, double,
                                           const ExtOpts&, int*, float*, float*, hipStream_t);

}  // namespace gh
