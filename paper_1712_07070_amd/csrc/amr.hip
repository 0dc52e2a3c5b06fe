// Coarse-fine coupling of AMR levels (GAMER-2 Sec. 2.1: patches of 8^3
// cells, refinement ratio 2, the 8 children of a coarse patch form one fine
// patch group; Sec. 2.2: restriction and flux fix-up after a coarse level is
// synchronized with its children; Sec. 3.2: ghost zones of fine groups filled
// from siblings or by interpolation from the coarse level).
//
// A level is a set of 16^3 groups at positions of its group lattice (level l:
// n_0 2^l per axis over the domain), with a dense lattice map (group index or
// -1) on the device for neighbour lookups.  One thread per cell or face:
//   amr_fill        padded groups [G][5][P^3] of a level: a ghost cell is
//                   copied from the sibling group that holds it, else
//                   interpolated from the coarse level, linearly in time
//                   between the coarse step's input and output ((1-a) U_old
//                   + a U_new) and conservatively linear in space (coarse
//                   value + minmod-limited slopes of the conserved variables
//                   times the child's offsets of +-1/4 cell, summed x, y, z);
//   amr_accumulate  flux registers R[G_f][6][5][8][8] on the sides of fine
//                   groups with no sibling: R += w (1/4) (sum of the 2x2 fine
//                   faces over a coarse face), w = dt_f / dt_c per substep;
//   amr_restrict    coarse cells covered by a fine group: mean of the 8
//                   children (summed pairwise: x, then y, then z);
//   amr_fixup       uncovered coarse cells next to the fine level: the coarse
//                   flux F_c of the shared face is replaced by the register
//                   R, U += dt_c/dx_c (R - F_c) on a low face, -= on a high
//                   face, sides in the order x-, x+, y-, y+, z-, z+ (one
//                   thread per coarse cell: deterministic).

#include "kernels.h"

namespace gh {

namespace {

struct LevelDev {
  const int* pos;  // [G][3]
  const int* map;  // [n2][n1][n0]
  int64_t G;
  int n[3];
  __device__ __forceinline__ int at(int gx, int gy, int gz) const {
    return map[(int64_t(gz) * n[1] + gy) * n[0] + gx];
  }
};

__device__ __forceinline__ int wrap(int i, int N, int lo, int hi) {
  if (i < 0) return lo == 0 ? i + N : 0;
  if (i >= N) return hi == 0 ? i - N : N - 1;
  return i;
}

template <typename T>
__device__ __forceinline__ T minmod2(T a, T b) {
  if (!(a * b > T(0))) return T(0);
  return fabs_(a) < fabs_(b) ? a : b;
}

struct Bc6 {
  int v[6];
};

template <typename T>
__global__ __launch_bounds__(256) void amr_fill_kernel(const T* __restrict__ Uf, LevelDev F, const T* __restrict__ Cold,
                                                       const T* __restrict__ Cnew, LevelDev C, T a, Bc6 bc, int ghost,
                                                       T* __restrict__ pad) {
  const int P = 16 + 2 * ghost;
  const int P3 = P * P * P;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P3) return;
  const int x = i % P, y = (i / P) % P, z = i / (P * P);
  const int N0 = 16 * F.n[0], N1 = 16 * F.n[1], N2 = 16 * F.n[2];
  for (int64_t g = blockIdx.y; g < F.G; g += gridDim.y) {
    const int X = wrap(16 * F.pos[3 * g] + x - ghost, N0, bc.v[0], bc.v[1]);
    const int Y = wrap(16 * F.pos[3 * g + 1] + y - ghost, N1, bc.v[2], bc.v[3]);
    const int Z = wrap(16 * F.pos[3 * g + 2] + z - ghost, N2, bc.v[4], bc.v[5]);
    const int gs = F.at(X >> 4, Y >> 4, Z >> 4);
    T v[5];
    if (gs >= 0) {
      const T* s = Uf + int64_t(gs) * 5 * 4096 + ((Z & 15) * 16 + (Y & 15)) * 16 + (X & 15);
#pragma unroll
      for (int q = 0; q < 5; ++q) v[q] = s[q * 4096];
    } else {
      const int M0 = 16 * C.n[0], M1 = 16 * C.n[1], M2 = 16 * C.n[2];
      const int c0 = X >> 1, c1 = Y >> 1, c2 = Z >> 1;
      const T off0 = (X & 1) ? T(0.25) : T(-0.25), off1 = (Y & 1) ? T(0.25) : T(-0.25),
              off2 = (Z & 1) ? T(0.25) : T(-0.25);
      auto at = [&](int dx, int dy, int dz, T u[5]) {
        const int xx = wrap(c0 + dx, M0, bc.v[0], bc.v[1]);
        const int yy = wrap(c1 + dy, M1, bc.v[2], bc.v[3]);
        const int zz = wrap(c2 + dz, M2, bc.v[4], bc.v[5]);
        const int64_t o = int64_t(C.at(xx >> 4, yy >> 4, zz >> 4)) * 5 * 4096 +
                          ((zz & 15) * 16 + (yy & 15)) * 16 + (xx & 15);
#pragma unroll
        for (int q = 0; q < 5; ++q) u[q] = (T(1) - a) * Cold[o + q * 4096] + a * Cnew[o + q * 4096];
      };
      T U0[5], Um[5], Up[5], s0[5], s1[5], s2[5];
      at(0, 0, 0, U0);
      at(-1, 0, 0, Um);
      at(1, 0, 0, Up);
#pragma unroll
      for (int q = 0; q < 5; ++q) s0[q] = minmod2(U0[q] - Um[q], Up[q] - U0[q]);
      at(0, -1, 0, Um);
      at(0, 1, 0, Up);
#pragma unroll
      for (int q = 0; q < 5; ++q) s1[q] = minmod2(U0[q] - Um[q], Up[q] - U0[q]);
      at(0, 0, -1, Um);
      at(0, 0, 1, Up);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        s2[q] = minmod2(U0[q] - Um[q], Up[q] - U0[q]);
        v[q] = ((U0[q] + s0[q] * off0) + s1[q] * off1) + s2[q] * off2;
      }
    }
    T* d = pad + g * 5 * int64_t(P3) + i;
#pragma unroll
    for (int q = 0; q < 5; ++q) d[q * int64_t(P3)] = v[q];
  }
}

// Side s = 2 axis + high of fine group g: the group across it is missing (a
// side on an outflow domain face has no interface).
__device__ __forceinline__ bool interface_side(const LevelDev& F, int64_t g, int s, const Bc6& bc) {
  const int d = s >> 1, hi = s & 1;
  int p[3] = {F.pos[3 * g], F.pos[3 * g + 1], F.pos[3 * g + 2]};
  p[d] += hi ? 1 : -1;
  if (p[d] < 0 || p[d] >= F.n[d]) {
    if (bc.v[2 * d + hi] != 0) return false;
    p[d] = (p[d] + F.n[d]) % F.n[d];
  }
  return F.at(p[0], p[1], p[2]) < 0;
}

template <typename T>
__global__ __launch_bounds__(256) void amr_accumulate_kernel(LevelDev F, const T* __restrict__ face_flux, T w, Bc6 bc,
                                                             T* __restrict__ R) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 6 * 5 * 64) return;
  const int s = t / 320, q = (t / 64) % 5, j = (t / 8) & 7, i = t & 7;
  const int d = s >> 1, k = (s & 1) ? 2 : 0;
  for (int64_t g = blockIdx.y; g < F.G; g += gridDim.y) {
    if (!interface_side(F, g, s, bc)) continue;
    const T* f = face_flux + ((g * 9 + d * 3 + k) * 5 + q) * 256;
    const T sum = (f[(2 * j) * 16 + 2 * i] + f[(2 * j) * 16 + 2 * i + 1]) +
                  (f[(2 * j + 1) * 16 + 2 * i] + f[(2 * j + 1) * 16 + 2 * i + 1]);
    T& r = R[(g * 6 + s) * 320 + q * 64 + j * 8 + i];
    r = r + w * (T(0.25) * sum);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void amr_restrict_kernel(const T* __restrict__ Uf, LevelDev F, T* __restrict__ Uc,
                                                           LevelDev C) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;  // < 512: a coarse cell of the parent patch
  const int x = t & 7, y = (t >> 3) & 7, z = t >> 6;
  for (int64_t g = blockIdx.y; g < F.G; g += gridDim.y) {
    const int px = F.pos[3 * g], py = F.pos[3 * g + 1], pz = F.pos[3 * g + 2];
    const int64_t gc = C.at(px >> 1, py >> 1, pz >> 1);
    const int cx = (px & 1) * 8 + x, cy = (py & 1) * 8 + y, cz = (pz & 1) * 8 + z;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const T* f = Uf + (g * 5 + q) * 4096 + ((2 * z) * 16 + 2 * y) * 16 + 2 * x;
      // pairwise: x pairs, then y, then z (a uniform state restricts exactly)
      const T s0 = (f[0] + f[1]) + (f[16] + f[17]);
      const T s1 = (f[256] + f[257]) + (f[272] + f[273]);
      Uc[(gc * 5 + q) * 4096 + (cz * 16 + cy) * 16 + cx] = T(0.125) * (s0 + s1);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void amr_fixup_kernel(T* __restrict__ Uc, LevelDev C, LevelDev F,
                                                        const T* __restrict__ cflux, const T* __restrict__ R, T dtdx,
                                                        Bc6 bc) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= C.G * 4096) return;
  const int64_t g = t >> 12;
  const int c = int(t & 4095);
  const int xyz[3] = {16 * C.pos[3 * g] + (c & 15), 16 * C.pos[3 * g + 1] + ((c >> 4) & 15),
                      16 * C.pos[3 * g + 2] + (c >> 8)};
  if (F.at(xyz[0] >> 3, xyz[1] >> 3, xyz[2] >> 3) >= 0) return;  // covered: restricted instead
  const int N[3] = {16 * C.n[0], 16 * C.n[1], 16 * C.n[2]};
  for (int s = 0; s < 6; ++s) {
    const int d = s >> 1, hi = s & 1;
    int nb[3] = {xyz[0], xyz[1], xyz[2]};
    nb[d] += hi ? 1 : -1;
    if (nb[d] < 0 || nb[d] >= N[d]) {
      if (bc.v[2 * d + hi] != 0) continue;
      nb[d] = (nb[d] + N[d]) % N[d];
    }
    const int gf = F.at(nb[0] >> 3, nb[1] >> 3, nb[2] >> 3);
    if (gf < 0) continue;
    const int k = ((xyz[d] & 15) + hi) >> 3;
    const int a = xyz[(d + 1) % 3] & 15, b = xyz[(d + 2) % 3] & 15;
    const T* Fc = cflux + (g * 9 + d * 3 + k) * 5 * 256 + b * 16 + a;
    const int fs = 2 * d + (hi ? 0 : 1);
    const int i = xyz[(d + 1) % 3] & 7, j = xyz[(d + 2) % 3] & 7;
    const T* r = R + (int64_t(gf) * 6 + fs) * 320 + j * 8 + i;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const T corr = dtdx * (r[q * 64] - Fc[q * 256]);
      T& u = Uc[(g * 5 + q) * 4096 + c];
      u = hi ? u - corr : u + corr;
    }
  }
}

LevelDev to_dev(const AmrLevelArgs& L) {
  LevelDev d;
  d.pos = L.pos;
  d.map = L.map;
  d.G = L.G;
  for (int i = 0; i < 3; ++i) d.n[i] = L.n[i];
  return d;
}

Bc6 to_bc(const int bc[6]) {
  Bc6 b;
  for (int i = 0; i < 6; ++i) b.v[i] = bc[i];
  return b;
}

unsigned gy(int64_t G) { return unsigned(G < 65535 ? G : 65535); }

}  // namespace

template <typename T>
hipError_t launch_amr_fill(const T* Uf, const AmrLevelArgs& F, const T* Cold, const T* Cnew, const AmrLevelArgs& C,
                           double a, const int bc[6], int ghost, T* pad, hipStream_t stream) {
  if (F.G == 0) return hipSuccess;
  const int P = 16 + 2 * ghost;
  hipLaunchKernelGGL(amr_fill_kernel<T>, dim3(unsigned((P * P * P + 255) / 256), gy(F.G)), dim3(256), 0, stream, Uf,
                     to_dev(F), Cold, Cnew, to_dev(C), T(a), to_bc(bc), ghost, pad);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_amr_accumulate(const AmrLevelArgs& F, const T* face_flux, double w, const int bc[6], T* R,
                                 hipStream_t stream) {
  if (F.G == 0) return hipSuccess;
  hipLaunchKernelGGL(amr_accumulate_kernel<T>, dim3(8u, gy(F.G)), dim3(256), 0, stream, to_dev(F), face_flux, T(w),
                     to_bc(bc), R);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_amr_restrict(const T* Uf, const AmrLevelArgs& F, T* Uc, const AmrLevelArgs& C, hipStream_t stream) {
  if (F.G == 0) return hipSuccess;
  hipLaunchKernelGGL(amr_restrict_kernel<T>, dim3(2u, gy(F.G)), dim3(256), 0, stream, Uf, to_dev(F), Uc, to_dev(C));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_amr_fixup(T* Uc, const AmrLevelArgs& C, const AmrLevelArgs& F, const T* cflux, const T* R,
                            double dtdx, const int bc[6], hipStream_t stream) {
  if (C.G == 0) return hipSuccess;
  const int64_t n = C.G * 4096;
  hipLaunchKernelGGL(amr_fixup_kernel<T>, dim3(unsigned((n + 255) / 256)), dim3(256), 0, stream, Uc, to_dev(C),
                     to_dev(F), cflux, R, T(dtdx), to_bc(bc));
  return hipGetLastError();
}

#define GH_AMR_INST(T)                                                                                             \
  template hipError_t launch_amr_fill<T>(const T*, const AmrLevelArgs&, const T*, const T*, const AmrLevelArgs&,    \
                                         double, const int*, int, T*, hipStream_t);                                 \
  template hipError_t launch_amr_accumulate<T>(const AmrLevelArgs&, const T*, double, const int*, T*, hipStream_t); \
  template hipError_t launch_amr_restrict<T>(const T*, const AmrLevelArgs&, T*, const AmrLevelArgs&, hipStream_t);  \
  template hipError_t launch_amr_fixup<T>(T*, const AmrLevelArgs&, const AmrLevelArgs&, const T*, const T*, double, \
                                          const int*, hipStream_t);
GH_AMR_INST(double)
GH_AMR_INST(float)
#undef GH_AMR_INST

}  // namespace gh
