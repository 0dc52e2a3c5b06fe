// Ghost-zone fill (Sec. 3.4, boundary conditions of Sec. 2.2) and the
// per-patch CFL time-step (Sec. 2.6 Eq. 2) of padded patch groups.

#include "mhm_group.h"

namespace gh {

namespace {

// ------------------------------------------------------------ ghost fill --
// One thread per padded cell: the source index along each axis is mapped
// independently (wrap for periodic faces, clamp for outflow faces).
__device__ __forceinline__ int bc_map(int i, int n, int lo, int hi) {
  if (i < 0) return lo == 0 ? i + n : 0;
  if (i >= n) return hi == 0 ? i - n : n - 1;
  return i;
}

struct BC6 {
  int b[6];
};

template <typename T>
__global__ __launch_bounds__(256) void fill_ghosts_kernel(const T* __restrict__ level, T* __restrict__ U_pad,
                                                          int ngx, int ngy, int ngz, int gh, BC6 bc) {
  // one workgroup per padded plane: (group g, field f, padded z); the plane's
  // P x P cells are written contiguously
  const int P = 16 + 2 * gh;
  const unsigned int blk = blockIdx.x;
  const int z = int(blk % unsigned(P));
  const int f = int((blk / unsigned(P)) % 5u);
  const unsigned int g = blk / unsigned(5 * P);
  const int gx = int(g % unsigned(ngx)), gy = int((g / unsigned(ngx)) % unsigned(ngy));
  const int gz = int(g / (unsigned(ngx) * unsigned(ngy)));
  const int Nx = ngx * 16, Ny = ngy * 16, Nz = ngz * 16;
  const int Z = bc_map(gz * 16 + z - gh, Nz, bc.b[4], bc.b[5]);
  T* dst = U_pad + (int64_t(blk / unsigned(P)) * P + z) * P * P;  // ((g*5 + f)*P + z)*P*P
  for (int i = threadIdx.x; i < P * P; i += blockDim.x) {
    const int x = i % P, y = i / P;
    const int X = bc_map(gx * 16 + x - gh, Nx, bc.b[0], bc.b[1]);
    const int Y = bc_map(gy * 16 + y - gh, Ny, bc.b[2], bc.b[3]);
    const int64_t sg = (int64_t(Z >> 4) * ngy + (Y >> 4)) * ngx + (X >> 4);
    dst[i] = level[((sg * 5 + f) * 16 + (Z & 15)) * 256 + (Y & 15) * 16 + (X & 15)];
  }
}

// ------------------------------------------------------------------ CFL ---
// One workgroup of 256 threads per group: thread (x, y) walks z; the maximum
// signal speed |u|+|v|+|w|+3c is reduced per 8^3 patch through LDS.
// cfl_signal_speed evaluates each cell in double for both state types with
// IEEE-rounded, uncontracted operations.  The maximum keeps the running value unless a speed is strictly larger (a
// NaN speed from an unphysical cell never wins; the step counts such cells).
template <typename T>
__global__ __launch_bounds__(256) void cfl_dt_kernel(const T* __restrict__ U_pad, int gh, double dx, double gamma,
                                                     double c_cfl, double* __restrict__ dt_patch,
                                                     unsigned long long* __restrict__ dt_min) {
  __shared__ double red[2][4][64];  // [pz][py*2 + px][cell column within the patch]
  const int P = 16 + 2 * gh;
  const int64_t P3 = int64_t(P) * P * P;
  const T* __restrict__ Ug = U_pad + int64_t(blockIdx.x) * 5 * P3;
  const int x = threadIdx.x & 15, y = threadIdx.x >> 4;
  double smax[2] = {0.0, 0.0};
  for (int z = 0; z < 16; ++z) {
    const int64_t o = (int64_t(z + gh) * P + (y + gh)) * P + (x + gh);
    const double s = cfl_signal_speed(double(Ug[o]), double(Ug[P3 + o]), double(Ug[2 * P3 + o]),
                                      double(Ug[3 * P3 + o]), double(Ug[4 * P3 + o]), gamma);
    if (s > smax[z >> 3]) smax[z >> 3] = s;
  }
  const int pxy = (y >> 3) * 2 + (x >> 3);
  const int col = (y & 7) * 8 + (x & 7);
  red[0][pxy][col] = smax[0];
  red[1][pxy][col] = smax[1];
  // patch p = (pz*2 + py)*2 + px owns red[p >> 2][p & 3][0..63]: the fused
  // step's epilogue layout and reduction (wave w: patches 2w, 2w+1)
  cfl_epilogue(&red[0][0][0], c_cfl * dx, dt_patch + int64_t(blockIdx.x) * 8, dt_min);
}

__global__ void set_inf_kernel(unsigned long long* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0x7ff0000000000000ull;
}

}  // namespace

template <typename T>
hipError_t launch_fill_ghosts(const T* level, T* U_pad, int ngx, int ngy, int ngz, int ghost, const int bc[6],
                              hipStream_t stream) {
  const int P = 16 + 2 * ghost;
  const int64_t planes = int64_t(ngx) * ngy * ngz * 5 * P;  // one workgroup per padded plane
  if (planes == 0) return hipSuccess;
  if (planes > (int64_t(1) << 31)) return hipErrorInvalidValue;
  BC6 b;
  for (int i = 0; i < 6; ++i) b.b[i] = bc[i];
  hipLaunchKernelGGL(fill_ghosts_kernel<T>, dim3(unsigned(planes)), dim3(256), 0, stream, level, U_pad, ngx, ngy,
                     ngz, ghost, b);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cfl_dt(const T* U_pad, int64_t n_groups, int ghost, double dx, double gamma, double c_cfl,
                         double* dt_patch, double* dt_min, hipStream_t stream) {
  unsigned long long* m = reinterpret_cast<unsigned long long*>(dt_min);
  if (m != nullptr) {
    hipLaunchKernelGGL(set_inf_kernel, dim3(1), dim3(64), 0, stream, m);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (n_groups == 0) return hipSuccess;
  const int64_t chunk = int64_t(1) << 30;
  const int P = 16 + 2 * ghost;
  const int64_t P3 = int64_t(P) * P * P;
  for (int64_t g0 = 0; g0 < n_groups; g0 += chunk) {
    const int64_t n = n_groups - g0 < chunk ? n_groups - g0 : chunk;
    hipLaunchKernelGGL(cfl_dt_kernel<T>, dim3(unsigned(n)), dim3(256), 0, stream, U_pad + g0 * 5 * P3, ghost, dx,
                       gamma, c_cfl, dt_patch + g0 * 8, m);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t launch_fill_ghosts<double>(const double*, double*, int, int, int, int, const int*,
                                               hipStream_t);
template hipError_t launch_fill_ghosts<float>(const float*, float*, int, int, int, int, const int*, hipStream_t);
template hipError_t launch_cfl_dt<double>(const double*, int64_t, int, double, double, double, double*, double*,
                                          hipStream_t);
template hipError_t launch_cfl_dt<float>(const float*, int64_t, int, double, double, double, double*, double*,
                                         hipStream_t);

}  // namespace gh
