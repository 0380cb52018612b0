// Ghost-cell fill, CFL time step and conservation sums.
#include "snap_internal.h"

namespace snap {

// One thread per ghost cell; the ghost cells are enumerated as three disjoint
// regions: z ghost levels (all y, x), y ghost rows of interior levels (all x),
// x ghost columns of interior rows. Threads start at `first` and stride by
// `stride` over the enumeration.
// The enumeration index has type I: 32-bit unsigned whenever the ghost cells
// of the grid number fewer than 2^31 (its divisions are then far cheaper),
// 64-bit otherwise.
template <typename T, typename I>
__device__ __forceinline__ void fill_ghosts_range(T* __restrict__ q, const GhostArgs& a,
                                                  I first, I stride) {
  const I nxp = (I)a.nxp, nyp = (I)a.nyp;
  const I nzr = (I)6 * nyp * nxp;
  const I nyr = a.d3 ? (I)a.nz * 6 * nxp : (I)0;
  const I nxr = (I)a.nz * (I)a.ny * 6;
  const I total = nzr + nyr + nxr;
  for (I g = first; g < total; g += stride) {
    int i, j, k;
    if (g < nzr) {
      const int ip = (int)(g % nxp);
      const I r = g / nxp;
      const int jp = (int)(r % nyp);
      const int kg = (int)(r / nyp);
      i = ip - NG;
      j = jp - a.gy;
      k = kg < 3 ? kg - 3 : a.nz + kg - 3;
    } else if (g < nzr + nyr) {
      const I h = g - nzr;
      const int ip = (int)(h % nxp);
      const I r = h / nxp;
      const int jg = (int)(r % 6);
      k = (int)(r / 6);
      i = ip - NG;
      j = jg < 3 ? jg - 3 : a.ny + jg - 3;
    } else {
      const I h = g - nzr - nyr;
      const int ig = (int)(h % 6);
      const I r = h / 6;
      j = (int)(r % (I)a.ny);
      k = (int)(r / (I)a.ny);
      i = ig < 3 ? ig - 3 : a.nx + ig - 3;
    }
    bool fx, fy = false, fz;
    const int si = ghost_src(i, a.nx, a.bcx, fx);
    const int sj = a.d3 ? ghost_src(j, a.ny, a.bcy, fy) : 0;
    const int sk = ghost_src(k, a.nz, a.bcz, fz);
    const long long dst = (long long)(k + NG) * a.sz + (long long)(j + a.gy) * a.sy + (i + NG);
    const long long src = (long long)(sk + NG) * a.sz + (long long)(sj + a.gy) * a.sy + (si + NG);
    // all loads first, then all stores: the ghost cell is never its own
    // source, but through one pointer the compiler cannot know that, and
    // interleaved load / store pairs would wait on memory once per variable
    T x[5 + MAX_TRACERS];
#pragma unroll
    for (int v = 0; v < 5 + MAX_TRACERS; ++v)
      if (v < a.nvar) x[v] = q[src + v * a.sv];
#pragma unroll
    for (int v = 0; v < 5 + MAX_TRACERS; ++v) {
      if (v < a.nvar) {
        const T y = (v == 1 && fx) || (v == 2 && fy) || (v == 3 && fz) ? -x[v] : x[v];
        q[dst + v * a.sv] = y;
      }
    }
  }
}

// Ghost cells of a grid (6 layers per axis, z layers over the whole padded
// plane), and whether their count fits the 32-bit enumeration.
__host__ __device__ inline long long ghost_count(const GhostArgs& a) {
  return 6LL * a.nyp * a.nxp + (a.d3 ? (long long)a.nz * 6 * a.nxp : 0) + (long long)a.nz * a.ny * 6;
}

template <typename T>
__device__ __forceinline__ void fill_ghosts_all(T* __restrict__ q, const GhostArgs& a) {
  const long long first = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  if (ghost_count(a) + stride < 0x7fffffffLL)
    fill_ghosts_range<T, unsigned>(q, a, (unsigned)first, (unsigned)stride);
  else
    fill_ghosts_range<T, long long>(q, a, first, stride);
}

template <typename T>
__global__ void k_fill_ghosts(T* __restrict__ q, GhostArgs a) {
  fill_ghosts_all<T>(q, a);
}

// All members of an ensemble: member blockIdx.y.
template <typename T>
__global__ void k_fill_ghosts_batched(const GhostDesc* __restrict__ d) {
  const GhostDesc g = d[blockIdx.y];
  fill_ghosts_all<T>(static_cast<T*>(g.q), g.a);
}

// ---------------------------------------------------------------------------
// CFL: per-cell signal speed sum_d (|u_d| + c) / dx_d in double precision
// (each term multiplied by the reciprocal spacing 1 / dx_d),
// written with the same operation order as the conserved -> primitive
// conversion, reduced to its maximum. A cell with rho <= 0 or p <= 0 (or NaN)
// contributes NaN, whose bit pattern exceeds every finite double and +inf when
// compared as an unsigned integer, so the reduction flags it.
// ---------------------------------------------------------------------------
__global__ void k_zero_u64(unsigned long long* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ULL;
}

// Raise *flag if the reduced maximum signal speed in *smax (IEEE bits) is not
// finite and positive (a cell with non-finite or non-positive density or
// pressure reduces to NaN).
__global__ void k_flag_speed(const unsigned long long* __restrict__ smax,
                             unsigned long long* __restrict__ flag) {
  if (threadIdx.x == 0) {
    const unsigned long long b = *smax;
    if (b == 0ULL || b >= 0x7FF0000000000000ULL) *flag = 1ULL;
  }
}

// One block per interior row (k, j) at a time, its threads along x: the
// row's offset is formed once, and no per-cell division is needed. NT: the
// tracer count under the mixture equation of state (0: the passive gas, whose
// tracers the signal speed does not read); a compile-time count lets a
// cell's tracer loads issue together with its five others.
template <typename T, int NT>
__global__ void __launch_bounds__(256) k_cfl(const T* __restrict__ q, CflArgs a,
                                             unsigned long long* __restrict__ out) {
  unsigned long long b = 0ULL;  // bit pattern of the running maximum
  const long long rows = (long long)a.ny * a.nz;
  for (long long row = blockIdx.x; row < rows; row += gridDim.x) {
   const int j = (int)(row % a.ny), k = (int)(row / a.ny);
   const long long base = (long long)(k + NG) * a.sz + (long long)(j + a.gy) * a.sy + NG;
   // perturbation storage: rho and p with the level references added back
   const double rbo = a.pert ? a.rbar_c[k + NG] : 0.0, pbo = a.pert ? a.pbar_c[k + NG] : 0.0;
   for (int i = threadIdx.x; i < a.nx; i += 256) {
    const long long o = base + i;
    double s;
    {
#pragma clang fp contract(off)
      const double rho = static_cast<double>(q[o]) + rbo, mx = q[o + a.sv], my = q[o + 2 * a.sv];
      const double mz = q[o + 3 * a.sv];
      const double E = q[o + 4 * a.sv];
      const double inv = 1.0 / rho;
      const double u = mx * inv, v = my * inv, w = mz * inv;
      const double K = 0.5 * ((mx * u + my * v) + mz * w);
      double p, gam;
      if constexpr (NT > 0) {
        // mixture equation of state: p and the parcel's effective gamma
        double A = 0.0, num = 1.0, den = 1.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {   // constant indices: the argument stays out of scratch
          const double rt = q[o + (5 + t) * a.sv];
          const double qt = rt * inv;
          A = t == 0 ? a.m.mu[0] * rt : A + a.m.mu[t] * rt;
          num = num + a.m.a[t] * qt;
          den = den + a.m.b[t] * qt;
        }
        const double ratio = num / den;
        p = (a.gm1 * ratio) * ((E - K) - A);
        gam = 1.0 + a.gm1 * ratio;
      } else {
        p = a.gm1 * (E - K) + pbo;
        gam = a.gamma;
      }
      const double cs = sqrt(gam * p / rho);
      s = (fabs(u) + cs) * a.dxi;
      if (a.d3) s = s + (fabs(v) + cs) * a.dyi;
      s = s + (fabs(w) + cs) * a.dzi;
      if (!(rho > 0.0) || !(p > 0.0)) s = __builtin_nan("");
    }
    const unsigned long long sb = (unsigned long long)__double_as_longlong(s);
    b = sb > b ? sb : b;
   }
  }
  // wave reduction of the unsigned bit patterns
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o2 = __shfl_xor(b, off, 64);
    b = o2 > b ? o2 : b;
  }
  __shared__ unsigned long long red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long x = red[0];
    for (int wv = 1; wv < 4; ++wv) x = red[wv] > x ? red[wv] : x;
    atomicMax(out, x);
  }
}

// ---------------------------------------------------------------------------
// Conservation sums: fixed grid of SUM_BLOCKS blocks, each summing a fixed
// strided subset of the interior in double precision and reducing it with a
// fixed tree; a single block then adds the partials in block order. The result
// is therefore reproducible from run to run.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_sums_partial(const T* __restrict__ q, SumArgs a,
                                                      double* __restrict__ part) {
  __shared__ double red[256];
  const long long n = (long long)a.nx * a.ny * a.nz;
  for (int v = 0; v < a.nvar; ++v) {
    double acc = 0.0;
    for (long long c = blockIdx.x * 256LL + threadIdx.x; c < n; c += (long long)gridDim.x * 256) {
      const int i = c % a.nx;
      const long long r = c / a.nx;
      const int j = r % a.ny;
      const int k = r / a.ny;
      const long long o = (long long)(k + NG) * a.sz + (long long)(j + a.gy) * a.sy + (i + NG);
      double x = static_cast<double>(q[o + v * a.sv]);
      if (a.pert && v == 0) x += a.rbar_c[k + NG];
      if (a.pert && v == 4) x += a.pbar_c[k + NG] * a.inv_gm1;
      acc += x;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(long long)v * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

__global__ void k_sums_final(const double* __restrict__ part, int nblk, int nvar,
                             double* __restrict__ out) {
  const int v = threadIdx.x;
  if (v < nvar) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(long long)v * nblk + b];
    out[v] = s;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int launch_fill_ghosts(int dtype, void* q, const GhostArgs& a, hipStream_t st) {
  const long long total = ghost_count(a);
  long long nb = (total + 255) / 256;
  if (nb > 65536) nb = 65536;
  if (nb < 1) nb = 1;
  if (dtype == 0)
    hipLaunchKernelGGL(k_fill_ghosts<double>, dim3((unsigned)nb), dim3(256), 0, st,
                       static_cast<double*>(q), a);
  else
    hipLaunchKernelGGL(k_fill_ghosts<float>, dim3((unsigned)nb), dim3(256), 0, st,
                       static_cast<float*>(q), a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_fill_ghosts_batched(int dtype, const GhostDesc* d, int n, long long max_ghosts,
                               hipStream_t st) {
  long long nb = (max_ghosts + 255) / 256;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  if (dtype == 0)
    hipLaunchKernelGGL(k_fill_ghosts_batched<double>, dim3((unsigned)nb, n), dim3(256), 0, st, d);
  else
    hipLaunchKernelGGL(k_fill_ghosts_batched<float>, dim3((unsigned)nb, n), dim3(256), 0, st, d);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_cfl(int dtype, const void* q, const CflArgs& a, unsigned long long* out,
               hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, out, 1);
  long long nb = (long long)a.ny * a.nz;   // rows
  if (nb > CFL_BLOCKS) nb = CFL_BLOCKS;
  if (nb < 1) nb = 1;
  const int nt = a.mix ? a.ntracer : 0;
  if (nt < 0 || nt > MAX_TRACERS) return -1;
  switch (nt) {
#define SNAP_CFL_CASE(N)                                                                  \
  case N:                                                                                 \
    if (dtype == 0)                                                                       \
      hipLaunchKernelGGL((k_cfl<double, N>), dim3((unsigned)nb), dim3(256), 0, st,        \
                         static_cast<const double*>(q), a, out);                          \
    else                                                                                  \
      hipLaunchKernelGGL((k_cfl<float, N>), dim3((unsigned)nb), dim3(256), 0, st,         \
                         static_cast<const float*>(q), a, out);                           \
    break;
    SNAP_CFL_CASE(0)
    SNAP_CFL_CASE(1)
    SNAP_CFL_CASE(2)
    SNAP_CFL_CASE(3)
    SNAP_CFL_CASE(4)
    SNAP_CFL_CASE(5)
    SNAP_CFL_CASE(6)
    SNAP_CFL_CASE(7)
    SNAP_CFL_CASE(8)
#undef SNAP_CFL_CASE
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_zero_u64(unsigned long long* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, p, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_flag_speed(const unsigned long long* smax, unsigned long long* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_flag_speed, dim3(1), dim3(64), 0, st, smax, flag);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_sums(int dtype, const void* q, const SumArgs& a, double* part, double* out,
                hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_sums_partial<double>, dim3(SUM_BLOCKS), dim3(256), 0, st,
                       static_cast<const double*>(q), a, part);
  else
    hipLaunchKernelGGL(k_sums_partial<float>, dim3(SUM_BLOCKS), dim3(256), 0, st,
                       static_cast<const float*>(q), a, part);
  hipLaunchKernelGGL(k_sums_final, dim3(1), dim3(64), 0, st, part, SUM_BLOCKS, a.nvar, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace snap

namespace snap {

TileShape batched_tile_f64(int ntracer, int v);
TileShape batched_tile_f32(int ntracer, int v);
int batched_occupancy_f64(int ntracer, int v, int form);
int batched_occupancy_f32(int ntracer, int v, int form);
int launch_stage2d_batched_f64(int ntracer, int v, int form, const StageArgs* d, const int* first,
                               int n, int nb, hipStream_t st);
int launch_stage2d_batched_f32(int ntracer, int v, int form, const StageArgs* d, const int* first,
                               int n, int nb, hipStream_t st);

TileShape batched_tile(int dtype, int ntracer, int variant) {
  if (variant < 0 || variant >= BATCH_VARIANTS) return TileShape{0, 0};
  return dtype == 0 ? batched_tile_f64(ntracer, variant) : batched_tile_f32(ntracer, variant);
}

int batched_occupancy(int dtype, int ntracer, int variant, int form) {
  return dtype == 0 ? batched_occupancy_f64(ntracer, variant, form)
                    : batched_occupancy_f32(ntracer, variant, form);
}

int launch_stage2d_batched(int dtype, int ntracer, int variant, int form, const StageArgs* descs,
                           const int* first, int n, int nblocks, hipStream_t st) {
  return dtype == 0
             ? launch_stage2d_batched_f64(ntracer, variant, form, descs, first, n, nblocks, st)
             : launch_stage2d_batched_f32(ntracer, variant, form, descs, first, n, nblocks, st);
}

}  // namespace snap
