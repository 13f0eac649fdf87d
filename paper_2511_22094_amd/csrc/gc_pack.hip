// Layout kernels: mask compaction (the memory-saving masking of paper §2.3.2,
// Fig. 3b), gathers into structure-of-arrays, scatters back to the grid,
// neighbour tables for the TV stencil, deterministic reductions, and the
// random-stream test kernels.
#include "gc_internal.hpp"
#include "gc_timing.hpp"

namespace gc {

// ------------------------------------------------------------ compaction
// Pass 1: masked voxels per tile of kTile grid voxels.
__global__ __launch_bounds__(kBlock) void tile_count_kernel(const uint8_t* __restrict__ mask,
                                                           int64_t n_grid,
                                                           int32_t* __restrict__ count) {
    __shared__ int lds[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    int c = 0;
#pragma unroll
    for (int i = 0; i < kTile / kBlock; ++i) {
        int64_t a = base + (int64_t)i * kBlock + threadIdx.x;
        if (a < n_grid) c += (mask == nullptr || mask[a]) ? 1 : 0;
    }
    int s = block_sum(c, lds);
    if (threadIdx.x == 0) count[blockIdx.x] = s;
}

// Pass 2 (one block): exclusive scan of the tile counts.
__global__ __launch_bounds__(1024) void tile_scan_kernel(const int32_t* __restrict__ count,
                                                        int64_t n_tiles,
                                                        int64_t* __restrict__ offset) {
    __shared__ int64_t part[1024];
    const int64_t per = (n_tiles + 1023) / 1024;
    const int64_t lo = threadIdx.x * per;
    int64_t s = 0;
    for (int64_t i = lo; i < lo + per && i < n_tiles; ++i) s += count[i];
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 1024 partial sums
    for (int o = 1; o < 1024; o <<= 1) {
        int64_t x = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    int64_t run = threadIdx.x == 0 ? 0 : part[threadIdx.x - 1];
    for (int64_t i = lo; i < lo + per && i < n_tiles; ++i) {
        offset[i] = run;
        run += count[i];
    }
    if (threadIdx.x == 1023) offset[n_tiles] = part[1023];
}

// Pass 3: compact indices.  Each thread owns kTile/kBlock consecutive voxels;
// a block-wide exclusive scan of the per-thread counts keeps grid order.
__global__ __launch_bounds__(kBlock) void tile_compact_kernel(const uint8_t* __restrict__ mask,
                                                             int64_t n_grid,
                                                             const int64_t* __restrict__ offset,
                                                             int32_t* __restrict__ g2c,
                                                             int32_t* __restrict__ c2g) {
    constexpr int PER = kTile / kBlock;
    __shared__ int wsum[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * PER;
    int flags[PER];
    int c = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        int64_t a = base + i;
        flags[i] = (a < n_grid) && (mask == nullptr || mask[a]) ? 1 : 0;
        c += flags[i];
    }
    // inclusive wave scan
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    int wbase = 0;
    for (int i = 0; i < wid; ++i) wbase += wsum[i];
    int64_t pos = offset[blockIdx.x] + wbase + x - c;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        int64_t a = base + i;
        if (a >= n_grid) break;
        if (flags[i]) {
            g2c[a] = (int32_t)pos;
            c2g[pos] = (int32_t)a;
            ++pos;
        } else {
            g2c[a] = -1;
        }
    }
}

hipError_t pack_index(const uint8_t* mask, PackPlan& plan, hipStream_t s) {
    const int nt = (int)plan.n_tiles;
    hipLaunchKernelGGL(tile_count_kernel, dim3(nt), dim3(kBlock), 0, s, mask, plan.n_grid,
                       plan.tile_count);
    hipLaunchKernelGGL(tile_scan_kernel, dim3(1), dim3(1024), 0, s, plan.tile_count,
                       plan.n_tiles, plan.tile_offset);
    hipLaunchKernelGGL(tile_compact_kernel, dim3(nt), dim3(kBlock), 0, s, mask, plan.n_grid,
                       plan.tile_offset, plan.g2c, plan.c2g);
    return hipGetLastError();
}

// ------------------------------------------------------------ gathers
// A thread reads its voxel's index once and moves kRowsPer rows of it, the
// reads all in flight before the writes (one row per thread re-read the
// index for every row and had one read in flight).
constexpr int kRowsPer = 8;

// dst[r][c] = src[r][c2g[c]] for r < rows; flags non-finite values.
__global__ __launch_bounds__(kBlock) void gather_rows_kernel(const float* __restrict__ src,
                                                            int64_t n_grid,
                                                            const int32_t* __restrict__ c2g,
                                                            int64_t n, int64_t rows,
                                                            float* __restrict__ dst,
                                                            int* __restrict__ flag) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    const int64_t r0 = (int64_t)blockIdx.y * kRowsPer;
    const int64_t a = c2g ? (int64_t)c2g[c] : c;
    float x[kRowsPer];
#pragma unroll
    for (int k = 0; k < kRowsPer; ++k) {
        // rows past the end re-read the last row (unconditional reads); not stored
        const int64_t r = r0 + k < rows ? r0 + k : rows - 1;
        x[k] = src[r * n_grid + a];
    }
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kRowsPer; ++k) {
        if (r0 + k < rows) {
            dst[(r0 + k) * n + c] = x[k];
            bad |= !isfinite(x[k]);
        }
    }
    if (flag && bad) atomicOr(flag, 1);
}

hipError_t gather_rows(const float* src, int64_t rows, int64_t n_grid, const int32_t* c2g,
                       int64_t n, float* dst, int* flag, hipStream_t s) {
    if (n == 0 || rows == 0) return hipSuccess;
    GC_LAUNCH(gather_rows_kernel,
              dim3((unsigned)((n + kBlock - 1) / kBlock), (unsigned)((rows + kRowsPer - 1) / kRowsPer)),
              dim3(kBlock), 0, s, src, n_grid, c2g, n, rows, dst, flag);
    return hipGetLastError();
}

// dst[r][a] = g2c[a] >= 0 ? src[r][g2c[a]] : 0, kRowsPer rows per thread
template <typename T>
__global__ __launch_bounds__(kBlock) void scatter_rows_kernel(const T* __restrict__ src,
                                                             int64_t n,
                                                             const int32_t* __restrict__ g2c,
                                                             int64_t n_grid, int64_t rows,
                                                             T* __restrict__ dst) {
    const int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (a >= n_grid) return;
    const int64_t r0 = (int64_t)blockIdx.y * kRowsPer;
    const int32_t c = g2c ? g2c[a] : (int32_t)a;
    T x[kRowsPer];
#pragma unroll
    for (int k = 0; k < kRowsPer; ++k) x[k] = (T)0;
    if (c >= 0) {   // voxels outside the mask read nothing (src may be empty)
#pragma unroll
        for (int k = 0; k < kRowsPer; ++k) {
            const int64_t r = r0 + k < rows ? r0 + k : rows - 1;
            x[k] = src[r * n + c];
        }
    }
#pragma unroll
    for (int k = 0; k < kRowsPer; ++k)
        if (r0 + k < rows) dst[(r0 + k) * n_grid + a] = x[k];
}

template <typename T>
static hipError_t scatter_t(const T* src, int64_t rows, int64_t n, const int32_t* g2c,
                            int64_t n_grid, T* dst, hipStream_t s) {
    if (n_grid == 0 || rows == 0) return hipSuccess;
    hipLaunchKernelGGL((scatter_rows_kernel<T>),
                       dim3((unsigned)((n_grid + kBlock - 1) / kBlock),
                            (unsigned)((rows + kRowsPer - 1) / kRowsPer)),
                       dim3(kBlock), 0, s, src, n, g2c, n_grid, rows, dst);
    return hipGetLastError();
}
hipError_t scatter_rows_f32(const float* src, int64_t rows, int64_t n, const int32_t* g2c,
                            int64_t n_grid, float* dst, hipStream_t s) {
    return scatter_t(src, rows, n, g2c, n_grid, dst, s);
}
hipError_t scatter_rows_f64(const double* src, int64_t rows, int64_t n, const int32_t* g2c,
                            int64_t n_grid, double* dst, hipStream_t s) {
    return scatter_t(src, rows, n, g2c, n_grid, dst, s);
}
hipError_t scatter_rows_i32(const int32_t* src, int64_t rows, int64_t n, const int32_t* g2c,
                            int64_t n_grid, int32_t* dst, hipStream_t s) {
    return scatter_t(src, rows, n, g2c, n_grid, dst, s);
}

// ------------------------------------------------------------ neighbours
// nbr[d][c], d = x-, x+, y-, y+, z-, z+ : compact index of the neighbour if it
// is inside the grid and the mask (z neighbours only for 3D TV), else -1.
__global__ __launch_bounds__(kBlock) void neighbour_kernel(const int32_t* __restrict__ c2g,
                                                          const int32_t* __restrict__ g2c,
                                                          int64_t n, int nx, int ny, int nz,
                                                          int tv_dim, int32_t* __restrict__ nbr) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    const int64_t a = c2g ? (int64_t)c2g[c] : c;
    const int x = (int)(a % nx), y = (int)((a / nx) % ny), z = (int)(a / ((int64_t)nx * ny));
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    auto at = [&](bool ok, int64_t b) -> int32_t {
        if (!ok) return -1;
        return g2c ? g2c[b] : (int32_t)b;
    };
    nbr[0 * n + c] = at(x > 0, a - 1);
    nbr[1 * n + c] = at(x + 1 < nx, a + 1);
    nbr[2 * n + c] = at(y > 0, a - sy);
    nbr[3 * n + c] = at(y + 1 < ny, a + sy);
    nbr[4 * n + c] = at(tv_dim == 3 && z > 0, a - sz);
    nbr[5 * n + c] = at(tv_dim == 3 && z + 1 < nz, a + sz);
}

hipError_t build_neighbours(const int32_t* c2g, const int32_t* g2c, int64_t n, int nx, int ny,
                            int nz, int tv_dim, int32_t* nbr, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(neighbour_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, c2g, g2c, n, nx, ny, nz, tv_dim, nbr);
    return hipGetLastError();
}

// ------------------------------------------------------------ reductions
// One block; each thread sums a strided slice in FP64 with Neumaier
// compensation, then a fixed-order tree: deterministic for a given count.
template <typename T>
__global__ __launch_bounds__(kBlock) void sum_partials_kernel(const T* __restrict__ p,
                                                             int64_t count,
                                                             double* __restrict__ out) {
    __shared__ double ss[kBlock], cc[kBlock];
    double s = 0.0, comp = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += kBlock) {
        const double x = (double)p[i];
        const double t = s + x;
        comp += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
        s = t;
    }
    ss[threadIdx.x] = s;
    cc[threadIdx.x] = comp;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double a = ss[threadIdx.x], b = ss[threadIdx.x + o];
            const double t = a + b;
            cc[threadIdx.x] += cc[threadIdx.x + o] + (fabs(a) >= fabs(b) ? (a - t) + b : (b - t) + a);
            ss[threadIdx.x] = t;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = ss[0] + cc[0];
}

hipError_t sum_partials(const float* partial, int64_t count, double* out, hipStream_t s) {
    hipLaunchKernelGGL((sum_partials_kernel<float>), dim3(1), dim3(kBlock), 0, s, partial, count,
                       out);
    return hipGetLastError();
}
hipError_t sum_partials_f64(const double* partial, int64_t count, double* out, hipStream_t s) {
    hipLaunchKernelGGL((sum_partials_kernel<double>), dim3(1), dim3(kBlock), 0, s, partial, count,
                       out);
    return hipGetLastError();
}

__global__ void fill_f32_kernel(float* p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}
hipError_t fill_f32(float* p, int64_t n, float v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, p, n, v);
    return hipGetLastError();
}

// flag |= 1 if any of p[0..n) is not a finite value > 0
__global__ void check_positive_kernel(const float* __restrict__ p, int64_t n, int* flag) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n && !(p[i] > 0.f && p[i] < INFINITY)) atomicOr(flag, 1);
}
hipError_t check_positive(const float* p, int64_t n, int* flag, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(check_positive_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, p, n, flag);
    return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}
hipError_t fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, p, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------------ random streams
__global__ __launch_bounds__(kBlock) void philox_kernel(uint32_t k0, uint32_t k1,
                                                       const uint32_t* __restrict__ ctr,
                                                       int64_t n, uint32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    U4 o = philox4x32_10(U4{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]}, k0, k1);
    out[4 * i] = o.x;
    out[4 * i + 1] = o.y;
    out[4 * i + 2] = o.z;
    out[4 * i + 3] = o.w;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void philox_un_kernel(uint32_t k0, uint32_t k1,
                                                          const uint32_t* __restrict__ ctr,
                                                          int64_t n, R* __restrict__ ou,
                                                          R* __restrict__ oz) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    U4 o = philox4x32_10(U4{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]}, k0, k1);
    const uint32_t w[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) ou[4 * i + k] = uniform01<R>(w[k]);
    // the same Box-Muller code path as the MH step draws
#pragma unroll
    for (int pr = 0; pr < 2; ++pr) {
        R u1 = uniform01<R>(w[2 * pr]), u2 = uniform01<R>(w[2 * pr + 1]);
        R r = Math<R>::sqrt(Math<R>::m2ln(u1));
        oz[4 * i + 2 * pr] = r * Math<R>::cos2pi(u2);
        oz[4 * i + 2 * pr + 1] = r * Math<R>::sin2pi(u2);
    }
}

hipError_t philox_batch(uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out,
                        hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(philox_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       (uint32_t)seed, (uint32_t)(seed >> 32), ctr, n, out);
    return hipGetLastError();
}

hipError_t philox_uniform_normal(uint64_t seed, const uint32_t* ctr, int64_t n, bool fp64,
                                 void* out_u, void* out_z, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const dim3 g((unsigned)((n + kBlock - 1) / kBlock));
    if (fp64)
        hipLaunchKernelGGL((philox_un_kernel<double>), g, dim3(kBlock), 0, s, (uint32_t)seed,
                           (uint32_t)(seed >> 32), ctr, n, (double*)out_u, (double*)out_z);
    else
        hipLaunchKernelGGL((philox_un_kernel<float>), g, dim3(kBlock), 0, s, (uint32_t)seed,
                           (uint32_t)(seed >> 32), ctr, n, (float*)out_u, (float*)out_z);
    return hipGetLastError();
}

}  // namespace gc
