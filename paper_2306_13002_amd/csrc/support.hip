// support.hip -- halo copy, periodic halo fill, the residual's final pass and
// the device scratch of the allocation-free run.
#include <mutex>

#include "internal.hpp"

namespace stn {
namespace {

// Enumerate the halo cells of a padded grid (x/y halo width r, z halo width
// rz; rz = 0 and nz = 1 for 2-D grids) as three segments: the z-halo planes,
// then the y-halo rows of interior planes, then the x-halo cells of interior
// rows.  Writes the padded (x, y, z) of halo cell t.
__device__ __forceinline__ void halo_cell(long long t, const Geom &g, int rz, long long &x, long long &y,
                                          long long &z) {
    const long long PX = g.nx + 2 * g.r, PY = g.ny + 2 * g.r;
    const long long cA = 2LL * rz * PY * PX, cB = (long long)g.nz * 2 * g.r * PX;
    if (t < cA) {
        const long long zz = t / (PY * PX), rem = t % (PY * PX);
        z = zz < rz ? zz : g.nz + zz;
        y = rem / PX;
        x = rem % PX;
    } else if (t < cA + cB) {
        t -= cA;
        const long long per = 2LL * g.r * PX;
        z = rz + t / per;
        const long long rem = t % per, yy = rem / PX;
        y = yy < g.r ? yy : g.ny + yy;
        x = rem % PX;
    } else {
        t -= cA + cB;
        const long long zy = t / (2 * g.r), xx = t % (2 * g.r);
        z = rz + zy / g.ny;
        y = g.r + zy % g.ny;
        x = xx < g.r ? xx : g.nx + xx;
    }
}

__host__ __device__ inline long long halo_count(const Geom &g, int rz) {
    const long long PX = g.nx + 2 * g.r, PY = g.ny + 2 * g.r;
    return 2LL * rz * PY * PX + (long long)g.nz * 2 * g.r * PX + (long long)g.nz * g.ny * 2 * g.r;
}

template <typename T>
__global__ void halo_copy_kernel(const T *__restrict__ src, T *__restrict__ dst, Geom g, int rz, long long n) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x) {
        long long x, y, z;
        halo_cell(t, g, rz, x, y, z);
        const long long q = z * g.pz + y * g.py + x;
        dst[q] = src[q];
    }
}

__device__ __forceinline__ long long wrap_into(long long c, int r, int n) {
    // padded coordinate -> padded coordinate of the interior cell it images
    long long i = (c - r) % n;
    if (i < 0) i += n;
    return i + r;
}

template <typename T>
__global__ void periodic_fill_kernel(T *__restrict__ buf, Geom g, int rz, long long n) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x) {
        long long x, y, z;
        halo_cell(t, g, rz, x, y, z);
        const long long sx = wrap_into(x, g.r, g.nx), sy = wrap_into(y, g.r, g.ny);
        const long long sz = rz ? wrap_into(z, rz, g.nz) : z;
        buf[z * g.pz + y * g.py + x] = buf[sz * g.pz + sy * g.py + sx];
    }
}

template <typename T>
__global__ void interior_copy_kernel(const T *__restrict__ src, T *__restrict__ dst, Geom g, long long n) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x) {
        const long long i = t % g.nx, jk = t / g.nx, j = jk % g.ny, k = jk / g.ny;
        const long long q = (k + g.r) * g.pz + (j + g.r) * g.py + (i + g.r);  // 2-D: pz = 0
        dst[q] = src[q];
    }
}

// Pass 1: block b sums the contiguous chunk [b*chunk, min((b+1)*chunk, n))
// (thread-strided, then the block sum); pass 2 (one block) sums the pass-1
// results.  The split depends only on n, so the total is reproducible.
__global__ void reduce_pass1_kernel(const double *__restrict__ part, long long n, long long chunk,
                                    double *__restrict__ out) {
    __shared__ double lds[4];
    const long long b0 = blockIdx.x * chunk, b1 = min(b0 + chunk, n);
    double s = 0.0;
    for (long long i = b0 + threadIdx.x; i < b1; i += 256) s += part[i];
    s = block_sum_f64(s, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

template <typename T>
__global__ void fill_kernel(T *__restrict__ buf, long long n, T v) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
        buf[t] = v;
}

// seg holds count begins, then count ends.
__global__ void segment_sums_kernel(const double *__restrict__ part, const int *__restrict__ seg, int count,
                                    double *__restrict__ out) {
    __shared__ double lds[4];
    const int b0 = seg[blockIdx.x], b1 = seg[count + blockIdx.x];
    double s = 0.0;
    for (int i = b0 + threadIdx.x; i < b1; i += 256) s += part[i];
    s = block_sum_f64(s, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

dim3 grid_for(long long n) {
    long long b = cdiv(n, 256);
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

}  // namespace

hipError_t launch_halo_copy(const void *src, void *dst, int eb, const Geom &g, int rz, hipStream_t s) {
    const long long n = halo_count(g, rz);
    if (n == 0) return hipSuccess;
    if (eb == 8)
        hipLaunchKernelGGL(halo_copy_kernel<double>, grid_for(n), dim3(256), 0, s, (const double *)src,
                           (double *)dst, g, rz, n);
    else
        hipLaunchKernelGGL(halo_copy_kernel<float>, grid_for(n), dim3(256), 0, s, (const float *)src,
                           (float *)dst, g, rz, n);
    return hipGetLastError();
}

hipError_t launch_periodic_fill(void *buf, int eb, const Geom &g, int rz, hipStream_t s) {
    const long long n = halo_count(g, rz);
    if (n == 0) return hipSuccess;
    if (eb == 8)
        hipLaunchKernelGGL(periodic_fill_kernel<double>, grid_for(n), dim3(256), 0, s, (double *)buf, g, rz, n);
    else
        hipLaunchKernelGGL(periodic_fill_kernel<float>, grid_for(n), dim3(256), 0, s, (float *)buf, g, rz, n);
    return hipGetLastError();
}

hipError_t launch_fill(void *buf, long long n, int eb, double v, hipStream_t s) {
    if (eb == 8)
        hipLaunchKernelGGL(fill_kernel<double>, grid_for(n), dim3(256), 0, s, (double *)buf, n, v);
    else
        hipLaunchKernelGGL(fill_kernel<float>, grid_for(n), dim3(256), 0, s, (float *)buf, n, (float)v);
    return hipGetLastError();
}

hipError_t launch_interior_copy(const void *src, void *dst, int eb, const Geom &g, int rz, hipStream_t s) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    Geom h = g;
    if (rz == 0) h.pz = 0;  // 2-D: a single plane
    if (eb == 8)
        hipLaunchKernelGGL(interior_copy_kernel<double>, grid_for(n), dim3(256), 0, s, (const double *)src,
                           (double *)dst, h, n);
    else
        hipLaunchKernelGGL(interior_copy_kernel<float>, grid_for(n), dim3(256), 0, s, (const float *)src,
                           (float *)dst, h, n);
    return hipGetLastError();
}

hipError_t launch_segment_sums(const double *part, const int *seg, int count, double *out, hipStream_t s) {
    hipLaunchKernelGGL(segment_sums_kernel, dim3(count), dim3(256), 0, s, part, seg, count, out);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const double *part, long long n, double *scratch, double *out, hipStream_t s) {
    long long chunk = cdiv(n, kReduceBlocks);
    if (chunk < 1024) chunk = 1024;
    const long long nb = cdiv(n, chunk);
    if (nb == 1) {
        // One chunk: a second pass would add zeros to this sum and return it
        // unchanged (residuals are sums of squares, never -0), so the single
        // block writes the total itself and one launch is saved.
        hipLaunchKernelGGL(reduce_pass1_kernel, dim3(1), dim3(256), 0, s, part, n, chunk, out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(reduce_pass1_kernel, dim3((unsigned)nb), dim3(256), 0, s, part, n, chunk, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_pass1_kernel, dim3(1), dim3(256), 0, s, (const double *)scratch, nb, nb, out);
    return hipGetLastError();
}

// Scratch of the allocation-free run: kNoallocPartials per-block residual
// partials, then kReduceBlocks first-pass sums of their reduction.  One copy
// per GPU, resident until the process ends.  In host code the array's name
// is not a device address: only the address hipGetSymbolAddress returns for
// the current device is passed to kernels.
static __device__ __align__(256) double scratch[kNoallocPartials + kReduceBlocks];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(double **out) {
    *out = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        double *ptr = nullptr;
        if ((e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace stn
