// stream.hip -- streaming kernels of known traffic: the HBM ceiling of the
// sweeps' access shapes, measured on the device.
//
// The leapfrog step reads three FP64 grids (u^n, u^{n-1}, vsq) and writes
// one, in place over u^{n-1}; every Jacobi sweep reads one grid and writes
// another.  These kernels do exactly that and nothing else, so their
// bandwidth is what a sweep of the same shape can at best reach, and their
// known byte counts calibrate the HBM byte counters of the profiler.
//
//   op 0 (copy):    d[i] = a[i]                        8 B read + 8 B written
//   op 1 (3R + 1W): d[i] = fma(c[i], a[i], 2a[i] - b[i])  24 B read + 8 B written
//
// W doubles per lane and access (1: 8-byte loads, 2: 16-byte loads); loads
// and stores may carry the nontemporal hint.  d may equal b (in place).
#include "internal.hpp"

namespace stn {
namespace {

typedef double dbl2 __attribute__((ext_vector_type(2)));

template <int W>
struct Vec;
template <>
struct Vec<1> {
    typedef double T;
};
template <>
struct Vec<2> {
    typedef dbl2 T;
};

template <bool NT, typename T>
__device__ __forceinline__ T ld(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool NT, typename T>
__device__ __forceinline__ void st(T *p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <int OP, int W, bool NTL, bool NTS>
__global__ __launch_bounds__(256) void stream_kernel(const double *a, const double *b, const double *c, double *d,
                                                     long long n) {
    typedef typename Vec<W>::T V;
    const long long nv = n / W;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < nv; v += stride) {
        const V x = ld<NTL>((const V *)a + v);
        if constexpr (OP == 0) {
            st<NTS>((V *)d + v, x);
        } else {
            const V y = ld<NTL>((const V *)b + v);
            const V z = ld<NTL>((const V *)c + v);
            V r;
            if constexpr (W == 1) {
                r = fma(z, x, 2.0 * x - y);
            } else {
                r.x = fma(z.x, x.x, 2.0 * x.x - y.x);
                r.y = fma(z.y, x.y, 2.0 * x.y - y.y);
            }
            st<NTS>((V *)d + v, r);
        }
    }
    // tail (n not a multiple of W): the first block's threads
    if (blockIdx.x == 0) {
        const long long i = nv * W + threadIdx.x;
        if (i < n) {
            if constexpr (OP == 0) d[i] = a[i];
            else d[i] = fma(c[i], a[i], 2.0 * a[i] - b[i]);
        }
    }
}

template <int OP, int W>
hipError_t launch_w(int flags, dim3 grid, hipStream_t s, const double *a, const double *b, const double *c,
                    double *d, long long n) {
    switch (flags & 3) {
    case 0: hipLaunchKernelGGL((stream_kernel<OP, W, false, false>), grid, dim3(256), 0, s, a, b, c, d, n); break;
    case 1: hipLaunchKernelGGL((stream_kernel<OP, W, true, false>), grid, dim3(256), 0, s, a, b, c, d, n); break;
    case 2: hipLaunchKernelGGL((stream_kernel<OP, W, false, true>), grid, dim3(256), 0, s, a, b, c, d, n); break;
    default: hipLaunchKernelGGL((stream_kernel<OP, W, true, true>), grid, dim3(256), 0, s, a, b, c, d, n); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stream(int op, const double *a, const double *b, const double *c, double *d, long long n,
                         int width, int flags, int grid, hipStream_t s) {
    const long long per_thread_pass = cdiv(n / width, 256);
    // one pass by default (at most 2^24 blocks; the loop covers the rest)
    const dim3 g(grid > 0 ? grid : (unsigned)std::min(1LL << 24, std::max(1LL, per_thread_pass)));
    if (op == 0) return width == 1 ? launch_w<0, 1>(flags, g, s, a, b, c, d, n) : launch_w<0, 2>(flags, g, s, a, b, c, d, n);
    return width == 1 ? launch_w<1, 1>(flags, g, s, a, b, c, d, n) : launch_w<1, 2>(flags, g, s, a, b, c, d, n);
}

}  // namespace stn
