// common.hpp -- device building blocks shared by the sweep kernels (gfx950).
//
// Layout: padded grid, x contiguous; interior point (i,j,k) at
// (k+r)*pz + (j+r)*py + (i+r) elements from the base pointer.
#pragma once

#if !defined(__HIPCC_RTC__)  // hipRTC (generated kernels) provides the runtime itself
#include <hip/hip_runtime.h>

#include <cstdint>
#endif

namespace stn {

struct Geom {
    int nx, ny, nz;    // interior extents
    int r;             // halo width
    long long py, pz;  // row / plane pitch in elements
    __host__ __device__ int PX() const { return nx + 2 * r; }
    __host__ __device__ int PY() const { return ny + 2 * r; }
    __host__ __device__ int PZ() const { return nz + 2 * r; }
};

// ---------------------------------------------------------------------------
// Wave64 FP64 sum with DPP.  Four DPP steps leave every lane of each 16-lane
// row holding that row's sum (quad swaps, then half-row and row mirrors);
// the four row sums are then combined in a fixed order through readlane.
// Every lane of the wave must be active (all block sizes here are multiples
// of 64 and no lane leaves before the reduction).  FP addition is
// commutative, so lanes that add the same pair in swapped order agree
// bit for bit, and the result is independent of scheduling.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
    const int hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi2, lo2);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror: lane i <- 7-i within 8
    v += dpp_f64<0x140>(v);  // row_mirror: lane i <- 15-i within 16
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Block sum: wave sums through LDS, added by thread 0 in wave order.
// Returns the block total in thread 0 (other threads: unspecified).
// lds must hold one double per wave.  Contains a barrier: every thread of
// the block must call it.
__device__ __forceinline__ double block_sum_f64(double v, double *lds) {
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthreads = blockDim.x * blockDim.y * blockDim.z;
    v = wave_sum_f64(v);
    if ((tid & 63) == 0) lds[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0)
        for (int w = 0; w < (nthreads >> 6); ++w) s += lds[w];
    return s;
}

__device__ __forceinline__ int block_linear_id() {
    return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

// Workgroups are handed to the eight XCDs round-robin in dispatch order
// (block L runs on XCD L % 8), and each XCD has its own L2.  With remap set,
// logical tiles are renumbered so that every XCD receives one contiguous run
// of them (x fastest, then y, then z): tiles that share halo rows, boundary
// cache lines and priming planes then meet in the same L2.  The map is a
// bijection of [0, N), so each tile is still computed exactly once.
__device__ __forceinline__ void tile_coords(int remap, int &bx, int &by, int &bz) {
    const int gx = gridDim.x, gy = gridDim.y;
    int L = block_linear_id();
    if (remap) {
        const int N = gx * gy * gridDim.z, q = N >> 3, rem = N & 7, x = L & 7;
        L = x * q + min(x, rem) + (L >> 3);
    }
    bx = L % gx;
    L /= gx;
    by = L % gy;
    bz = L / gy;
}

// ---------------------------------------------------------------------------
// Raw buffer access to one plane: the plane's base address lives in a scalar
// buffer resource (4 SGPRs) and each lane passes a 32-bit byte offset, so a
// streaming kernel holds no 64-bit address per lane and per plane.  Word 3 is
// the untyped 32-bit data format of gfx9-family raw buffers; the record count
// is the full 32-bit range (offsets stay inside the plane, which the host
// keeps below 4 GiB for kernels that use these).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *plane) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(plane), (short)0, -1, 0x00020000);
}
__device__ __forceinline__ double buf_ld_f64(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void buf_st_f64(__amdgpu_buffer_rsrc_t r, unsigned off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                          off, 0, 0);
}

// ---------------------------------------------------------------------------
// Halo stager: the cells of an xy tile's halo ring of width R (TX x TY
// interior cells, LDS tile (TY+2R) x (TX+2R)), spread over the block's
// threads.  With CORNERS = false the four R x R corner squares are skipped
// (star stencils never read them).  Each thread keeps at most HR cells: their
// LDS index, in-plane global offset and validity are computed once; load()
// issues the global loads of one plane into registers (early, one plane
// ahead) and store() writes them into LDS.  LW: the LDS row stride (the
// tile width unless the caller pads its rows).
template <typename T, int TX, int TY, int R, bool CORNERS, int NT, int LW = TX + 2 * R>
struct HaloStager {
    static constexpr int W = TX + 2 * R;
    static constexpr int BW = CORNERS ? W : TX;
    static constexpr int NH = 2 * R * BW + 2 * R * TY;
    static constexpr int HR = (NH + NT - 1) / NT;
    int lidx[HR];
    long long goff[HR];
    bool has[HR];  // this thread owns ring cell s
    bool ok[HR];   // ... and it lies inside the padded array (else it stages 0)
    T val[HR];

    // x0p, y0p: padded coordinates of the tile's first interior cell.
    __device__ __forceinline__ void init(int tid, int x0p, int y0p, long long py, int PX, int PY) {
#pragma unroll
        for (int s = 0; s < HR; ++s) {
            int h = tid + s * NT;
            has[s] = h < NH;
            ok[s] = false;
            lidx[s] = 0;
            goff[s] = 0;
            val[s] = T(0);
            if (h < NH) {
                int lx, ly;
                if (h < R * BW) {
                    ly = h / BW;
                    lx = h % BW + (CORNERS ? 0 : R);
                } else if (h < 2 * R * BW) {
                    h -= R * BW;
                    ly = TY + R + h / BW;
                    lx = h % BW + (CORNERS ? 0 : R);
                } else if (h < 2 * R * BW + R * TY) {
                    h -= 2 * R * BW;
                    ly = R + h / R;
                    lx = h % R;
                } else {
                    h -= 2 * R * BW + R * TY;
                    ly = R + h / R;
                    lx = TX + R + h % R;
                }
                const int gx = x0p - R + lx, gy = y0p - R + ly;
                ok[s] = gx >= 0 && gx < PX && gy >= 0 && gy < PY;
                lidx[s] = ly * LW + lx;
                goff[s] = (long long)gy * py + gx;
            }
        }
    }
    __device__ __forceinline__ void load(const T *__restrict__ plane) {
#pragma unroll
        for (int s = 0; s < HR; ++s) val[s] = ok[s] ? plane[goff[s]] : T(0);
    }
    // L: the LDS element type (a wider type widens exactly on store)
    template <typename L>
    __device__ __forceinline__ void store(L *lds) const {
#pragma unroll
        for (int s = 0; s < HR; ++s)
            if (has[s]) lds[lidx[s]] = (L)val[s];
    }
};

}  // namespace stn
