// Signed-distance grid from a lidar point cloud: voxel occupancy, exact
// squared Euclidean distance transforms (separable: one 1-D lower-envelope
// pass per axis over integer squared distances), and the signed field at
// voxel centres.  Every pass is exact integer arithmetic, so the squared
// distances are bit-identical to any other exact method.
#include <algorithm>

#include "launch.h"

namespace cp {

constexpr int32_t kEdtInf = 1 << 29;  // larger than any squared distance on a grid of <= 4096 per axis

__global__ void k_fill_u8(uint8_t *p, size_t n, uint8_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// occupied = voxel holding at least one point; index floor((p - o) / h) in
// double precision; points outside the grid are dropped
__global__ void k_occupancy(const float *__restrict__ pts, int64_t N, int nx, int ny, int nz, double ox, double oy,
                            double oz, double h, uint8_t *__restrict__ occ) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const double gx = floor(((double)pts[3 * i] - ox) / h);
        const double gy = floor(((double)pts[3 * i + 1] - oy) / h);
        const double gz = floor(((double)pts[3 * i + 2] - oz) / h);
        if (gx >= 0.0 && gx < nx && gy >= 0.0 && gy < ny && gz >= 0.0 && gz < nz)
            occ[((size_t)gz * ny + (size_t)gy) * nx + (size_t)gx] = 1;
    }
}

// pass along x: g(x) = min over target voxels x' of the row of (x - x')^2
__global__ __launch_bounds__(256) void k_edt_x(const uint8_t *__restrict__ occ, uint8_t target, int nx,
                                               int32_t *__restrict__ out) {
    extern __shared__ int32_t row[];
    const size_t base = (size_t)blockIdx.x * nx;
    for (int x = threadIdx.x; x < nx; x += blockDim.x) row[x] = occ[base + x] == target ? 0 : kEdtInf;
    __syncthreads();
    for (int x = threadIdx.x; x < nx; x += blockDim.x) {
        int32_t best = kEdtInf;
        for (int x2 = 0; x2 < nx; ++x2) {
            const int32_t d = x - x2;
            const int32_t v = row[x2] + d * d;
            best = v < best ? v : best;
        }
        out[base + x] = best;
    }
}

// pass along a strided axis of length L (y: stride nx; z: stride nx*ny):
// out(l) = min over l' of in(l') + (l - l')^2, for 32 consecutive x at once
constexpr int kEdtCols = 32;

__global__ __launch_bounds__(256) void k_edt_strided(const int32_t *__restrict__ in, int32_t *__restrict__ out, int L,
                                                     size_t stride, size_t outer_stride, int nx) {
    extern __shared__ int32_t tile[];  // [L][kEdtCols]
    const int x0 = blockIdx.x * kEdtCols;
    const size_t base = (size_t)blockIdx.y * outer_stride + x0;
    const int ncol = min(kEdtCols, nx - x0);
    for (int idx = threadIdx.x; idx < L * kEdtCols; idx += blockDim.x) {
        const int l = idx / kEdtCols, c = idx % kEdtCols;
        tile[idx] = c < ncol ? in[base + (size_t)l * stride + c] : kEdtInf;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < L * kEdtCols; idx += blockDim.x) {
        const int l = idx / kEdtCols, c = idx % kEdtCols;
        if (c >= ncol) continue;
        int32_t best = kEdtInf;
        for (int l2 = 0; l2 < L; ++l2) {
            const int32_t d = l - l2;
            const int32_t f = tile[l2 * kEdtCols + c];
            const int32_t v = f >= kEdtInf ? kEdtInf : f + d * d;
            best = v < best ? v : best;
        }
        out[base + (size_t)l * stride + c] = best;
    }
}

__global__ void k_edt_finish(int32_t *__restrict__ e, size_t n, int32_t none) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        if (e[i] >= kEdtInf) e[i] = none;
}

// free voxels: h (sqrt(EDT to occupied) - 1/2); occupied: -h (sqrt(EDT to free) - 1/2)
__global__ void k_sdf_sign(const uint8_t *__restrict__ occ, const int32_t *__restrict__ e_occ,
                           const int32_t *__restrict__ e_free, size_t n, float h, float *__restrict__ sdf) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        if (occ[i])
            sdf[i] = -h * (sqrtf((float)e_free[i]) - 0.5f);
        else
            sdf[i] = h * (sqrtf((float)e_occ[i]) - 0.5f);
    }
}

static hipError_t edt3(const uint8_t *occ, uint8_t target, int nx, int ny, int nz, int32_t *out, int32_t *tmp,
                       hipStream_t st) {
    // x pass into out, y pass out -> tmp, z pass tmp -> out
    hipLaunchKernelGGL(k_edt_x, dim3(ny * nz), dim3(256), nx * sizeof(int32_t), st, occ, target, nx, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int cx = (nx + kEdtCols - 1) / kEdtCols;
    hipLaunchKernelGGL(k_edt_strided, dim3(cx, nz), dim3(256), ny * kEdtCols * sizeof(int32_t), st, out, tmp, ny,
                       (size_t)nx, (size_t)nx * ny, nx);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_edt_strided, dim3(cx, ny), dim3(256), nz * kEdtCols * sizeof(int32_t), st, tmp, out, nz,
                       (size_t)nx * ny, (size_t)nx, nx);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const size_t n = (size_t)nx * ny * nz;
    const int32_t none = nx * nx + ny * ny + nz * nz;
    hipLaunchKernelGGL(k_edt_finish, dim3(1024), dim3(256), 0, st, out, n, none);
    return hipGetLastError();
}

hipError_t launch_sdf_build(const float *points, int64_t N, const int32_t dims[3], const float origin[3], float voxel,
                            float *sdf, uint8_t *occ, int32_t *edt_occ, int32_t *edt_free, int32_t *work,
                            hipStream_t st) {
    const int nx = dims[0], ny = dims[1], nz = dims[2];
    const size_t n = (size_t)nx * ny * nz;
    hipLaunchKernelGGL(k_fill_u8, dim3(1024), dim3(256), 0, st, occ, n, (uint8_t)0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (N > 0) {
        const unsigned blocks = (unsigned)std::min<int64_t>((N + 255) / 256, 65535);
        hipLaunchKernelGGL(k_occupancy, dim3(blocks), dim3(256), 0, st, points, N, nx, ny, nz, (double)origin[0],
                           (double)origin[1], (double)origin[2], (double)voxel, occ);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = edt3(occ, 1, nx, ny, nz, edt_occ, work, st)) != hipSuccess) return e;
    if ((e = edt3(occ, 0, nx, ny, nz, edt_free, work, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sdf_sign, dim3(1024), dim3(256), 0, st, occ, edt_occ, edt_free, n, voxel, sdf);
    return hipGetLastError();
}

}  // namespace cp
