// Signed-distance grid from a lidar point cloud: voxel occupancy, exact
// squared Euclidean distance transforms (separable: a two-sweep nearest-target
// pass along x, O(L) per line, then one pass per other axis over integer
// squared distances: the lower envelope of parabolas, O(L) per line, for
// long lines and the plain minimum, O(L^2) per line but parallel over every
// output, for short ones), and the signed field at voxel centres.  Every pass is exact integer arithmetic, so the squared distances
// are bit-identical to any other exact method.
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

// LDS budget of one block of the line passes (lines are staged as a tile
// [L][lines per block], L <= 4096 per axis)
constexpr size_t kEdtLds = 48u << 10;

// lines per block of a pass whose tile takes `bytes` per entry (a power of two,
// 1..64)
static int edt_lines(int L, size_t bytes) {
    int nl = 64;
    while (nl > 1 && (size_t)L * nl * bytes > kEdtLds) nl >>= 1;
    return nl;
}

// pass along x: squared distance along the row to the nearest target voxel.
// A block stages nl rows (coalesced reads along x) transposed into LDS; each
// thread then takes one row in two sweeps (nearest target at or before x,
// then at or after it: O(nx) per row) and the block stores the results
// coalesced.
__global__ __launch_bounds__(64) void k_edt_row(const uint8_t *__restrict__ occ, uint8_t target, int nx, int rows,
                                                int32_t *__restrict__ out) {
    extern __shared__ int32_t lds[];
    const int nl = blockDim.x, t = threadIdx.x;
    const int r0 = blockIdx.x * nl;
    const int nr = min(nl, rows - r0);
    int32_t *res = lds;                                         // [nx][nl]
    uint8_t *hit = reinterpret_cast<uint8_t *>(lds + (size_t)nx * nl);  // [nx][nl]
    for (int idx = t; idx < nr * nx; idx += nl) {
        const int c = idx / nx, x = idx - c * nx;
        hit[x * nl + c] = occ[(size_t)(r0 + c) * nx + x] == target;
    }
    __syncthreads();
    if (t < nr) {
        int last = -1;
        for (int x = 0; x < nx; ++x) {
            if (hit[x * nl + t]) last = x;
            res[x * nl + t] = last < 0 ? kEdtInf : (x - last) * (x - last);
        }
        last = -1;
        for (int x = nx - 1; x >= 0; --x) {
            if (hit[x * nl + t]) last = x;
            if (last >= 0) {
                const int32_t d = (last - x) * (last - x);
                if (d < res[x * nl + t]) res[x * nl + t] = d;
            }
        }
    }
    __syncthreads();
    for (int idx = t; idx < nr * nx; idx += nl) {
        const int c = idx / nx, x = idx - c * nx;
        out[(size_t)(r0 + c) * nx + x] = res[x * nl + c];
    }
}

// the same pass for rows of at most 256 voxels: one wave per row, four
// consecutive voxels per lane.  Each lane finds its own nearest target at or
// before / at or after each of its voxels; the nearest one in the lanes
// before / after it comes from a ballot of the lanes holding a target, the
// bit of the closest such lane, and one shuffle of that lane's last / first
// target.  The same integers as the two sweeps above.
__global__ __launch_bounds__(256) void k_edt_row_wave(const uint8_t *__restrict__ occ, uint8_t target, int nx,
                                                      int rows, int32_t *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= rows) return;  // whole waves leave together
    const uint8_t *src = occ + (size_t)row * nx;
    const int x0 = 4 * lane;
    bool hit[4];
    int first = -1, last = -1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        hit[j] = x0 + j < nx && src[x0 + j] == target;
        if (hit[j]) {
            if (first < 0) first = x0 + j;
            last = x0 + j;
        }
    }
    const unsigned long long m = __ballot(last >= 0);
    const unsigned long long below = m & ((1ull << lane) - 1ull);
    const unsigned long long above = lane == 63 ? 0ull : m & ~((2ull << lane) - 1ull);
    const int src_b = below ? 63 - __clzll((long long)below) : 0;
    const int src_a = above ? __ffsll((long long)above) - 1 : 0;
    const int last_before = __shfl(last, src_b);
    const int first_after = __shfl(first, src_a);
    int prev = below ? last_before : -1;
    int next = above ? first_after : -1;
    // forward within the lane: the nearest target at or before each voxel
    int pv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (hit[j]) prev = x0 + j;
        pv[j] = prev;
    }
    int32_t *dst = out + (size_t)row * nx;
#pragma unroll
    for (int j = 3; j >= 0; --j) {
        if (hit[j]) next = x0 + j;
        const int x = x0 + j;
        int32_t r = pv[j] < 0 ? kEdtInf : (x - pv[j]) * (x - pv[j]);
        if (next >= 0) {
            const int32_t d = (next - x) * (next - x);
            if (d < r) r = d;
        }
        if (x < nx) dst[x] = r;
    }
}

// pass along a strided axis of length L (y: stride nx; z: stride nx*ny):
// out(q) = min over l of f(l) + (q - l)^2, the lower envelope of the
// parabolas rooted at the finite samples (Felzenszwalb and Huttenlocher,
// "Distance Transforms of Sampled Functions", 2012), one thread per line,
// O(L) per line.  The envelope's breakpoints are rationals
// s(a, b) = (h_a - h_b) / (2 (a - b)), h_l = f(l) + l^2; they are never
// formed: every comparison of two of them, or of one with an integer q, is
// made by cross-multiplication in 64-bit integers, so the result is exact
// (the same minimum as the brute-force definition).  A block takes nl lines
// of consecutive x (coalesced reads and writes of each sample) and stages
// their samples in LDS ([L][nl] int32) beside the stack of envelope roots
// ([L][nl] int16).
__global__ __launch_bounds__(64) void k_edt_envelope(const int32_t *__restrict__ in, int32_t *__restrict__ out, int L,
                                                     size_t stride, size_t outer_stride, int nx, int lines) {
    extern __shared__ int32_t lds[];
    const int nl = blockDim.x, t = threadIdx.x;
    const int l0 = blockIdx.x * nl;
    const int nln = min(nl, lines - l0);
    int32_t *f = lds;                                                   // [L][nl]
    int16_t *stk = reinterpret_cast<int16_t *>(lds + (size_t)L * nl);  // [L][nl]
    auto base_of = [&](int line) { return (size_t)(line / nx) * outer_stride + (line % nx); };
    for (int idx = t; idx < L * nln; idx += nl) {
        const int q = idx / nln, c = idx - q * nln;
        f[q * nl + c] = in[base_of(l0 + c) + (size_t)q * stride];
    }
    __syncthreads();
    if (t >= nln) return;  // (no barrier below)
    int32_t *o = out + base_of(l0 + t);
    auto h = [&](int l) { return (int64_t)f[l * nl + t] + (int64_t)l * l; };
    // envelope: stk[0..k], roots in increasing order
    int k = -1;
    int v = 0;        // root at the top
    int64_t hv = 0;   // its h
    for (int q = 0; q < L; ++q) {
        const int32_t fq = f[q * nl + t];
        if (fq >= kEdtInf) continue;
        const int64_t hq = (int64_t)fq + (int64_t)q * q;
        // pop while the new parabola's breakpoint with the top is at or before
        // the top's own breakpoint with the one below it
        while (k >= 1) {
            const int u = stk[(k - 1) * nl + t];
            const int64_t hu = h(u);
            if ((hq - hv) * (int64_t)(v - u) <= (hv - hu) * (int64_t)(q - v)) {
                --k;
                v = u;
                hv = hu;
            } else {
                break;
            }
        }
        stk[++k * nl + t] = (int16_t)q;
        v = q;
        hv = hq;
    }
    if (k < 0) {
        for (int q = 0; q < L; ++q) o[(size_t)q * stride] = kEdtInf;
        return;
    }
    const int top = k;
    k = 0;
    v = stk[t];
    hv = h(v);
    int w = top > 0 ? stk[nl + t] : 0;
    int64_t hw = top > 0 ? h(w) : 0;
    for (int q = 0; q < L; ++q) {
        // advance while the breakpoint of roots k and k + 1 lies before q
        while (k < top && hw - hv < 2 * (int64_t)q * (w - v)) {
            ++k;
            v = w;
            hv = hw;
            if (k < top) {
                w = stk[(k + 1) * nl + t];
                hw = h(w);
            }
        }
        o[(size_t)q * stride] = (int32_t)(hv - (int64_t)v * v + (int64_t)(q - v) * (q - v));
    }
}

// The same pass for short lines (L <= kEdtShort): every output takes the plain
// minimum over the line's samples, O(L) per output and O(L^2) per line, but
// every output is independent, so the whole grid works in parallel; at the
// lengths of the workloads (128 and 256) this measures faster than the
// envelope's sequential walk per line (one thread per line leaves the chip
// mostly idle).  32 lines of consecutive x per block, staged in LDS
// ([L][32] int32, at most 64 KiB).
constexpr int kEdtShort = 512;
constexpr int kEdtCols = 32;

__global__ __launch_bounds__(256) void k_edt_short(const int32_t *__restrict__ in, int32_t *__restrict__ out, int L,
                                                   size_t stride, size_t outer_stride, int nx) {
    extern __shared__ int32_t tile[];  // [L][kEdtCols]
    const int x0 = blockIdx.x * kEdtCols;
    const size_t base = (size_t)blockIdx.y * outer_stride + x0;
    const int ncol = min(kEdtCols, nx - x0);
    // staged as g(l) = f(l) + l^2, so that f(l') + (l - l')^2 = g(l') - 2 l l' + l^2:
    // one 24-bit multiply-add and a minimum per sample (l, l' < 512).  A sample
    // without a target (f = kEdtInf) keeps g >= kEdtInf + l'^2, so its terms stay
    // at or above kEdtInf, above every finite squared distance (< 2^26).
    for (int idx = threadIdx.x; idx < L * kEdtCols; idx += blockDim.x) {
        const int l = idx / kEdtCols, c = idx % kEdtCols;
        const int32_t f = c < ncol ? in[base + (size_t)l * stride + c] : kEdtInf;
        tile[idx] = min(f, kEdtInf) + l * l;
    }
    __syncthreads();
    // eight outputs per thread, rows l0 + 8 r of one column (the block covers 8
    // rows per pass): each staged sample read from LDS serves all eight
    constexpr int kRows = 8;
    const int rows_per_pass = blockDim.x / kEdtCols;
    for (int idx = threadIdx.x; idx < L * kEdtCols; idx += blockDim.x * kRows) {
        const int l0 = idx / kEdtCols, c = idx % kEdtCols;
        if (c >= ncol) continue;
        int m2l[kRows];
        int32_t best[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            m2l[r] = -2 * (l0 + r * rows_per_pass);
            best[r] = 2 * kEdtInf;
        }
        for (int l2 = 0; l2 < L; ++l2) {
            const int32_t v = tile[l2 * kEdtCols + c];
#pragma unroll
            for (int r = 0; r < kRows; ++r) best[r] = min(best[r], v + __mul24(m2l[r], l2));
        }
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const int l = l0 + r * rows_per_pass;
            if (l < L) out[base + (size_t)l * stride + c] = min(best[r] + l * l, kEdtInf);
        }
    }
}

// one strided pass: the plain minimum for short lines, the envelope for long ones
static hipError_t edt_pass(const int32_t *in, int32_t *out, int L, size_t stride, size_t outer_stride, int nx,
                           int n_outer, hipStream_t st) {
    if (L <= kEdtShort) {
        hipLaunchKernelGGL(k_edt_short, dim3((nx + kEdtCols - 1) / kEdtCols, n_outer), dim3(256),
                           (size_t)L * kEdtCols * sizeof(int32_t), st, in, out, L, stride, outer_stride, nx);
    } else {
        const int lines = nx * n_outer, nl = edt_lines(L, 6);
        hipLaunchKernelGGL(k_edt_envelope, dim3((lines + nl - 1) / nl), dim3(nl), (size_t)L * nl * 6, st, in, out, L,
                           stride, outer_stride, nx, lines);
    }
    return hipGetLastError();
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
    const int rows = ny * nz;
    if (nx <= 256) {
        hipLaunchKernelGGL(k_edt_row_wave, dim3((rows + 3) / 4), dim3(256), 0, st, occ, target, nx, rows, out);
    } else {
        const int xl = edt_lines(nx, 5);
        hipLaunchKernelGGL(k_edt_row, dim3((rows + xl - 1) / xl), dim3(xl), (size_t)nx * xl * 5, st, occ, target, nx,
                           rows, out);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // y lines: (x, z), stride nx; z lines: (x, y), stride nx * ny
    if ((e = edt_pass(out, tmp, ny, (size_t)nx, (size_t)nx * ny, nx, nz, st)) != hipSuccess) return e;
    if ((e = edt_pass(tmp, out, nz, (size_t)nx * ny, (size_t)nx, nx, ny, st)) != hipSuccess) return e;
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
