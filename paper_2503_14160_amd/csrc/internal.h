// Internal device-side tables and helpers of the craneplan library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "craneplan.h"

namespace cp {

constexpr int kWave = 64;
constexpr float kInf = __builtin_huge_valf();

// One joint: fixed offset, then motion about / along a unit axis.
struct JointDev {
    int32_t type;
    float ax, ay, az;
    float ox, oy, oz;
    float qmin, qmax, qhold;
    int32_t active;
    int32_t pad;
};

// Spheres are stored sorted by frame; `orig` is the caller's sphere index.
struct SphereDev {
    float lx, ly, lz, r;
    int32_t frame, orig, pad0, pad1;
};

// Cylinders that share one vertical extent form a group.  Within a group the
// minimum over cylinders of (radial distance - R) is taken first and the
// height term applied once (the cylinder SDF is non-decreasing in the radial
// term for a fixed height offset, so this equals the minimum of the SDFs).
// A uniform 2-D grid over the group's cylinder centres (about three per cell)
// lets a wave visit only the cylinders near its own spheres: the group's
// cylinders are also stored sorted by cell (row-major), so the cylinders of a
// run of cells in one row are contiguous.
struct GroupDev {
    int32_t start, count;  // into the sorted cylinder tables; count is a multiple of 4
    float zc, hz;          // centre and half height of the shared extent
    float rmax;            // largest radius in the group
    float gx0, gy0;        // grid: lower corner,
    float gh, ginv;        //       cell edge and its reciprocal,
    int32_t gnx, gny;      //       cells per axis,
    int32_t gcell;         //       offset of the group's first cell in cell_start
    // A finer square grid of hints: per cell, the cyl_cell index of the
    // cylinder nearest to the cell's centre (in the radial term); any one
    // cylinder gives an upper bound of a minimum, a near one a tight bound.
    float hx0, hy0;        // lower corner
    float hinv;            // reciprocal of the cell edge
    int32_t hn;            // cells per axis
    int32_t hoff;          // offset of the group's first cell in hint
    int32_t pad[3];
};
static_assert(sizeof(GroupDev) == 80, "GroupDev layout");

// Within a group, cylinders are sorted by polar angle about the world z axis;
// kAngleBins start offsets per group let a wave begin its scan at the
// cylinders nearest its own azimuth.
constexpr int kAngleBins = 64;

// Everything a kernel needs about a plan, passed by value.
struct PlanView {
    int32_t n_joints, n_spheres, n_groups, n_box, n_cyl, has_ground;
    float ground_z;
    int32_t K, M, ns, interp, jp_mode, hinge;
    float margin, lambda_c, w_c, w_l;
    const JointDev *joints;       // [n_joints]
    const SphereDev *spheres;     // [n_spheres], sorted by frame
    const int32_t *sphere_slot;   // [n_spheres]: position in spheres of the caller's sphere i
    const int32_t *frame_start;   // [n_joints + 2]: spheres of frame f are [frame_start[f], frame_start[f+1])
    const float4 *cyl;            // [sum of group counts] (x, y, R, unused), grouped
    const GroupDev *groups;       // [n_groups]
    const int32_t *angle_start;   // [n_groups][kAngleBins] scan start (multiple of 4) per azimuth bin
    int32_t pair_filter;          // 1: skip the square root of pairs that cannot lower the minimum
    const float4 *cyl_cell;       // (x, y, R, caller index as int bits), sorted by grid cell within each group
    const int32_t *cell_start;    // per group [gny * gnx + 1]: first cyl_cell index of each cell
    const int32_t *hint;          // per group [hn * hn]: cyl_cell index of a near cylinder per cell
    const float4 *cyl_orig;       // [n_cyl] (x, y, R, group) in the caller's order
    const float4 *box;            // [n_box][2]: (cx, cy, cz, hx), (hy, hz, -, -)
    const float *qs, *qg;         // [n_joints]
    const float *sdf;             // [nz][ny][nx] or null
    int32_t sdf_n[3];
    float sdf_o[3], sdf_inv_h, sdf_h;
    // per block of 2 x 2 x 2 grid cells, a lower bound of every trilinear
    // value computed in the block (null: not in use; the launchers that
    // refresh it from the current grid set it)
    const float *sdf_lb;
    float *sdf_lb_buf;            // the plan's buffer for it (null without a grid)
    int32_t sdf_lbn[3];           // blocks per axis
    // clearance grid over the obstacles' footprints (null: not in use): per
    // cell a lower bound of the horizontal signed distance from any point of
    // the cell to every cylinder (radial term) and every box footprint
    const float *clr;
    float clr_x0, clr_y0, clr_h, clr_inv;
    int32_t clr_nx, clr_ny;
    int32_t lead_frame;           // with clr: frame taken first (1..n), or -1
    // self-collision: frame pairs (fa, fb), fa < fb, sorted, both with
    // spheres; per frame a bounding sphere of its spheres (local centre, radius)
    int32_t n_self;
    const int2 *self_pairs;
    const float4 *frame_bound;    // [n_joints + 1]
    float tip[3];                 // end-effector point in the last frame
    // separating-axis narrow phase (narrow = CP_NARROW_SAT): the link hulls
    // and the scene's oriented boxes, four float4 per box:
    // (cx, cy, cz, hx), (R00, R01, R02, hy), (R10, R11, R12, hz),
    // (R20, R21, R22, frame as int bits; 0 for scene boxes)
    int32_t narrow;
    int32_t n_hulls, n_obb, n_hull_self;
    const float4 *hulls;          // [n_hulls][4], caller order
    const float4 *obb;            // [n_obb][4]
    const int2 *hull_self;        // [n_hull_self] hull pairs (k < m) of listed frame pairs, sorted
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Load through a global-address-space pointer.  Table pointers that reach a
// kernel through device memory (the batched launch) lose their address space,
// which would turn wave-uniform table reads into vector flat loads; loading
// through this helper keeps them scalar (and lane-varying ones global).
// (The host compilation pass also instantiates these templates; it only needs
// a well-formed body, so it gets the plain load.)
template <class T>
__device__ __forceinline__ T ldg(const T *p, int64_t i = 0) {
#if defined(__HIP_DEVICE_COMPILE__)
    T v;
    __builtin_memcpy(&v, (const __attribute__((address_space(1))) T *)p + i, sizeof(T));
    return v;
#else
    return p[i];
#endif
}

// signed distance of a vertical cylinder with radial term a and height term b
// (exact Euclidean SDF of the solid: inside part + outside part)
__device__ __forceinline__ float cyl_combine(float a, float b) {
    float ap = fmaxf(a, 0.0f), bp = fmaxf(b, 0.0f);
    return fminf(fmaxf(a, b), 0.0f) + fsqrt(__builtin_fmaf(ap, ap, bp * bp));
}

__device__ __forceinline__ float cyl_radial(float cx, float cy, float4 c) {
    float dx = cx - c.x, dy = cy - c.y;
    return fsqrt(__builtin_fmaf(dx, dx, dy * dy)) - c.z;
}

__device__ __forceinline__ float box_sd(float cx, float cy, float cz, float4 b0, float4 b1) {
    float qx = fabsf(cx - b0.x) - b0.w;
    float qy = fabsf(cy - b0.y) - b1.x;
    float qz = fabsf(cz - b0.z) - b1.y;
    float px = fmaxf(qx, 0.0f), py = fmaxf(qy, 0.0f), pz = fmaxf(qz, 0.0f);
    float o2 = __builtin_fmaf(px, px, __builtin_fmaf(py, py, pz * pz));
    return fsqrt(o2) + fminf(fmaxf(qx, fmaxf(qy, qz)), 0.0f);
}

// grid cell of a point (clamped to the grid) and its fractional position
__device__ __forceinline__ void sdf_cell(const PlanView &P, float cx, float cy, float cz, int (&i0)[3],
                                         float (&f)[3], float (&dg)[3]) {
    float g[3] = {(cx - P.sdf_o[0]) * P.sdf_inv_h - 0.5f, (cy - P.sdf_o[1]) * P.sdf_inv_h - 0.5f,
                  (cz - P.sdf_o[2]) * P.sdf_inv_h - 0.5f};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float fl = floorf(g[a]);
        float hi = (float)(P.sdf_n[a] - 2);
        float il = fminf(fmaxf(fl, 0.0f), hi);
        float fr = g[a] - il;
        dg[a] = (fr >= 0.0f && fr <= 1.0f) ? 1.0f : 0.0f;
        fr = fminf(fmaxf(fr, 0.0f), 1.0f);
        i0[a] = (int)il;
        f[a] = fr;
    }
}

// lower bound of every primitive obstacle's signed distance at horizontal
// position (x, y), the ground excepted (P.clr set, x and y finite): a
// cylinder's distance is never below its radial term and a box's never below
// the signed distance to its footprint rectangle
//
// A point outside the grid takes the cell of its projection onto the grid's
// rectangle: every obstacle lies inside that rectangle, and projecting onto
// a convex set brings a point no closer to any point of the set.
__device__ __forceinline__ float clearance_bound(const PlanView &P, float x, float y) {
    const int ix = (int)__builtin_amdgcn_fmed3f((x - P.clr_x0) * P.clr_inv, 0.0f, (float)(P.clr_nx - 1));
    const int iy = (int)__builtin_amdgcn_fmed3f((y - P.clr_y0) * P.clr_inv, 0.0f, (float)(P.clr_ny - 1));
    return P.clr[iy * P.clr_nx + ix];
}

// grid cells per bound block along each axis: 1 << kSdfBlockLog2
constexpr int kSdfBlockLog2 = 1;

// lower bound of the trilinear value anywhere in cell i0 (P.sdf_lb set)
__device__ __forceinline__ float sdf_cell_bound(const PlanView &P, const int (&i0)[3]) {
    const int k = kSdfBlockLog2;
    return P.sdf_lb[((size_t)(i0[2] >> k) * P.sdf_lbn[1] + (i0[1] >> k)) * P.sdf_lbn[0] + (i0[0] >> k)];
}

// trilinear interpolation in cell i0 at fractional position f
__device__ __forceinline__ float sdf_interp(const PlanView &P, const int (&i0)[3], const float (&f)[3],
                                           const float (&dg)[3], float *grad) {
    const int nx = P.sdf_n[0], ny = P.sdf_n[1];
    const float *base = P.sdf + ((size_t)i0[2] * ny + i0[1]) * nx + i0[0];
    const size_t sy = nx, sz = (size_t)nx * ny;
    float v000 = base[0], v001 = base[1], v010 = base[sy], v011 = base[sy + 1];
    float v100 = base[sz], v101 = base[sz + 1], v110 = base[sz + sy], v111 = base[sz + sy + 1];
    // interpolate along x, then y, then z
    float c00 = __builtin_fmaf(f[0], v001 - v000, v000);
    float c01 = __builtin_fmaf(f[0], v011 - v010, v010);
    float c10 = __builtin_fmaf(f[0], v101 - v100, v100);
    float c11 = __builtin_fmaf(f[0], v111 - v110, v110);
    float c0 = __builtin_fmaf(f[1], c01 - c00, c00);
    float c1 = __builtin_fmaf(f[1], c11 - c10, c10);
    float phi = __builtin_fmaf(f[2], c1 - c0, c0);
    if (grad) {
        float dx0 = __builtin_fmaf(f[1], (v011 - v010) - (v001 - v000), v001 - v000);
        float dx1 = __builtin_fmaf(f[1], (v111 - v110) - (v101 - v100), v101 - v100);
        float gx = __builtin_fmaf(f[2], dx1 - dx0, dx0);
        float gy = __builtin_fmaf(f[2], c11 - c10 - (c01 - c00), c01 - c00);
        float gz = c1 - c0;
        grad[0] = gx * dg[0] * P.sdf_inv_h;
        grad[1] = gy * dg[1] * P.sdf_inv_h;
        grad[2] = gz * dg[2] * P.sdf_inv_h;
    }
    return phi;
}

// trilinear signed-distance lookup (voxel-centre samples, clamped coordinates)
__device__ __forceinline__ float sdf_query(const PlanView &P, float cx, float cy, float cz, float *grad) {
    int i0[3];
    float f[3], dg[3];
    sdf_cell(P, cx, cy, cz, i0, f, dg);
    return sdf_interp(P, i0, f, dg, grad);
}

// gradient of the signed distance of obstacle o at c (same case split as the
// exact SDFs); returns the signed distance
__device__ __forceinline__ float obstacle_sd_grad(const PlanView &P, uint32_t o, float cx, float cy, float cz,
                                                  float (&gr)[3]) {
    if (o == CP_OBS_SDF) return sdf_query(P, cx, cy, cz, gr);
    if (o == 0) {
        gr[0] = 0.0f; gr[1] = 0.0f; gr[2] = 1.0f;
        return cz - P.ground_z;
    }
    if ((int)o <= P.n_cyl) {
        const float4 c = P.cyl_orig[o - 1];
        const GroupDev g = P.groups[__float_as_int(c.w)];
        float dx = cx - c.x, dy = cy - c.y, dz = cz - g.zc;
        float rho = fsqrt(__builtin_fmaf(dx, dx, dy * dy));
        float a = rho - c.z, b = fabsf(dz) - g.hz;
        float sd = cyl_combine(a, b);
        float inv = rho > 0.0f ? 1.0f / rho : 0.0f;
        float gax = dx * inv, gay = dy * inv, gbz = dz >= 0.0f ? 1.0f : -1.0f;
        if (a > 0.0f && b > 0.0f) {
            float out = sd;  // sqrt(a^2 + b^2) here
            gr[0] = a * gax / out; gr[1] = a * gay / out; gr[2] = b * gbz / out;
        } else if (a > 0.0f || (b <= 0.0f && a >= b)) {
            gr[0] = gax; gr[1] = gay; gr[2] = 0.0f;
        } else {
            gr[0] = 0.0f; gr[1] = 0.0f; gr[2] = gbz;
        }
        return sd;
    }
    const int bi = (int)o - 1 - P.n_cyl;
    const float4 b0 = P.box[2 * bi], b1 = P.box[2 * bi + 1];
    float d[3] = {cx - b0.x, cy - b0.y, cz - b0.z};
    float h[3] = {b0.w, b1.x, b1.y};
    float qv[3], sg[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) { sg[i] = d[i] >= 0.0f ? 1.0f : -1.0f; qv[i] = fabsf(d[i]) - h[i]; }
    float sd = box_sd(cx, cy, cz, b0, b1);
    float px = fmaxf(qv[0], 0.0f), py = fmaxf(qv[1], 0.0f), pz = fmaxf(qv[2], 0.0f);
    float o2 = __builtin_fmaf(px, px, __builtin_fmaf(py, py, pz * pz));
    if (o2 > 0.0f) {
        float inv = 1.0f / fsqrt(o2);
        gr[0] = sg[0] * px * inv; gr[1] = sg[1] * py * inv; gr[2] = sg[2] * pz * inv;
    } else {
        int am = 0;
        if (qv[1] > qv[am]) am = 1;
        if (qv[2] > qv[am]) am = 2;
        gr[0] = am == 0 ? sg[0] : 0.0f;
        gr[1] = am == 1 ? sg[1] : 0.0f;
        gr[2] = am == 2 ? sg[2] : 0.0f;
    }
    return sd;
}

// ---------------------------------------------------------------------------
// uniform cubic B-spline blend on one span (closed form of the degree-3 basis
// on uniform knots) and its backward difference over one checkpoint step h,
// written without cancellation: db_t(u) = b_t(u) - b_t(u - h)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void bspline_blend(float u, float h, float b[4], float db[4]) {
    float v = 1.0f - u;
    float u2 = u * u, v2 = v * v;
    b[0] = v2 * v * (1.0f / 6.0f);
    b[1] = __builtin_fmaf(u2, __builtin_fmaf(0.5f, u, -1.0f), 2.0f / 3.0f);
    b[2] = __builtin_fmaf(v2, __builtin_fmaf(0.5f, v, -1.0f), 2.0f / 3.0f);
    b[3] = u2 * u * (1.0f / 6.0f);
    // cube differences: u^3 - (u-h)^3 = h (3u^2 - 3uh + h^2); v^3 - (v+h)^3 = -h (3v^2 + 3vh + h^2)
    float h2 = h * h;
    float Au = __builtin_fmaf(3.0f * u, u - h, h2);
    float Av = __builtin_fmaf(3.0f * v, v + h, h2);
    float du2 = h * (2.0f * u - h);   // u^2 - (u-h)^2
    db[0] = -h * Av * (1.0f / 6.0f);
    db[3] = h * Au * (1.0f / 6.0f);
    // b1 = u^3/2 - u^2 + 2/3 ; b2 = v^3/2 - v^2 + 2/3 with v = 1 - u
    db[1] = __builtin_fmaf(0.5f * h, Au, -du2);
    float dv2 = -h * (2.0f * v + h);  // v^2 - (v+h)^2
    db[2] = __builtin_fmaf(-0.5f * h, Av, -dv2);
}

// Control point i of path b (B-spline polygon: 3 x start, W, 3 x goal;
// linear polygon: start, W, goal).
__device__ __forceinline__ const float *control_point(const PlanView &P, const float *Wb, int i) {
    const int lead = P.interp == CP_INTERP_BSPLINE ? 3 : 1;
    if (i < lead) return P.qs;
    if (i < lead + P.K) return Wb + (size_t)(i - lead) * P.n_joints;
    return P.qg;
}

// Position of checkpoint k (1..n_s): first control point j of its span
// window, blend weights b[4] and difference weights db[4] so that
//   q_k = sum_t b_t P_{j+t},  q_k - q_{k-1} = sum_t db_t P_{j+t}.
__device__ __forceinline__ void checkpoint_weights(const PlanView &P, int k, int &j, float b[4], float db[4]) {
    j = (k - 1) / P.M;
    int i = k - j * P.M;  // 1..M
    float h = 1.0f / (float)P.M;
    float u = (float)i * h;
    if (P.interp == CP_INTERP_BSPLINE) {
        bspline_blend(u, h, b, db);
    } else {
        b[0] = 1.0f - u; b[1] = u; b[2] = 0.0f; b[3] = 0.0f;
        db[0] = -h; db[1] = h; db[2] = 0.0f; db[3] = 0.0f;
    }
}

__device__ __forceinline__ int n_ctrl_points(const PlanView &P) {
    return P.interp == CP_INTERP_BSPLINE ? P.K + 6 : P.K + 2;
}

// Rigid transform in registers: R row-major, p.
struct Xf {
    float r[9];
    float p[3];
};

__device__ __forceinline__ void xf_identity(Xf &T) {
#pragma unroll
    for (int i = 0; i < 9; ++i) T.r[i] = (i % 4 == 0) ? 1.0f : 0.0f;
    T.p[0] = T.p[1] = T.p[2] = 0.0f;
}

// T <- T * Trans(origin) * Motion(q) for joint J
__device__ __forceinline__ void xf_joint(Xf &T, const JointDev &J, float q) {
    float ox = J.ox, oy = J.oy, oz = J.oz;
    if (J.type == CP_PRISMATIC) {
        ox = __builtin_fmaf(q, J.ax, ox);
        oy = __builtin_fmaf(q, J.ay, oy);
        oz = __builtin_fmaf(q, J.az, oz);
    }
    float np[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        np[i] = __builtin_fmaf(T.r[3 * i], ox, __builtin_fmaf(T.r[3 * i + 1], oy, __builtin_fmaf(T.r[3 * i + 2], oz, T.p[i])));
    T.p[0] = np[0]; T.p[1] = np[1]; T.p[2] = np[2];
    if (J.type == CP_REVOLUTE) {
        float s, c;
        sincosf(q, &s, &c);
        float v = 1.0f - c;
        float x = J.ax, y = J.ay, z = J.az;
        float R[9];
        R[0] = __builtin_fmaf(x * x, v, c);
        R[1] = __builtin_fmaf(x * y, v, -z * s);
        R[2] = __builtin_fmaf(x * z, v, y * s);
        R[3] = __builtin_fmaf(y * x, v, z * s);
        R[4] = __builtin_fmaf(y * y, v, c);
        R[5] = __builtin_fmaf(y * z, v, -x * s);
        R[6] = __builtin_fmaf(z * x, v, -y * s);
        R[7] = __builtin_fmaf(z * y, v, x * s);
        R[8] = __builtin_fmaf(z * z, v, c);
        float nr[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                nr[3 * i + k] = __builtin_fmaf(T.r[3 * i], R[k], __builtin_fmaf(T.r[3 * i + 1], R[3 + k], T.r[3 * i + 2] * R[6 + k]));
#pragma unroll
        for (int i = 0; i < 9; ++i) T.r[i] = nr[i];
    }
}

__device__ __forceinline__ void xf_point(const Xf &T, float lx, float ly, float lz, float &cx, float &cy, float &cz) {
    cx = __builtin_fmaf(T.r[0], lx, __builtin_fmaf(T.r[1], ly, __builtin_fmaf(T.r[2], lz, T.p[0])));
    cy = __builtin_fmaf(T.r[3], lx, __builtin_fmaf(T.r[4], ly, __builtin_fmaf(T.r[5], lz, T.p[1])));
    cz = __builtin_fmaf(T.r[6], lx, __builtin_fmaf(T.r[7], ly, __builtin_fmaf(T.r[8], lz, T.p[2])));
}

// q[j] with a wave-uniform index j (avoids dynamic register indexing)
__device__ __forceinline__ float pick(const float q[CP_MAX_JOINTS], int j) {
    float v = q[0];
#pragma unroll
    for (int i = 1; i < CP_MAX_JOINTS; ++i) v = (j == i) ? q[i] : v;
    return v;
}

__device__ __forceinline__ float hinge_value(const PlanView &P, float d, float &dphi) {
    float m = P.margin, lam = P.lambda_c;
    if (P.hinge == CP_HINGE_HARD) {
        dphi = d < m ? -lam : 0.0f;
        return d < m ? lam * (m - d) : 0.0f;
    }
    if (d < 0.0f) {
        dphi = -lam;
        return lam * (0.5f * m - d);
    }
    if (d < m) {
        float e = m - d;
        dphi = -lam * e / m;
        return lam * e * e / (2.0f * m);
    }
    dphi = 0.0f;
    return 0.0f;
}

// The gradient polish's step on an elite path (a clipped gradient step, which
// the paper does not specify): W' = W - eta g / max(1, |g| / g_max) on the
// sampled joints (|g| over those joints only), the other joints copied,
// applied by the adjoint to each path right after its gradient is complete
// and written to W_out, a buffer distinct from the adjoint's input; W_out
// null: no step.
struct PolishStep {
    float *W_out;                  // [B][K][n] stepped waypoints
    int32_t act[CP_MAX_JOINTS];    // sampled joint ids
    uint32_t act_mask;             // bit j set: joint j is sampled
    float eta, clip;
    int32_t D, n_act;
};

// path b's cost (FP64 sum of its checkpoints' partial sums, in wave order),
// minimum distance and collision flag from the evaluation's partial sums
__device__ __forceinline__ void reduce_one(const double2 *__restrict__ partial, int slots, int ns, float margin,
                                           float *__restrict__ cost, float *__restrict__ min_dist,
                                           uint8_t *__restrict__ flags, int b) {
    const int64_t g0 = (int64_t)b * ns, g1 = g0 + ns - 1;
    double s = 0.0;
    float m = kInf;
    for (int64_t w = g0 / kWave; w <= g1 / kWave; ++w) {
        const int p0 = (int)((w * kWave) / ns);
        const double2 v = partial[w * slots + (b - p0)];
        s += v.x;
        m = fminf(m, (float)v.y);
    }
    cost[b] = (float)s;
    if (min_dist) min_dist[b] = m;
    if (flags) flags[b] = (uint8_t)(m < margin);
}

// order key of a cost: increasing in the cost, -0 equal to +0, and NaN equal
// to +inf (the two then go by index); 0xFFFFFFFF is above every cost's key
__device__ __forceinline__ uint32_t cost_key(float c) {
    if (c != c) return 0xFF800000u;
    if (c == 0.0f) c = 0.0f;
    uint32_t u = __float_as_uint(c);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// a value known to be equal on every lane, moved to scalar registers
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// wave reductions (butterfly over all 64 lanes; fixed order, so deterministic)
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, kWave));
    return v;
}

// Minimum / maximum over the 64 lanes of a wave, returned as a wave-uniform
// value: DPP-fused min/max steps exchange within quads and rows, then the row
// broadcasts (lane 15 into rows 1 and 3, lane 31 into rows 2 and 3) leave the
// total in lane 63.  Six VALU instructions and no LDS traffic.  Every lane of
// the wave must be active; rows that a broadcast leaves out keep their value.
// Each DPP read of a register written by the previous VALU instruction needs
// two wait states, hence the s_nop 1 before every step.  Inputs must not be
// signalling NaNs (they are arithmetic results or constants here).
__device__ __forceinline__ float wave_min_u(float v) {
    asm("s_nop 1\n\t"
        "v_min_f32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_min_f32_dpp %0, %0, %0 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_min_f32_dpp %0, %0, %0 row_half_mirror row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_min_f32_dpp %0, %0, %0 row_mirror row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_min_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_min_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "s_nop 1"
        : "+v"(v));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), kWave - 1));
}
__device__ __forceinline__ float wave_max_u(float v) {
    asm("s_nop 1\n\t"
        "v_max_f32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_max_f32_dpp %0, %0, %0 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_max_f32_dpp %0, %0, %0 row_half_mirror row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_max_f32_dpp %0, %0, %0 row_mirror row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_max_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_max_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "s_nop 1"
        : "+v"(v));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), kWave - 1));
}

// Four independent wave reductions in one sequence: the four chains are
// interleaved, so consecutive DPP reads of one register are four instructions
// apart and need no wait states of their own.  OPn is "min" or "max".
#define CP_DPP4(OA, OB, OC, OD, CTRL)                  \
    "v_" OA "_f32_dpp %0, %0, %0 " CTRL "\n\t"       \
    "v_" OB "_f32_dpp %1, %1, %1 " CTRL "\n\t"       \
    "v_" OC "_f32_dpp %2, %2, %2 " CTRL "\n\t"       \
    "v_" OD "_f32_dpp %3, %3, %3 " CTRL "\n\t"
#define CP_WAVE_REDUCE4(OA, OB, OC, OD, a, b, c, d)                                         \
    asm("s_nop 1\n\t"                                                                    \
        CP_DPP4(OA, OB, OC, OD, "quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf")           \
        CP_DPP4(OA, OB, OC, OD, "quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf")           \
        CP_DPP4(OA, OB, OC, OD, "row_half_mirror row_mask:0xf bank_mask:0xf")               \
        CP_DPP4(OA, OB, OC, OD, "row_mirror row_mask:0xf bank_mask:0xf")                    \
        CP_DPP4(OA, OB, OC, OD, "row_bcast:15 row_mask:0xa bank_mask:0xf")                  \
        CP_DPP4(OA, OB, OC, OD, "row_bcast:31 row_mask:0xc bank_mask:0xf")                  \
        "s_nop 1"                                                                           \
        : "+v"(a), "+v"(b), "+v"(c), "+v"(d))

__device__ __forceinline__ float lane63(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), kWave - 1));
}

// wave-uniform sum of one value (fixed order, so deterministic)
__device__ __forceinline__ float wave_sum_u(float v) {
    asm("s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_half_mirror row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_mirror row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "s_nop 1"
        : "+v"(v));
    return lane63(v);
}

// wave-uniform (min a, max b, min c, max d)
__device__ __forceinline__ void wave_box(float &a, float &b, float &c, float &d) {
    CP_WAVE_REDUCE4("min", "max", "min", "max", a, b, c, d);
    a = lane63(a); b = lane63(b); c = lane63(c); d = lane63(d);
}
// wave-uniform minima / maxima of four values
__device__ __forceinline__ void wave_min4(float &a, float &b, float &c, float &d) {
    CP_WAVE_REDUCE4("min", "min", "min", "min", a, b, c, d);
    a = lane63(a); b = lane63(b); c = lane63(c); d = lane63(d);
}
__device__ __forceinline__ void wave_max4(float &a, float &b, float &c, float &d) {
    CP_WAVE_REDUCE4("max", "max", "max", "max", a, b, c, d);
    a = lane63(a); b = lane63(b); c = lane63(c); d = lane63(d);
}

// min(a, b) as one v_min_f32, for operands known not to be signalling NaNs
// (fminf adds a canonicalising instruction when it cannot prove that).
__device__ __forceinline__ float fmin_q(float a, float b) {
    float r;
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// ---------------------------------------------------------------------------
// every sphere-obstacle pair of G sphere centres per lane, obstacle records
// wave-uniform (the path evaluation's plain and lane-filtered modes, and the
// inverse kinematics' distance)
// ---------------------------------------------------------------------------

// Four cylinders against G spheres: running minimum of (radial distance - R).
template <int G>
__device__ __forceinline__ void cyl_chunk(const float (&cx)[G], const float (&cy)[G], const float4 *c, float (&a)[G]) {
    const float4 c0 = ldg(c, 0), c1 = ldg(c, 1), c2 = ldg(c, 2), c3 = ldg(c, 3);
#pragma unroll
    for (int s = 0; s < G; ++s) {
        float r0 = cyl_radial(cx[s], cy[s], c0);
        float r1 = cyl_radial(cx[s], cy[s], c1);
        float r2 = cyl_radial(cx[s], cy[s], c2);
        float r3 = cyl_radial(cx[s], cy[s], c3);
        a[s] = fminf(a[s], fminf(fminf(r0, r1), fminf(r2, r3)));
    }
}

// Same result with the square root taken only where it can matter: a pair
// lowers the running minimum a only if rho - R < a, which needs
// rho^2 < (a + R_max)^2.  The threshold carries 1e-4 m plus a relative 1e-6
// of slack, far above the rounding of the threshold and of the square root
// (both a few 1e-7 relative), so rounding never hides a pair that would lower
// a; pairs that are skipped cannot change the minimum, so the result is
// bitwise that of cyl_chunk.
// The test is a wave-wide ballot (compares OR-ed in scalar registers) and the
// candidate block runs for the whole wave when any lane has a candidate:
// lanes without one only recompute values that cannot lower their minimum.
// Per skipped pair this costs two subtractions, a multiply, a multiply-add and
// a compare, all in 32-bit (VOP2/VOPC) encodings, instead of the same four
// operations plus a square root, a subtraction and a minimum.
constexpr float kRelSlack = 1.000001f;

template <int G>
__device__ __forceinline__ void cyl_chunk_filtered(const float (&cx)[G], const float (&cy)[G], const float4 *c,
                                                   float (&a)[G], float (&thr)[G], float reach) {
    const float4 cc[4] = {ldg(c, 0), ldg(c, 1), ldg(c, 2), ldg(c, 3)};
    float d2[G][4];
    uint64_t need = 0;
#pragma unroll
    for (int s = 0; s < G; ++s)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            float dx = cx[s] - cc[u].x, dy = cy[s] - cc[u].y;
            d2[s][u] = __builtin_fmaf(dx, dx, dy * dy);
            need |= __builtin_amdgcn_ballot_w64(d2[s][u] < thr[s]);
        }
    if (need) {
#pragma unroll
        for (int s = 0; s < G; ++s) {
            // fsqrt(d2) - R is exactly cyl_radial of the pair
            float r0 = fsqrt(d2[s][0]) - cc[0].z, r1 = fsqrt(d2[s][1]) - cc[1].z;
            float r2 = fsqrt(d2[s][2]) - cc[2].z, r3 = fsqrt(d2[s][3]) - cc[3].z;
            a[s] = fminf(a[s], fminf(fminf(r0, r1), fminf(r2, r3)));
            float t = fmaxf(a[s] + reach, 0.0f) * kRelSlack;
            thr[s] = t * t;
        }
    }
}

__device__ __forceinline__ float first_lane(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Minimum signed distance over the primitive obstacles (ground, cylinders,
// boxes) for G sphere centres; the grid term is taken by the caller.
template <int G>
__device__ __forceinline__ void spheres_min_sd(const PlanView &P, const float (&cx)[G], const float (&cy)[G],
                                               const float (&cz)[G], float (&v)[G]) {
#pragma unroll
    for (int s = 0; s < G; ++s) v[s] = P.has_ground ? cz[s] - P.ground_z : kInf;
    for (int g = 0; g < P.n_groups; ++g) {
        const GroupDev gr = ldg(P.groups, g);
        const float4 *c = P.cyl + gr.start;
        float a[G];
#pragma unroll
        for (int s = 0; s < G; ++s) a[s] = kInf;
        if (P.pair_filter) {
            // start at the cylinders around the azimuth of the wave's first sphere
            const float ang = atan2f(first_lane(cy[0]), first_lane(cx[0]));
            int bin = (int)((ang + 3.14159265f) * (kAngleBins / 6.28318531f));
            bin = min(max(bin, 0), kAngleBins - 1);
            const int start = ldg(P.angle_start, g * kAngleBins + bin);
            const float reach = gr.rmax + 1e-4f;
            float thr[G];
#pragma unroll
            for (int s = 0; s < G; ++s) thr[s] = kInf;
            for (int o = start; o < gr.count; o += 4) cyl_chunk_filtered<G>(cx, cy, c + o, a, thr, reach);
            for (int o = 0; o < start; o += 4) cyl_chunk_filtered<G>(cx, cy, c + o, a, thr, reach);
        } else {
            for (int o = 0; o < gr.count; o += 4) cyl_chunk<G>(cx, cy, c + o, a);
        }
#pragma unroll
        for (int s = 0; s < G; ++s) v[s] = fminf(v[s], cyl_combine(a[s], fabsf(cz[s] - gr.zc) - gr.hz));
    }
    for (int o = 0; o < P.n_box; ++o) {
        const float4 b0 = ldg(P.box, 2 * o), b1 = ldg(P.box, 2 * o + 1);
#pragma unroll
        for (int s = 0; s < G; ++s) v[s] = fminf(v[s], box_sd(cx[s], cy[s], cz[s], b0, b1));
    }
}

// ---------------------------------------------------------------------------
// one configuration per lane: interpolation, per-checkpoint terms, per-path sums
// ---------------------------------------------------------------------------

// Configuration of checkpoint k of path b: q (all joints) and the step
// q_k - q_{k-1}; also the span window start j and the weights.
__device__ __forceinline__ void interpolate(const PlanView &P, const float *Wb, int k, float (&q)[CP_MAX_JOINTS],
                                            float (&dq)[CP_MAX_JOINTS], int &j, float (&bw)[4], float (&db)[4]) {
    checkpoint_weights(P, k, j, bw, db);
    const float *p0 = control_point(P, Wb, j), *p1 = control_point(P, Wb, j + 1);
    const float *p2 = control_point(P, Wb, j + 2), *p3 = control_point(P, Wb, j + 3);
#pragma unroll
    for (int i = 0; i < CP_MAX_JOINTS; ++i) {
        if (i < P.n_joints) {
            float a0 = ldg(p0, i), a1 = ldg(p1, i), a2 = ldg(p2, i), a3 = ldg(p3, i);
            q[i] = __builtin_fmaf(bw[0], a0, __builtin_fmaf(bw[1], a1, __builtin_fmaf(bw[2], a2, bw[3] * a3)));
            // differences centred on the second control point (the db sum to zero)
            dq[i] = __builtin_fmaf(db[0], a0 - a1, __builtin_fmaf(db[2], a2 - a1, db[3] * (a3 - a1)));
        } else {
            q[i] = 0.0f;
            dq[i] = 0.0f;
        }
    }
}

// J_p and J_l terms of one checkpoint
__device__ __forceinline__ void step_terms(const PlanView &P, const float (&q)[CP_MAX_JOINTS],
                                           const float (&dq)[CP_MAX_JOINTS], float &jp, float &jl) {
    float sq = 0.0f, lim = 0.0f;
#pragma unroll
    for (int i = 0; i < CP_MAX_JOINTS; ++i) {
        if (i < P.n_joints) {
            sq = __builtin_fmaf(dq[i], dq[i], sq);
            const JointDev J = ldg(P.joints, i);
            float hi = fmaxf(q[i] - J.qmax, 0.0f), lo = fmaxf(J.qmin - q[i], 0.0f);
            lim = __builtin_fmaf(hi, hi, __builtin_fmaf(lo, lo, lim));
        }
    }
    jp = P.jp_mode == CP_JP_SQUARED ? sq : fsqrt(sq);
    jl = lim;
}

// Per-path sums of a wave: lane l holds checkpoint cost c and distance d of
// path b (b = -1: a lane past the end); the wave covers paths p0..p1 and
// writes, per path, the FP64 sum of its lanes' costs and their minimum
// distance to partial[w * slots + (p - p0)] (fixed-order reductions).
__device__ __forceinline__ void path_partials(int b, float c, float d, int p0, int p1, int64_t w,
                                              double2 *__restrict__ partial, int slots) {
    if (b < 0) { c = 0.0f; d = kInf; }
    for (int p = p0; p <= p1; ++p) {
        double s = wave_sum_d(b == p ? (double)c : 0.0);
        float m = wave_min(b == p ? d : kInf);
        if ((threadIdx.x & (kWave - 1)) == 0) partial[w * slots + (p - p0)] = make_double2(s, (double)m);
    }
}

}  // namespace cp
