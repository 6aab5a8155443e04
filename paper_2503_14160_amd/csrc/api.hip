// C ABI of the craneplan library: argument validation, plan / optimizer
// objects and their device tables, and the step sequencing of Algorithm 1.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <atomic>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "launch.h"

using namespace cp;

namespace {

thread_local std::string g_err;
// an error a HIP call made before the current entry point had left behind
// (the launch checks read the thread's last error, so it is taken first)
thread_local hipError_t g_stale = hipSuccess;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    std::string msg = std::string(what) + ": " + hipGetErrorString(e);
    if (g_stale != hipSuccess)
        msg += std::string(" (an earlier HIP call on this thread, before this entry point, had failed with: ") +
               hipGetErrorString(g_stale) + ")";
    return fail(e == hipErrorOutOfMemory ? CP_ERR_NOMEM : CP_ERR_HIP, msg);
}

// takes any error left by earlier HIP calls, so the checks of this entry
// point's launches see their own
void take_stale_error() { g_stale = hipGetLastError(); }

#define CP_HIP(call, what)                               \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// makes the object's device current for the duration of a call
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        take_stale_error();
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

template <class T>
hipError_t upload(T **dst, const std::vector<T> &src) {
    *dst = nullptr;
    const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
    hipError_t e = hipMalloc((void **)dst, bytes);
    if (e != hipSuccess) return e;
    if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

bool finite(float x) { return std::isfinite(x); }

// CP_PAIRS_AUTO: the wave-level culling pays off from a few dozen obstacles on
// (measured crossover between 32 and 64 for a 64-sphere crane)
constexpr int kAutoCullObstacles = 48;
int resolve_pairs(int mode, int n_obstacles) {
    if (mode != CP_PAIRS_AUTO) return mode;
    return n_obstacles >= kAutoCullObstacles ? CP_PAIRS_WAVE : CP_PAIRS_LANE;
}

// Scratch of the allocation-free evaluation (cp_eval_paths_noalloc): the
// per-wave partial sums of one evaluation, in a static array that every GPU
// the library runs on holds until the process ends.  In host code `scratch`
// is only a stand-in for the symbol: its device address, per device, comes
// from hipGetSymbolAddress at plan creation and is the only way host code
// refers to this memory.
constexpr size_t kNoAllocScratchBytes = (size_t)24 << 20;
static __device__ __align__(256) double2 scratch[kNoAllocScratchBytes / sizeof(double2)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double2 *g_scratch_ptr[kMaxDevices] = {};

// the address of `scratch` on `dev`, which must be the current device
hipError_t scratch_on(int dev, double2 **out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double2 *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

struct cp_plan {
    // the caller's handle plus one per optimizer created on the plan: the
    // plan is freed when the last of them lets go (cp_plan_destroy and
    // cp_optimizer_destroy may come in either order)
    std::atomic<int> refs{1};
    int device = 0;
    int n = 0, S = 0, K = 0, M = 0, ns = 0, max_B = 0;
    int n_cyl = 0, n_box = 0;
    cp_cost_params cost{};
    std::vector<JointDev> joints;
    JointDev *d_joints = nullptr;
    SphereDev *d_spheres = nullptr;
    int32_t *d_sphere_slot = nullptr;
    int32_t *d_frame_start = nullptr;
    float4 *d_cyl = nullptr;
    float4 *d_cyl_cell = nullptr;
    int32_t *d_cell_start = nullptr;
    int32_t *d_hint = nullptr;
    GroupDev *d_groups = nullptr;
    int2 *d_self_pairs = nullptr;
    float4 *d_frame_bound = nullptr;
    int32_t *d_angle_start = nullptr;
    float4 *d_cyl_orig = nullptr;
    float4 *d_box = nullptr;
    float *d_qs = nullptr, *d_qg = nullptr;
    double2 *d_partial = nullptr;
    float *d_sdf_lb = nullptr;
    float *d_clr = nullptr;
    float4 *d_hulls = nullptr, *d_obb = nullptr;
    int2 *d_hull_self = nullptr;
    PlanView view{};

    ~cp_plan() {
        DeviceGuard g(device);
        void *bufs[] = {d_joints, d_spheres, d_sphere_slot, d_frame_start, d_cyl,  d_cyl_cell, d_cell_start, d_hint, d_groups,
                        d_angle_start, d_cyl_orig, d_box, d_qs, d_qg, d_partial, d_sdf_lb, d_clr,
                        d_self_pairs, d_frame_bound, d_hulls, d_obb, d_hull_self};
        for (void *p : bufs)
            if (p) (void)hipFree(p);
    }
};

struct cp_opt {
    cp_plan *plan = nullptr;
    cp_opt_params prm{};
    int D = 0, n_act = 0, npol = 0;
    OptView view{};
    uint32_t *d_tape_p = nullptr;
    std::vector<void *> bufs;
    // the population's argmin tape and unit path weights (cp_optimizer_record_tape)
    uint32_t *d_tape = nullptr;
    float *d_ones_B = nullptr;
    // evaluation timing (cp_optimizer_time_eval): one event pair per timed
    // evaluation launch, used in order until cp_optimizer_eval_time reads them
    std::vector<EvalEvents> ev;
    size_t ev_used = 0;

    void drop_events() {
        for (EvalEvents &e : ev) {
            (void)hipEventDestroy(e.begin);
            (void)hipEventDestroy(e.end);
        }
        ev.clear();
        ev_used = 0;
    }
    void drop_tape() {
        if (d_tape) (void)hipFree(d_tape);
        if (d_ones_B) (void)hipFree(d_ones_B);
        d_tape = nullptr;
        d_ones_B = nullptr;
    }
    ~cp_opt() {
        DeviceGuard g(plan->device);
        (void)hipDeviceSynchronize();
        drop_events();
        drop_tape();
        for (void *p : bufs)
            if (p) (void)hipFree(p);
    }
    // the next event pair, or null when timing is off or every pair is in use
    const EvalEvents *next_events() { return ev_used < ev.size() ? &ev[ev_used++] : nullptr; }
    template <class T>
    hipError_t alloc(T **p, size_t count) {
        *p = nullptr;
        hipError_t e = hipMalloc((void **)p, std::max<size_t>(1, count) * sizeof(T));
        if (e == hipSuccess) bufs.push_back((void *)*p);
        return e;
    }
};

extern "C" {

const char *cp_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------

static int validate_plan_args(const cp_robot_desc *r, const cp_scene_desc *s, const cp_cost_params *c) {
    if (!r || !s || !c) return fail(CP_ERR_INVALID_ARG, "null descriptor");
    if (r->n_joints < 1 || r->n_joints > CP_MAX_JOINTS) return fail(CP_ERR_SIZE, "n_joints out of range");
    if (!r->type || !r->axis || !r->origin || !r->q_min || !r->q_max || !r->q_hold || !r->active)
        return fail(CP_ERR_INVALID_ARG, "null joint table");
    for (int j = 0; j < r->n_joints; ++j) {
        if (r->type[j] != CP_REVOLUTE && r->type[j] != CP_PRISMATIC) return fail(CP_ERR_INVALID_ARG, "bad joint type");
        const float *a = r->axis + 3 * j;
        const double nrm = std::sqrt((double)a[0] * a[0] + (double)a[1] * a[1] + (double)a[2] * a[2]);
        if (!(std::fabs(nrm - 1.0) < 1e-4)) return fail(CP_ERR_INVALID_ARG, "joint axis is not a unit vector");
        for (int i = 0; i < 3; ++i)
            if (!finite(r->origin[3 * j + i])) return fail(CP_ERR_INVALID_ARG, "non-finite joint origin");
        if (!finite(r->q_min[j]) || !finite(r->q_max[j]) || !(r->q_min[j] <= r->q_max[j]) || !finite(r->q_hold[j]))
            return fail(CP_ERR_INVALID_ARG, "bad joint limits");
    }
    if (r->n_spheres < 1 || r->n_spheres > CP_MAX_SPHERES) return fail(CP_ERR_SIZE, "n_spheres out of range");
    if (!r->sphere_frame || !r->sphere_center || !r->sphere_radius) return fail(CP_ERR_INVALID_ARG, "null sphere table");
    for (int i = 0; i < r->n_spheres; ++i) {
        if (r->sphere_frame[i] < 0 || r->sphere_frame[i] > r->n_joints) return fail(CP_ERR_INVALID_ARG, "bad sphere frame");
        if (!(r->sphere_radius[i] > 0.0f) || !finite(r->sphere_radius[i])) return fail(CP_ERR_INVALID_ARG, "bad sphere radius");
    }
    if (r->n_self_pairs < 0 || r->n_self_pairs > 64) return fail(CP_ERR_SIZE, "n_self_pairs out of range (0..64)");
    if (r->n_self_pairs > 0 && !r->self_pairs) return fail(CP_ERR_INVALID_ARG, "null self_pairs");
    for (int i = 0; i < r->n_self_pairs; ++i) {
        const int a = r->self_pairs[2 * i], b = r->self_pairs[2 * i + 1];
        if (a < 0 || a > r->n_joints || b < 0 || b > r->n_joints || a == b)
            return fail(CP_ERR_INVALID_ARG, "bad self-collision frame pair");
    }
    for (int i = 0; i < 3; ++i)
        if (!finite(r->tip[i])) return fail(CP_ERR_INVALID_ARG, "non-finite tip");
    // obstacle numbers stay below CP_OBS_SELF
    if (s->n_cyl < 0 || s->n_box < 0 || s->n_cyl + s->n_box > (int)CP_OBS_SELF - 1)
        return fail(CP_ERR_SIZE, "obstacle count out of range");
    if ((s->n_cyl > 0 && !s->cyl) || (s->n_box > 0 && !s->box)) return fail(CP_ERR_INVALID_ARG, "null obstacle table");
    for (int o = 0; o < s->n_cyl; ++o) {
        const float *y = s->cyl + 5 * o;
        for (int i = 0; i < 5; ++i)
            if (!finite(y[i])) return fail(CP_ERR_INVALID_ARG, "non-finite cylinder");
        if (!(y[2] >= 0.0f) || !(y[4] >= y[3])) return fail(CP_ERR_INVALID_ARG, "bad cylinder");
    }
    for (int o = 0; o < s->n_box; ++o) {
        const float *y = s->box + 6 * o;
        for (int i = 0; i < 6; ++i)
            if (!finite(y[i])) return fail(CP_ERR_INVALID_ARG, "non-finite box");
        if (!(y[3] >= 0.0f && y[4] >= 0.0f && y[5] >= 0.0f)) return fail(CP_ERR_INVALID_ARG, "bad box");
    }
    if (s->d_sdf) {
        for (int a = 0; a < 3; ++a)
            if (s->sdf_dims[a] < 2) return fail(CP_ERR_SIZE, "sdf dims must be >= 2");
        if (!(s->voxel > 0.0f)) return fail(CP_ERR_INVALID_ARG, "sdf voxel must be > 0");
    }
    if (s->narrow != CP_NARROW_SPHERES && s->narrow != CP_NARROW_SAT) return fail(CP_ERR_INVALID_ARG, "bad narrow");
    if (r->n_hulls < 0 || r->n_hulls > CP_MAX_HULLS) return fail(CP_ERR_SIZE, "n_hulls out of range");
    if (r->n_hulls > 0 && (!r->hull_frame || !r->hull_box)) return fail(CP_ERR_INVALID_ARG, "null hull table");
    if (s->n_obb < 0 || s->n_obb > (int)CP_OBS_SELF - 1) return fail(CP_ERR_SIZE, "n_obb out of range");
    if (s->n_obb > 0 && !s->obb) return fail(CP_ERR_INVALID_ARG, "null obb table");
    if (s->narrow == CP_NARROW_SAT && r->n_hulls < 1)
        return fail(CP_ERR_INVALID_ARG, "the SAT narrow phase needs the robot's hulls");
    if (s->narrow == CP_NARROW_SAT && s->d_sdf) return fail(CP_ERR_INVALID_ARG, "the SAT narrow phase takes no grid");
    for (int k = 0; k < r->n_hulls + s->n_obb; ++k) {
        const bool hull = k < r->n_hulls;
        const float *b = hull ? r->hull_box + 15 * k : s->obb + 15 * (k - r->n_hulls);
        if (hull && (r->hull_frame[k] < 0 || r->hull_frame[k] > r->n_joints))
            return fail(CP_ERR_INVALID_ARG, "bad hull frame");
        for (int i = 0; i < 15; ++i)
            if (!finite(b[i])) return fail(CP_ERR_INVALID_ARG, "non-finite box");
        if (!(b[12] > 0.0f && b[13] > 0.0f && b[14] > 0.0f)) return fail(CP_ERR_INVALID_ARG, "box half extents must be > 0");
        // the rotation must be orthonormal (R^T R = I)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double d = 0.0;
                for (int m = 0; m < 3; ++m) d += (double)b[3 + 3 * m + i] * b[3 + 3 * m + j];
                if (std::fabs(d - (i == j ? 1.0 : 0.0)) > 1e-4)
                    return fail(CP_ERR_INVALID_ARG, "box rotation is not orthonormal");
            }
    }
    if (c->K < 1 || c->K > CP_MAX_K || c->M < 1) return fail(CP_ERR_SIZE, "K or M out of range");
    if (c->interp != CP_INTERP_BSPLINE && c->interp != CP_INTERP_LINEAR) return fail(CP_ERR_INVALID_ARG, "bad interp");
    if (c->jp_mode != CP_JP_SQUARED && c->jp_mode != CP_JP_L2) return fail(CP_ERR_INVALID_ARG, "bad jp_mode");
    if (c->hinge != CP_HINGE_HARD && c->hinge != CP_HINGE_SMOOTH) return fail(CP_ERR_INVALID_ARG, "bad hinge");
    if (c->pair_filter < CP_PAIRS_ALL || c->pair_filter > CP_PAIRS_AUTO)
        return fail(CP_ERR_INVALID_ARG, "bad pair_filter");
    if (!(c->margin >= 0.0f) || (c->hinge == CP_HINGE_SMOOTH && !(c->margin > 0.0f)))
        return fail(CP_ERR_INVALID_ARG, "bad margin");
    if (!finite(c->lambda_c) || !finite(c->w_c) || !finite(c->w_l)) return fail(CP_ERR_INVALID_ARG, "bad weights");
    if (c->max_B < 1) return fail(CP_ERR_SIZE, "max_B must be >= 1");
    const int64_t ns = (int64_t)(c->interp == CP_INTERP_BSPLINE ? c->K + 3 : c->K + 1) * c->M;
    if (ns > (1 << 24) || (int64_t)c->max_B * ns > ((int64_t)1 << 31) - 256)
        return fail(CP_ERR_SIZE, "max_B * n_s exceeds 2^31");
    return CP_OK;
}

int cp_plan_create(const cp_robot_desc *robot, const cp_scene_desc *scene, const cp_cost_params *cost, int device,
                   cp_plan **out) {
    if (!out) return fail(CP_ERR_INVALID_ARG, "null out");
    *out = nullptr;
    int rc = validate_plan_args(robot, scene, cost);
    if (rc) return rc;
    int ndev = 0;
    CP_HIP(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(CP_ERR_INVALID_ARG, "bad device");
    DeviceGuard guard(device);
    {
        // the allocation-free evaluation's scratch address on this device
        double2 *sp = nullptr;
        CP_HIP(scratch_on(device, &sp), "scratch address");
    }
    cp_plan *p = new (std::nothrow) cp_plan();
    if (!p) return fail(CP_ERR_NOMEM, "host allocation");
    p->device = device;
    p->n = robot->n_joints;
    p->S = robot->n_spheres;
    p->K = cost->K;
    p->M = cost->M;
    p->ns = (cost->interp == CP_INTERP_BSPLINE ? cost->K + 3 : cost->K + 1) * cost->M;
    p->max_B = cost->max_B;
    p->cost = *cost;
    p->n_cyl = scene->n_cyl;
    p->n_box = scene->n_box;
    auto bail = [&](int code) {
        delete p;
        return code;
    };

    // joints
    for (int j = 0; j < p->n; ++j) {
        JointDev J{};
        J.type = robot->type[j];
        J.ax = robot->axis[3 * j]; J.ay = robot->axis[3 * j + 1]; J.az = robot->axis[3 * j + 2];
        J.ox = robot->origin[3 * j]; J.oy = robot->origin[3 * j + 1]; J.oz = robot->origin[3 * j + 2];
        J.qmin = robot->q_min[j]; J.qmax = robot->q_max[j]; J.qhold = robot->q_hold[j];
        J.active = robot->active[j] ? 1 : 0;
        p->joints.push_back(J);
    }
    // spheres sorted by frame (stable), with per-frame ranges
    std::vector<int> order(p->S);
    for (int i = 0; i < p->S; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return robot->sphere_frame[a] < robot->sphere_frame[b]; });
    std::vector<SphereDev> spheres;
    for (int i : order) {
        SphereDev s{};
        s.lx = robot->sphere_center[3 * i]; s.ly = robot->sphere_center[3 * i + 1]; s.lz = robot->sphere_center[3 * i + 2];
        s.r = robot->sphere_radius[i];
        s.frame = robot->sphere_frame[i];
        s.orig = i;
        spheres.push_back(s);
    }
    std::vector<int32_t> sphere_slot(p->S);
    for (int k = 0; k < p->S; ++k) sphere_slot[spheres[k].orig] = k;
    std::vector<int32_t> frame_start(p->n + 2, 0);
    for (int f = 0; f <= p->n + 1; ++f) {
        int c = 0;
        for (const SphereDev &s : spheres) c += s.frame < f;
        frame_start[f] = c;
    }
    // cylinders grouped by shared vertical extent, each group padded to a
    // multiple of 4 with far-away zero-radius entries
    std::vector<std::pair<float, float>> ext;
    std::vector<std::vector<int>> members;
    std::vector<float4> cyl_orig(p->n_cyl);
    for (int o = 0; o < p->n_cyl; ++o) {
        const float *y = scene->cyl + 5 * o;
        std::pair<float, float> e(y[3], y[4]);
        int g = -1;
        for (size_t i = 0; i < ext.size(); ++i)
            if (ext[i] == e) { g = (int)i; break; }
        if (g < 0) {
            g = (int)ext.size();
            ext.push_back(e);
            members.emplace_back();
        }
        members[g].push_back(o);
        int gbits;
        std::memcpy(&gbits, &g, sizeof(int));
        float gf;
        std::memcpy(&gf, &gbits, sizeof(float));
        cyl_orig[o] = make_float4(y[0], y[1], y[2], gf);
    }
    // within a group, cylinders sorted by polar angle about the z axis, with a
    // per-azimuth-bin scan start (one bin behind, aligned to the chunk of 4)
    std::vector<float4> cyl, cyl_cell;
    std::vector<GroupDev> groups;
    std::vector<int32_t> angle_start, cell_start, hint;
    const double kPi = 3.14159265358979323846;
    for (size_t g = 0; g < ext.size(); ++g) {
        GroupDev G{};
        G.start = (int)cyl.size();
        std::vector<std::pair<double, int>> by_angle;
        float rmax = 0.0f;
        for (int o : members[g]) {
            const float *y = scene->cyl + 5 * o;
            by_angle.emplace_back(std::atan2((double)y[1], (double)y[0]), o);
            rmax = std::max(rmax, y[2]);
        }
        std::stable_sort(by_angle.begin(), by_angle.end(),
                         [](const std::pair<double, int> &a, const std::pair<double, int> &b) { return a.first < b.first; });
        for (const auto &ao : by_angle) {
            const float *y = scene->cyl + 5 * ao.second;
            cyl.push_back(make_float4(y[0], y[1], y[2], 0.0f));
        }
        while ((cyl.size() - G.start) % 4) cyl.push_back(make_float4(1e15f, 1e15f, 0.0f, 0.0f));
        G.count = (int)cyl.size() - G.start;
        G.zc = (float)(0.5 * ((double)ext[g].first + (double)ext[g].second));
        G.hz = (float)(0.5 * ((double)ext[g].second - (double)ext[g].first));
        G.rmax = rmax;
        // the grid: about three cylinder centres per cell, at most 256 cells per axis
        double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
        for (int o : members[g]) {
            const float *y = scene->cyl + 5 * o;
            x0 = std::min(x0, (double)y[0]); x1 = std::max(x1, (double)y[0]);
            y0 = std::min(y0, (double)y[1]); y1 = std::max(y1, (double)y[1]);
        }
        const double gw = x1 - x0, gd = y1 - y0;
        double h = std::sqrt(std::max(gw * gd, 1e-6) * 3.0 / (double)members[g].size());
        h = std::max({h, 1e-3, gw / 255.0, gd / 255.0});
        const int nx = std::min(256, (int)std::floor(gw / h) + 1), ny = std::min(256, (int)std::floor(gd / h) + 1);
        std::vector<std::pair<int, int>> by_cell;  // (cell, caller index), stable in caller order
        for (int o : members[g]) {
            const float *y = scene->cyl + 5 * o;
            const int ix = std::min(nx - 1, std::max(0, (int)std::floor(((double)y[0] - x0) / h)));
            const int iy = std::min(ny - 1, std::max(0, (int)std::floor(((double)y[1] - y0) / h)));
            by_cell.emplace_back(iy * nx + ix, o);
        }
        std::stable_sort(by_cell.begin(), by_cell.end(),
                         [](const std::pair<int, int> &a, const std::pair<int, int> &b) { return a.first < b.first; });
        G.gx0 = (float)x0; G.gy0 = (float)y0;
        G.gh = (float)h; G.ginv = (float)(1.0 / h);
        G.gnx = nx; G.gny = ny;
        G.gcell = (int)cell_start.size();
        size_t next = 0;
        for (int c = 0; c <= nx * ny; ++c) {
            while (next < by_cell.size() && by_cell[next].first < c) ++next;
            cell_start.push_back(G.start + (int)next);
        }
        for (const auto &co : by_cell) {
            const float *y = scene->cyl + 5 * co.second;
            float idx_bits;  // the caller's index, as integer bits
            std::memcpy(&idx_bits, &co.second, sizeof(float));
            cyl_cell.push_back(make_float4(y[0], y[1], y[2], idx_bits));
        }
        // hints: a square grid over the cylinders' extent plus 10 m on every
        // side, about four cells per cylinder cell edge (at most 128 per axis);
        // per cell the cylinder minimising (distance to the centre - R), found
        // among the 5 x 5 cylinder cells around it, else among all
        {
            const double span = std::max(gw, gd) + 20.0;
            const double hh = std::max(h / 4.0, span / 128.0);
            const int hn = std::min(128, (int)std::ceil(span / hh));
            const double hx0 = 0.5 * (x0 + x1) - 0.5 * hn * hh, hy0 = 0.5 * (y0 + y1) - 0.5 * hn * hh;
            G.hx0 = (float)hx0; G.hy0 = (float)hy0;
            G.hinv = (float)(1.0 / hh);
            G.hn = hn;
            G.hoff = (int)hint.size();
            const int n_mem = (int)by_cell.size();
            for (int iy = 0; iy < hn; ++iy)
                for (int ix = 0; ix < hn; ++ix) {
                    const double px = hx0 + (ix + 0.5) * hh, py = hy0 + (iy + 0.5) * hh;
                    const int cx = std::min(nx - 1, std::max(0, (int)std::floor((px - x0) / h)));
                    const int cy = std::min(ny - 1, std::max(0, (int)std::floor((py - y0) / h)));
                    double best = HUGE_VAL;
                    int arg = 0;
                    auto visit = [&](int c) {
                        const float *y = scene->cyl + 5 * by_cell[c].second;
                        const double d = std::hypot(px - y[0], py - y[1]) - y[2];
                        if (d < best) { best = d; arg = c; }
                    };
                    for (int jy = std::max(0, cy - 2); jy <= std::min(ny - 1, cy + 2); ++jy)
                        for (int jx = std::max(0, cx - 2); jx <= std::min(nx - 1, cx + 2); ++jx)
                            for (int c = cell_start[G.gcell + jy * nx + jx] - G.start;
                                 c < cell_start[G.gcell + jy * nx + jx + 1] - G.start; ++c)
                                visit(c);
                    if (best == HUGE_VAL)
                        for (int c = 0; c < n_mem; ++c) visit(c);
                    hint.push_back(G.start + arg);
                }
        }
        while (cyl_cell.size() < cyl.size()) cyl_cell.push_back(make_float4(1e15f, 1e15f, 0.0f, 0.0f));
        groups.push_back(G);
        for (int b = 0; b < kAngleBins; ++b) {
            const double lo = -kPi + (b - 1) * (2.0 * kPi / kAngleBins);
            int first = 0;
            while (first < (int)by_angle.size() && by_angle[first].first < lo) ++first;
            if (first >= (int)by_angle.size()) first = 0;
            angle_start.push_back(first & ~3);
        }
    }
    if (angle_start.empty()) angle_start.assign(kAngleBins, 0);
    if (cell_start.empty()) cell_start.assign(1, 0);
    if (hint.empty()) hint.assign(1, 0);
    const int pair_filter = resolve_pairs(cost->pair_filter, p->n_cyl + p->n_box);
    std::vector<float4> box;
    for (int o = 0; o < p->n_box; ++o) {
        const float *y = scene->box + 6 * o;
        box.push_back(make_float4(y[0], y[1], y[2], y[3]));
        box.push_back(make_float4(y[4], y[5], 0.0f, 0.0f));
    }
    // self-collision: frame pairs (fa < fb) with spheres on both, sorted and
    // unique; per frame the bounding sphere of its spheres (centre of their
    // box, radius rounded up)
    std::vector<int2> self_pairs;
    for (int i = 0; i < robot->n_self_pairs; ++i) {
        const int a = std::min(robot->self_pairs[2 * i], robot->self_pairs[2 * i + 1]);
        const int b = std::max(robot->self_pairs[2 * i], robot->self_pairs[2 * i + 1]);
        if (frame_start[a + 1] == frame_start[a] || frame_start[b + 1] == frame_start[b]) continue;
        self_pairs.push_back(make_int2(a, b));
    }
    std::sort(self_pairs.begin(), self_pairs.end(),
              [](const int2 &u, const int2 &w) { return u.x != w.x ? u.x < w.x : u.y < w.y; });
    self_pairs.erase(std::unique(self_pairs.begin(), self_pairs.end(),
                                 [](const int2 &u, const int2 &w) { return u.x == w.x && u.y == w.y; }),
                     self_pairs.end());
    std::vector<float4> frame_bound(p->n + 1, make_float4(0.0f, 0.0f, 0.0f, 0.0f));
    for (int f = 0; f <= p->n; ++f) {
        if (frame_start[f + 1] == frame_start[f]) continue;
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int k = frame_start[f]; k < frame_start[f + 1]; ++k) {
            const double l[3] = {spheres[k].lx, spheres[k].ly, spheres[k].lz};
            for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], l[a]); hi[a] = std::max(hi[a], l[a]); }
        }
        const double c[3] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])};
        double rad = 0.0;
        for (int k = frame_start[f]; k < frame_start[f + 1]; ++k) {
            const double dx = spheres[k].lx - c[0], dy = spheres[k].ly - c[1], dz = spheres[k].lz - c[2];
            rad = std::max(rad, std::sqrt(dx * dx + dy * dy + dz * dz) + (double)spheres[k].r);
        }
        frame_bound[f] = make_float4((float)c[0], (float)c[1], (float)c[2], (float)(rad * (1.0 + 1e-6) + 1e-6));
    }
    // separating-axis narrow phase: hulls (caller order) and scene boxes as
    // four float4 each, the hull's frame in the last word; hull pairs of the
    // listed frame pairs (k < m), sorted
    auto pack_box = [](const float *b, int frame, std::vector<float4> &out) {
        out.push_back(make_float4(b[0], b[1], b[2], b[12]));
        out.push_back(make_float4(b[3], b[4], b[5], b[13]));
        out.push_back(make_float4(b[6], b[7], b[8], b[14]));
        float fw;
        std::memcpy(&fw, &frame, sizeof(fw));
        out.push_back(make_float4(b[9], b[10], b[11], fw));
    };
    std::vector<float4> hulls, obb;
    for (int k = 0; k < robot->n_hulls; ++k) pack_box(robot->hull_box + 15 * k, robot->hull_frame[k], hulls);
    for (int o = 0; o < scene->n_obb; ++o) pack_box(scene->obb + 15 * o, 0, obb);
    std::vector<int2> hull_self;
    for (int k = 0; k < robot->n_hulls; ++k)
        for (int m = k + 1; m < robot->n_hulls; ++m) {
            const int fa = robot->hull_frame[k], fb = robot->hull_frame[m];
            bool listed = false;
            for (int i = 0; i < robot->n_self_pairs; ++i) {
                const int a = robot->self_pairs[2 * i], b = robot->self_pairs[2 * i + 1];
                listed = listed || (a == fa && b == fb) || (a == fb && b == fa);
            }
            if (listed) hull_self.push_back(make_int2(k, m));
        }
    std::vector<float> hold(robot->q_hold, robot->q_hold + p->n);
    hipError_t e;
    if ((e = upload(&p->d_hulls, hulls)) != hipSuccess || (e = upload(&p->d_obb, obb)) != hipSuccess ||
        (e = upload(&p->d_hull_self, hull_self)) != hipSuccess)
        return bail(hip_fail(e, "plan hull tables"));
    if ((e = upload(&p->d_joints, p->joints)) != hipSuccess || (e = upload(&p->d_spheres, spheres)) != hipSuccess ||
        (e = upload(&p->d_sphere_slot, sphere_slot)) != hipSuccess ||
        (e = upload(&p->d_frame_start, frame_start)) != hipSuccess || (e = upload(&p->d_cyl, cyl)) != hipSuccess ||
        (e = upload(&p->d_cyl_cell, cyl_cell)) != hipSuccess || (e = upload(&p->d_cell_start, cell_start)) != hipSuccess ||
        (e = upload(&p->d_hint, hint)) != hipSuccess ||
        (e = upload(&p->d_groups, groups)) != hipSuccess || (e = upload(&p->d_angle_start, angle_start)) != hipSuccess ||
        (e = upload(&p->d_cyl_orig, cyl_orig)) != hipSuccess ||
        (e = upload(&p->d_box, box)) != hipSuccess || (e = upload(&p->d_qs, hold)) != hipSuccess ||
        (e = upload(&p->d_self_pairs, self_pairs)) != hipSuccess ||
        (e = upload(&p->d_frame_bound, frame_bound)) != hipSuccess ||
        (e = upload(&p->d_qg, hold)) != hipSuccess)
        return bail(hip_fail(e, "plan tables"));
    e = hipMalloc((void **)&p->d_partial, eval_partial_count(p->max_B, p->ns) * sizeof(double2));
    if (e != hipSuccess) return bail(hip_fail(e, "plan workspace"));

    PlanView &v = p->view;
    v.n_joints = p->n;
    v.n_spheres = p->S;
    v.n_groups = (int)groups.size();
    v.n_box = p->n_box;
    v.n_cyl = p->n_cyl;
    v.has_ground = scene->has_ground ? 1 : 0;
    v.ground_z = scene->ground_z;
    v.K = p->K; v.M = p->M; v.ns = p->ns;
    v.interp = cost->interp; v.jp_mode = cost->jp_mode; v.hinge = cost->hinge;
    v.margin = cost->margin; v.lambda_c = cost->lambda_c; v.w_c = cost->w_c; v.w_l = cost->w_l;
    v.joints = p->d_joints; v.spheres = p->d_spheres; v.frame_start = p->d_frame_start;
    v.sphere_slot = p->d_sphere_slot;
    v.cyl = p->d_cyl; v.groups = p->d_groups; v.cyl_orig = p->d_cyl_orig; v.box = p->d_box;
    v.angle_start = p->d_angle_start;
    v.cyl_cell = p->d_cyl_cell;
    v.cell_start = p->d_cell_start;
    v.hint = p->d_hint;
    v.pair_filter = pair_filter;
    v.qs = p->d_qs; v.qg = p->d_qg;
    v.n_self = (int)self_pairs.size();
    v.self_pairs = p->d_self_pairs;
    v.frame_bound = p->d_frame_bound;
    for (int a = 0; a < 3; ++a) v.tip[a] = robot->tip[a];
    v.narrow = scene->narrow;
    v.n_hulls = robot->n_hulls;
    v.n_obb = scene->n_obb;
    v.n_hull_self = (int)hull_self.size();
    v.hulls = p->d_hulls;
    v.obb = p->d_obb;
    v.hull_self = p->d_hull_self;
    v.sdf = scene->d_sdf;
    for (int a = 0; a < 3; ++a) {
        v.sdf_n[a] = scene->d_sdf ? scene->sdf_dims[a] : 2;
        v.sdf_o[a] = scene->sdf_origin[a];
    }
    v.sdf_h = scene->d_sdf ? scene->voxel : 1.0f;
    v.sdf_inv_h = 1.0f / v.sdf_h;
    // block lower bounds of the grid, refreshed from the grid by every launch
    // that uses them (the grid is borrowed and may change between calls)
    v.sdf_lb = nullptr;
    v.sdf_lb_buf = nullptr;
    if (scene->d_sdf) {
        size_t nb = 1;
        for (int a = 0; a < 3; ++a) nb *= (size_t)(v.sdf_lbn[a] = ((v.sdf_n[a] - 2) >> kSdfBlockLog2) + 1);
        e = hipMalloc((void **)&p->d_sdf_lb, nb * sizeof(float));
        if (e != hipSuccess) return bail(hip_fail(e, "plan workspace"));
        v.sdf_lb_buf = p->d_sdf_lb;
    }
    // clearance grid (wave culling, primitive scenes; on the small scenes of
    // the other modes the per-group test costs more than it saves): over the
    // obstacles' footprints plus 2 m on every side, cells of at least 0.1 m,
    // at most 512 per axis
    v.clr = nullptr;
    v.lead_frame = -1;
    if (!scene->d_sdf && pair_filter == CP_PAIRS_WAVE && (p->n_cyl > 0 || p->n_box > 0)) {
        double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
        for (int o = 0; o < p->n_cyl; ++o) {
            const float *y = scene->cyl + 5 * o;
            x0 = std::min(x0, (double)y[0] - y[2]); x1 = std::max(x1, (double)y[0] + y[2]);
            y0 = std::min(y0, (double)y[1] - y[2]); y1 = std::max(y1, (double)y[1] + y[2]);
        }
        for (int o = 0; o < p->n_box; ++o) {
            const float *y = scene->box + 6 * o;
            x0 = std::min(x0, (double)y[0] - y[3]); x1 = std::max(x1, (double)y[0] + y[3]);
            y0 = std::min(y0, (double)y[1] - y[4]); y1 = std::max(y1, (double)y[1] + y[4]);
        }
        const double pad = 2.0;
        x0 -= pad; y0 -= pad; x1 += pad; y1 += pad;
        const double h = std::max({0.1, (x1 - x0) / 512.0, (y1 - y0) / 512.0});
        v.clr_nx = std::max(1, (int)std::ceil((x1 - x0) / h));
        v.clr_ny = std::max(1, (int)std::ceil((y1 - y0) / h));
        v.clr_x0 = (float)x0; v.clr_y0 = (float)y0;
        v.clr_h = (float)h; v.clr_inv = (float)(1.0 / h);
        e = hipMalloc((void **)&p->d_clr, (size_t)v.clr_nx * v.clr_ny * sizeof(float));
        if (e != hipSuccess) return bail(hip_fail(e, "plan workspace"));
        if ((e = launch_clearance(v, p->d_clr, nullptr)) != hipSuccess) return bail(hip_fail(e, "clearance grid"));
        v.clr = p->d_clr;
        // the frame with the most spheres (the lowest on ties) is evaluated
        // first; frame 0 needs no reordering
        int lead = 0;
        for (int f = 1; f <= p->n; ++f)
            if (frame_start[f + 1] - frame_start[f] > frame_start[lead + 1] - frame_start[lead]) lead = f;
        v.lead_frame = lead > 0 ? lead : -1;
    }
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return bail(hip_fail(e, "plan create"));
    *out = p;
    return CP_OK;
}

static void plan_release(cp_plan *plan) {
    if (plan->refs.fetch_sub(1) == 1) delete plan;
}

int cp_plan_destroy(cp_plan *plan) {
    if (!plan) return CP_OK;
    {
        DeviceGuard g(plan->device);
        (void)hipDeviceSynchronize();
    }
    plan_release(plan);
    return CP_OK;
}

int cp_plan_set_endpoints(cp_plan *plan, const float *q_start, const float *q_goal) {
    if (!plan || !q_start || !q_goal) return fail(CP_ERR_INVALID_ARG, "null argument");
    for (int j = 0; j < plan->n; ++j)
        if (!finite(q_start[j]) || !finite(q_goal[j])) return fail(CP_ERR_INVALID_ARG, "non-finite endpoint");
    DeviceGuard g(plan->device);
    CP_HIP(hipDeviceSynchronize(), "sync");
    CP_HIP(hipMemcpy(plan->d_qs, q_start, plan->n * sizeof(float), hipMemcpyHostToDevice), "endpoints");
    CP_HIP(hipMemcpy(plan->d_qg, q_goal, plan->n * sizeof(float), hipMemcpyHostToDevice), "endpoints");
    return CP_OK;
}

int cp_plan_n_checkpoints(const cp_plan *plan, int32_t *n_s) {
    if (!plan || !n_s) return fail(CP_ERR_INVALID_ARG, "null argument");
    *n_s = plan->ns;
    return CP_OK;
}

int cp_eval_paths(cp_plan *plan, const float *d_waypoints, int32_t B, float *d_cost, float *d_min_dist,
                  uint8_t *d_flags, uint32_t *d_tape, cp_stream_t stream) {
    if (!plan || !d_waypoints || !d_cost || !d_min_dist) return fail(CP_ERR_INVALID_ARG, "null argument");
    if (B < 1 || B > plan->max_B) return fail(CP_ERR_SIZE, "B out of range (1..max_B)");
    DeviceGuard g(plan->device);
    CP_HIP(launch_eval_fwd(plan->view, d_waypoints, B, plan->d_partial, d_tape, d_cost, d_min_dist, d_flags,
                           (hipStream_t)stream),
           "eval launch");
    return CP_OK;
}

int cp_eval_paths_noalloc(cp_plan *plan, const float *d_waypoints, int32_t B, float *d_cost, float *d_min_dist,
                          uint8_t *d_flags, uint32_t *d_tape, cp_stream_t stream) {
    if (!plan || !d_waypoints || !d_cost || !d_min_dist) return fail(CP_ERR_INVALID_ARG, "null argument");
    if (B < 1 || B > plan->max_B) return fail(CP_ERR_SIZE, "B out of range (1..max_B)");
    if (eval_partial_count(B, plan->ns) * sizeof(double2) > kNoAllocScratchBytes)
        return fail(CP_ERR_SIZE, "B * n_s exceeds the static scratch of cp_eval_paths_noalloc (24 MiB of per-wave "
                                 "partial sums); use cp_eval_paths");
    DeviceGuard g(plan->device);
    double2 *sp = nullptr;
    CP_HIP(scratch_on(plan->device, &sp), "scratch address");
    CP_HIP(launch_eval_fwd(plan->view, d_waypoints, B, sp, d_tape, d_cost, d_min_dist, d_flags, (hipStream_t)stream),
           "eval launch");
    return CP_OK;
}

int cp_eval_paths_backward(cp_plan *plan, const float *d_waypoints, int32_t B, const uint32_t *d_tape,
                           const float *d_grad_cost, float *d_grad_waypoints, cp_stream_t stream) {
    if (!plan || !d_waypoints || !d_grad_cost || !d_grad_waypoints) return fail(CP_ERR_INVALID_ARG, "null argument");
    if (B < 1 || B > plan->max_B) return fail(CP_ERR_SIZE, "B out of range (1..max_B)");
    if (plan->view.narrow == CP_NARROW_SAT) return fail(CP_ERR_INVALID_ARG, "the SAT narrow phase has no adjoint");
    DeviceGuard g(plan->device);
    CP_HIP(launch_eval_bwd(plan->view, d_waypoints, B, d_tape, d_grad_cost, d_grad_waypoints, (hipStream_t)stream),
           "backward launch");
    return CP_OK;
}

int cp_debug_fk(cp_plan *plan, const float *d_q, int32_t N, float *d_centers, float *d_frames, cp_stream_t stream) {
    if (!plan || !d_q) return fail(CP_ERR_INVALID_ARG, "null argument");
    if (N < 1) return fail(CP_ERR_SIZE, "N must be >= 1");
    DeviceGuard g(plan->device);
    CP_HIP(launch_debug_fk(plan->view, d_q, N, d_centers, d_frames, (hipStream_t)stream), "fk launch");
    return CP_OK;
}

int cp_debug_eval_configs(cp_plan *plan, const float *d_q, int32_t N, float *d_dist, uint32_t *d_argmin,
                          cp_stream_t stream) {
    if (!plan || !d_q || !d_dist) return fail(CP_ERR_INVALID_ARG, "null argument");
    if (N < 1) return fail(CP_ERR_SIZE, "N must be >= 1");
    DeviceGuard g(plan->device);
    CP_HIP(launch_debug_configs(plan->view, d_q, N, d_dist, d_argmin, (hipStream_t)stream), "configs launch");
    return CP_OK;
}

int cp_debug_select(const float *d_cost, int32_t B, int32_t nu, int32_t *d_elite, cp_stream_t stream) {
    if (!d_cost || !d_elite) return fail(CP_ERR_INVALID_ARG, "null argument");
    if (B < 1 || nu < 1 || nu > B || nu > CP_MAX_ELITES) return fail(CP_ERR_SIZE, "B or nu out of range");
    take_stale_error();
    OptView v{};
    v.cost = const_cast<float *>(d_cost);
    v.B = B;
    v.nu = nu;
    v.elite0 = d_elite;
    CP_HIP(launch_select(v, (hipStream_t)stream), "select launch");
    return CP_OK;
}

// ---------------------------------------------------------------------------
// collision-free inverse kinematics
// ---------------------------------------------------------------------------

static int validate_ik_params(const cp_ik_params *p) {
    if (!p) return fail(CP_ERR_INVALID_ARG, "null IK parameters");
    const float lam[4] = {p->lambda_q, p->lambda_c, p->lambda_e, p->lambda_r};
    for (float v : lam)
        if (!finite(v) || v < 0.0f) return fail(CP_ERR_INVALID_ARG, "IK weights must be finite and >= 0");
    if (p->max_iters < 0 || p->max_iters > 1000) return fail(CP_ERR_INVALID_ARG, "max_iters out of range (0..1000)");
    if (!finite(p->tau) || p->tau <= 0.0f) return fail(CP_ERR_INVALID_ARG, "tau must be finite and > 0");
    if (!finite(p->eps_grad) || p->eps_grad < 0.0f || !finite(p->eps_step) || p->eps_step < 0.0f)
        return fail(CP_ERR_INVALID_ARG, "IK tolerances must be finite and >= 0");
    return CP_OK;
}

constexpr int32_t kMaxIkRows = 1 << 20;

int cp_ik_solve(cp_plan *plan, const cp_ik_params *params, const float *d_target, const float *d_q_init,
                const float *d_q_ref, int32_t N, int32_t restarts, float *d_q, float *d_info, int32_t *d_status,
                int32_t *d_best, cp_stream_t stream) {
    if (!plan || !d_target || !d_q_init || !d_q) return fail(CP_ERR_INVALID_ARG, "null argument");
    if (int rc = validate_ik_params(params)) return rc;
    if (N < 1 || N > kMaxIkRows) return fail(CP_ERR_SIZE, "N out of range (1..1048576)");
    if (restarts < 1 || N % restarts != 0) return fail(CP_ERR_SIZE, "N must be a positive multiple of restarts");
    if (d_best && !d_info) return fail(CP_ERR_INVALID_ARG, "d_best needs d_info (the rows' costs)");
    if (plan->view.narrow == CP_NARROW_SAT) return fail(CP_ERR_INVALID_ARG, "the IK takes the sphere narrow phase");
    DeviceGuard g(plan->device);
    CP_HIP(launch_ik_solve(plan->view, *params, d_target, d_q_init, d_q_ref, N, restarts, d_q, d_info, d_status,
                           d_best, (hipStream_t)stream),
           "IK launch");
    return CP_OK;
}

int cp_debug_ik_residual(cp_plan *plan, const cp_ik_params *params, const float *d_target, const float *d_q,
                         const float *d_q_ref, int32_t N, float *d_r, float *d_J, cp_stream_t stream) {
    if (!plan || !d_target || !d_q) return fail(CP_ERR_INVALID_ARG, "null argument");
    if (int rc = validate_ik_params(params)) return rc;
    if (N < 1 || N > kMaxIkRows) return fail(CP_ERR_SIZE, "N out of range (1..1048576)");
    if (plan->view.narrow == CP_NARROW_SAT) return fail(CP_ERR_INVALID_ARG, "the IK takes the sphere narrow phase");
    DeviceGuard g(plan->device);
    CP_HIP(launch_ik_residual(plan->view, *params, d_target, d_q, d_q_ref, N, d_r, d_J, (hipStream_t)stream),
           "IK residual launch");
    return CP_OK;
}

// ---------------------------------------------------------------------------
// step two: direct collocation
// ---------------------------------------------------------------------------

static int validate_traj(const cp_plan *plan, const cp_traj_params *p, int *act, int *n_act) {
    if (!plan || !p) return fail(CP_ERR_INVALID_ARG, "null argument");
    if (p->N < 2 || p->N > 400) return fail(CP_ERR_SIZE, "N out of range (2..400)");
    auto ok = [](double v) { return std::isfinite(v); };
    if (!ok(p->omega_s) || p->omega_s < 0.0 || !ok(p->omega_t) || p->omega_t < 0.0 || !ok(p->grav) ||
        !ok(p->damping) || p->damping < 0.0 || !ok(p->mu0) || !(p->mu0 > 0.0) || !ok(p->mu_factor) ||
        !(p->mu_factor >= 1.0) || !ok(p->tau) || !(p->tau > 0.0) || !ok(p->eps_grad) || p->eps_grad < 0.0 ||
        !ok(p->eps_step) || p->eps_step < 0.0 || !ok(p->fd_q) || !(p->fd_q > 0.0) || !ok(p->t_f0) ||
        !(p->t_f0 > 0.0))
        return fail(CP_ERR_INVALID_ARG, "step-two parameters out of range");
    if (p->outer < 1 || p->outer > 20 || p->max_iters < 0 || p->max_iters > 500)
        return fail(CP_ERR_INVALID_ARG, "outer (1..20) or max_iters (0..500) out of range");
    for (int j = 0; j < plan->n; ++j)
        if (!ok(p->v_max[j]) || !(p->v_max[j] > 0.0)) return fail(CP_ERR_INVALID_ARG, "v_max must be > 0");
    *n_act = 0;
    for (int j = 0; j < plan->n; ++j)
        if (plan->joints[j].active) act[(*n_act)++] = j;
    if (2 * plan->n + *n_act > kTrajBlock) return fail(CP_ERR_SIZE, "2 n + actuated joints exceeds 16");
    return CP_OK;
}

int cp_traj_workspace_size(const cp_plan *plan, const cp_traj_params *params, int32_t P, size_t *bytes) {
    int act[CP_MAX_JOINTS], na = 0;
    if (int rc = validate_traj(plan, params, act, &na)) return rc;
    if (!bytes) return fail(CP_ERR_INVALID_ARG, "null bytes");
    if (P < 1) return fail(CP_ERR_SIZE, "P must be >= 1");
    *bytes = traj_workspace_bytes(params->N, plan->n, na, P);
    return CP_OK;
}

int cp_traj_refine(cp_plan *plan, const cp_traj_params *params, const float *d_q_start, const float *d_q_goal,
                   const float *d_q_star, int32_t P, void *d_work, size_t work_bytes, float *d_x, float *d_u,
                   float *d_t_f, float *d_info, cp_stream_t stream) {
    int act[CP_MAX_JOINTS], na = 0;
    if (int rc = validate_traj(plan, params, act, &na)) return rc;
    if (!d_q_start || !d_q_goal || !d_q_star || !d_work || !d_x || !d_u || !d_t_f)
        return fail(CP_ERR_INVALID_ARG, "null argument");
    if (P < 1 || P > (1 << 20)) return fail(CP_ERR_SIZE, "P out of range (1..1048576)");
    if (work_bytes < traj_workspace_bytes(params->N, plan->n, na, P)) return fail(CP_ERR_SIZE, "workspace too small");
    if (reinterpret_cast<uintptr_t>(d_work) % 8 != 0) return fail(CP_ERR_INVALID_ARG, "workspace not 8-byte aligned");
    DeviceGuard g(plan->device);
    CP_HIP(launch_traj_refine(plan->view, *params, act, na, d_q_start, d_q_goal, d_q_star, P, d_work, d_x, d_u, d_t_f,
                              d_info, (hipStream_t)stream),
           "step-two launch");
    return CP_OK;
}

// ---------------------------------------------------------------------------
// optimizer
// ---------------------------------------------------------------------------

int cp_optimizer_create(cp_plan *plan, const cp_opt_params *prm, cp_opt **out) {
    if (!out) return fail(CP_ERR_INVALID_ARG, "null out");
    *out = nullptr;
    if (!plan || !prm) return fail(CP_ERR_INVALID_ARG, "null argument");
    if (prm->B < 1 || prm->B > plan->max_B) return fail(CP_ERR_SIZE, "B out of range (1..max_B)");
    if (prm->nu < 1 || prm->nu > prm->B || prm->nu > CP_MAX_ELITES) return fail(CP_ERR_SIZE, "nu out of range");
    if (!(prm->sigma0 > 0.0f) || !finite(prm->sigma0)) return fail(CP_ERR_INVALID_ARG, "sigma0 must be > 0");
    if (!(prm->eps >= 0.0) || !std::isfinite(prm->eps)) return fail(CP_ERR_INVALID_ARG, "eps must be >= 0");
    if (prm->polish_elites < 0 || prm->polish_elites > prm->nu || prm->polish_steps < 0)
        return fail(CP_ERR_SIZE, "polish settings out of range");
    if (prm->polish_elites > 0 && prm->polish_steps > 0 &&
        (!(prm->polish_eta >= 0.0f) || !(prm->polish_clip > 0.0f)))
        return fail(CP_ERR_INVALID_ARG, "bad polish step");
    if (prm->polish_elites > 0 && prm->polish_steps > 0 && plan->view.narrow == CP_NARROW_SAT)
        return fail(CP_ERR_INVALID_ARG, "the polish needs the adjoint, which the SAT narrow phase has not");
    int n_act = 0;
    int act[CP_MAX_JOINTS] = {0};
    for (int j = 0; j < plan->n; ++j)
        if (plan->joints[j].active) act[n_act++] = j;
    if (n_act < 1) return fail(CP_ERR_INVALID_ARG, "no sampled joint");
    const int D = plan->K * n_act;
    if (D > CP_MAX_DIM) return fail(CP_ERR_SIZE, "K * sampled joints exceeds CP_MAX_DIM");
    DeviceGuard guard(plan->device);
    cp_opt *o = new (std::nothrow) cp_opt();
    if (!o) return fail(CP_ERR_NOMEM, "host allocation");
    o->plan = plan;
    o->prm = *prm;
    o->D = D;
    o->n_act = n_act;
    o->npol = (prm->polish_steps > 0) ? prm->polish_elites : 0;
    OptView &v = o->view;
    v.B = prm->B; v.nu = prm->nu; v.D = D; v.n_act = n_act; v.npol = o->npol;
    for (int a = 0; a < CP_MAX_JOINTS; ++a) v.act[a] = act[a];
    v.eps = prm->eps; v.seed = prm->seed; v.problem_id = prm->problem_id;
    v.eta = prm->polish_eta; v.clip = prm->polish_clip;
    const size_t per = (size_t)plan->K * plan->n;
    const size_t np = std::max(1, o->npol);
    hipError_t e;
    if ((e = o->alloc(&v.mu, D)) != hipSuccess || (e = o->alloc(&v.C, (size_t)D * D)) != hipSuccess ||
        (e = o->alloc(&v.L, (size_t)D * D)) != hipSuccess || (e = o->alloc(&v.xi, (size_t)prm->B * D)) != hipSuccess ||
        (e = o->alloc(&v.W, prm->B * per)) != hipSuccess || (e = o->alloc(&v.cost, prm->B)) != hipSuccess ||
        (e = o->alloc(&v.min_dist, prm->B)) != hipSuccess || (e = o->alloc(&v.elite, prm->nu)) != hipSuccess ||
        (e = o->alloc(&v.elite0, prm->nu)) != hipSuccess || (e = o->alloc(&v.Wp, np * per)) != hipSuccess ||
        (e = o->alloc(&v.Wp2, np * per)) != hipSuccess || (e = o->alloc(&v.md_p, np)) != hipSuccess ||
        (e = o->alloc(&v.cost_p, np)) != hipSuccess || (e = o->alloc(&v.grad_p, np * per)) != hipSuccess ||
        (e = o->alloc(&v.ones, np)) != hipSuccess || (e = o->alloc(&v.w, prm->nu)) != hipSuccess ||
        (e = o->alloc(&v.t, 1)) != hipSuccess || (e = o->alloc(&v.status, 1)) != hipSuccess ||
        (e = o->alloc(&v.best_cost, 1)) != hipSuccess || (e = o->alloc(&v.best_W, per)) != hipSuccess ||
        (e = o->alloc(&o->d_tape_p, np * plan->ns)) != hipSuccess) {
        delete o;
        return hip_fail(e, "optimizer buffers");
    }
    if (o->npol == 0) v.elite0 = v.elite;  // no polish: selection writes the final ranking
    std::vector<float> ones(np, 1.0f);
    e = hipMemcpy(v.ones, ones.data(), np * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_init_state(plan->view, v, prm->sigma0, nullptr);
    if (e == hipSuccess) e = launch_chol(v, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        delete o;
        return hip_fail(e, "optimizer init");
    }
    plan->refs.fetch_add(1);
    *out = o;
    return CP_OK;
}

int cp_optimizer_destroy(cp_opt *opt) {
    if (!opt) return CP_OK;
    cp_plan *plan = opt->plan;
    {
        DeviceGuard g(plan->device);
        (void)hipDeviceSynchronize();
    }
    delete opt;
    plan_release(plan);
    return CP_OK;
}

// The gradient polish of the selected elites (elite0[0..npol)), their
// re-evaluation and the re-ranking of the elites.  Each step reads the
// waypoints from one of two buffers and writes the stepped ones to the other;
// the gather picks the first buffer so that the last step writes v.Wp.
static int enqueue_polish(cp_opt *opt, hipStream_t st) {
    cp_plan *p = opt->plan;
    const OptView &v = opt->view;
    const PlanView &P = p->view;
    float *buf[2] = {v.Wp, v.Wp2};
    int cur = opt->prm.polish_steps & 1;
    CP_HIP(launch_polish_gather(P, v, buf[cur], st), "polish gather");
    PolishStep ps{};
    for (int a = 0; a < CP_MAX_JOINTS; ++a) ps.act[a] = v.act[a];
    for (int a = 0; a < v.n_act; ++a) ps.act_mask |= 1u << v.act[a];
    ps.eta = v.eta;
    ps.clip = v.clip;
    ps.D = v.D;
    ps.n_act = v.n_act;
    for (int s = 0; s < opt->prm.polish_steps; ++s) {
        // (only the argmin tape of this evaluation is used)
        CP_HIP(launch_eval_fwd(P, buf[cur], opt->npol, p->d_partial, opt->d_tape_p, nullptr, nullptr, nullptr, st),
               "polish eval");
        // the adjoint applies each path's gradient step itself
        ps.W_out = buf[cur ^ 1];
        CP_HIP(launch_eval_bwd(P, buf[cur], opt->npol, opt->d_tape_p, v.ones, v.grad_p, st, &ps),
               "polish adjoint and step");
        cur ^= 1;
    }
    CP_HIP(launch_eval_fwd(P, v.Wp, opt->npol, p->d_partial, nullptr, v.cost_p, v.md_p, nullptr, st), "polish eval");
    CP_HIP(launch_rerank(v, st), "rerank");
    return CP_OK;
}

int cp_optimizer_step(cp_opt *opt, int32_t n_iters, cp_stream_t stream) {
    if (!opt) return fail(CP_ERR_INVALID_ARG, "null optimizer");
    if (n_iters < 0) return fail(CP_ERR_SIZE, "n_iters must be >= 0");
    cp_plan *p = opt->plan;
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    const OptView &v = opt->view;
    const PlanView &P = p->view;
    for (int it = 0; it < n_iters; ++it) {
        CP_HIP(launch_sample(P, v, st), "sample");
        const EvalEvents *ev = opt->next_events();
        if (reduce_select_fits(v.B)) {
            CP_HIP(launch_eval_fwd(P, v.W, v.B, p->d_partial, opt->d_tape, nullptr, nullptr, nullptr, st, ev), "eval");
            CP_HIP(launch_reduce_select(p->d_partial, eval_slots(P.ns), P.ns, P.margin, v, st), "select");
        } else {
            CP_HIP(launch_eval_fwd(P, v.W, v.B, p->d_partial, opt->d_tape, v.cost, v.min_dist, nullptr, st, ev),
                   "eval");
            CP_HIP(launch_select(v, st), "select");
        }
        if (opt->npol > 0) {
            const int rc = enqueue_polish(opt, st);
            if (rc) return rc;
        }
        CP_HIP(launch_update(P, v, st), "update");
        CP_HIP(launch_chol(v, st), "cholesky");
    }
    return CP_OK;
}

int cp_optimizer_record_tape(cp_opt *opt, int32_t enable) {
    if (!opt) return fail(CP_ERR_INVALID_ARG, "null optimizer");
    if (enable && opt->plan->view.narrow == CP_NARROW_SAT)
        return fail(CP_ERR_INVALID_ARG, "the population gradient needs the adjoint, which the SAT narrow phase has not");
    DeviceGuard g(opt->plan->device);
    CP_HIP(hipDeviceSynchronize(), "sync");
    if (!enable) {
        opt->drop_tape();
        return CP_OK;
    }
    if (opt->d_tape) return CP_OK;
    const OptView &v = opt->view;
    hipError_t e = hipMalloc((void **)&opt->d_tape, (size_t)v.B * opt->plan->ns * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&opt->d_ones_B, (size_t)v.B * sizeof(float));
    if (e == hipSuccess) {
        std::vector<float> ones(v.B, 1.0f);
        e = hipMemcpy(opt->d_ones_B, ones.data(), v.B * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        opt->drop_tape();
        return hip_fail(e, "tape buffers");
    }
    return CP_OK;
}

int cp_optimizer_population_grad(cp_opt *opt, float *d_grad_waypoints, cp_stream_t stream) {
    if (!opt || !d_grad_waypoints) return fail(CP_ERR_INVALID_ARG, "null argument");
    if (!opt->d_tape) return fail(CP_ERR_STATE, "no tape: call cp_optimizer_record_tape first");
    cp_plan *p = opt->plan;
    DeviceGuard g(p->device);
    const OptView &v = opt->view;
    CP_HIP(launch_eval_bwd(p->view, v.W, v.B, opt->d_tape, opt->d_ones_B, d_grad_waypoints, (hipStream_t)stream),
           "population adjoint");
    return CP_OK;
}

int cp_optimizer_time_eval(cp_opt *opt, int32_t max_launches) {
    if (!opt) return fail(CP_ERR_INVALID_ARG, "null optimizer");
    if (max_launches < 0 || max_launches > 65536) return fail(CP_ERR_SIZE, "max_launches out of range (0..65536)");
    DeviceGuard g(opt->plan->device);
    CP_HIP(hipDeviceSynchronize(), "sync");
    opt->drop_events();
    for (int i = 0; i < max_launches; ++i) {
        EvalEvents e{};
        CP_HIP(hipEventCreate(&e.begin), "event");
        hipError_t er = hipEventCreate(&e.end);
        if (er != hipSuccess) {
            (void)hipEventDestroy(e.begin);
            return hip_fail(er, "event");
        }
        opt->ev.push_back(e);
    }
    return CP_OK;
}

int cp_optimizer_eval_time(cp_opt *opt, double *total_ms, int32_t *launches) {
    if (!opt || !total_ms || !launches) return fail(CP_ERR_INVALID_ARG, "null argument");
    DeviceGuard g(opt->plan->device);
    double sum = 0.0;
    for (size_t i = 0; i < opt->ev_used; ++i) {
        CP_HIP(hipEventSynchronize(opt->ev[i].end), "event sync");
        float ms = 0.0f;
        CP_HIP(hipEventElapsedTime(&ms, opt->ev[i].begin, opt->ev[i].end), "event time");
        sum += ms;
    }
    *total_ms = sum;
    *launches = (int32_t)opt->ev_used;
    opt->ev_used = 0;
    return CP_OK;
}

int cp_debug_update(cp_opt *opt, const int32_t *d_elite, cp_stream_t stream) {
    if (!opt || !d_elite) return fail(CP_ERR_INVALID_ARG, "null argument");
    cp_plan *p = opt->plan;
    DeviceGuard g(p->device);
    const OptView &v = opt->view;
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> idx(v.nu);
    CP_HIP(hipStreamSynchronize(st), "sync");
    CP_HIP(hipMemcpy(idx.data(), d_elite, v.nu * sizeof(int32_t), hipMemcpyDeviceToHost), "elites");
    for (int32_t i : idx)
        if (i < 0 || i >= v.B) return fail(CP_ERR_INVALID_ARG, "elite index out of range");
    CP_HIP(hipMemcpyAsync(v.elite0, d_elite, v.nu * sizeof(int32_t), hipMemcpyDeviceToDevice, st), "elites");
    if (opt->npol > 0) {
        const int rc = enqueue_polish(opt, st);
        if (rc) return rc;
    }
    CP_HIP(launch_update(p->view, v, st), "update");
    return CP_OK;
}

int cp_optimizer_last_polished(cp_opt *opt, float *d_waypoints, float *d_cost, cp_stream_t stream) {
    if (!opt) return fail(CP_ERR_INVALID_ARG, "null optimizer");
    if (opt->npol == 0) return fail(CP_ERR_STATE, "the optimizer has no polish");
    DeviceGuard g(opt->plan->device);
    const OptView &v = opt->view;
    hipStream_t st = (hipStream_t)stream;
    const size_t per = (size_t)opt->plan->K * opt->plan->n;
    if (d_waypoints)
        CP_HIP(hipMemcpyAsync(d_waypoints, v.Wp, opt->npol * per * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
    if (d_cost) CP_HIP(hipMemcpyAsync(d_cost, v.cost_p, opt->npol * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
    return CP_OK;
}

int cp_optimizer_last_elites(cp_opt *opt, int32_t *d_idx, float *d_cost, cp_stream_t stream) {
    return cp_optimizer_last(opt, nullptr, d_cost, d_idx, stream);
}

int cp_optimizer_get_state(cp_opt *opt, double *mu, double *C, int64_t *iter, float *best_cost,
                           float *best_waypoints) {
    if (!opt) return fail(CP_ERR_INVALID_ARG, "null optimizer");
    DeviceGuard g(opt->plan->device);
    const OptView &v = opt->view;
    CP_HIP(hipDeviceSynchronize(), "sync");
    const size_t per = (size_t)opt->plan->K * opt->plan->n;
    if (mu) CP_HIP(hipMemcpy(mu, v.mu, opt->D * sizeof(double), hipMemcpyDeviceToHost), "state");
    if (C) CP_HIP(hipMemcpy(C, v.C, (size_t)opt->D * opt->D * sizeof(double), hipMemcpyDeviceToHost), "state");
    if (iter) CP_HIP(hipMemcpy(iter, v.t, sizeof(int64_t), hipMemcpyDeviceToHost), "state");
    if (best_cost) CP_HIP(hipMemcpy(best_cost, v.best_cost, sizeof(float), hipMemcpyDeviceToHost), "state");
    if (best_waypoints) CP_HIP(hipMemcpy(best_waypoints, v.best_W, per * sizeof(float), hipMemcpyDeviceToHost), "state");
    int32_t status = 0;
    CP_HIP(hipMemcpy(&status, v.status, sizeof(int32_t), hipMemcpyDeviceToHost), "state");
    if (status) {
        const int32_t zero = 0;
        CP_HIP(hipMemcpy(v.status, &zero, sizeof(int32_t), hipMemcpyHostToDevice), "state");
        return fail(CP_ERR_NOT_PD, "covariance was not positive definite (previous factor kept)");
    }
    return CP_OK;
}

int cp_optimizer_set_state(cp_opt *opt, const double *mu, const double *C, int64_t iter) {
    if (!opt || !mu || !C) return fail(CP_ERR_INVALID_ARG, "null argument");
    if (iter < 0) return fail(CP_ERR_INVALID_ARG, "iter must be >= 0");
    for (int i = 0; i < opt->D; ++i)
        if (!std::isfinite(mu[i])) return fail(CP_ERR_INVALID_ARG, "non-finite mu");
    for (int i = 0; i < opt->D * opt->D; ++i)
        if (!std::isfinite(C[i])) return fail(CP_ERR_INVALID_ARG, "non-finite C");
    DeviceGuard g(opt->plan->device);
    const OptView &v = opt->view;
    CP_HIP(hipDeviceSynchronize(), "sync");
    CP_HIP(hipMemcpy(v.mu, mu, opt->D * sizeof(double), hipMemcpyHostToDevice), "state");
    CP_HIP(hipMemcpy(v.C, C, (size_t)opt->D * opt->D * sizeof(double), hipMemcpyHostToDevice), "state");
    CP_HIP(hipMemcpy(v.t, &iter, sizeof(int64_t), hipMemcpyHostToDevice), "state");
    const float inf = INFINITY;
    CP_HIP(hipMemcpy(v.best_cost, &inf, sizeof(float), hipMemcpyHostToDevice), "state");
    CP_HIP(launch_chol(v, nullptr), "cholesky");
    CP_HIP(hipDeviceSynchronize(), "sync");
    int32_t status = 0;
    CP_HIP(hipMemcpy(&status, v.status, sizeof(int32_t), hipMemcpyDeviceToHost), "state");
    if (status) {
        const int32_t zero = 0;
        CP_HIP(hipMemcpy(v.status, &zero, sizeof(int32_t), hipMemcpyHostToDevice), "state");
        return fail(CP_ERR_NOT_PD, "covariance is not positive definite");
    }
    return CP_OK;
}

int cp_optimizer_last(cp_opt *opt, float *d_waypoints, float *d_cost, int32_t *d_elite, cp_stream_t stream) {
    if (!opt) return fail(CP_ERR_INVALID_ARG, "null optimizer");
    DeviceGuard g(opt->plan->device);
    const OptView &v = opt->view;
    hipStream_t st = (hipStream_t)stream;
    const size_t per = (size_t)opt->plan->K * opt->plan->n;
    if (d_waypoints)
        CP_HIP(hipMemcpyAsync(d_waypoints, v.W, v.B * per * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
    if (d_cost) CP_HIP(hipMemcpyAsync(d_cost, v.cost, v.B * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
    if (d_elite) CP_HIP(hipMemcpyAsync(d_elite, v.elite, v.nu * sizeof(int32_t), hipMemcpyDeviceToDevice, st), "copy");
    return CP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batches of problems
// ---------------------------------------------------------------------------

struct cp_batch {
    int device = 0, n = 0, max_B = 0, n_cu = 0;
    std::vector<cp_plan *> plans;
    std::vector<cp_opt *> opts;
    std::vector<int> order;           // problems, costliest configuration first
    BatchProblem *d_probs = nullptr;
    int2 *d_items = nullptr;
    size_t items_cap = 0;
    int n_items = 0;
    double2 *d_partial = nullptr;     // per-wave partial sums of every problem, back to back
    BatchTuning tune{4, 4};
    bool cull = false;                // wave-level culling (CP_PAIRS_WAVE)
    hipStream_t capture_stream = nullptr;
    std::map<int, std::pair<hipGraph_t, hipGraphExec_t>> graphs;

    void drop_graphs() {
        for (auto &kv : graphs) {
            (void)hipGraphExecDestroy(kv.second.second);
            (void)hipGraphDestroy(kv.second.first);
        }
        graphs.clear();
    }
    ~cp_batch() {
        DeviceGuard g(device);
        (void)hipDeviceSynchronize();
        drop_graphs();
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
        if (d_probs) (void)hipFree(d_probs);
        if (d_items) (void)hipFree(d_items);
        if (d_partial) (void)hipFree(d_partial);
        for (cp_opt *o : opts) delete o;
        for (cp_plan *p : plans) delete p;
    }
    // work items (problem, first configuration) for the current tuning
    hipError_t build_items() {
        std::vector<int2> items;
        const int64_t chunk = 256 * (int64_t)tune.rounds;
        for (int p : order) {
            const int64_t N = (int64_t)opts[p]->prm.B * plans[p]->ns;
            for (int64_t g0 = 0; g0 < N; g0 += chunk) items.push_back(make_int2(p, (int)g0));
        }
        n_items = (int)items.size();
        if (items.size() > items_cap) {
            if (d_items) (void)hipFree(d_items);
            d_items = nullptr;
            hipError_t e = hipMalloc((void **)&d_items, items.size() * sizeof(int2));
            if (e != hipSuccess) return e;
            items_cap = items.size();
        }
        return hipMemcpy(d_items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice);
    }
    int grid() const { return tune.wg_per_cu > 0 ? n_cu * tune.wg_per_cu : std::max(1, n_items); }
};

extern "C" {

int cp_batch_create(int32_t n, const cp_robot_desc *robots, const cp_scene_desc *scenes, const cp_cost_params *costs,
                    const cp_opt_params *opts, const float *q_start, const float *q_goal, int device,
                    cp_batch **out) {
    if (!out) return fail(CP_ERR_INVALID_ARG, "null out");
    *out = nullptr;
    if (n < 1) return fail(CP_ERR_SIZE, "n must be >= 1");
    if (!robots || !scenes || !costs || !opts || !q_start || !q_goal) return fail(CP_ERR_INVALID_ARG, "null argument");
    for (int i = 0; i < n; ++i) {
        if (opts[i].polish_steps > 0 && opts[i].polish_elites > 0)
            return fail(CP_ERR_INVALID_ARG, "polish is not supported in a batch");
        if (costs[i].max_B < opts[i].B) return fail(CP_ERR_SIZE, "cost max_B below opt B");
        if (costs[i].pair_filter != costs[0].pair_filter)
            return fail(CP_ERR_INVALID_ARG, "every problem of a batch needs the same pair_filter");
        if (scenes[i].narrow != CP_NARROW_SPHERES)
            return fail(CP_ERR_INVALID_ARG, "batches take the sphere narrow phase");
    }
    cp_batch *b = new (std::nothrow) cp_batch();
    if (!b) return fail(CP_ERR_NOMEM, "host allocation");
    b->device = device;
    b->n = n;
    b->cull = costs[0].pair_filter == CP_PAIRS_WAVE;
    for (int i = 0; i < n && costs[0].pair_filter == CP_PAIRS_AUTO; ++i)
        if (resolve_pairs(CP_PAIRS_AUTO, scenes[i].n_cyl + scenes[i].n_box) == CP_PAIRS_WAVE) b->cull = true;
    size_t qoff = 0;
    for (int i = 0; i < n; ++i) {
        cp_plan *p = nullptr;
        int rc = cp_plan_create(robots + i, scenes + i, costs + i, device, &p);
        if (rc) {
            delete b;
            return fail(rc, "problem " + std::to_string(i) + ": " + g_err);
        }
        b->plans.push_back(p);
        rc = cp_plan_set_endpoints(p, q_start + qoff, q_goal + qoff);
        qoff += robots[i].n_joints;
        cp_opt *o = nullptr;
        if (!rc) rc = cp_optimizer_create(p, opts + i, &o);
        if (rc) {
            delete b;
            return fail(rc, "problem " + std::to_string(i) + ": " + g_err);
        }
        b->opts.push_back(o);
        b->max_B = std::max(b->max_B, opts[i].B);
    }
    DeviceGuard guard(device);
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "device properties");
    }
    b->n_cu = prop.multiProcessorCount;
    std::vector<BatchProblem> probs(n);
    std::vector<std::pair<double, int>> cost_of(n);
    int64_t partial_total = 0;
    for (int i = 0; i < n; ++i) {
        probs[i].P = b->plans[i]->view;
        probs[i].O = b->opts[i]->view;
        probs[i].O.elite0 = probs[i].O.elite;  // no polish: selection writes the final ranking
        probs[i].partial_off = partial_total;
        probs[i].slots = eval_slots(b->plans[i]->ns);
        partial_total += (int64_t)eval_partial_count(opts[i].B, b->plans[i]->ns);
        cost_of[i] = {-(double)b->plans[i]->S * (b->plans[i]->n_cyl + b->plans[i]->n_box + 1), i};
    }
    std::stable_sort(cost_of.begin(), cost_of.end());
    for (auto &c : cost_of) b->order.push_back(c.second);
    if ((e = hipMalloc((void **)&b->d_partial, (size_t)partial_total * sizeof(double2))) != hipSuccess) {
        delete b;
        return hip_fail(e, "batch workspace");
    }
    if ((e = upload(&b->d_probs, probs)) != hipSuccess ||
        (e = b->build_items()) != hipSuccess || (e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking)) != hipSuccess) {
        delete b;
        return hip_fail(e, "batch tables");
    }
    *out = b;
    return CP_OK;
}

int cp_batch_destroy(cp_batch *batch) {
    delete batch;
    return CP_OK;
}

int cp_batch_run(cp_batch *b, int32_t n_iters, cp_stream_t stream) {
    if (!b) return fail(CP_ERR_INVALID_ARG, "null batch");
    if (n_iters < 0) return fail(CP_ERR_SIZE, "n_iters must be >= 0");
    if (n_iters == 0) return CP_OK;
    DeviceGuard g(b->device);
    auto it = b->graphs.find(n_iters);
    if (it == b->graphs.end()) {
        hipStream_t cs = b->capture_stream;
        CP_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "graph capture");
        hipError_t e = hipSuccess;
        for (int i = 0; i < n_iters && e == hipSuccess; ++i)
            e = launch_batch_iteration(b->d_probs, b->d_partial, b->n, b->max_B, b->d_items, b->n_items,
                                       b->tune.rounds, b->grid(), b->cull, cs);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(e, "graph capture");
        }
        if (e2 != hipSuccess) return hip_fail(e2, "graph capture end");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(e, "graph instantiate");
        }
        it = b->graphs.emplace(n_iters, std::make_pair(graph, exec)).first;
    }
    CP_HIP(hipGraphLaunch(it->second.second, (hipStream_t)stream), "graph launch");
    return CP_OK;
}

int cp_batch_eval(cp_batch *b, cp_stream_t stream) {
    if (!b) return fail(CP_ERR_INVALID_ARG, "null batch");
    DeviceGuard g(b->device);
    CP_HIP(launch_batch_eval(b->d_probs, b->d_partial, b->n, b->max_B, b->d_items, b->n_items, b->tune.rounds,
                             b->grid(), b->cull, (hipStream_t)stream),
           "batch eval");
    return CP_OK;
}

int cp_batch_get_state(cp_batch *b, int32_t p, double *mu, double *C, int64_t *iter, float *best_cost,
                       float *best_waypoints) {
    if (!b) return fail(CP_ERR_INVALID_ARG, "null batch");
    if (p < 0 || p >= b->n) return fail(CP_ERR_SIZE, "problem index out of range");
    return cp_optimizer_get_state(b->opts[p], mu, C, iter, best_cost, best_waypoints);
}

int cp_batch_last(cp_batch *b, int32_t p, float *d_waypoints, float *d_cost, int32_t *d_elite, cp_stream_t stream) {
    if (!b) return fail(CP_ERR_INVALID_ARG, "null batch");
    if (p < 0 || p >= b->n) return fail(CP_ERR_SIZE, "problem index out of range");
    return cp_optimizer_last(b->opts[p], d_waypoints, d_cost, d_elite, stream);
}

int cp_batch_set_tuning(cp_batch *b, const cp_batch_tuning *t) {
    if (!b || !t) return fail(CP_ERR_INVALID_ARG, "null argument");
    if (t->rounds < 1 || t->rounds > 64 || t->wg_per_cu < 0 || t->wg_per_cu > 16)
        return fail(CP_ERR_SIZE, "tuning out of range");
    DeviceGuard g(b->device);
    CP_HIP(hipDeviceSynchronize(), "sync");
    b->drop_graphs();
    b->tune.rounds = t->rounds;
    b->tune.wg_per_cu = t->wg_per_cu;
    CP_HIP(b->build_items(), "work items");
    return CP_OK;
}

int cp_batch_get_tuning(const cp_batch *b, cp_batch_tuning *t) {
    if (!b || !t) return fail(CP_ERR_INVALID_ARG, "null argument");
    t->rounds = b->tune.rounds;
    t->wg_per_cu = b->tune.wg_per_cu;
    return CP_OK;
}

int cp_batch_tune(cp_batch *b, const char *cache_path, cp_batch_tuning *chosen) {
    if (!b) return fail(CP_ERR_INVALID_ARG, "null batch");
    DeviceGuard g(b->device);
    // signature of the batch shape and the device (FNV-1a)
    hipDeviceProp_t prop;
    CP_HIP(hipGetDeviceProperties(&prop, b->device), "device properties");
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](uint64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 0xFF;
            h *= 1099511628211ull;
        }
    };
    mix((uint64_t)b->n);
    for (int i = 0; i < b->n; ++i) {
        mix((uint64_t)b->opts[i]->prm.B);
        mix((uint64_t)b->plans[i]->ns);
        mix((uint64_t)b->plans[i]->S);
        mix((uint64_t)b->plans[i]->n_cyl);
        mix((uint64_t)b->plans[i]->n_box);
    }
    for (const char *c = prop.gcnArchName; *c; ++c) mix((uint64_t)(unsigned char)*c);
    mix((uint64_t)prop.multiProcessorCount);
    char key[32];
    std::snprintf(key, sizeof(key), "%016llx", (unsigned long long)h);
    cp_batch_tuning best{0, 0};
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "r")) {
            char k[64];
            int r, w;
            double ms;
            while (std::fscanf(f, "%63s %d %d %lf", k, &r, &w, &ms) == 4)
                if (std::strcmp(k, key) == 0) best = {r, w};
            std::fclose(f);
        }
    }
    if (best.rounds == 0) {
        // current populations for timing: one sampling pass (does not advance t)
        hipStream_t st = b->capture_stream;
        CP_HIP(launch_batch_sample(b->d_probs, b->n, b->max_B, st), "tune sample");
        hipEvent_t e0, e1;
        CP_HIP(hipEventCreate(&e0), "event");
        CP_HIP(hipEventCreate(&e1), "event");
        double best_ms = 1e300;
        // every launch shape: rounds of 256 configurations per work item, and
        // resident workgroups per compute unit (0: one workgroup per item);
        // each timed three times after a warm-up launch, the median kept
        const int rounds_c[] = {1, 2, 4, 8, 16, 32};
        const int wg_c[] = {0, 1, 2, 4, 8};
        constexpr int kReps = 3;
        for (int r : rounds_c)
            for (int w : wg_c) {
                cp_batch_tuning t{r, w};
                int rc = cp_batch_set_tuning(b, &t);
                if (rc) return rc;
                float ms[kReps];
                hipError_t e = launch_batch_eval(b->d_probs, b->d_partial, b->n, b->max_B, b->d_items, b->n_items, r,
                                                 b->grid(), b->cull, st);
                for (int k = 0; k < kReps && e == hipSuccess; ++k) {
                    e = hipEventRecord(e0, st);
                    if (e == hipSuccess)
                        e = launch_batch_eval(b->d_probs, b->d_partial, b->n, b->max_B, b->d_items, b->n_items, r,
                                              b->grid(), b->cull, st);
                    if (e == hipSuccess) e = hipEventRecord(e1, st);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms[k], e0, e1);
                }
                if (e != hipSuccess) return hip_fail(e, "tune timing");
                std::sort(ms, ms + kReps);
                if (ms[kReps / 2] < best_ms) {
                    best_ms = ms[kReps / 2];
                    best = t;
                }
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (cache_path) {
            if (FILE *f = std::fopen(cache_path, "a")) {
                std::fprintf(f, "%s %d %d %.4f\n", key, best.rounds, best.wg_per_cu, best_ms);
                std::fclose(f);
            }
        }
    }
    int rc = cp_batch_set_tuning(b, &best);
    if (rc) return rc;
    if (chosen) *chosen = best;
    return CP_OK;
}

// ---------------------------------------------------------------------------
// signed-distance grid
// ---------------------------------------------------------------------------

int cp_sdf_build(const float *d_points, int64_t N, const int32_t dims[3], const float origin[3], float voxel,
                 float *d_sdf, uint8_t *d_occ, int32_t *d_edt_occ, int32_t *d_edt_free, cp_stream_t stream) {
    if (!dims || !origin || !d_sdf || (N > 0 && !d_points)) return fail(CP_ERR_INVALID_ARG, "null argument");
    if (N < 0) return fail(CP_ERR_SIZE, "N must be >= 0");
    for (int a = 0; a < 3; ++a) {
        if (dims[a] < 2 || dims[a] > 4096) return fail(CP_ERR_SIZE, "dims must be in 2..4096");
        if (!finite(origin[a])) return fail(CP_ERR_INVALID_ARG, "non-finite origin");
    }
    if (!(voxel > 0.0f) || !finite(voxel)) return fail(CP_ERR_INVALID_ARG, "voxel must be > 0");
    const size_t n = (size_t)dims[0] * dims[1] * dims[2];
    if (n > ((size_t)1 << 31)) return fail(CP_ERR_SIZE, "grid too large");
    take_stale_error();
    int dev;
    CP_HIP(hipGetDevice(&dev), "device");
    hipStream_t st = (hipStream_t)stream;
    uint8_t *occ = d_occ;
    int32_t *eo = d_edt_occ, *ef = d_edt_free;
    // the output grid doubles as the transforms' scratch (the sign pass, which
    // writes it, runs last)
    int32_t *work = reinterpret_cast<int32_t *>(d_sdf);
    std::vector<void *> owned;
    auto cleanup = [&]() {
        for (void *q : owned) (void)hipFree(q);
    };
    auto get = [&](void **q, size_t bytes) {
        hipError_t e = hipMalloc(q, bytes);
        if (e == hipSuccess) owned.push_back(*q);
        return e;
    };
    hipError_t e = hipSuccess;
    if (!occ) e = get((void **)&occ, n);
    if (e == hipSuccess && !eo) e = get((void **)&eo, n * 4);
    if (e == hipSuccess && !ef) e = get((void **)&ef, n * 4);
    if (e == hipSuccess) e = launch_sdf_build(d_points, N, dims, origin, voxel, d_sdf, occ, eo, ef, work, st);
    if (e == hipSuccess && !owned.empty()) e = hipStreamSynchronize(st);
    cleanup();
    if (e != hipSuccess) return hip_fail(e, "sdf build");
    return CP_OK;
}

int cp_tune(cp_plan *plan, cp_batch *batch, const char *cache_path) {
    if (!plan && !batch) return fail(CP_ERR_INVALID_ARG, "null plan and batch");
    if (batch) return cp_batch_tune(batch, cache_path, nullptr);
    return CP_OK;
}

}  // extern "C"
