// Path evaluation (Algorithm 1, step 2) and its adjoint.
//
// Forward: one lane per checkpoint configuration (path b, checkpoint k),
// configurations flattened over all paths so that every wave is full.  Each
// lane interpolates its configuration from four control points, runs the
// kinematic chain in registers, and takes the minimum signed distance of its
// spheres to the scene.  Obstacle records are wave-uniform, so they are read
// with scalar loads into SGPRs and consumed directly by the vector ALU; no LDS
// or vector memory traffic sits in the pair loop.  Per-path sums are formed by
// a fixed-order wave reduction per path segment and a second fixed-order pass
// over waves, so results are bitwise reproducible.
#include "launch.h"

namespace cp {

// Wave-level culling.  The configurations of a wave are consecutive
// checkpoints of at most NS paths, so each sphere's centres over the lanes of
// one path (a segment) lie in a small box.  Per sphere and segment:
//  1. the box [xl, xh] x [yl, yh] (wave reductions);
//  2. U = min over cylinders o of (farthest box point to o's axis - R_o), an
//     upper bound of every segment lane's final minimum a;
//  3. a cylinder is a candidate only if the nearest box point comes within
//     U + R_o (+ slack) of its axis; the others cannot lower any lane's a.
// Steps 2 and 3 put one cylinder on each lane (64 per pass), and the
// candidates are then evaluated by every lane with the same arithmetic as the
// all-pairs loop.  Boxes are culled the same way against the wave maximum of
// the running minimum v, with the 3-D gap between the obstacle and the union
// of the group's sphere boxes as the lower bound.  The per-axis bounds are exact in floating point (rounding is
// monotone, so the nearest box point's squared distance never exceeds a
// lane's and the farthest one's is never below it); only the square roots and
// the threshold carry rounding, covered by 1e-4 m plus 1e-6 relative slack.
// Results are therefore bitwise those of the all-pairs evaluation.
constexpr float kCullAbs = 1e-4f;
constexpr float kCullRel = 1e-6f;

// Grid cell range [c0, c1] along one axis covering the interval [x0, x1]
// (clamped to the grid; widened by a hair so that a centre on a cell border,
// binned in double precision on the host, is never missed).
__device__ __forceinline__ void cell_span(float x0, float x1, float g0, float ginv, int n, int &c0, int &c1) {
    const float slack = 1e-3f + 4e-7f * (fabsf(x0) + fabsf(x1) + fabsf(g0)) * ginv;
    const float f0 = floorf((x0 - g0) * ginv - slack), f1 = floorf((x1 - g0) * ginv + slack);
    c0 = (int)fminf(fmaxf(f0, 0.0f), (float)(n - 1));
    c1 = (int)fminf(fmaxf(f1, 0.0f), (float)(n - 1));
}

// Calls f(idx) once per 64 cylinders of the cells overlapping
// [x0, x1] x [y0, y1] (every cell when `whole` is set or a bound is not
// finite); on each call lane l holds the cyl_cell index of one cylinder or -1.
// A row's cells are contiguous in cyl_cell, so the region is a list of row
// runs, packed onto the lanes in order.
template <class F>
__device__ __forceinline__ void for_cells(const PlanView &P, const GroupDev &gr, float x0, float x1, float y0,
                                          float y1, bool whole, int lane, F &&f) {
    int cx0 = 0, cx1 = gr.gnx - 1, cy0 = 0, cy1 = gr.gny - 1;
    if (!whole && fabsf(x0) < 1e30f && fabsf(x1) < 1e30f && fabsf(y0) < 1e30f && fabsf(y1) < 1e30f) {
        cell_span(x0, x1, gr.gx0, gr.ginv, gr.gnx, cx0, cx1);
        cell_span(y0, y1, gr.gy0, gr.ginv, gr.gny, cy0, cy1);
    }
    cx0 = __builtin_amdgcn_readfirstlane(cx0);
    cx1 = __builtin_amdgcn_readfirstlane(cx1);
    cy0 = __builtin_amdgcn_readfirstlane(cy0);
    cy1 = __builtin_amdgcn_readfirstlane(cy1);
    const int32_t *cs = P.cell_start + gr.gcell;
    const int nx = gr.gnx;
    int total = 0;
    for (int iy = cy0; iy <= cy1; ++iy) total += ldg(cs, iy * nx + cx1 + 1) - ldg(cs, iy * nx + cx0);
    for (int t0 = 0; t0 < total; t0 += kWave) {
        int idx = -1, acc = 0;
        for (int iy = cy0; iy <= cy1 && acc < t0 + kWave; ++iy) {
            const int s0 = ldg(cs, iy * nx + cx0), len = ldg(cs, iy * nx + cx1 + 1) - s0;
            const int t = t0 + lane - acc;
            if (t >= 0 && t < len) idx = s0 + t;
            acc += len;
        }
        f(idx);
    }
}

// The minima over the primitive obstacles are exact for the lanes with `in`
// set (one segment); the other lanes' results are unspecified.  With `all` set (a non-finite centre in the
// segment, where the box bounds do not hold) every obstacle is a candidate.
template <int G>
__device__ __forceinline__ void spheres_min_sd_culled(const PlanView &P, const float (&cx)[G], const float (&cy)[G],
                                                      const float (&cz)[G], bool in, bool all, float (&v)[G]) {
    const int lane = (int)(threadIdx.x & (kWave - 1));
    // one box around the centres of all the group's spheres over the
    // segment's lanes
    float bxl = cx[0], bxh = cx[0], byl = cy[0], byh = cy[0];
#pragma unroll
    for (int s = 1; s < G; ++s) {
        bxl = fminf(bxl, cx[s]); bxh = fmaxf(bxh, cx[s]);
        byl = fminf(byl, cy[s]); byh = fmaxf(byh, cy[s]);
    }
    bxl = in ? bxl : kInf;
    bxh = in ? bxh : -kInf;
    byl = in ? byl : kInf;
    byh = in ? byh : -kInf;
    wave_box(bxl, bxh, byl, byh);
#pragma unroll
    for (int s = 0; s < G; ++s) v[s] = P.has_ground ? cz[s] - P.ground_z : kInf;
    const float4 kFar = make_float4(1e15f, 1e15f, 0.0f, 0.0f);
    for (int g = 0; g < P.n_groups; ++g) {
        const GroupDev gr = ldg(P.groups, g);
        // upper bounds U_s: every lane's distance from sphere s to one
        // cylinder near that lane's spheres (the hint of the hint-grid cell
        // holding the centre of the group's middle sphere), maximised over the
        // segment's lanes.  Each lane's final minimum a_s is at most its own
        // value for that cylinder, computed with the same arithmetic.  (A hint
        // per lane rather than one for the wave keeps U close to the largest
        // of the lanes' true minima; one per group of spheres rather than per
        // sphere measured faster.)
        float umax = -kInf;  // max over the spheres of U + slack
        {
            float r[4];
            float4 c = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (!all) {
                const int m = G / 2;
                const float hx = (cx[m] - gr.hx0) * gr.hinv;
                const float hy = (cy[m] - gr.hy0) * gr.hinv;
                const int ix = (int)fminf(fmaxf(hx, 0.0f), (float)(gr.hn - 1));
                const int iy = (int)fminf(fmaxf(hy, 0.0f), (float)(gr.hn - 1));
                c = ldg(P.cyl_cell, ldg(P.hint, gr.hoff + iy * gr.hn + ix));
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                r[s] = s < G ? kInf : -kInf;
                if (s < G && !all) {
                    const float dx = cx[s] - c.x, dy = cy[s] - c.y;
                    r[s] = in ? fsqrt(__builtin_fmaf(dx, dx, dy * dy)) - c.z : -kInf;
                }
            }
            // one wave maximum over the lanes' largest U_s: each sphere's
            // threshold U_s + slack(|U_s|) is at most U + slack(max(|U|, R_max))
            // since -R_max <= U_s <= U
            float rl = r[0];
#pragma unroll
            for (int s = 1; s < G; ++s) rl = fmaxf(rl, r[s]);
            const float U = wave_max_u(rl);
            umax = U + (kCullAbs + kCullRel * (fmaxf(fabsf(U), gr.rmax) + 2.0f * gr.rmax));
        }
        const float e2 = fmaxf(umax + gr.rmax, 0.0f);
        // candidates: a cylinder can lower sphere s's minimum only if its
        // axis comes within U_s + R (+ slack) of s's centres, so within
        // max_s U_s + R of the group's box (within e2 of it for the grid
        // cells); a candidate is evaluated exactly for every sphere of the
        // group, its entry fetched once through the scalar cache (by the
        // index read out of its lane).  (Per-sphere boxes would
        // cull a few more pairs, about 7 % at c1, for four times the box
        // reductions and tests.)
        float a[G];
#pragma unroll
        for (int s = 0; s < G; ++s) a[s] = kInf;
        for_cells(P, gr, bxl - e2, bxh + e2, byl - e2, byh + e2, all, lane, [&](int idx) {
            float4 cc = ldg(P.cyl_cell, max(idx, 0));
            if (idx < 0) cc = kFar;
            const float ex = fmaxf(fmaxf(bxl - cc.x, cc.x - bxh), 0.0f);
            const float ey = fmaxf(fmaxf(byl - cc.y, cc.y - byh), 0.0f);
            const float n2 = __builtin_fmaf(ex, ex, ey * ey);
            const float th = fmaxf(umax + cc.z, 0.0f);
            uint64_t any = __builtin_amdgcn_ballot_w64(idx >= 0 && (all || n2 < th * th));
            while (any) {
                const int l = (int)__builtin_ctzll(any);
                any &= any - 1;
                const float4 o = ldg(P.cyl_cell, __builtin_amdgcn_readlane(idx, l));
                const float ox = o.x, oy = o.y, R = o.z;
#pragma unroll
                for (int s = 0; s < G; ++s) {
                    const float dx = cx[s] - ox, dy = cy[s] - oy;
                    a[s] = fmin_q(a[s], fsqrt(__builtin_fmaf(dx, dx, dy * dy)) - R);
                }
            }
        });
#pragma unroll
        for (int s = 0; s < G; ++s) v[s] = fminf(v[s], cyl_combine(a[s], fabsf(cz[s] - gr.zc) - gr.hz));
    }
    if (P.n_box > 0) {
        // one test per obstacle box for the whole sphere group: the gap between
        // the union of the spheres' boxes and the obstacle, against the wave
        // maximum of the running minima (obstacle boxes that pass are
        // evaluated for every sphere of the group)
        float zlo = cz[0], zhi = cz[0], vmax = v[0], unused = 0.0f;
#pragma unroll
        for (int s = 1; s < G; ++s) {
            zlo = fminf(zlo, cz[s]);
            zhi = fmaxf(zhi, cz[s]);
            vmax = fmaxf(vmax, v[s]);
        }
        zlo = in ? zlo : kInf;
        zhi = in ? zhi : -kInf;
        vmax = in ? vmax : -kInf;
        wave_box(zlo, zhi, unused, vmax);
        const float th = fmaxf(vmax + (kCullAbs + kCullRel * fabsf(vmax)), 0.0f);
        for (int o0 = 0; o0 < P.n_box; o0 += kWave) {
            const int ob = min(o0 + lane, P.n_box - 1);
            const float4 b0 = ldg(P.box, 2 * ob), b1 = ldg(P.box, 2 * ob + 1);
            const bool real = o0 + lane < P.n_box;
            // per axis: distance of the box of centres from the obstacle's slab
            const float gx = fmaxf(fmaxf(fmaxf(bxl - b0.x, b0.x - bxh), 0.0f) - b0.w, 0.0f);
            const float gy = fmaxf(fmaxf(fmaxf(byl - b0.y, b0.y - byh), 0.0f) - b1.x, 0.0f);
            const float gz = fmaxf(fmaxf(fmaxf(zlo - b0.z, b0.z - zhi), 0.0f) - b1.y, 0.0f);
            const float g2 = __builtin_fmaf(gx, gx, __builtin_fmaf(gy, gy, gz * gz));
            const bool cand = all || g2 <= 0.0f || g2 < th * th;
            uint64_t m = __builtin_amdgcn_ballot_w64(cand && real);
            while (m) {
                const int o = o0 + (int)__builtin_ctzll(m);
                m &= m - 1;
                const float4 c0 = ldg(P.box, 2 * o), c1 = ldg(P.box, 2 * o + 1);
#pragma unroll
                for (int s = 0; s < G; ++s) v[s] = fminf(v[s], box_sd(cx[s], cy[s], cz[s], c0, c1));
            }
        }
    }
}

// Lane state of the running minimum over spheres.
struct Best {
    float d;
    int s;           // caller's sphere index
    float r;         // its radius
    float v;         // its minimum signed distance over the obstacles (d = v - r)
    float cx, cy, cz;
    int sb;          // a self-collision pair (s, sb), s < sb; -1: a scene obstacle
};

// Pair order on equal distances: the lower sphere, then (for the same
// sphere) its scene obstacles before its self pairs, self pairs by the other
// sphere.  Candidate (d, s, sb) (sb = -1: a scene obstacle) beats `best`?
__device__ __forceinline__ bool pair_before(float d, int s, int sb, const Best &best) {
    if (d != best.d) return d < best.d;
    if (s != best.s) return s < best.s;
    if (sb < 0) return best.sb >= 0;
    return best.sb >= 0 && sb < best.sb;
}

// How the lanes of a wave split into paths for the wave-level culling: n
// segments (1 or 2) and this lane's segment (-1: result unused).
struct WaveSeg {
    int n;
    int lane;
};

template <int G, bool ARG, bool CULL>
__device__ __forceinline__ void sphere_group(const PlanView &P, const Xf &T, int s0, Best &best, WaveSeg ws) {
    float cx[G], cy[G], cz[G], v[G];
    bool finite = true;
#pragma unroll
    for (int i = 0; i < G; ++i) {
        const SphereDev sp = ldg(P.spheres, s0 + i);
        xf_point(T, sp.lx, sp.ly, sp.lz, cx[i], cy[i], cz[i]);
        finite = finite && fabsf(cx[i]) < kInf && fabsf(cy[i]) < kInf && fabsf(cz[i]) < kInf;
    }
    if (CULL && P.clr) {
        // the whole group is skipped when, on every lane, a lower bound of
        // each of its spheres' distances (the clearance grid and the ground)
        // is strictly above the lane's running minimum: no pair of the group
        // could lower it or tie with it
        bool above = finite;
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const SphereDev sp = ldg(P.spheres, s0 + i);
            float lb = clearance_bound(P, cx[i], cy[i]);
            if (P.has_ground) lb = fminf(lb, cz[i] - P.ground_z);
            above = above && lb - sp.r > best.d;
        }
        if (__builtin_amdgcn_ballot_w64(ws.lane >= 0 && !above) == 0) return;
    }
    if (CULL) {
        // the box bounds hold only for finite centres: a wave with a
        // non-finite one (from non-finite waypoints) evaluates every pair
        const bool all = __builtin_amdgcn_ballot_w64(ws.lane >= 0 && !finite) != 0;
        // one pass per path segment (a wave holding the end of one path and
        // the start of the next bounds the two separately)
        spheres_min_sd_culled<G>(P, cx, cy, cz, ws.n == 2 ? ws.lane == 0 : ws.lane >= 0, all, v);
        if (ws.n == 2) {
            float vt[G];
            spheres_min_sd_culled<G>(P, cx, cy, cz, ws.lane == 1, all, vt);
#pragma unroll
            for (int i = 0; i < G; ++i) v[i] = ws.lane == 1 ? vt[i] : v[i];
        }
    } else {
        spheres_min_sd<G>(P, cx, cy, cz, v);
    }
#pragma unroll
    for (int i = 0; i < G; ++i) {
        const SphereDev sp = ldg(P.spheres, s0 + i);
        if (P.sdf) {
            // the grid term; skipped where the block's lower bound shows it
            // cannot bring this sphere below the lane's running minimum
            // (strictly, so ties keep their order)
            int i0[3];
            float f[3], dg[3];
            sdf_cell(P, cx[i], cy[i], cz[i], i0, f, dg);
            if (!P.sdf_lb || !(sdf_cell_bound(P, i0) - sp.r > best.d))
                v[i] = fminf(v[i], sdf_interp(P, i0, f, dg, nullptr));
        }
        float d = v[i] - sp.r;
        if (ARG) {
            if (pair_before(d, sp.orig, -1, best)) {
                best.d = d; best.s = sp.orig; best.r = sp.r; best.v = v[i];
                best.cx = cx[i]; best.cy = cy[i]; best.cz = cz[i]; best.sb = -1;
            }
        } else {
            best.d = fminf(best.d, d);
        }
    }
}

// Self-collision (Sec. 3.2 names it beside collision with the scene): the
// minimum over every sphere pair of the listed frame pairs of
// |c_a - c_b| - r_a - r_b, taken after the scene.  Frame pairs come sorted by
// (fa, fb), fa < fb: the chain runs once from the base to each fa and on
// from there to its fb's.  Outside CP_PAIRS_ALL a frame pair is skipped when
// on every lane a lower bound of all its sphere pairs (the distance between
// the frames' bounding spheres, less a rounding slack far above FP32 error)
// lies strictly above the lane's running minimum: such pairs cannot lower or
// tie it, so results are bitwise those of taking every pair.
template <bool ARG>
__device__ __forceinline__ void self_min(const PlanView &P, const float (&q)[CP_MAX_JOINTS], Best &best, WaveSeg ws) {
    int i = 0;
    while (i < P.n_self) {
        const int fa = ldg(P.self_pairs, i).x;
        Xf Ta;
        xf_identity(Ta);
        for (int j = 0; j < fa; ++j) xf_joint(Ta, ldg(P.joints, j), pick(q, j));
        Xf T = Ta;
        int cur = fa;
        for (; i < P.n_self && ldg(P.self_pairs, i).x == fa; ++i) {
            const int fb = ldg(P.self_pairs, i).y;
            for (; cur < fb; ++cur) xf_joint(T, ldg(P.joints, cur), pick(q, cur));
            if (P.pair_filter != CP_PAIRS_ALL) {
                const float4 ba = ldg(P.frame_bound, fa), bb = ldg(P.frame_bound, fb);
                float ax, ay, az, bx, by, bz;
                xf_point(Ta, ba.x, ba.y, ba.z, ax, ay, az);
                xf_point(T, bb.x, bb.y, bb.z, bx, by, bz);
                const float dx = ax - bx, dy = ay - by, dz = az - bz;
                const float lb = fsqrt(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz))) - ba.w - bb.w -
                                 (1e-3f + 1e-5f * (fabsf(ax) + fabsf(ay) + fabsf(az) + fabsf(bx) + fabsf(by) + fabsf(bz)));
                if (__builtin_amdgcn_ballot_w64(ws.lane >= 0 && !(lb > best.d)) == 0) continue;
            }
            const int a1 = ldg(P.frame_start, fa + 1), b0 = ldg(P.frame_start, fb), b1 = ldg(P.frame_start, fb + 1);
            for (int sa = ldg(P.frame_start, fa); sa < a1; ++sa) {
                const SphereDev pa = ldg(P.spheres, sa);
                float cx, cy, cz;
                xf_point(Ta, pa.lx, pa.ly, pa.lz, cx, cy, cz);
                for (int sb = b0; sb < b1; ++sb) {
                    const SphereDev pb = ldg(P.spheres, sb);
                    float ex, ey, ez;
                    xf_point(T, pb.lx, pb.ly, pb.lz, ex, ey, ez);
                    const float dx = cx - ex, dy = cy - ey, dz = cz - ez;
                    const float d = fsqrt(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz))) - pa.r - pb.r;
                    if (ARG) {
                        const int lo = min(pa.orig, pb.orig), hi = max(pa.orig, pb.orig);
                        if (pair_before(d, lo, hi, best)) {
                            best.d = d; best.s = lo; best.sb = hi;
                        }
                    } else {
                        best.d = fminf(best.d, d);
                    }
                }
            }
        }
    }
}

// d(q) for one configuration; with ARG also the minimising sphere and its centre.
// With split > 1 only the sphere groups numbered part, part + split, ... are
// taken (their minimum is merged with the other parts' by the caller).
template <bool ARG, bool CULL>
__device__ __forceinline__ Best config_distance(const PlanView &P, const float (&q)[CP_MAX_JOINTS], WaveSeg ws,
                                                int part = 0, int split = 1) {
    Best best;
    best.d = kInf; best.s = 0x7fffffff; best.r = 0.0f; best.v = kInf;
    best.cx = best.cy = best.cz = 0.0f;
    best.sb = -1;
    Xf T;
    xf_identity(T);
    int gi = 0;
    // With the group skip, the frame holding the most spheres goes first (its
    // early minimum lets more of the other groups be skipped), then the rest
    // base first; the chain of transforms is rebuilt from the base when the
    // order steps back.  The minimum does not depend on the order.
    const int lead = CULL && P.clr ? P.lead_frame : -1;
    int cur = 0;  // frame of T
    for (int step = 0; step <= P.n_joints; ++step) {
        const int f = lead < 0 ? step : step == 0 ? lead : step <= lead ? step - 1 : step;
        if (f < cur) {
            xf_identity(T);
            cur = 0;
        }
        for (; cur < f; ++cur) xf_joint(T, ldg(P.joints, cur), pick(q, cur));
        const int s1 = ldg(P.frame_start, f + 1);
        int s = ldg(P.frame_start, f);
        for (; s + 4 <= s1; s += 4, ++gi)
            if (gi % split == part) sphere_group<4, ARG, CULL>(P, T, s, best, ws);
        if (s < s1 && gi++ % split == part) {
            switch (s1 - s) {
                case 3: sphere_group<3, ARG, CULL>(P, T, s, best, ws); break;
                case 2: sphere_group<2, ARG, CULL>(P, T, s, best, ws); break;
                case 1: sphere_group<1, ARG, CULL>(P, T, s, best, ws); break;
                default: break;
            }
        }
    }
    if (P.n_self > 0 && part == 0) self_min<ARG>(P, q, best, ws);
    return best;
}

// Obstacle of the minimising pair for centre c (lowest number on ties):
// recomputes every obstacle's signed distance with the same arithmetic as the
// forward pass, in the caller's table order.
__device__ __forceinline__ uint32_t argmin_obstacle(const PlanView &P, float cx, float cy, float cz) {
    float bv = kInf;
    uint32_t bo = 0;
    if (P.has_ground) { bv = cz - P.ground_z; bo = 0; }
    for (int o = 0; o < P.n_cyl; ++o) {
        const float4 c = ldg(P.cyl_orig, o);
        const GroupDev gr = ldg(P.groups, __float_as_int(c.w));
        float val = cyl_combine(cyl_radial(cx, cy, c), fabsf(cz - gr.zc) - gr.hz);
        if (val < bv) { bv = val; bo = 1u + (uint32_t)o; }
    }
    for (int o = 0; o < P.n_box; ++o) {
        float val = box_sd(cx, cy, cz, ldg(P.box, 2 * o), ldg(P.box, 2 * o + 1));
        if (val < bv) { bv = val; bo = 1u + (uint32_t)(P.n_cyl + o); }
    }
    if (P.sdf) {
        float val = sdf_query(P, cx, cy, cz, nullptr);
        if (val < bv) { bv = val; bo = CP_OBS_SDF; }
    }
    return bo;
}

// The same choice as argmin_obstacle when v is the minimum over the
// obstacles at c (the value the evaluation found): a cylinder's signed
// distance is never below its radial term, so only cylinders whose axis lies
// within v + R_max (+ slack) of c can attain v, and those are read from the
// cell grid; ties keep the lowest obstacle number, as in the full scan.
__device__ __forceinline__ uint32_t argmin_obstacle_near(const PlanView &P, float cx, float cy, float cz, float v) {
    if (!(fabsf(cx) < kInf && fabsf(cy) < kInf && fabsf(cz) < kInf && fabsf(v) < kInf))
        return argmin_obstacle(P, cx, cy, cz);
    float bv = kInf;
    uint32_t bo = 0;
    if (P.has_ground) { bv = cz - P.ground_z; bo = 0; }
    for (int g = 0; g < P.n_groups; ++g) {
        const GroupDev gr = ldg(P.groups, g);
        const float E = fmaxf(v + gr.rmax + kCullAbs +
                                  kCullRel * (fabsf(v) + 2.0f * gr.rmax + fabsf(cx) + fabsf(cy)),
                              0.0f);
        int cx0, cx1, cy0, cy1;
        cell_span(cx - E, cx + E, gr.gx0, gr.ginv, gr.gnx, cx0, cx1);
        cell_span(cy - E, cy + E, gr.gy0, gr.ginv, gr.gny, cy0, cy1);
        const int32_t *cs = P.cell_start + gr.gcell;
        const float bz = fabsf(cz - gr.zc) - gr.hz;
        for (int iy = cy0; iy <= cy1; ++iy) {
            const int e1 = ldg(cs, iy * gr.gnx + cx1 + 1);
            for (int e = ldg(cs, iy * gr.gnx + cx0); e < e1; ++e) {
                const float4 c = ldg(P.cyl_cell, e);
                const float val = cyl_combine(cyl_radial(cx, cy, c), bz);
                const uint32_t id = 1u + (uint32_t)__float_as_int(c.w);
                if (val < bv || (val == bv && id < bo)) { bv = val; bo = id; }
            }
        }
    }
    for (int o = 0; o < P.n_box; ++o) {
        float val = box_sd(cx, cy, cz, ldg(P.box, 2 * o), ldg(P.box, 2 * o + 1));
        if (val < bv) { bv = val; bo = 1u + (uint32_t)(P.n_cyl + o); }
    }
    if (P.sdf) {
        float val = sdf_query(P, cx, cy, cz, nullptr);
        if (val < bv) { bv = val; bo = CP_OBS_SDF; }
    }
    return bo;
}

// The obstacle of the winning pair of a configuration.  In a scene of the
// ground and a grid alone it follows from the minimum itself: the winning
// sphere's minimum over the two is one of them exactly (where its grid term
// was skipped, the grid's lower bound already lay above the ground term), and
// a tie keeps the ground, the lower number, as the full rescan does.  A
// non-finite centre or minimum takes the rescan.
template <bool CULL>
__device__ __forceinline__ uint32_t argmin_of(const PlanView &P, const Best &best) {
    if (best.sb >= 0) return CP_OBS_SELF + (uint32_t)best.sb;
    if (P.sdf && P.n_cyl == 0 && P.n_box == 0 && fabsf(best.cz) < kInf && fabsf(best.v) < kInf) {
        if (P.has_ground && best.cz - P.ground_z == best.v) return 0;
        return best.v < kInf ? CP_OBS_SDF : 0u;
    }
    return CULL ? argmin_obstacle_near(P, best.cx, best.cy, best.cz, best.v)
                : argmin_obstacle(P, best.cx, best.cy, best.cz);
}

// Per-lane minima of the waves of a workgroup (up to 8), for merging split parts.
struct MergeBuf {
    float d[8][kWave], r[8][kWave], v[8][kWave], cx[8][kWave], cy[8][kWave], cz[8][kWave];
    int s[8][kWave], sb[8][kWave];
};

// One configuration per lane: g is the flattened (path, checkpoint) index;
// all 64 lanes of a wave hold consecutive g (some may lie past the end).
// SPLIT: `split` consecutive waves of the workgroup hold the same
// configurations and share out the sphere groups; the first of them merges
// the others' minima (the minimum over all pairs, and with the tape the
// lowest sphere among equal minima, do not depend on the order) and finishes.
template <bool TAPE, bool CULL, bool SPLIT = false>
__device__ __forceinline__ void eval_one(const PlanView &P, const float *__restrict__ W, int B,
                                         double2 *__restrict__ partial, int slots, uint32_t *__restrict__ tape,
                                         int64_t g, int part = 0, int split = 1, MergeBuf *mb = nullptr) {
    const int64_t N = (int64_t)B * P.ns;
    const bool active = g < N;
    const int b = active ? (int)(g / P.ns) : B - 1;
    const int k = active ? (int)(g - (int64_t)b * P.ns) + 1 : 1;
    const float *Wb = W + (size_t)b * P.K * P.n_joints;

    float q[CP_MAX_JOINTS], dq[CP_MAX_JOINTS], bw[4], db[4];
    int j;
    interpolate(P, Wb, k, q, dq, j, bw, db);
    float jp, jl;
    step_terms(P, q, dq, jp, jl);

    // paths p0..p1 of this wave (contiguous; wave-uniform, kept in scalar registers)
    const int64_t g_first = uniform_i64(g & ~(int64_t)(kWave - 1));
    const int64_t w = g_first / kWave;
    const int64_t g_last = min(g_first + kWave - 1, N - 1);
    const int p0 = (int)(g_first / P.ns), p1 = (int)(g_last / P.ns);
    // (a wave over more than two paths, only when a path has fewer than 64
    // checkpoints, is bounded as one segment: still exact, culls less)
    WaveSeg ws;
    ws.n = p1 - p0 == 1 ? 2 : 1;
    ws.lane = active ? (ws.n == 2 ? b - p0 : 0) : -1;
    Best best = config_distance<TAPE, CULL>(P, q, ws, part, split);
    if (SPLIT) {
        const int wv = threadIdx.x >> 6, ln = threadIdx.x & (kWave - 1);
        if (part != 0) {
            mb->d[wv][ln] = best.d;
            if (TAPE) {
                mb->s[wv][ln] = best.s; mb->r[wv][ln] = best.r; mb->v[wv][ln] = best.v; mb->sb[wv][ln] = best.sb;
                mb->cx[wv][ln] = best.cx; mb->cy[wv][ln] = best.cy; mb->cz[wv][ln] = best.cz;
            }
        }
        __syncthreads();
        if (part != 0) return;
        for (int u = 1; u < split; ++u) {
            const float d = mb->d[wv + u][ln];
            if (TAPE) {
                const int so = mb->s[wv + u][ln], sbo = mb->sb[wv + u][ln];
                if (pair_before(d, so, sbo, best)) {
                    best.d = d; best.s = so; best.sb = sbo; best.r = mb->r[wv + u][ln]; best.v = mb->v[wv + u][ln];
                    best.cx = mb->cx[wv + u][ln]; best.cy = mb->cy[wv + u][ln]; best.cz = mb->cz[wv + u][ln];
                }
            } else {
                best.d = fminf(best.d, d);
            }
        }
    }
    float dphi;
    float phi = hinge_value(P, best.d, dphi);
    float c = __builtin_fmaf(P.w_c, phi, __builtin_fmaf(P.w_l, jl, jp));
    if (TAPE && active) {
        tape[g] = ((uint32_t)best.s << 16) | argmin_of<CULL>(P, best);
    }
    path_partials(active ? b : -1, c, best.d, p0, p1, w, partial, slots);
}

// The culling path holds more state than the plain pair loop; five waves per
// SIMD (at most 96 registers per lane) measured faster than the compiler's
// unconstrained four, and six spill.
template <bool TAPE, bool CULL>
__global__ __launch_bounds__(256, CULL ? 5 : 1) void k_eval_fwd(PlanView P, const float *__restrict__ W, int B,
                                                  double2 *__restrict__ partial, int slots, uint32_t *__restrict__ tape) {
    eval_one<TAPE, CULL>(P, W, B, partial, slots, tape, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Small launches (too few waves to fill the chip): each group of `split`
// waves (2, 4 or 8) of a workgroup of NW waves takes one wave's 64
// configurations and shares out their sphere groups, so the per-wave chain is
// up to `split` times shorter.  With the tape, four waves per SIMD (128
// registers): at five the merge state spills heavily.
template <bool TAPE, bool CULL, int NW>
__global__ __launch_bounds__(NW * 64, NW == 4 ? (CULL ? (TAPE ? 4 : 5) : 1) : (CULL ? 2 : 1)) void k_eval_fwd_split(
    PlanView P, const float *__restrict__ W, int B, double2 *__restrict__ partial, int slots,
    uint32_t *__restrict__ tape, int split) {
    __shared__ MergeBuf mb;
    const int wv = threadIdx.x >> 6;
    const int64_t cw = (int64_t)blockIdx.x * (NW / split) + wv / split;
    eval_one<TAPE, CULL, true>(P, W, B, partial, slots, tape, cw * kWave + (threadIdx.x & (kWave - 1)), wv % split,
                               split, &mb);
}

// Many problems in one launch: the work items (problem, first configuration)
// are listed costliest problem first and dealt to the workgroups round robin
// (workgroup w takes items w, w + G, w + 2G, ...); an item covers `rounds` x
// 256 consecutive configurations of one problem.  With a grid of a few
// workgroups per compute unit the workgroups are persistent and the deal
// balances to within one item; with one workgroup per item the hardware
// dispatcher hands items out in order as compute units free up.
// Every configuration runs exactly the single-problem code, so results are
// bitwise those of k_eval_fwd on each problem.  (The kernel has no atomics and
// stores only through the restrict-qualified partial-sum base pointer, so the
// compiler can prove the tables unchanged and keeps their wave-uniform reads
// in scalar loads; a global work counter would turn them into vector loads.)
template <bool CULL>
__global__ __launch_bounds__(256, CULL ? 5 : 6) void k_eval_persistent(const BatchProblem *__restrict__ probs,
                                                         double2 *__restrict__ partial,
                                                         const int2 *__restrict__ items, int n_items, int rounds) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = ldg(items, it);
        const int p = item.x, g0 = item.y;
        // only what the evaluation needs (the optimizer state stays in memory)
        const BatchProblem *bp = probs + p;
        const PlanView P = ldg(&bp->P);
        const float *W = ldg(&bp->O.W);
        const int B = ldg(&bp->O.B);
        const int slots = ldg(&bp->slots);
        double2 *part = partial + ldg(&bp->partial_off);
        for (int r = 0; r < rounds; ++r)
            eval_one<false, CULL>(P, W, B, part, slots, nullptr, (int64_t)g0 + r * 256 + threadIdx.x);
    }
}

__global__ __launch_bounds__(256) void k_eval_reduce(const double2 *__restrict__ partial, int slots, int B, int ns,
                                                     float margin, float *__restrict__ cost,
                                                     float *__restrict__ min_dist, uint8_t *__restrict__ flags) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) reduce_one(partial, slots, ns, margin, cost, min_dist, flags, b);
}

// per-problem path sums of a batch: blockIdx.y = problem
__global__ __launch_bounds__(256) void k_reduce_batched(const BatchProblem *__restrict__ probs,
                                                        const double2 *__restrict__ partial) {
    const BatchProblem &bp = probs[blockIdx.y];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < bp.O.B)
        reduce_one(partial + bp.partial_off, bp.slots, bp.P.ns, bp.P.margin, bp.O.cost, bp.O.min_dist, nullptr, b);
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------

// d cost_k / d q for the collision term through the tape's pair (s, o):
// recomputes the chain, the sphere centre and the pair's signed distance.  A
// self-collision pair (o = CP_OBS_SELF + b) differentiates
// |c_s - c_b| - r_s - r_b through both spheres' chains.
__device__ __forceinline__ void collision_grad(const PlanView &P, const float (&q)[CP_MAX_JOINTS], int s_orig,
                                               uint32_t o, float (&gq)[CP_MAX_JOINTS]) {
    const bool self = o >= CP_OBS_SELF && o < CP_OBS_SDF;
    const int b_orig = self ? (int)(o - CP_OBS_SELF) : 0;
    // locate the spheres (table sorted by frame; `orig` is the caller's index)
    const int si = (s_orig >= 0 && s_orig < P.n_spheres) ? ldg(P.sphere_slot, s_orig) : 0;
    const int bi = (self && b_orig < P.n_spheres) ? ldg(P.sphere_slot, b_orig) : 0;
    const SphereDev sp = ldg(P.spheres, si);
    const SphereDev sq = ldg(P.spheres, bi);
    float aw[CP_MAX_JOINTS][3], pj[CP_MAX_JOINTS][3];
    float cx = 0.0f, cy = 0.0f, cz = 0.0f, ex = 0.0f, ey = 0.0f, ez = 0.0f;
    Xf T;
    xf_identity(T);
    if (sp.frame == 0) xf_point(T, sp.lx, sp.ly, sp.lz, cx, cy, cz);
    if (sq.frame == 0) xf_point(T, sq.lx, sq.ly, sq.lz, ex, ey, ez);
#pragma unroll
    for (int f = 1; f <= CP_MAX_JOINTS; ++f) {
        if (f <= P.n_joints) {
            const JointDev J = ldg(P.joints, f - 1);
            // world axis of joint f-1: R_{f-1} a (unchanged by its own rotation)
            aw[f - 1][0] = __builtin_fmaf(T.r[0], J.ax, __builtin_fmaf(T.r[1], J.ay, T.r[2] * J.az));
            aw[f - 1][1] = __builtin_fmaf(T.r[3], J.ax, __builtin_fmaf(T.r[4], J.ay, T.r[5] * J.az));
            aw[f - 1][2] = __builtin_fmaf(T.r[6], J.ax, __builtin_fmaf(T.r[7], J.ay, T.r[8] * J.az));
            xf_joint(T, J, q[f - 1]);
            pj[f - 1][0] = T.p[0]; pj[f - 1][1] = T.p[1]; pj[f - 1][2] = T.p[2];
            if (sp.frame == f) xf_point(T, sp.lx, sp.ly, sp.lz, cx, cy, cz);
            if (sq.frame == f) xf_point(T, sq.lx, sq.ly, sq.lz, ex, ey, ez);
        }
    }
    // a tape entry that names no pair of this plan contributes nothing
    const bool valid = self ? (P.n_self > 0 && b_orig < P.n_spheres)
                            : (o == CP_OBS_SDF) ? (P.sdf != nullptr)
                                                : (o == 0 ? P.has_ground != 0 : (int)o <= P.n_cyl + P.n_box);
    if (!valid || s_orig >= P.n_spheres) return;
    float gr[3];
    float sd;
    if (self) {
        // gradient of |c_s - c_b| with respect to c_s (minus it for c_b)
        const float dx = cx - ex, dy = cy - ey, dz = cz - ez;
        const float len = fsqrt(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz)));
        const float inv = len > 0.0f ? 1.0f / len : 0.0f;
        gr[0] = dx * inv; gr[1] = dy * inv; gr[2] = dz * inv;
        sd = len - sq.r;
    } else {
        sd = obstacle_sd_grad(P, o, cx, cy, cz, gr);
    }
    float dphi;
    hinge_value(P, sd - sp.r, dphi);
    float scale = P.w_c * dphi;
#pragma unroll
    for (int jj = 0; jj < CP_MAX_JOINTS; ++jj) {
        if (jj < P.n_joints && scale != 0.0f && (jj < sp.frame || (self && jj < sq.frame))) {
            const bool rev = P.joints[jj].type == CP_REVOLUTE;
            float jx = 0.0f, jy = 0.0f, jz = 0.0f;
            if (jj < sp.frame) {
                if (rev) {
                    float rx = cx - pj[jj][0], ry = cy - pj[jj][1], rz = cz - pj[jj][2];
                    jx = aw[jj][1] * rz - aw[jj][2] * ry;
                    jy = aw[jj][2] * rx - aw[jj][0] * rz;
                    jz = aw[jj][0] * ry - aw[jj][1] * rx;
                } else {
                    jx = aw[jj][0]; jy = aw[jj][1]; jz = aw[jj][2];
                }
            }
            if (self && jj < sq.frame) {
                if (rev) {
                    float rx = ex - pj[jj][0], ry = ey - pj[jj][1], rz = ez - pj[jj][2];
                    jx -= aw[jj][1] * rz - aw[jj][2] * ry;
                    jy -= aw[jj][2] * rx - aw[jj][0] * rz;
                    jz -= aw[jj][0] * ry - aw[jj][1] * rx;
                } else {
                    jx -= aw[jj][0]; jy -= aw[jj][1]; jz -= aw[jj][2];
                }
            }
            gq[jj] += scale * __builtin_fmaf(gr[0], jx, __builtin_fmaf(gr[1], jy, gr[2] * jz));
        }
    }
}

constexpr int kMaxCtrl = CP_MAX_K + 6;
// control points one wave can touch: 64 checkpoints span at most 64 windows
// of four consecutive control points
constexpr int kWaveCtrl = kWave + 3;

// One workgroup per path.  Each lane takes one checkpoint and forms its
// contribution to the four control points of its span window; per wave and
// control point the contributions are summed by DPP reductions (fixed order)
// and the wave sums are added in wave order in double precision.  A
// workgroup of NW waves takes 64 NW checkpoints per round; since every wave
// covers the same 64 checkpoints whatever NW, and the wave sums are added in
// the same order, the gradient does not depend on NW (16 for small launches,
// whose few workgroups would otherwise run several rounds each).
template <bool TAPE, bool CULL, int NW>
__global__ __launch_bounds__(NW * 64) void k_eval_bwd(PlanView P, const float *__restrict__ W, int B,
                                                          const uint32_t *__restrict__ tape,
                                                          const float *__restrict__ grad_cost,
                                                          float *__restrict__ grad_W, PolishStep pol) {
    constexpr int kBwdThreads = NW * kWave, kBwdWaves = NW;
    __shared__ float part[kBwdWaves][kWaveCtrl][CP_MAX_JOINTS];
    __shared__ int wlo[kBwdWaves], whi[kBwdWaves];
    __shared__ double acc[kMaxCtrl * CP_MAX_JOINTS];
    const int b = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int n = P.n_joints;
    // (the windows of the linear mode reach past its last control point: those
    // entries receive zero weights and are never read out)
    for (int i = tid; i < kMaxCtrl * CP_MAX_JOINTS; i += kBwdThreads) acc[i] = 0.0;
    const float *Wb = W + (size_t)b * P.K * n;
    for (int k0 = 1; k0 <= P.ns; k0 += kBwdThreads) {
        const int k = k0 + tid;
        const bool active = k <= P.ns;
        const int kk = active ? k : P.ns;
        float q[CP_MAX_JOINTS], dq[CP_MAX_JOINTS], bw[4], db[4];
        int j;
        interpolate(P, Wb, kk, q, dq, j, bw, db);
        float gq[CP_MAX_JOINTS], gd[CP_MAX_JOINTS];
        float sq = 0.0f;
#pragma unroll
        for (int i = 0; i < CP_MAX_JOINTS; ++i) sq = __builtin_fmaf(dq[i], dq[i], sq);
        float len = fsqrt(sq);
        float inv = len > 0.0f ? 1.0f / len : 0.0f;
#pragma unroll
        for (int i = 0; i < CP_MAX_JOINTS; ++i) {
            gd[i] = P.jp_mode == CP_JP_SQUARED ? 2.0f * dq[i] : dq[i] * inv;
            gq[i] = 0.0f;
            if (i < n) {
                const JointDev J = ldg(P.joints, i);
                float hi = fmaxf(q[i] - J.qmax, 0.0f), lo = fmaxf(J.qmin - q[i], 0.0f);
                gq[i] = P.w_l * (2.0f * hi - 2.0f * lo);
            }
        }
        int s_orig;
        uint32_t o;
        if (TAPE) {
            uint32_t t = tape[(size_t)b * P.ns + (kk - 1)];
            s_orig = (int)(t >> 16);
            o = t & 0xFFFFu;
        } else {
            // a block's lanes all hold checkpoints of path b (inactive ones repeat the last)
            WaveSeg ws;
            ws.n = 1;
            ws.lane = 0;
            Best best = config_distance<true, CULL>(P, q, ws);
            s_orig = best.s;
            o = argmin_of<CULL>(P, best);
        }
        collision_grad(P, q, s_orig, o, gq);
        float c[4][CP_MAX_JOINTS];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < CP_MAX_JOINTS; ++i) c[t][i] = active ? __builtin_fmaf(bw[t], gq[i], db[t] * gd[i]) : 0.0f;
        // this wave's control points: windows are non-decreasing along the lanes
        const int jlo = __builtin_amdgcn_readfirstlane(j);
        const int jhi = __builtin_amdgcn_readlane(j, kWave - 1);
        for (int cp = jlo; cp <= jhi + 3; ++cp) {
            const int t = cp - j;
#pragma unroll
            for (int i = 0; i < CP_MAX_JOINTS; ++i) {
                if (i < n) {
                    const float v = t == 0 ? c[0][i] : t == 1 ? c[1][i] : t == 2 ? c[2][i] : t == 3 ? c[3][i] : 0.0f;
                    const float sum = wave_sum_u(v);
                    if (lane == 0) part[wv][cp - jlo][i] = sum;
                }
            }
        }
        if (lane == 0) {
            wlo[wv] = jlo;
            whi[wv] = jhi + 3;
        }
        __syncthreads();
        // each control point: the waves' sums in wave order
        const int lo = wlo[0], hi = whi[kBwdWaves - 1];
        for (int idx = tid; idx < (hi - lo + 1) * n; idx += kBwdThreads) {
            const int cp = lo + idx / n, i = idx % n;
            double s = acc[cp * n + i];
#pragma unroll
            for (int w = 0; w < kBwdWaves; ++w)
                if (cp >= wlo[w] && cp <= whi[w]) s += (double)part[w][cp - wlo[w]][i];
            acc[cp * n + i] = s;
        }
        __syncthreads();
    }
    const float gc = grad_cost[b];
    const int lead = P.interp == CP_INTERP_BSPLINE ? 3 : 1;
    for (int idx = tid; idx < P.K * n; idx += kBwdThreads) {
        const int i = idx / n, jj = idx % n;
        grad_W[(size_t)b * P.K * n + idx] = gc * (float)acc[(i + lead) * n + jj];
    }
    if (pol.W_out && wv == 0) {
        // the polish step on this path, written to the step's output buffer
        // (the input W is only read): the gradient entries as written above,
        // squared and summed per lane then across the wave, then the clipped
        // step on the sampled joints; the other entries are copied
        float s = 0.0f;
        for (int e = lane; e < pol.D; e += kWave) {
            const int k = e / pol.n_act, jj = pol.act[e % pol.n_act];
            const float g = gc * (float)acc[(k + lead) * n + jj];
            s = __builtin_fmaf(g, g, s);
        }
        s = wave_sum(s);
        const float scale = pol.eta / fmaxf(1.0f, fsqrt(s) / pol.clip);
        float *Wo = pol.W_out + (size_t)b * P.K * n;
        for (int idx = lane; idx < P.K * n; idx += kWave) {
            const int k = idx / n, jj = idx - k * n;
            const float w = Wb[idx];
            if ((pol.act_mask >> jj) & 1u) {
                const float g = gc * (float)acc[(k + lead) * n + jj];
                Wo[idx] = w - scale * g;
            } else {
                Wo[idx] = w;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// test exports
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_debug_fk(PlanView P, const float *__restrict__ Q, int N,
                                                  float *__restrict__ centers, float *__restrict__ frames) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float q[CP_MAX_JOINTS];
#pragma unroll
    for (int jj = 0; jj < CP_MAX_JOINTS; ++jj) q[jj] = jj < P.n_joints ? Q[(size_t)i * P.n_joints + jj] : 0.0f;
    Xf T;
    xf_identity(T);
    for (int f = 0; f <= P.n_joints; ++f) {
        if (f > 0) xf_joint(T, ldg(P.joints, f - 1), pick(q, f - 1));
        if (frames) {
            float *fr = frames + ((size_t)i * (P.n_joints + 1) + f) * 12;
            for (int e = 0; e < 9; ++e) fr[e] = T.r[e];
            for (int e = 0; e < 3; ++e) fr[9 + e] = T.p[e];
        }
        if (centers) {
            for (int s = P.frame_start[f]; s < P.frame_start[f + 1]; ++s) {
                const SphereDev sp = P.spheres[s];
                float cx, cy, cz;
                xf_point(T, sp.lx, sp.ly, sp.lz, cx, cy, cz);
                float *c = centers + ((size_t)i * P.n_spheres + sp.orig) * 3;
                c[0] = cx; c[1] = cy; c[2] = cz;
            }
        }
    }
}

template <bool CULL>
__global__ __launch_bounds__(256) void k_debug_configs(PlanView P, const float *__restrict__ Q, int N,
                                                       float *__restrict__ dist, uint32_t *__restrict__ arg) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int ii = i < N ? i : N - 1;
    float q[CP_MAX_JOINTS];
#pragma unroll
    for (int jj = 0; jj < CP_MAX_JOINTS; ++jj) q[jj] = jj < P.n_joints ? Q[(size_t)ii * P.n_joints + jj] : 0.0f;
    // unrelated configurations: one segment (culling still exact, rarely useful)
    WaveSeg ws;
    ws.n = 1;
    ws.lane = 0;
    Best best = config_distance<true, CULL>(P, q, ws);
    uint32_t o = best.sb >= 0 ? CP_OBS_SELF + (uint32_t)best.sb : argmin_obstacle(P, best.cx, best.cy, best.cz);
    if (i < N) {
        dist[i] = best.d;
        if (arg) arg[i] = ((uint32_t)best.s << 16) | o;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

int eval_slots(int ns) { return kWave / ns + 2; }

// the wave-level culling runs when asked for and there is something to cull
// (a grid-only scene has neither cylinders nor boxes)
static bool use_cull(const PlanView &P) { return P.pair_filter == CP_PAIRS_WAVE && (P.n_groups > 0 || P.n_box > 0); }

// split launches from which the group-skip test is left out
constexpr int kNoClearanceSplit = 4;

// Waves per configuration wave: launches of fewer than about twelve waves
// per SIMD (1024 SIMDs) share each wave's sphere groups out over 8, 4 or 2
// waves (measured on the polish, c0 and c2 launches).
static int eval_split(int64_t waves) {
    if (waves <= 1024) return 8;
    if (waves <= 2048) return 4;
    if (waves <= 12288) return 2;
    return 1;
}

size_t eval_partial_count(int B, int ns) {
    const int64_t N = (int64_t)B * ns;
    return (size_t)((N + kWave - 1) / kWave) * eval_slots(ns);
}

// Clearance grid: per cell, the least horizontal signed distance from its
// centre to a cylinder (radial term) or a box footprint, less half the cell
// diagonal (the distance is 1-Lipschitz) and a margin for the rounding of the
// evaluation's FP32 distances: a lower bound of every such distance the
// evaluation computes anywhere in the cell.
__global__ __launch_bounds__(256) void k_clearance(PlanView P, float *__restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.clr_nx * P.clr_ny) return;
    const double px = P.clr_x0 + (c % P.clr_nx + 0.5) * (double)P.clr_h;
    const double py = P.clr_y0 + (c / P.clr_nx + 0.5) * (double)P.clr_h;
    double d = 1e30;
    for (int o = 0; o < P.n_cyl; ++o) {
        const float4 q = P.cyl_orig[o];
        d = fmin(d, sqrt((px - q.x) * (px - q.x) + (py - q.y) * (py - q.y)) - q.z);
    }
    for (int o = 0; o < P.n_box; ++o) {
        // signed distance to the footprint rectangle: below the box's signed
        // distance everywhere, inside the box included
        const float4 b0 = P.box[2 * o], b1 = P.box[2 * o + 1];
        const double qx = fabs(px - b0.x) - b0.w, qy = fabs(py - b0.y) - b1.x;
        const double ex = fmax(qx, 0.0), ey = fmax(qy, 0.0);
        d = fmin(d, sqrt(ex * ex + ey * ey) + fmin(fmax(qx, qy), 0.0));
    }
    const double m = 0.7072 * P.clr_h + 1e-4 + 1e-6 * (fabs(px) + fabs(py) + fabs(d) + 1.0);
    out[c] = (float)(d - m);
}

hipError_t launch_clearance(const PlanView &P, float *out, hipStream_t st) {
    const int n = P.clr_nx * P.clr_ny;
    hipLaunchKernelGGL(k_clearance, dim3((n + 255) / 256), dim3(256), 0, st, P, out);
    return hipGetLastError();
}

// Per block of cells (2 x 2 x 2), the smallest grid sample any of its cells
// interpolates, less a margin for the rounding of the three interpolation
// steps (each loses at most 3 units in the last place of the largest sample
// magnitude A; the margin is 1e-6 (A + 1)): a lower bound of every value
// sdf_interp computes in the block.
__global__ __launch_bounds__(256) void k_sdf_bound(PlanView P) {
    const int nbx = P.sdf_lbn[0], nby = P.sdf_lbn[1], nbz = P.sdf_lbn[2];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbx * nby * nbz) return;
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int nx = P.sdf_n[0], ny = P.sdf_n[1], nz = P.sdf_n[2];
    float mn = kInf, mx = 0.0f;
    const int w = 1 << kSdfBlockLog2;
    for (int z = w * bz; z <= min(w * bz + w, nz - 1); ++z)
        for (int y = w * by; y <= min(w * by + w, ny - 1); ++y)
            for (int x = w * bx; x <= min(w * bx + w, nx - 1); ++x) {
                const float val = P.sdf[((size_t)z * ny + y) * nx + x];
                mn = fminf(mn, val);
                mx = fmaxf(mx, fabsf(val));
            }
    P.sdf_lb_buf[b] = mn - (1e-6f + 1e-6f * mx);
}

// The view the evaluation kernels get: with a grid, its block bounds are
// refreshed from the current grid first and switched on (not in the
// every-pair mode, which takes every grid lookup too).
static hipError_t view_with_sdf_bound(const PlanView &P, PlanView &Q, hipStream_t st) {
    Q = P;
    if (!P.sdf || !P.sdf_lb_buf || P.pair_filter == CP_PAIRS_ALL) return hipSuccess;
    const int nb = P.sdf_lbn[0] * P.sdf_lbn[1] * P.sdf_lbn[2];
    hipLaunchKernelGGL(k_sdf_bound, dim3((nb + 255) / 256), dim3(256), 0, st, P);
    Q.sdf_lb = P.sdf_lb_buf;
    return hipGetLastError();
}

hipError_t launch_eval_fwd(const PlanView &P0, const float *W, int B, double2 *partial, uint32_t *tape,
                           float *cost, float *min_dist, uint8_t *flags, hipStream_t st, const EvalEvents *ev) {
    PlanView P;
    const hipError_t eb = view_with_sdf_bound(P0, P, st);
    if (eb != hipSuccess) return eb;
    if (ev) {
        const hipError_t er = hipEventRecord(ev->begin, st);
        if (er != hipSuccess) return er;
    }
    const int64_t N = (int64_t)B * P.ns;
    const int slots = eval_slots(P.ns);
    if (P.narrow == CP_NARROW_SAT) {
        hipError_t e = launch_eval_fwd_sat(P, W, B, partial, tape, st);
        if (e != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev->end, st)) != hipSuccess) return e;
        if (!cost && !min_dist && !flags) return hipSuccess;
        hipLaunchKernelGGL(k_eval_reduce, dim3((B + 255) / 256), dim3(256), 0, st, partial, slots, B, P.ns, P.margin,
                           cost, min_dist, flags);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((N + 255) / 256));
    const bool cull = use_cull(P);
    const int64_t waves = (N + kWave - 1) / kWave;
    const int split = eval_split(waves);
    // with the sphere groups shared out, each wave's running minimum covers
    // few groups and seldom lets one be skipped: no clearance test there
    if (split >= kNoClearanceSplit) P.clr = nullptr;
    if (split == 8) {
        const dim3 sg((unsigned)waves);
        if (tape && cull)
            hipLaunchKernelGGL((k_eval_fwd_split<true, true, 8>), sg, dim3(512), 0, st, P, W, B, partial, slots, tape,
                               split);
        else if (tape)
            hipLaunchKernelGGL((k_eval_fwd_split<true, false, 8>), sg, dim3(512), 0, st, P, W, B, partial, slots, tape,
                               split);
        else if (cull)
            hipLaunchKernelGGL((k_eval_fwd_split<false, true, 8>), sg, dim3(512), 0, st, P, W, B, partial, slots, tape,
                               split);
        else
            hipLaunchKernelGGL((k_eval_fwd_split<false, false, 8>), sg, dim3(512), 0, st, P, W, B, partial, slots,
                               tape, split);
    } else if (split > 1) {
        const dim3 sg((unsigned)((waves * split + 3) / 4));
        if (tape && cull)
            hipLaunchKernelGGL((k_eval_fwd_split<true, true, 4>), sg, dim3(256), 0, st, P, W, B, partial, slots, tape,
                               split);
        else if (tape)
            hipLaunchKernelGGL((k_eval_fwd_split<true, false, 4>), sg, dim3(256), 0, st, P, W, B, partial, slots, tape,
                               split);
        else if (cull)
            hipLaunchKernelGGL((k_eval_fwd_split<false, true, 4>), sg, dim3(256), 0, st, P, W, B, partial, slots, tape,
                               split);
        else
            hipLaunchKernelGGL((k_eval_fwd_split<false, false, 4>), sg, dim3(256), 0, st, P, W, B, partial, slots,
                               tape, split);
    } else if (tape && cull)
        hipLaunchKernelGGL((k_eval_fwd<true, true>), grid, dim3(256), 0, st, P, W, B, partial, slots, tape);
    else if (tape)
        hipLaunchKernelGGL((k_eval_fwd<true, false>), grid, dim3(256), 0, st, P, W, B, partial, slots, tape);
    else if (cull)
        hipLaunchKernelGGL((k_eval_fwd<false, true>), grid, dim3(256), 0, st, P, W, B, partial, slots, tape);
    else
        hipLaunchKernelGGL((k_eval_fwd<false, false>), grid, dim3(256), 0, st, P, W, B, partial, slots, tape);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev->end, st)) != hipSuccess) return e;
    // no outputs: the caller takes the per-path sums itself, or wants only the tape
    if (!cost && !min_dist && !flags) return hipSuccess;
    hipLaunchKernelGGL(k_eval_reduce, dim3((B + 255) / 256), dim3(256), 0, st, partial, slots, B, P.ns, P.margin,
                       cost, min_dist, flags);
    return hipGetLastError();
}

hipError_t launch_batch_eval(const BatchProblem *probs, double2 *partial, int n, int max_B, const int2 *items,
                             int n_items, int rounds, int grid, bool cull, hipStream_t st) {
    if (cull)
        hipLaunchKernelGGL(k_eval_persistent<true>, dim3(grid), dim3(256), 0, st, probs, partial, items, n_items,
                           rounds);
    else
        hipLaunchKernelGGL(k_eval_persistent<false>, dim3(grid), dim3(256), 0, st, probs, partial, items, n_items,
                           rounds);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_batched, dim3((max_B + 255) / 256, n), dim3(256), 0, st, probs, partial);
    return hipGetLastError();
}

// paths up to which the adjoint runs 16 waves per path
constexpr int kBwdWidePaths = 256;

hipError_t launch_eval_bwd(const PlanView &P0, const float *W, int B, const uint32_t *tape, const float *grad_cost,
                           float *grad_W, hipStream_t st, const PolishStep *pol) {
    PolishStep ps{};
    if (pol) ps = *pol;
    // without a tape the minimising pair is found again (grid bounds in use)
    PlanView P = P0;
    if (!tape) {
        const hipError_t eb = view_with_sdf_bound(P0, P, st);
        if (eb != hipSuccess) return eb;
    }
    // one workgroup per path: 4 waves, or 16 when there are few paths
    const bool wide = B <= kBwdWidePaths;
    if (tape && wide)
        hipLaunchKernelGGL((k_eval_bwd<true, false, 16>), dim3(B), dim3(1024), 0, st, P, W, B, tape, grad_cost, grad_W, ps);
    else if (tape)
        hipLaunchKernelGGL((k_eval_bwd<true, false, 4>), dim3(B), dim3(256), 0, st, P, W, B, tape, grad_cost, grad_W, ps);
    else if (use_cull(P) && wide)
        hipLaunchKernelGGL((k_eval_bwd<false, true, 16>), dim3(B), dim3(1024), 0, st, P, W, B, tape, grad_cost,
                           grad_W, ps);
    else if (use_cull(P))
        hipLaunchKernelGGL((k_eval_bwd<false, true, 4>), dim3(B), dim3(256), 0, st, P, W, B, tape, grad_cost, grad_W, ps);
    else if (wide)
        hipLaunchKernelGGL((k_eval_bwd<false, false, 16>), dim3(B), dim3(1024), 0, st, P, W, B, tape, grad_cost,
                           grad_W, ps);
    else
        hipLaunchKernelGGL((k_eval_bwd<false, false, 4>), dim3(B), dim3(256), 0, st, P, W, B, tape, grad_cost, grad_W, ps);
    return hipGetLastError();
}

hipError_t launch_debug_fk(const PlanView &P, const float *Q, int N, float *centers, float *frames, hipStream_t st) {
    hipLaunchKernelGGL(k_debug_fk, dim3((N + 255) / 256), dim3(256), 0, st, P, Q, N, centers, frames);
    return hipGetLastError();
}

hipError_t launch_debug_configs(const PlanView &P, const float *Q, int N, float *dist, uint32_t *arg, hipStream_t st) {
    if (P.narrow == CP_NARROW_SAT) return launch_debug_configs_sat(P, Q, N, dist, arg, st);
    if (use_cull(P))
        hipLaunchKernelGGL(k_debug_configs<true>, dim3((N + 255) / 256), dim3(256), 0, st, P, Q, N, dist, arg);
    else
        hipLaunchKernelGGL(k_debug_configs<false>, dim3((N + 255) / 256), dim3(256), 0, st, P, Q, N, dist, arg);
    return hipGetLastError();
}

}  // namespace cp
