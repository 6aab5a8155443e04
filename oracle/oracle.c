/*
 * Plain FP64 CPU oracle for the crane path optimizer's evaluation step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or constant with the HIP library; both sides only take the same
 * seeded input arrays.
 *
 * Every quantity is the plain definition written out, in double precision,
 * built with -ffp-contract=off (no fused multiply-add) and no fast-math:
 *   - forward kinematics of a serial chain (Sec. 2: FK(q) -> H_g),
 *   - signed distances of link spheres to the scene (Sec. 3.1: d(q) < 0 in
 *     collision), minimum over every (sphere, obstacle) pair,
 *   - the cubic B-spline path (Sec. 4.1, eq. for q(s)) by the Cox-de Boor
 *     recursion on a uniform knot vector with four copies of the start and
 *     goal configuration at the ends,
 *   - the path cost J = J_p + w_c J_c + w_l J_l (Sec. 4.1, eqs. path-length,
 *     collision and feasibility costs, s_k = k / n_s),
 *   - its analytic gradient with respect to the free control points,
 *   - Philox4x32-10 (Salmon et al., SC'11) and Box-Muller normals for the
 *     sampling step of Algorithm 1,
 *   - voxel occupancy of a point cloud and exact squared Euclidean distance
 *     transforms (by brute force, and by 1-D passes that each take the plain
 *     minimum over a grid line), and the trilinear signed-distance query.
 * Paths are independent, so the path loop runs under OpenMP; each path's sums
 * are formed in a fixed order, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXJ 16
#define ORC_REVOLUTE 0
#define ORC_PRISMATIC 1

typedef struct {
    int32_t n_joints;
    const int32_t *type;      /* [n] */
    const float *axis;        /* [n,3] */
    const float *origin;      /* [n,3] */
    const float *q_min, *q_max, *q_hold;  /* [n] */
    const uint8_t *active;    /* [n] */
    int32_t n_spheres;
    const int32_t *sphere_frame;   /* [S] 0..n */
    const float *sphere_center;    /* [S,3] */
    const float *sphere_radius;    /* [S] */
    const float *tip;              /* [3] */
    int32_t n_self;                /* frame pairs checked for self-collision */
    const int32_t *self_pairs;     /* [n_self][2] frame indices */
    int32_t n_hulls;               /* convex hulls (oriented boxes) of the links */
    const int32_t *hull_frame;     /* [H] frame of each hull */
    const float *hull_box;         /* [H][15] centre, rotation (row-major, box axes as columns), half extents */
} orc_robot;

typedef struct {
    int32_t has_ground;
    float ground_z;
    int32_t n_cyl;
    const float *cyl;         /* [n,5] x y R z0 z1 */
    int32_t n_box;
    const float *box;         /* [n,6] cx cy cz hx hy hz */
    const float *sdf;         /* optional [nz][ny][nx] signed distance at voxel centres */
    int32_t sdf_dims[3];      /* nx ny nz */
    float sdf_origin[3];
    float voxel;
    int32_t narrow;           /* 0: spheres against the primitives above; 1: hulls against obb (SAT) */
    int32_t n_obb;
    const float *obb;         /* [n_obb][15] oriented boxes, the layout of hull_box, world coordinates */
} orc_scene;

typedef struct {
    int32_t K, M, interp, jp_mode, hinge;
    float margin, lambda_c, w_c, w_l;
} orc_cost;

/* ------------------------------------------------------------------------ */
/* forward kinematics (Sec. 2)                                               */
/* ------------------------------------------------------------------------ */

typedef struct { double R[9]; double p[3]; } xform;

static void xf_identity(xform *T) {
    memset(T, 0, sizeof(*T));
    T->R[0] = T->R[4] = T->R[8] = 1.0;
}

/* A = A * B for rigid transforms */
static void xf_mul(const xform *A, const xform *B, xform *out) {
    xform r;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A->R[3 * i + k] * B->R[3 * k + j];
            r.R[3 * i + j] = s;
        }
        double s = A->p[i];
        for (int k = 0; k < 3; ++k) s += A->R[3 * i + k] * B->p[k];
        r.p[i] = s;
    }
    *out = r;
}

/* rotation by angle q about the unit axis a (Rodrigues' formula) */
static void rot_axis(const double a[3], double q, double R[9]) {
    double c = cos(q), s = sin(q), v = 1.0 - c;
    double x = a[0], y = a[1], z = a[2];
    R[0] = c + x * x * v;     R[1] = x * y * v - z * s; R[2] = x * z * v + y * s;
    R[3] = y * x * v + z * s; R[4] = c + y * y * v;     R[5] = y * z * v - x * s;
    R[6] = z * x * v - y * s; R[7] = z * y * v + x * s; R[8] = c + z * z * v;
}

/* frames[0] = world; frames[j] = frames[j-1] * Trans(origin_j) * Motion_j(q_j) */
static void fk_frames(const orc_robot *rb, const double *q, xform *frames) {
    xf_identity(&frames[0]);
    for (int j = 0; j < rb->n_joints; ++j) {
        xform step;
        double a[3] = {rb->axis[3 * j], rb->axis[3 * j + 1], rb->axis[3 * j + 2]};
        xf_identity(&step);
        for (int i = 0; i < 3; ++i) step.p[i] = rb->origin[3 * j + i];
        if (rb->type[j] == ORC_REVOLUTE) {
            rot_axis(a, q[j], step.R);
        } else {
            for (int i = 0; i < 3; ++i) step.p[i] += q[j] * a[i];
        }
        xf_mul(&frames[j], &step, &frames[j + 1]);
    }
}

static void xf_apply(const xform *T, const double l[3], double out[3]) {
    for (int i = 0; i < 3; ++i)
        out[i] = T->R[3 * i] * l[0] + T->R[3 * i + 1] * l[1] + T->R[3 * i + 2] * l[2] + T->p[i];
}

static void sphere_local(const orc_robot *rb, int s, double l[3]) {
    for (int i = 0; i < 3; ++i) l[i] = rb->sphere_center[3 * s + i];
}

/* Frames as [n+1][12] (row-major R then p), sphere centres [S][3], tip [3]. */
void orc_fk(const orc_robot *rb, const double *q, double *frames_out, double *centers, double *tip) {
    xform F[ORC_MAXJ + 1];
    fk_frames(rb, q, F);
    if (frames_out)
        for (int j = 0; j <= rb->n_joints; ++j) {
            memcpy(frames_out + 12 * j, F[j].R, 9 * sizeof(double));
            memcpy(frames_out + 12 * j + 9, F[j].p, 3 * sizeof(double));
        }
    if (centers)
        for (int s = 0; s < rb->n_spheres; ++s) {
            double l[3];
            sphere_local(rb, s, l);
            xf_apply(&F[rb->sphere_frame[s]], l, centers + 3 * s);
        }
    if (tip) {
        double l[3] = {rb->tip[0], rb->tip[1], rb->tip[2]};
        xf_apply(&F[rb->n_joints], l, tip);
    }
}

/* ------------------------------------------------------------------------ */
/* signed distances (Sec. 3.1): exact Euclidean SDF of each solid             */
/* ------------------------------------------------------------------------ */

static double sgn(double x) { return x >= 0.0 ? 1.0 : -1.0; }

/* vertical solid cylinder; optional gradient with respect to the point */
double orc_sd_cylinder(const double c[3], const float *cy, double *grad) {
    double x0 = cy[0], y0 = cy[1], R = cy[2], z0 = cy[3], z1 = cy[4];
    double zc = 0.5 * (z0 + z1), hz = 0.5 * (z1 - z0);
    double dx = c[0] - x0, dy = c[1] - y0, dz = c[2] - zc;
    double rho = sqrt(dx * dx + dy * dy);
    double a = rho - R, b = fabs(dz) - hz;
    double ap = a > 0.0 ? a : 0.0, bp = b > 0.0 ? b : 0.0;
    double inside = fmin(fmax(a, b), 0.0);
    double outside = sqrt(ap * ap + bp * bp);
    if (grad) {
        double ga[3] = {rho > 0.0 ? dx / rho : 0.0, rho > 0.0 ? dy / rho : 0.0, 0.0};
        double gb[3] = {0.0, 0.0, sgn(dz)};
        if (a > 0.0 && b > 0.0) {
            for (int i = 0; i < 3; ++i) grad[i] = (a * ga[i] + b * gb[i]) / outside;
        } else if (a > 0.0) {
            for (int i = 0; i < 3; ++i) grad[i] = ga[i];
        } else if (b > 0.0) {
            for (int i = 0; i < 3; ++i) grad[i] = gb[i];
        } else {
            for (int i = 0; i < 3; ++i) grad[i] = a >= b ? ga[i] : gb[i];
        }
    }
    return inside + outside;
}

/* axis-aligned solid box */
double orc_sd_box(const double c[3], const float *bx, double *grad) {
    double q[3], s[3];
    for (int i = 0; i < 3; ++i) {
        double d = c[i] - bx[i];
        s[i] = sgn(d);
        q[i] = fabs(d) - bx[3 + i];
    }
    double o2 = 0.0;
    for (int i = 0; i < 3; ++i) {
        double qp = q[i] > 0.0 ? q[i] : 0.0;
        o2 += qp * qp;
    }
    double outside = sqrt(o2);
    double m = fmax(q[0], fmax(q[1], q[2]));
    double inside = fmin(m, 0.0);
    if (grad) {
        if (outside > 0.0) {
            for (int i = 0; i < 3; ++i) grad[i] = s[i] * (q[i] > 0.0 ? q[i] : 0.0) / outside;
        } else {
            int am = 0;
            for (int i = 1; i < 3; ++i)
                if (q[i] > q[am]) am = i;
            for (int i = 0; i < 3; ++i) grad[i] = 0.0;
            grad[am] = s[am];
        }
    }
    return outside + inside;
}

/* trilinear interpolation of a signed-distance grid sampled at voxel centres;
 * the continuous voxel coordinate is clamped to the grid */
double orc_sdf_query(const orc_scene *sc, const double c[3], double *grad) {
    int n[3] = {sc->sdf_dims[0], sc->sdf_dims[1], sc->sdf_dims[2]};
    double h = sc->voxel;
    int i0[3];
    double f[3], dfdg[3];
    for (int a = 0; a < 3; ++a) {
        double g = (c[a] - (double)sc->sdf_origin[a]) / h - 0.5;
        double fl = floor(g);
        int ii = (int)fl;
        if (fl < 0.0) ii = 0;
        if (fl > (double)(n[a] - 2)) ii = n[a] - 2;
        double fr = g - (double)ii;
        dfdg[a] = 1.0;
        if (fr < 0.0) { fr = 0.0; dfdg[a] = 0.0; }
        if (fr > 1.0) { fr = 1.0; dfdg[a] = 0.0; }
        i0[a] = ii;
        f[a] = fr;
    }
    double v[2][2][2];
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                size_t idx = ((size_t)(i0[2] + dz) * n[1] + (size_t)(i0[1] + dy)) * n[0] + (size_t)(i0[0] + dx);
                v[dz][dy][dx] = sc->sdf[idx];
            }
    double phi = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double wx = dx ? f[0] : 1.0 - f[0];
                double wy = dy ? f[1] : 1.0 - f[1];
                double wz = dz ? f[2] : 1.0 - f[2];
                double sx = dx ? 1.0 : -1.0, sy = dy ? 1.0 : -1.0, sz = dz ? 1.0 : -1.0;
                phi += wx * wy * wz * v[dz][dy][dx];
                gx += sx * wy * wz * v[dz][dy][dx];
                gy += wx * sy * wz * v[dz][dy][dx];
                gz += wx * wy * sz * v[dz][dy][dx];
            }
    if (grad) {
        grad[0] = gx * dfdg[0] / h;
        grad[1] = gy * dfdg[1] / h;
        grad[2] = gz * dfdg[2] / h;
    }
    return phi;
}

/* obstacle numbering of the tape: 0 = ground, 1..n_cyl = cylinders,
 * n_cyl+1.. = boxes, 0xFFFF = the signed-distance grid; a self-collision pair
 * of spheres (a, b), a < b, is recorded as sphere a and obstacle 0xFF00 + b */
#define ORC_OBS_SDF 0xFFFF
#define ORC_OBS_SELF 0xFF00

/* whether the frame pair {fa, fb} is listed for self-collision checks */
static int self_listed(const orc_robot *rb, int fa, int fb) {
    for (int i = 0; i < rb->n_self; ++i) {
        int a = rb->self_pairs[2 * i], b = rb->self_pairs[2 * i + 1];
        if ((a == fa && b == fb) || (a == fb && b == fa)) return 1;
    }
    return 0;
}

static double sd_obstacle(const orc_scene *sc, int o, const double c[3], double *grad) {
    if (o == ORC_OBS_SDF) return orc_sdf_query(sc, c, grad);
    if (o == 0) {
        if (grad) { grad[0] = 0.0; grad[1] = 0.0; grad[2] = 1.0; }
        return c[2] - (double)sc->ground_z;
    }
    if (o <= sc->n_cyl) return orc_sd_cylinder(c, sc->cyl + 5 * (o - 1), grad);
    return orc_sd_box(c, sc->box + 6 * (o - 1 - sc->n_cyl), grad);
}

/* ------------------------------------------------------------------------ */
/* separating-axis narrow phase on oriented boxes (Sec. 3.1)                 */
/* ------------------------------------------------------------------------ */

typedef struct { double c[3], R[9], h[3]; } orc_obb;

/* Gap of the projections of two boxes onto the unit axis n: the distance
 * between their centres along n less the two half-widths of the projections
 * (a box's half-width along n is the sum over its axes of h_i |a_i . n|).
 * Positive: n separates them by that much; negative: they overlap along n. */
static double sat_gap(const orc_obb *A, const orc_obb *B, const double n[3]) {
    double t = 0.0, ra = 0.0, rb = 0.0;
    for (int i = 0; i < 3; ++i) t += (B->c[i] - A->c[i]) * n[i];
    for (int i = 0; i < 3; ++i) {
        double pa = A->R[i] * n[0] + A->R[3 + i] * n[1] + A->R[6 + i] * n[2];
        double pb = B->R[i] * n[0] + B->R[3 + i] * n[1] + B->R[6 + i] * n[2];
        ra += A->h[i] * fabs(pa);
        rb += B->h[i] * fabs(pb);
    }
    return fabs(t) - ra - rb;
}

/* a cross-product axis a_i x b_j is taken only when |a_i x b_j|^2 exceeds
 * this (edges more than about 5.7 degrees from parallel): for parallel edges
 * the face axes already contain every separating direction, and for nearly
 * parallel ones the axis direction is ill-determined (a rotation error e
 * turns it by about e / |a_i x b_j|), so single-precision placements could
 * not reproduce its gap */
#define ORC_SAT_PARALLEL 1e-2

/* SAT signed distance of two oriented boxes: the largest projection gap over
 * the fifteen candidate axes of the separating axis theorem (the three face
 * normals of each box and the cross products of their edge directions,
 * near-parallel edge pairs excepted).
 * Positive: the boxes are disjoint and at least this far apart (exactly this
 * far when the nearest features are a face and anything, or two edges);
 * negative or zero: they intersect, and minus the value is the penetration
 * depth along the best axis (for boxes the minimum over all directions). */
double orc_sat_obb(const orc_obb *A, const orc_obb *B) {
    double best = -INFINITY;
    for (int i = 0; i < 3; ++i) {
        double na[3] = {A->R[i], A->R[3 + i], A->R[6 + i]};
        double nb[3] = {B->R[i], B->R[3 + i], B->R[6 + i]};
        double ga = sat_gap(A, B, na), gb = sat_gap(A, B, nb);
        if (ga > best) best = ga;
        if (gb > best) best = gb;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a[3] = {A->R[i], A->R[3 + i], A->R[6 + i]};
            double b[3] = {B->R[j], B->R[3 + j], B->R[6 + j]};
            double n[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
            double l2 = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
            if (!(l2 > ORC_SAT_PARALLEL)) continue;
            double l = sqrt(l2);
            for (int k = 0; k < 3; ++k) n[k] /= l;
            double g = sat_gap(A, B, n);
            if (g > best) best = g;
        }
    return best;
}

static void obb_load(const float *f, orc_obb *o) {
    for (int i = 0; i < 3; ++i) o->c[i] = f[i];
    for (int i = 0; i < 9; ++i) o->R[i] = f[3 + i];
    for (int i = 0; i < 3; ++i) o->h[i] = f[12 + i];
}

/* hull k of the robot in world coordinates at frames F */
static void hull_world(const orc_robot *rb, const xform *F, int k, orc_obb *o) {
    orc_obb l;
    obb_load(rb->hull_box + 15 * k, &l);
    const xform *T = &F[rb->hull_frame[k]];
    xf_apply(T, l.c, o->c);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int m = 0; m < 3; ++m) s += T->R[3 * i + m] * l.R[3 * m + j];
            o->R[3 * i + j] = s;
        }
    for (int i = 0; i < 3; ++i) o->h[i] = l.h[i];
}

/* signed distance of a box above the ground plane: its lowest point's height */
static double obb_ground(const orc_obb *o, double gz) {
    return o->c[2] - (o->h[0] * fabs(o->R[6]) + o->h[1] * fabs(o->R[7]) + o->h[2] * fabs(o->R[8])) - gz;
}

/* d(q) with the SAT narrow phase: the minimum over every (hull, obstacle)
 * pair, the obstacles being the ground (0) and the scene's boxes (1..n_obb),
 * and over the hull pairs of listed frame pairs (recorded as hull a and
 * obstacle 0xFF00 + b, a < b).  Ties keep the lowest hull, then its obstacles
 * in number order, then its self pairs by the other hull. */
static double config_distance_sat(const orc_robot *rb, const orc_scene *sc, const double *q, int32_t *arg_s,
                                  int32_t *arg_o, double *second) {
    xform F[ORC_MAXJ + 1];
    fk_frames(rb, q, F);
    double best = INFINITY, best2 = INFINITY;
    int bs = -1, bo = -1;
    orc_obb hw[64];
    int H = rb->n_hulls < 64 ? rb->n_hulls : 64;
    for (int k = 0; k < H; ++k) hull_world(rb, F, k, &hw[k]);
    for (int k = 0; k < H; ++k) {
        for (int o = 0; o <= sc->n_obb; ++o) {
            double d;
            if (o == 0) {
                if (!sc->has_ground) continue;
                d = obb_ground(&hw[k], (double)sc->ground_z);
            } else {
                orc_obb b;
                obb_load(sc->obb + 15 * (o - 1), &b);
                d = orc_sat_obb(&hw[k], &b);
            }
            if (d < best) { best2 = best; best = d; bs = k; bo = o; }
            else if (d < best2) best2 = d;
        }
        for (int m = k + 1; m < H; ++m) {
            if (rb->n_self == 0 || !self_listed(rb, rb->hull_frame[k], rb->hull_frame[m])) continue;
            double d = orc_sat_obb(&hw[k], &hw[m]);
            if (d < best) { best2 = best; best = d; bs = k; bo = ORC_OBS_SELF + m; }
            else if (d < best2) best2 = d;
        }
    }
    if (arg_s) *arg_s = bs;
    if (arg_o) *arg_o = bo;
    if (second) *second = best2;
    return best;
}

/* SAT distance of two boxes given as 15 floats each (tests) */
double orc_sat_obb_f(const double *a, const double *b) {
    orc_obb A, B;
    for (int i = 0; i < 3; ++i) { A.c[i] = a[i]; B.c[i] = b[i]; A.h[i] = a[12 + i]; B.h[i] = b[12 + i]; }
    for (int i = 0; i < 9; ++i) { A.R[i] = a[3 + i]; B.R[i] = b[3 + i]; }
    return orc_sat_obb(&A, &B);
}

/* the robot's hulls in world coordinates at q, [H][15] */
void orc_hulls_world(const orc_robot *rb, const double *q, double *out) {
    xform F[ORC_MAXJ + 1];
    fk_frames(rb, q, F);
    for (int k = 0; k < rb->n_hulls; ++k) {
        orc_obb o;
        hull_world(rb, F, k, &o);
        for (int i = 0; i < 3; ++i) out[15 * k + i] = o.c[i];
        for (int i = 0; i < 9; ++i) out[15 * k + 3 + i] = o.R[i];
        for (int i = 0; i < 3; ++i) out[15 * k + 12 + i] = o.h[i];
    }
}

/* d(q): minimum over every (sphere, obstacle) pair of sd(centre) - radius,
 * and over every self-collision pair (spheres a < b on a listed frame pair)
 * of |c_a - c_b| - r_a - r_b (Sec. 3.2 names self-collision beside collision
 * with the environment).  Ties keep the lowest sphere, then its obstacles in
 * number order, then its self pairs by the other sphere. */
double orc_config_distance(const orc_robot *rb, const orc_scene *sc, const double *q,
                           int32_t *arg_s, int32_t *arg_o, double *second) {
    if (sc->narrow == 1) return config_distance_sat(rb, sc, q, arg_s, arg_o, second);
    xform F[ORC_MAXJ + 1];
    fk_frames(rb, q, F);
    double best = INFINITY, best2 = INFINITY;
    int bs = -1, bo = -1;
    for (int s = 0; s < rb->n_spheres; ++s) {
        double l[3], c[3];
        sphere_local(rb, s, l);
        xf_apply(&F[rb->sphere_frame[s]], l, c);
        double r = rb->sphere_radius[s];
        int n_obs = 1 + sc->n_cyl + sc->n_box;
        for (int o = 0; o <= n_obs; ++o) {
            int code = o;
            if (o == n_obs) {
                if (!sc->sdf) continue;
                code = ORC_OBS_SDF;
            } else if (o == 0 && !sc->has_ground) {
                continue;
            }
            double d = sd_obstacle(sc, code, c, NULL) - r;
            if (d < best) {
                best2 = best;
                best = d; bs = s; bo = code;
            } else if (d < best2) {
                best2 = d;
            }
        }
        for (int b = s + 1; b < rb->n_spheres; ++b) {
            if (rb->n_self == 0 || !self_listed(rb, rb->sphere_frame[s], rb->sphere_frame[b])) continue;
            double lb[3], cb[3];
            sphere_local(rb, b, lb);
            xf_apply(&F[rb->sphere_frame[b]], lb, cb);
            double dx = c[0] - cb[0], dy = c[1] - cb[1], dz = c[2] - cb[2];
            double d = sqrt(dx * dx + dy * dy + dz * dz) - r - (double)rb->sphere_radius[b];
            if (d < best) {
                best2 = best;
                best = d; bs = s; bo = ORC_OBS_SELF + b;
            } else if (d < best2) {
                best2 = d;
            }
        }
    }
    if (arg_s) *arg_s = bs;
    if (arg_o) *arg_o = bo;
    if (second) *second = best2;
    return best;
}

/* ------------------------------------------------------------------------ */
/* path: cubic B-spline by Cox-de Boor, or piecewise linear (Sec. 4.1)       */
/* ------------------------------------------------------------------------ */

/* N_{i,p}(t) on the uniform knot vector t_i = i */
static double bspline_basis(int i, int p, double t) {
    if (p == 0) return (t >= (double)i && t < (double)(i + 1)) ? 1.0 : 0.0;
    double left = (t - (double)i) / (double)p * bspline_basis(i, p - 1, t);
    double right = ((double)(i + p + 1) - t) / (double)p * bspline_basis(i + 1, p - 1, t);
    return left + right;
}

int orc_n_checkpoints(const orc_cost *cp) {
    return (cp->interp == 0 ? cp->K + 3 : cp->K + 1) * cp->M;
}

/* control polygon of the B-spline: 4 x start, the K waypoints, 4 x goal */
static void control_point(const orc_robot *rb, const orc_cost *cp, const double *qs, const double *qg,
                          const double *W, int i, double *out) {
    int n = rb->n_joints;
    const int lead = cp->interp == 0 ? 4 : 1;
    if (i < lead) {
        for (int j = 0; j < n; ++j) out[j] = qs[j];
    } else if (i < lead + cp->K) {
        for (int j = 0; j < n; ++j) out[j] = W[(size_t)(i - lead) * n + j];
    } else {
        for (int j = 0; j < n; ++j) out[j] = qg[j];
    }
}

/* weights of every control point at path parameter s (n_ctrl entries) */
static int path_weights(const orc_cost *cp, double s, double *w) {
    if (cp->interp == 0) {
        int n_ctrl = cp->K + 8;
        /* the four leading copies make span [3,4) constant; the path runs over
         * the K+3 spans between t = 4 and t = K+7 */
        double t = 4.0 + s * (double)(cp->K + 3);
        for (int i = 0; i < n_ctrl; ++i) w[i] = bspline_basis(i, 3, t);
        return n_ctrl;
    } else {
        int n_ctrl = cp->K + 2;
        for (int i = 0; i < n_ctrl; ++i) w[i] = 0.0;
        double x = s * (double)(cp->K + 1);
        int j = (int)floor(x);
        if (j >= cp->K + 1) { w[cp->K + 1] = 1.0; return n_ctrl; }
        double u = x - (double)j;
        w[j] = 1.0 - u;
        w[j + 1] = u;
        return n_ctrl;
    }
}

/* q(s_k) for k = 0..n_s, written to out [n_s+1][n] */
void orc_path_points(const orc_robot *rb, const orc_cost *cp, const double *qs_f, const double *qg_f,
                     const double *W, double *out) {
    int n = rb->n_joints, ns = orc_n_checkpoints(cp);
    double qs[ORC_MAXJ], qg[ORC_MAXJ], w[64], P[ORC_MAXJ];
    for (int j = 0; j < n; ++j) { qs[j] = qs_f[j]; qg[j] = qg_f[j]; }
    for (int k = 0; k <= ns; ++k) {
        double s = (double)k / (double)ns;
        int nc = path_weights(cp, s, w);
        for (int j = 0; j < n; ++j) out[(size_t)k * n + j] = 0.0;
        for (int i = 0; i < nc; ++i) {
            if (w[i] == 0.0) continue;
            control_point(rb, cp, qs, qg, W, i, P);
            for (int j = 0; j < n; ++j) out[(size_t)k * n + j] += w[i] * P[j];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* cost (Sec. 4.1) and its gradient                                          */
/* ------------------------------------------------------------------------ */

static double hinge(const orc_cost *cp, double d, double *dphi) {
    double m = cp->margin, lam = cp->lambda_c;
    if (cp->hinge == 0 || m <= 0.0) {
        if (dphi) *dphi = d < m ? -lam : 0.0;
        return d < m ? lam * (m - d) : 0.0;
    }
    if (d < 0.0) {
        if (dphi) *dphi = -lam;
        return lam * (0.5 * m - d);
    }
    if (d < m) {
        if (dphi) *dphi = -lam * (m - d) / m;
        return lam * (m - d) * (m - d) / (2.0 * m);
    }
    if (dphi) *dphi = 0.0;
    return 0.0;
}

static double limit_cost(const orc_robot *rb, const double *q, double *grad) {
    double J = 0.0;
    for (int j = 0; j < rb->n_joints; ++j) {
        double hi = q[j] - (double)rb->q_max[j], lo = (double)rb->q_min[j] - q[j];
        double hp = hi > 0.0 ? hi : 0.0, lp = lo > 0.0 ? lo : 0.0;
        J += hp * hp + lp * lp;
        if (grad) grad[j] = 2.0 * hp - 2.0 * lp;
    }
    return J;
}

/* d c / d q_j for a point c rigidly attached to frame f, into dc */
static void point_jacobian_col(const orc_robot *rb, const xform *F, int j, const double c[3], double dc[3]) {
    /* joint j moves frame j+1; its axis in world coordinates is R_j a_j
     * and passes through the origin of frame j+1 */
    double a[3], aw[3];
    for (int i = 0; i < 3; ++i) a[i] = rb->axis[3 * j + i];
    for (int i = 0; i < 3; ++i)
        aw[i] = F[j].R[3 * i] * a[0] + F[j].R[3 * i + 1] * a[1] + F[j].R[3 * i + 2] * a[2];
    if (rb->type[j] == ORC_REVOLUTE) {
        double r[3] = {c[0] - F[j + 1].p[0], c[1] - F[j + 1].p[1], c[2] - F[j + 1].p[2]};
        dc[0] = aw[1] * r[2] - aw[2] * r[1];
        dc[1] = aw[2] * r[0] - aw[0] * r[2];
        dc[2] = aw[0] * r[1] - aw[1] * r[0];
    } else {
        dc[0] = aw[0]; dc[1] = aw[1]; dc[2] = aw[2];
    }
}

/* gradient of d(q) with respect to q through the minimising pair */
static void distance_grad_q(const orc_robot *rb, const orc_scene *sc, const double *q, int s, int o,
                            double *gq) {
    if (sc->narrow == 1) {  /* no gradient for the separating-axis distance (refused by the wrapper) */
        for (int j = 0; j < rb->n_joints; ++j) gq[j] = 0.0;
        return;
    }
    xform F[ORC_MAXJ + 1];
    fk_frames(rb, q, F);
    double l[3], c[3], gc[3];
    sphere_local(rb, s, l);
    xf_apply(&F[rb->sphere_frame[s]], l, c);
    for (int j = 0; j < rb->n_joints; ++j) gq[j] = 0.0;
    if (o >= ORC_OBS_SELF && o < ORC_OBS_SDF) {
        /* self pair: d = |c_s - c_b| - r_s - r_b, dd/dq = n . (dc_s/dq - dc_b/dq) */
        int b = o - ORC_OBS_SELF;
        double lb[3], cb[3];
        sphere_local(rb, b, lb);
        xf_apply(&F[rb->sphere_frame[b]], lb, cb);
        double n[3] = {c[0] - cb[0], c[1] - cb[1], c[2] - cb[2]};
        double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (!(len > 0.0)) return;
        for (int i = 0; i < 3; ++i) n[i] /= len;
        for (int j = 0; j < rb->n_joints; ++j) {
            double da[3] = {0.0, 0.0, 0.0}, db[3] = {0.0, 0.0, 0.0};
            if (j < rb->sphere_frame[s]) point_jacobian_col(rb, F, j, c, da);
            if (j < rb->sphere_frame[b]) point_jacobian_col(rb, F, j, cb, db);
            gq[j] = n[0] * (da[0] - db[0]) + n[1] * (da[1] - db[1]) + n[2] * (da[2] - db[2]);
        }
        return;
    }
    sd_obstacle(sc, o, c, gc);
    int f = rb->sphere_frame[s];
    for (int j = 0; j < f; ++j) {
        double dc[3];
        point_jacobian_col(rb, F, j, c, dc);
        gq[j] = gc[0] * dc[0] + gc[1] * dc[1] + gc[2] * dc[2];
    }
}

/*
 * One path: cost, min distance over checkpoints, collision flag, optional
 * per-checkpoint distance / argmin / runner-up distance, optional gradient
 * d cost / d W [K][n] (scaled by grad_scale).
 */
static double eval_path(const orc_robot *rb, const orc_scene *sc, const orc_cost *cp,
                        const double *qs_f, const double *qg_f, const double *W,
                        double *min_dist_out, double *dk_out, int32_t *tape_out, double *second_out,
                        double *grad_out, double *parts_out) {
    int n = rb->n_joints, ns = orc_n_checkpoints(cp), K = cp->K;
    int nc = cp->interp == 0 ? K + 8 : K + 2;
    int lead = cp->interp == 0 ? 4 : 1;
    double *pts = (double *)malloc(sizeof(double) * (size_t)(ns + 1) * n);
    orc_path_points(rb, cp, qs_f, qg_f, W, pts);
    double Jp = 0.0, Jc = 0.0, Jl = 0.0, dmin = INFINITY;
    double *gP = NULL, *wk = NULL, *wk1 = NULL;
    if (grad_out) {
        gP = (double *)calloc((size_t)nc * n, sizeof(double));
        wk = (double *)malloc(sizeof(double) * nc);
        wk1 = (double *)malloc(sizeof(double) * nc);
    }
    for (int k = 1; k <= ns; ++k) {
        const double *q = pts + (size_t)k * n, *qp = pts + (size_t)(k - 1) * n;
        double delta[ORC_MAXJ], sq = 0.0;
        for (int j = 0; j < n; ++j) { delta[j] = q[j] - qp[j]; sq += delta[j] * delta[j]; }
        double len = sqrt(sq);
        Jp += cp->jp_mode == 0 ? sq : len;
        int32_t as, ao;
        double second;
        double d = orc_config_distance(rb, sc, q, &as, &ao, &second);
        if (d < dmin) dmin = d;
        double dphi;
        Jc += hinge(cp, d, &dphi);
        double glim[ORC_MAXJ];
        Jl += limit_cost(rb, q, glim);
        if (dk_out) dk_out[k - 1] = d;
        if (tape_out) tape_out[k - 1] = (int32_t)(((uint32_t)as << 16) | ((uint32_t)ao & 0xFFFFu));
        if (second_out) second_out[k - 1] = second;
        if (grad_out) {
            double gq[ORC_MAXJ], gd[ORC_MAXJ], gjp[ORC_MAXJ];
            for (int j = 0; j < n; ++j) gd[j] = 0.0;
            if (dphi != 0.0) distance_grad_q(rb, sc, q, as, ao, gd);
            for (int j = 0; j < n; ++j) {
                if (cp->jp_mode == 0) gjp[j] = 2.0 * delta[j];
                else gjp[j] = len > 0.0 ? delta[j] / len : 0.0;
                gq[j] = (double)cp->w_c * dphi * gd[j] + (double)cp->w_l * glim[j];
            }
            double s = (double)k / (double)ns, s1 = (double)(k - 1) / (double)ns;
            path_weights(cp, s, wk);
            path_weights(cp, s1, wk1);
            /* J_p term k depends on q_k (+) and q_{k-1} (-) */
            for (int i = 0; i < nc; ++i)
                for (int j = 0; j < n; ++j)
                    gP[(size_t)i * n + j] += wk[i] * (gq[j] + gjp[j]) - wk1[i] * gjp[j];
        }
    }
    double cost = Jp + (double)cp->w_c * Jc + (double)cp->w_l * Jl;
    if (min_dist_out) *min_dist_out = dmin;
    if (parts_out) { parts_out[0] = Jp; parts_out[1] = Jc; parts_out[2] = Jl; }
    if (grad_out) {
        for (int i = 0; i < K; ++i)
            for (int j = 0; j < n; ++j) grad_out[(size_t)i * n + j] = gP[(size_t)(i + lead) * n + j];
        free(gP); free(wk); free(wk1);
    }
    free(pts);
    return cost;
}

/* Batch of paths W [B][K][n] -> cost [B], min_dist [B], flags [B]; optional
 * per-checkpoint outputs [B][n_s] and parts [B][3] = (J_p, J_c, J_l). */
void orc_eval_paths(const orc_robot *rb, const orc_scene *sc, const orc_cost *cp, const double *qs,
                    const double *qg, const double *W, int64_t B, double *cost, double *min_dist,
                    uint8_t *flags, double *dk, int32_t *tape, double *second, double *parts) {
    int ns = orc_n_checkpoints(cp);
    size_t stride = (size_t)cp->K * rb->n_joints;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < B; ++b) {
        double md;
        double c = eval_path(rb, sc, cp, qs, qg, W + (size_t)b * stride, &md,
                             dk ? dk + (size_t)b * ns : NULL, tape ? tape + (size_t)b * ns : NULL,
                             second ? second + (size_t)b * ns : NULL, NULL,
                             parts ? parts + 3 * (size_t)b : NULL);
        cost[b] = c;
        if (min_dist) min_dist[b] = md;
        if (flags) flags[b] = (uint8_t)(md < (double)cp->margin);
    }
}

/* analytic gradient d cost_b / d W_b for every path, [B][K][n] */
void orc_grad_paths(const orc_robot *rb, const orc_scene *sc, const orc_cost *cp, const double *qs,
                    const double *qg, const double *W, int64_t B, double *cost, double *grad) {
    size_t stride = (size_t)cp->K * rb->n_joints;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < B; ++b) {
        double md;
        cost[b] = eval_path(rb, sc, cp, qs, qg, W + (size_t)b * stride, &md, NULL, NULL, NULL,
                            grad + (size_t)b * stride, NULL);
    }
}

/* per-configuration distance and argmin for N joint vectors */
void orc_eval_configs(const orc_robot *rb, const orc_scene *sc, const double *q, int64_t N,
                      double *d, int32_t *arg_s, int32_t *arg_o, double *second) {
    int n = rb->n_joints;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int32_t s, o;
        double sec;
        d[i] = orc_config_distance(rb, sc, q + (size_t)i * n, &s, &o, &sec);
        if (arg_s) arg_s[i] = s;
        if (arg_o) arg_o[i] = o;
        if (second) second[i] = sec;
    }
}

/* ------------------------------------------------------------------------ */
/* collision-free inverse kinematics (Sec. 3.2, eq. IK opt)                  */
/* ------------------------------------------------------------------------ */

static void cross3(const double a[3], const double b[3], double out[3]) {
    double x = a[1] * b[2] - a[2] * b[1];
    double y = a[2] * b[0] - a[0] * b[2];
    double z = a[0] * b[1] - a[1] * b[0];
    out[0] = x; out[1] = y; out[2] = z;
}

/* Logarithm of SO(3): the rotation vector w = theta n (theta in [0, pi]) of
 * the rotation R (row-major).  With v = vee(R - R^T) = 2 sin(theta) n and
 * cos(theta) = (tr R - 1) / 2, theta = atan2(|v| / 2, cos theta); the axis is
 * v / |v|, except close to theta = pi, where v vanishes and the axis comes
 * from the symmetric part (R + R^T) / 2 - cos(theta) I = (1 - cos theta) n n^T
 * (its largest diagonal entry, sign taken so that n . v >= 0). */
void orc_so3_log(const double *R, double *w) {
    double v[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
    double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    double th = atan2(0.5 * vn, c);
    if (c > -0.9) {
        for (int i = 0; i < 3; ++i) w[i] = vn > 0.0 ? th * v[i] / vn : 0.0;
        return;
    }
    double S[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) S[3 * i + j] = 0.5 * (R[3 * i + j] + R[3 * j + i]) - (i == j ? c : 0.0);
    int k = 0;
    for (int i = 1; i < 3; ++i)
        if (S[4 * i] > S[4 * k]) k = i;
    double n[3];
    double nk = sqrt(S[4 * k] / (1.0 - c));
    for (int i = 0; i < 3; ++i) n[i] = i == k ? nk : S[3 * k + i] / ((1.0 - c) * nk);
    double dot = n[0] * v[0] + n[1] * v[1] + n[2] * v[2];
    double sg = dot < 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < 3; ++i) w[i] = sg * th * n[i];
}

/* Inverse of the right Jacobian of SO(3) at w: the derivative of
 * Log(Exp(w) Exp(e)) with respect to e at e = 0,
 *   J_r^-1(w) = I + [w]/2 + (1/theta^2 - (1 + cos theta) / (2 theta sin theta)) [w]^2,
 * the last coefficient by its series 1/12 + theta^2/720 + theta^4/30240 for
 * small theta (cancellation). */
void orc_so3_jr_inv(const double w[3], double *Ji) {
    double t2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(t2);
    double k;
    if (th < 1e-2)
        k = 1.0 / 12.0 + t2 / 720.0 + t2 * t2 / 30240.0;
    else
        k = 1.0 / t2 - (1.0 + cos(th)) / (2.0 * th * sin(th));
    double W[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int l = 0; l < 3; ++l) s += W[3 * i + l] * W[3 * l + j];
            Ji[3 * i + j] = (i == j ? 1.0 : 0.0) + 0.5 * W[3 * i + j] + k * s;
        }
}

/* d^2 p / dq_i dq_j of a point p rigidly attached to the last frame: with
 * u = min(i, j), v = max(i, j), world axes a and pivots o (origin of the
 * frame each joint moves),
 *   v revolute:  a_u x (a_v x (p - o_v)) if u is revolute, 0 if prismatic;
 *   v prismatic: a_u x a_v if u < v is revolute, 0 otherwise. */
static void point_hessian(const orc_robot *rb, const double aw[][3], const double piv[][3], const double p[3],
                          int i, int j, double out[3]) {
    int u = i < j ? i : j, v = i < j ? j : i;
    out[0] = out[1] = out[2] = 0.0;
    if (rb->type[v] == ORC_REVOLUTE) {
        if (rb->type[u] != ORC_REVOLUTE) return;
        double r[3] = {p[0] - piv[v][0], p[1] - piv[v][1], p[2] - piv[v][2]}, t[3];
        cross3(aw[v], r, t);
        cross3(aw[u], t, out);
    } else {
        if (u == v || rb->type[u] != ORC_REVOLUTE) return;
        cross3(aw[u], aw[v], out);
    }
}

/*
 * Residual of the IK problem at q and its Jacobian (Sec. 3.2):
 *   r[0..2] = p_g - p_d                       (position of the tip point)
 *   r[3..5] = lambda_q Log(R_d^T R_g)         (orientation of the last frame)
 *   r[6]    = lambda_c ReLU(-d(q))            (collision, scene and self)
 *   r[7]    = lambda_e |g_p|^2                (equilibrium of the passive joints)
 *   r[8..]  = lambda_r (q - q_ref)            (regularisation, n entries)
 * g_p is the gravitational generalised force on the joints that are not
 * actuated (active[j] = 0) of a unit weight at the tip: g_p,j = dz_tip/dq_j
 * (the crane's mass model is not given; the load hangs at the tip).
 * lam = (lambda_q, lambda_c, lambda_e, lambda_r); target = R_d (row-major)
 * then p_d.  J [8+n][n] row-major (may be NULL).  info (may be NULL):
 * |p_g - p_d|, |Log(R_d^T R_g)|, d(q), |g_p|, argmin sphere, argmin obstacle.
 */
void orc_ik_residual(const orc_robot *rb, const orc_scene *sc, const double *lam, const double *target,
                     const double *q, const double *q_ref, double *r, double *J, double *info) {
    const int n = rb->n_joints, m = 8 + n;
    xform F[ORC_MAXJ + 1];
    fk_frames(rb, q, F);
    double tl[3] = {rb->tip[0], rb->tip[1], rb->tip[2]}, p[3];
    xf_apply(&F[n], tl, p);
    double aw[ORC_MAXJ][3], piv[ORC_MAXJ][3], dp[ORC_MAXJ][3];
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < 3; ++i)
            aw[j][i] = F[j].R[3 * i] * rb->axis[3 * j] + F[j].R[3 * i + 1] * rb->axis[3 * j + 1] +
                       F[j].R[3 * i + 2] * rb->axis[3 * j + 2];
        for (int i = 0; i < 3; ++i) piv[j][i] = F[j + 1].p[i];
        point_jacobian_col(rb, F, j, p, dp[j]);
    }
    /* position */
    for (int i = 0; i < 3; ++i) r[i] = p[i] - target[9 + i];
    /* orientation: E = R_d^T R_g */
    double E[9], w[3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int l = 0; l < 3; ++l) s += target[3 * l + i] * F[n].R[3 * l + j];
            E[3 * i + j] = s;
        }
    orc_so3_log(E, w);
    for (int i = 0; i < 3; ++i) r[3 + i] = lam[0] * w[i];
    /* collision */
    int32_t as, ao;
    double d = orc_config_distance(rb, sc, q, &as, &ao, NULL);
    r[6] = d < 0.0 ? lam[1] * (-d) : 0.0;
    /* equilibrium of the passive joints */
    double gp2 = 0.0;
    for (int j = 0; j < n; ++j)
        if (!rb->active[j]) gp2 += dp[j][2] * dp[j][2];
    r[7] = lam[2] * gp2;
    for (int j = 0; j < n; ++j) r[8 + j] = lam[3] * (q[j] - q_ref[j]);
    if (info) {
        info[0] = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        info[1] = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        info[2] = d;
        info[3] = sqrt(gp2);
        info[4] = as;
        info[5] = ao;
    }
    if (!J) return;
    for (int k = 0; k < m * n; ++k) J[k] = 0.0;
    double Ji[9];
    orc_so3_jr_inv(w, Ji);
    double gd[ORC_MAXJ];
    if (d < 0.0) distance_grad_q(rb, sc, q, as, ao, gd);
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < 3; ++i) J[i * n + j] = dp[j][i];
        if (rb->type[j] == ORC_REVOLUTE) {
            /* rotating about the world axis a_j is R_g -> R_g Exp(dq R_g^T a_j) */
            double b[3];
            for (int i = 0; i < 3; ++i)
                b[i] = F[n].R[i] * aw[j][0] + F[n].R[3 + i] * aw[j][1] + F[n].R[6 + i] * aw[j][2];
            for (int i = 0; i < 3; ++i)
                J[(3 + i) * n + j] = lam[0] * (Ji[3 * i] * b[0] + Ji[3 * i + 1] * b[1] + Ji[3 * i + 2] * b[2]);
        }
        if (d < 0.0) J[6 * n + j] = -lam[1] * gd[j];
        double s = 0.0;
        for (int k = 0; k < n; ++k) {
            if (rb->active[k]) continue;
            double h[3];
            point_hessian(rb, aw, piv, p, k, j, h);
            s += dp[k][2] * h[2];
        }
        J[7 * n + j] = 2.0 * lam[2] * s;
        J[(8 + j) * n + j] = lam[3];
    }
}

/* ------------------------------------------------------------------------ */
/* reduced dynamics (Sec. 2.1) and trapezoidal defects (Sec. 4.2)            */
/* ------------------------------------------------------------------------ */

/*
 * Joint accelerations of the reduced dynamics: the actuated joints
 * (active[j] = 1) take the commanded accelerations u (in joint order, one per
 * actuated joint); the passive ones follow from their rows of
 * M(q) qdd + b(q, qd) = tau with no torque there,
 *   qdd_p = -M_pp^-1 (M_pa qdd_a + b_p) - damping qd_p.
 * Mass model (the crane's own is not given): a unit load at the tip on
 * massless links, so M = J^T J and b = J^T (c + g e_z), with J = d tip / dq
 * and c = sum_ij H_ij qd_i qd_j the tip's velocity-product acceleration
 * (H_ij = d^2 tip / dq_i dq_j).  With the passive rows of M invertible this
 * is the load's equation of motion projected on the passive joints.
 */
void orc_crane_accel(const orc_robot *rb, const double *q, const double *qd, const double *u, double grav,
                     double damping, double *qdd) {
    const int n = rb->n_joints;
    xform F[ORC_MAXJ + 1];
    fk_frames(rb, q, F);
    double tl[3] = {rb->tip[0], rb->tip[1], rb->tip[2]}, p[3];
    xf_apply(&F[n], tl, p);
    double aw[ORC_MAXJ][3], piv[ORC_MAXJ][3], J[ORC_MAXJ][3];
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < 3; ++i)
            aw[j][i] = F[j].R[3 * i] * rb->axis[3 * j] + F[j].R[3 * i + 1] * rb->axis[3 * j + 1] +
                       F[j].R[3 * i + 2] * rb->axis[3 * j + 2];
        for (int i = 0; i < 3; ++i) piv[j][i] = F[j + 1].p[i];
        point_jacobian_col(rb, F, j, p, J[j]);
    }
    /* c = sum_ij H_ij qd_i qd_j */
    double c[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double h[3];
            point_hessian(rb, aw, piv, p, i, j, h);
            for (int k = 0; k < 3; ++k) c[k] += h[k] * qd[i] * qd[j];
        }
    /* tip acceleration from the actuated joints, plus c and gravity */
    double a[3] = {c[0], c[1], c[2] + grav};
    int pas[ORC_MAXJ], np_ = 0, ia = 0;
    for (int j = 0; j < n; ++j) {
        if (rb->active[j]) {
            qdd[j] = u[ia++];
            for (int k = 0; k < 3; ++k) a[k] += J[j][k] * qdd[j];
        } else {
            pas[np_++] = j;
        }
    }
    if (np_ == 0) return;
    /* M_pp x = -J_p^T a (Gaussian elimination with partial pivoting) */
    double Mp[ORC_MAXJ][ORC_MAXJ + 1];
    for (int r = 0; r < np_; ++r) {
        for (int s2 = 0; s2 < np_; ++s2) {
            double m = 0.0;
            for (int k = 0; k < 3; ++k) m += J[pas[r]][k] * J[pas[s2]][k];
            Mp[r][s2] = m;
        }
        double b = 0.0;
        for (int k = 0; k < 3; ++k) b += J[pas[r]][k] * a[k];
        Mp[r][np_] = -b;
    }
    for (int col = 0; col < np_; ++col) {
        int piv_r = col;
        for (int r = col + 1; r < np_; ++r)
            if (fabs(Mp[r][col]) > fabs(Mp[piv_r][col])) piv_r = r;
        if (piv_r != col)
            for (int k = 0; k <= np_; ++k) { double t = Mp[col][k]; Mp[col][k] = Mp[piv_r][k]; Mp[piv_r][k] = t; }
        for (int r = col + 1; r < np_; ++r) {
            double f = Mp[r][col] / Mp[col][col];
            for (int k = col; k <= np_; ++k) Mp[r][k] -= f * Mp[col][k];
        }
    }
    double x[ORC_MAXJ];
    for (int r = np_ - 1; r >= 0; --r) {
        double t = Mp[r][np_];
        for (int k = r + 1; k < np_; ++k) t -= Mp[r][k] * x[k];
        x[r] = t / Mp[r][r];
    }
    for (int r = 0; r < np_; ++r) qdd[pas[r]] = x[r] - damping * qd[pas[r]];
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11) and Box-Muller normals                           */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in (0, 1) from the top 23 bits: (2 (x >> 9) + 1) / 2^24 */
double orc_uniform(uint32_t x) { return (2.0 * (double)(x >> 9) + 1.0) / 16777216.0; }

/* z [B][D]: element e of path b in iteration t of problem p uses Philox
 * counter (e / 4, b, t, p) and key (seed lo, seed hi); the four words give
 * two Box-Muller pairs (w0, w1) and (w2, w3):
 *   r = sqrt(-2 ln u_first), z = r cos(2 pi u_second), r sin(2 pi u_second). */
void orc_normals(uint64_t seed, uint32_t t, uint32_t problem, int64_t B, int32_t D, double *z) {
    const double two_pi = 6.283185307179586476925286766559;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < B; ++b) {
        for (int g = 0; 4 * g < D; ++g) {
            uint32_t ctr[4] = {(uint32_t)g, (uint32_t)b, t, problem}, x[4];
            orc_philox4x32_10(ctr, key, x);
            double zz[4];
            for (int h = 0; h < 2; ++h) {
                double u1 = orc_uniform(x[2 * h]), u2 = orc_uniform(x[2 * h + 1]);
                double r = sqrt(-2.0 * log(u1));
                zz[2 * h] = r * cos(two_pi * u2);
                zz[2 * h + 1] = r * sin(two_pi * u2);
            }
            for (int h = 0; h < 4 && 4 * g + h < D; ++h) z[(size_t)b * D + 4 * g + h] = zz[h];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* voxel occupancy and exact squared Euclidean distance transforms           */
/* ------------------------------------------------------------------------ */

/* occupied = voxel holding at least one point; index floor((p - o) / h)
 * computed in double precision; points outside the grid are dropped */
void orc_occupancy(const float *pts, int64_t N, const int32_t dims[3], const float origin[3], float voxel,
                   uint8_t *occ) {
    size_t nvox = (size_t)dims[0] * dims[1] * dims[2];
    memset(occ, 0, nvox);
    for (int64_t i = 0; i < N; ++i) {
        int64_t ix[3];
        int ok = 1;
        for (int a = 0; a < 3; ++a) {
            double g = ((double)pts[3 * i + a] - (double)origin[a]) / (double)voxel;
            double fl = floor(g);
            if (!(fl >= 0.0 && fl < (double)dims[a])) { ok = 0; break; }
            ix[a] = (int64_t)fl;
        }
        if (ok) occ[((size_t)ix[2] * dims[1] + (size_t)ix[1]) * dims[0] + (size_t)ix[0]] = 1;
    }
}

static int64_t no_target_value(const int32_t dims[3]) {
    return (int64_t)dims[0] * dims[0] + (int64_t)dims[1] * dims[1] + (int64_t)dims[2] * dims[2];
}

/* definition: min over every target voxel of the squared index distance */
void orc_edt_brute(const uint8_t *mask, uint8_t target, const int32_t dims[3], int64_t *out) {
    int nx = dims[0], ny = dims[1], nz = dims[2];
    int64_t none = no_target_value(dims);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t best = -1;
                for (int z2 = 0; z2 < nz; ++z2)
                    for (int y2 = 0; y2 < ny; ++y2)
                        for (int x2 = 0; x2 < nx; ++x2) {
                            if (mask[((size_t)z2 * ny + y2) * nx + x2] != target) continue;
                            int64_t d = (int64_t)(x - x2) * (x - x2) + (int64_t)(y - y2) * (y - y2) +
                                        (int64_t)(z - z2) * (z - z2);
                            if (best < 0 || d < best) best = d;
                        }
                out[((size_t)z * ny + y) * nx + x] = best < 0 ? none : best;
            }
}

/* the squared distance separates over axes:
 *   D(x,y,z) = min_z' [(z-z')^2 + min_y' [(y-y')^2 + min_x' [(x-x')^2 + F(x',y',z')]]]
 * with F = 0 on target voxels and +inf elsewhere; each 1-D stage below is the
 * plain minimum over the grid line */
void orc_edt_separable(const uint8_t *mask, uint8_t target, const int32_t dims[3], int64_t *out) {
    int nx = dims[0], ny = dims[1], nz = dims[2];
    const int64_t INF = INT64_MAX / 4;
    size_t nvox = (size_t)nx * ny * nz;
    int64_t *a = (int64_t *)malloc(nvox * sizeof(int64_t));
    int64_t *b = (int64_t *)malloc(nvox * sizeof(int64_t));
    for (size_t i = 0; i < nvox; ++i) a[i] = mask[i] == target ? 0 : INF;
    /* x stage */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
            const int64_t *f = a + ((size_t)z * ny + y) * nx;
            int64_t *g = b + ((size_t)z * ny + y) * nx;
            for (int x = 0; x < nx; ++x) {
                int64_t best = INF;
                for (int x2 = 0; x2 < nx; ++x2) {
                    if (f[x2] >= INF) continue;
                    int64_t v = f[x2] + (int64_t)(x - x2) * (x - x2);
                    if (v < best) best = v;
                }
                g[x] = best;
            }
        }
    /* y stage */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int x = 0; x < nx; ++x) {
            for (int y = 0; y < ny; ++y) {
                int64_t best = INF;
                for (int y2 = 0; y2 < ny; ++y2) {
                    int64_t f = b[((size_t)z * ny + y2) * nx + x];
                    if (f >= INF) continue;
                    int64_t v = f + (int64_t)(y - y2) * (y - y2);
                    if (v < best) best = v;
                }
                a[((size_t)z * ny + y) * nx + x] = best;
            }
        }
    /* z stage */
#pragma omp parallel for collapse(2) schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            for (int z = 0; z < nz; ++z) {
                int64_t best = INF;
                for (int z2 = 0; z2 < nz; ++z2) {
                    int64_t f = a[((size_t)z2 * ny + y) * nx + x];
                    if (f >= INF) continue;
                    int64_t v = f + (int64_t)(z - z2) * (z - z2);
                    if (v < best) best = v;
                }
                b[((size_t)z * ny + y) * nx + x] = best;
            }
        }
    int64_t none = no_target_value(dims);
    for (size_t i = 0; i < nvox; ++i) out[i] = b[i] >= INF ? none : b[i];
    free(a);
    free(b);
}

/* signed field at voxel centres: free voxels h (sqrt(EDT to occupied) - 1/2),
 * occupied voxels -h (sqrt(EDT to free) - 1/2) */
void orc_sdf_from_edt(const uint8_t *occ, const int64_t *edt_occ, const int64_t *edt_free, size_t nvox,
                      float voxel, double *phi) {
    double h = voxel;
    for (size_t i = 0; i < nvox; ++i)
        phi[i] = occ[i] ? -h * (sqrt((double)edt_free[i]) - 0.5) : h * (sqrt((double)edt_occ[i]) - 0.5);
}
