/*
 * sgtp_ref.c -- plain CPU oracle for SGTP (Sampling-based Game-Theoretic Planning).
 *
 * TEST INFRASTRUCTURE.  This file is the slow, obviously-correct reference that
 * the GPU planner is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the planner never calls it.
 * It shares no source with the HIP implementation.
 *
 * Precision: float64 everywhere, except the Gaussian transform of the noise,
 * which is specified as an exact sequence of IEEE float32 operations so that the
 * drawn perturbations are reproducible bit for bit on any conforming device
 * (see gauss_pair below).  Build with -ffp-contract=off and without fast-math.
 *
 * What is computed (paper section / equation / algorithm):
 *   - Alg. 1 (SGTP): initialisation, L_IBR Jacobi sweeps of best responses
 *     with opponents fixed at the previous sweep, one extra ego response.
 *   - Sec. III (sampling): K Gaussian control perturbations about the nominal
 *     sequence, clipped to the admissible box, rolled out through f.
 *   - Sec. II: kinematic bicycle model; the full-scale workloads use a dynamic
 *     single-track model with a simplified Magic-Formula tyre (reading below).
 *   - Sec. III-A: game-aware cost, eqs. (game_cost), (c_contest), (c_long),
 *     (c_block), (Dmin), (c_safety); tracking cost eq. (ctrack); total eq. (allc).
 *   - Sec. III-B: boundary check eq. (selection-boundary), collision check
 *     eq. (selection-vehicle), selection eq. (selection), least-violation fallback.
 *
 * Readings where the paper is silent (each one is also listed in the design notes):
 *   - integrator: classic RK4 with the control held over dt; the derivative uses
 *     max(v_x, 0) and v_x is clamped at 0 after each interval (no reversing).
 *   - Frenet projection: polyline through the nodes with unit normals
 *     interpolated linearly along each segment; the foot parameter solves
 *     cross(p - c(t), n(t)) = 0, which makes s and d continuous.  A point is in
 *     segment i when it lies between the normal lines of nodes i and i+1; the
 *     per-step search starts at the previous segment and moves at most
 *     `max_moves` segments.
 *   - reference states: linear interpolation of node values at s^r.
 *   - heading error wrapped to [-pi, pi]; only (x, y, psi, v_x) are weighted by Q.
 *   - footprint: discs along the heading; d_min of eq. (Dmin) is the smallest
 *     centre distance over disc pairs and steps 1..H.
 *   - ties: lowest sample index; a non-finite sample is infeasible with
 *     violation +inf.
 *   - noise: Philox4x32-10 (Salmon et al., SC'11) with counter
 *     (k, floor(tau/2), agent | phase << 16, plan_step) and key = seed; each
 *     call yields the two Gaussian pairs of steps 2*floor(tau/2) and +1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REF_MAX_OPP 15
#define REF_MAX_N 64

/* Scalar types of the per-sample arithmetic (perturbation, rollout, projection and
 * scoring of one candidate): double and float here.  opcount.cpp compiles this file as
 * C++ with operation-counting types in their place (REF_COUNTING) to count that work per
 * sample-step.  Values that do not depend on the candidate (parameters, raceline rows,
 * opponent predictions, the vehicle's current state) stay double and are not counted. */
#ifndef REF_COUNTING
typedef double real;
typedef float real32;
#define REF_D(x) (x)
#define REF_F(x) (x)
#endif

/* ------------------------------------------------------------------------ */
/* Interface types (mirrored by ctypes in ref.py)                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int model; /* 0 dynamic single-track, 1 kinematic bicycle */
    int N;
    double dt;
    double a_min, a_max, d_min, d_max;
    double sigma_a, sigma_d;
    double Q[4], R[2], S[2];
    double w_game, w_contest, w_long, w_block, w_safety;
    double s_contest, s_role, eps_alpha;
    int n_tail, n_disc;
    double g_safe, m_bd, d_col;
    double disc_off[4];
    double m, Iz, lf, lr, B, C, mu, g, v_eps;
    int max_moves, pad0;
    /* best-response update: 0 = feasibility selection (Sec. III-B); 1 = path-integral
     * update of the nominal (the paper's GA-IBR-MPPI ablation, Sec. IV-A) with
     * temperature mppi_lambda on the score c + mppi_w_viol * nu */
    int update, pad1;
    double mppi_lambda, mppi_w_viol;
    /* perturbation of the opponents' predicted positions (robustness experiment,
     * Sec. IV-F, Table II): standard deviations along / across the predicted heading */
    double pred_sig_lon, pred_sig_lat;
} ref_params;

typedef struct {
    const double *nodes; /* [n][8] x, y, psi, kappa, wL, wR, vref, s */
    int n, closed;
    double length, psi_lap;
} ref_track;

typedef struct {
    int n_agents, ego, K, pad0;
    unsigned long long seed;
    unsigned int plan_step, pad1;
    const double *x;       /* [n][6] world states */
    const double *s_prev;  /* [n] previous unwrapped progress, or NULL */
    const double *v_scale; /* [n] */
    const double *u_nom;   /* [n][N][2] */
    const int *agent_id;   /* [n] identity used in the noise counter, or NULL (= index) */
    const double *prop;    /* [n][N][4] proposal (mu_a, mu_d, sigma_a, sigma_d), or NULL */
    int K_prop, pad2;      /* samples k < K_prop are drawn from the proposal */
} ref_race;

typedef struct {
    int k;          /* oracle's own selection */
    int fallback;   /* 1 when no sample was feasible */
    int n_feasible;
    int k_used;     /* sample whose controls were adopted (forced or own) */
    double cost;    /* cost of k (feasible) */
    double viol;    /* violation of k */
    double cost2;   /* second-lowest feasible cost (or +inf) */
    double cost_used, scale_used, viol_used;
    int flags_used, pad0;
} ref_choice;

typedef struct { /* optional per-sample outputs, any pointer may be NULL */
    double *cost, *scale, *viol, *rho_bd, *rho_obs, *x_final, *s_final, *contest_margin, *max_abs_d;
    int *flags; /* bit0 b, bit1 o, bit2 h, bit3 search limit hit, bit4 non-finite */
    float *noise; /* [K][N][2] */
} ref_sample_out;

enum { F_B = 1, F_O = 2, F_H = 4, F_LIMIT = 8, F_NONFINITE = 16 };

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): 10 rounds of two 32x32->64 multiplies with the  */
/* published multipliers and Weyl key increments.                            */
/* ------------------------------------------------------------------------ */

void ref_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Gaussian pair from two 32-bit words: Box-Muller, specified as an exact    */
/* float32 operation sequence (IEEE add/mul/fma/div/sqrt, round to nearest). */
/*   u1 = (2*(r_even >> 9) + 1) * 2^-24  in (0, 1)                           */
/*   u2 = (r_odd >> 8) * 2^-24           in [0, 1)                           */
/*   rho = sqrt(-2 ln u1), (z_a, z_d) = rho * (cos 2 pi u2, sin 2 pi u2)     */
/* ln: u1 = m 2^e with m in [sqrt(1/2), sqrt 2); ln m = 2 atanh((m-1)/(m+1)) */
/* summed to z^13.  sin/cos: exact quarter-turn split of u2, then Taylor     */
/* polynomials of sin(2 pi r), cos(2 pi r) for |r| <= 1/8 turn.              */
/* ------------------------------------------------------------------------ */

static float f_from_bits(uint32_t b) { float f; memcpy(&f, &b, 4); return f; }
static uint32_t bits_from_f(float f) { uint32_t b; memcpy(&b, &f, 4); return b; }

void ref_gauss_pair(uint32_t r_even, uint32_t r_odd, float out[2])
{
    const float L3 = 0x1.555556p-1f, L5 = 0x1.99999ap-2f, L7 = 0x1.24924ap-2f;
    const float L9 = 0x1.c71c72p-3f, L11 = 0x1.745d18p-3f, L13 = 0x1.3b13b2p-3f;
    const float LN2_HI = 0x1.62e4p-1f, LN2_LO = 0x1.7f7d1cp-20f;
    const float SQRT2 = 0x1.6a09e6p+0f;
    const float S1 = 0x1.921fb6p+2f, S3 = -0x1.4abbcep+5f, S5 = 0x1.466bc6p+6f;
    const float S7 = -0x1.32d2ccp+6f, S9 = 0x1.507834p+5f;
    const float C2 = -0x1.3bd3ccp+4f, C4 = 0x1.03c1f0p+6f, C6 = -0x1.55d3c8p+6f;
    const float C8 = 0x1.e1f506p+5f, C10 = -0x1.a6d1f2p+4f;

    /* ---- radius ---- */
    real32 u1 = (real32)(float)(2u * (r_even >> 9) + 1u) * 0x1p-24f;
    uint32_t b = bits_from_f(REF_F(u1));
    int e = (int)((b >> 23) & 0xffu) - 127;
    real32 m = f_from_bits((b & 0x7fffffu) | 0x3f800000u); /* [1, 2) */
    if (m > SQRT2) {
        m = m * 0.5f;
        e = e + 1;
    }
    real32 f = m - 1.0f;
    real32 z = f / (m + 1.0f);
    real32 w = z * z;
    real32 p = fmaf(L13, w, L11);
    p = fmaf(p, w, L9);
    p = fmaf(p, w, L7);
    p = fmaf(p, w, L5);
    p = fmaf(p, w, L3);
    p = p * w;
    real32 lnm = fmaf(z, p, z + z);
    real32 ef = (real32)(float)e;
    real32 lnu = fmaf(ef, LN2_HI, fmaf(ef, LN2_LO, lnm));
    real32 rho = sqrtf(-2.0f * lnu);

    /* ---- angle ---- */
    uint32_t j = r_odd >> 8;                       /* u2 = j * 2^-24 */
    uint32_t q = (j + (1u << 21)) >> 22;           /* nearest quarter turn */
    int32_t ri = (int32_t)j - (int32_t)(q << 22);  /* remainder in [-2^21, 2^21) */
    real32 r = (real32)(float)ri * 0x1p-24f;      /* turns, |r| <= 1/8 */
    real32 r2 = r * r;
    real32 ps = fmaf(S9, r2, S7);
    ps = fmaf(ps, r2, S5);
    ps = fmaf(ps, r2, S3);
    ps = fmaf(ps, r2, S1);
    real32 sn = ps * r;
    real32 pc = fmaf(C10, r2, C8);
    pc = fmaf(pc, r2, C6);
    pc = fmaf(pc, r2, C4);
    pc = fmaf(pc, r2, C2);
    real32 cs = fmaf(pc, r2, 1.0f);
    real32 sin_t, cos_t;
    switch (q & 3u) {
    case 0: sin_t = sn; cos_t = cs; break;
    case 1: sin_t = cs; cos_t = -sn; break;
    case 2: sin_t = -sn; cos_t = -cs; break;
    default: sin_t = -cs; cos_t = sn; break;
    }
    out[0] = REF_F(rho * cos_t);
    out[1] = REF_F(rho * sin_t);
}

/* The transform on n given word pairs: out[2 i], out[2 i + 1]. */
void ref_gauss_pairs(int n, const uint32_t *r_even, const uint32_t *r_odd, float *out)
{
    for (int i = 0; i < n; ++i) ref_gauss_pair(r_even[i], r_odd[i], out + 2 * (size_t)i);
}

/* Perturbations of sample k, steps 0..N-1, as float32 [N][2]. */
void ref_noise_seq(unsigned long long seed, unsigned int plan_step, int agent, int phase, int k, int N,
                   float *z)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int m = 0; 2 * m < N; ++m) {
        uint32_t ctr[4] = {(uint32_t)k, (uint32_t)m, (uint32_t)agent | ((uint32_t)phase << 16), plan_step};
        uint32_t r[4];
        ref_philox4x32_10(ctr, key, r);
        ref_gauss_pair(r[0], r[1], z + 4 * m);
        if (2 * m + 1 < N)
            ref_gauss_pair(r[2], r[3], z + 4 * m + 2);
    }
}

/* ------------------------------------------------------------------------ */
/* Vehicle models (Sec. II) and RK4                                          */
/* ------------------------------------------------------------------------ */

/* x = (x, y, psi, vx, vy, omega); u = (a, delta). */
void ref_deriv(const ref_params *p, const real *x, const real *u, real *dx)
{
    const double L = p->lf + p->lr;
    /* negative speeds reached inside an RK4 stage do not move the vehicle backwards */
    const real psi = x[2], vx = fmax(x[3], 0.0), vy = x[4], om = x[5];
    const real a = u[0], delta = u[1];
    if (p->model == 1) {
        /* kinematic bicycle, reference point at the centre of gravity */
        real beta = atan(p->lr * tan(delta) / L);
        dx[0] = vx * cos(psi + beta);
        dx[1] = vx * sin(psi + beta);
        dx[2] = vx * sin(beta) / p->lr;
        dx[3] = a;
        dx[4] = 0.0;
        dx[5] = 0.0;
        return;
    }
    /* dynamic single-track with F_y = mu F_z sin(C atan(B alpha)) */
    real vh = fmax(vx, p->v_eps);
    real alpha_f = delta - atan((vy + p->lf * om) / vh);
    real alpha_r = -atan((vy - p->lr * om) / vh);
    double Fzf = p->m * p->g * p->lr / L;
    double Fzr = p->m * p->g * p->lf / L;
    real Fyf = p->mu * Fzf * sin(p->C * atan(p->B * alpha_f));
    real Fyr = p->mu * Fzr * sin(p->C * atan(p->B * alpha_r));
    const real cpsi = cos(psi), spsi = sin(psi), cdel = cos(delta), sdel = sin(delta);
    dx[0] = vx * cpsi - vy * spsi;
    dx[1] = vx * spsi + vy * cpsi;
    dx[2] = om;
    dx[3] = a - Fyf * sdel / p->m + vy * om;
    dx[4] = (Fyr + Fyf * cdel) / p->m - vx * om;
    dx[5] = (p->lf * Fyf * cdel - p->lr * Fyr) / p->Iz;
}

/* One control interval: classic RK4 with u held, then v_x <- max(v_x, 0). */
void ref_step(const ref_params *p, real *x, const real *u)
{
    real k1[6], k2[6], k3[6], k4[6], xt[6];
    const double h = p->dt;
    ref_deriv(p, x, u, k1);
    for (int i = 0; i < 6; ++i) xt[i] = x[i] + 0.5 * h * k1[i];
    ref_deriv(p, xt, u, k2);
    for (int i = 0; i < 6; ++i) xt[i] = x[i] + 0.5 * h * k2[i];
    ref_deriv(p, xt, u, k3);
    for (int i = 0; i < 6; ++i) xt[i] = x[i] + h * k3[i];
    ref_deriv(p, xt, u, k4);
    for (int i = 0; i < 6; ++i) x[i] = x[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    if (x[3] < 0.0) x[3] = 0.0;
}

/* ------------------------------------------------------------------------ */
/* Track access and Frenet projection (Sec. II: s(x;G), d(x;G))              */
/* ------------------------------------------------------------------------ */

typedef struct {
    double x, y, psi, wL, wR, vref, s;
} node_t;

static long floordiv(long a, long b) { long q = a / b; if ((a % b) != 0 && ((a < 0) != (b < 0))) --q; return q; }

/* Node i of an unwrapped index: closed tracks repeat with s + length, psi + psi_lap per lap. */
static node_t node_at(const ref_track *T, long i)
{
    node_t nd;
    long lap = 0, b = i;
    if (T->closed) {
        lap = floordiv(i, T->n);
        b = i - lap * T->n;
    } else {
        if (b < 0) b = 0;
        if (b > T->n - 1) b = T->n - 1;
    }
    const double *r = T->nodes + 8 * b;
    nd.x = r[0];
    nd.y = r[1];
    nd.psi = r[2] + (double)lap * T->psi_lap;
    nd.wL = r[4];
    nd.wR = r[5];
    nd.vref = r[6];
    nd.s = r[7] + (double)lap * T->length;
    return nd;
}

/* Position of p relative to the normal line at node i: > 0 ahead of it. */
static real ahead_of(const ref_track *T, long i, const real *p)
{
    node_t nd = node_at(T, i);
    double nx = -sin(nd.psi), ny = cos(nd.psi);
    return (p[0] - nd.x) * ny - (p[1] - nd.y) * nx;
}

typedef struct {
    real s, d, t, wL, wR;
} foot_t;

/* Foot of p on segment i with linearly interpolated normals. */
static foot_t foot_on_segment(const ref_track *T, long i, const real *p)
{
    node_t a = node_at(T, i), b = node_at(T, i + 1);
    double n0x = -sin(a.psi), n0y = cos(a.psi);
    double n1x = -sin(b.psi), n1y = cos(b.psi);
    real rx = p[0] - a.x, ry = p[1] - a.y;
    double Dx = b.x - a.x, Dy = b.y - a.y;
    double dnx = n1x - n0x, dny = n1y - n0y;
    /* cross(r - t D, n0 + t dn) = C + B t + A t^2 */
    real Cc = rx * n0y - ry * n0x;
    real Bc = (rx * dny - ry * dnx) - (Dx * n0y - Dy * n0x);
    double Ac = -(Dx * dny - Dy * dnx);
    real disc = Bc * Bc - 4.0 * Ac * Cc;
    if (disc < 0.0) disc = 0.0;
    real den = -Bc - copysign(sqrt(disc), Bc);
    real t = (den != 0.0) ? 2.0 * Cc / den : (real)0.0;
    if (!(t >= 0.0)) t = 0.0; /* also maps NaN to 0 */
    if (t > 1.0) t = 1.0;
    real cx = a.x + t * Dx, cy = a.y + t * Dy;
    real nx = n0x + t * dnx, ny = n0y + t * dny;
    foot_t f;
    f.t = t;
    f.d = ((p[0] - cx) * nx + (p[1] - cy) * ny) / sqrt(nx * nx + ny * ny);
    f.s = a.s + t * (b.s - a.s);
    f.wL = a.wL + t * (b.wL - a.wL);
    f.wR = a.wR + t * (b.wR - a.wR);
    return f;
}

static int can_advance(const ref_track *T, long i) { return T->closed || i + 1 <= T->n - 2; }
static int can_retreat(const ref_track *T, long i) { return T->closed || i > 0; }

/* Local search from segment `seg`; returns the new segment, sets *limit when the
 * point is still outside the segment's normal lines after the search. */
static long walk(const ref_track *T, int max_moves, const real *p, long seg, int *limit)
{
    long i = seg;
    int moves = 0;
    while (moves < max_moves && can_advance(T, i) && ahead_of(T, i + 1, p) > 0.0) {
        ++i;
        ++moves;
    }
    while (moves < max_moves && can_retreat(T, i) && ahead_of(T, i, p) < 0.0) {
        --i;
        ++moves;
    }
    *limit = !(ahead_of(T, i, p) >= 0.0 && ahead_of(T, i + 1, p) <= 0.0);
    return i;
}

/* Global projection: among segments whose normal lines enclose p, the one with the
 * smallest |d| (lowest index on ties); if none encloses p, the segment starting at
 * the nearest node.  Returns the segment in [0, n) and writes (s, d, t). */
long ref_project_global(const ref_track *T, const double *p_in, double *out3)
{
    const real p[2] = {p_in[0], p_in[1]};
    long nseg = T->closed ? T->n : T->n - 1;
    long best = -1;
    double best_ad = INFINITY;
    for (long i = 0; i < nseg; ++i) {
        if (ahead_of(T, i, p) >= 0.0 && ahead_of(T, i + 1, p) <= 0.0) {
            foot_t f = foot_on_segment(T, i, p);
            if (fabs(REF_D(f.d)) < best_ad) {
                best_ad = fabs(REF_D(f.d));
                best = i;
            }
        }
    }
    if (best < 0) {
        double bd = INFINITY;
        for (long i = 0; i < nseg; ++i) {
            node_t nd = node_at(T, i);
            double dd = (p_in[0] - nd.x) * (p_in[0] - nd.x) + (p_in[1] - nd.y) * (p_in[1] - nd.y);
            if (dd < bd) {
                bd = dd;
                best = i;
            }
        }
    }
    foot_t f = foot_on_segment(T, best, p);
    out3[0] = REF_D(f.s);
    out3[1] = REF_D(f.d);
    out3[2] = REF_D(f.t);
    return best;
}

/* Local projection from a segment hint: out = (s, d, t, wL, wR, limit). */
long ref_project_walk(const ref_track *T, int max_moves, const double *p_in, long seg, double *out6)
{
    const real p[2] = {p_in[0], p_in[1]};
    int limit = 0;
    long i = walk(T, max_moves, p, seg, &limit);
    foot_t f = foot_on_segment(T, i, p);
    out6[0] = REF_D(f.s);
    out6[1] = REF_D(f.d);
    out6[2] = REF_D(f.t);
    out6[3] = REF_D(f.wL);
    out6[4] = REF_D(f.wR);
    out6[5] = (double)limit;
    return i;
}

/* Interpolated node values at arc length s; *hint is moved to the segment holding s. */
static void interp_at_s(const ref_track *T, double s, long *hint, double *x, double *y, double *psi, double *vref)
{
    long i = *hint;
    for (int it = 0; it < 1000000; ++it) {
        node_t a = node_at(T, i), b = node_at(T, i + 1);
        if (s < a.s && can_retreat(T, i)) {
            --i;
            continue;
        }
        if (s >= b.s && can_advance(T, i)) {
            ++i;
            continue;
        }
        double t = (s - a.s) / (b.s - a.s);
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
        *x = a.x + t * (b.x - a.x);
        *y = a.y + t * (b.y - a.y);
        *psi = a.psi + t * (b.psi - a.psi);
        *vref = a.vref + t * (b.vref - a.vref);
        break;
    }
    *hint = i;
}

/* Reference recursion of Sec. III-A (overall ranking):
 * s^r_0 = s0, s^r_{tau+1} = s^r_tau + dt * lam * v^r(s^r_tau);
 * xr[tau] = (x^r, y^r, psi^r, lam * v^r) at s^r_{tau+1}, tau = 0..N-1. */
void ref_reference(const ref_track *T, const ref_params *p, long seg0, double s0, double lam, double *xr)
{
    long hint = seg0;
    double sr = s0, x, y, psi, v;
    for (int tau = 0; tau < p->N; ++tau) {
        interp_at_s(T, sr, &hint, &x, &y, &psi, &v);
        sr = sr + p->dt * lam * v;
        interp_at_s(T, sr, &hint, &x, &y, &psi, &v);
        xr[4 * tau + 0] = x;
        xr[4 * tau + 1] = y;
        xr[4 * tau + 2] = psi;
        xr[4 * tau + 3] = lam * v;
    }
}

/* ------------------------------------------------------------------------ */
/* Rollouts                                                                  */
/* ------------------------------------------------------------------------ */

static real clampd(real v, double lo, double hi) { return v < lo ? (real)lo : (v > hi ? (real)hi : v); }

/* Noise-free rollout of a control sequence (already admissible after clipping):
 * traj[tau] = (x, y, psi, vx, vy, omega, s, d) for tau = 0..N (tau = 0 is x0). */
void ref_rollout_controls(const ref_track *T, const ref_params *p, const double *x0, long seg0, double s0,
                          double d0, const double *U, double *traj)
{
    real x[6];
    for (int i = 0; i < 6; ++i) x[i] = x0[i];
    long seg = seg0;
    for (int i = 0; i < 6; ++i) traj[i] = x0[i];
    traj[6] = s0;
    traj[7] = d0;
    for (int tau = 0; tau < p->N; ++tau) {
        real u[2] = {clampd(U[2 * tau], p->a_min, p->a_max), clampd(U[2 * tau + 1], p->d_min, p->d_max)};
        ref_step(p, x, u);
        int limit;
        seg = walk(T, p->max_moves, x, seg, &limit);
        foot_t f = foot_on_segment(T, seg, x);
        double *o = traj + 8 * (tau + 1);
        for (int i = 0; i < 6; ++i) o[i] = REF_D(x[i]);
        o[6] = REF_D(f.s);
        o[7] = REF_D(f.d);
    }
}

/* Everything one best response of agent i needs (Sec. III, per vehicle i). */
typedef struct {
    int agent, phase, n_opp, K;
    long seg0;
    double s0;
    double w_game;
    unsigned long long seed;
    unsigned int plan_step, pad0;
    const double *x0;       /* [6] */
    const double *xr;       /* [N][4] */
    const double *ubar;     /* [N][2] */
    const double *opp_traj; /* [n_opp][N+1][8] */
    const double *opp_s0;   /* [n_opp] */
    const double *prop;     /* [N][4] proposal (mu_a, mu_d, sigma_a, sigma_d), or NULL */
    int K_prop, pad1;
} ref_br_in;

typedef struct {
    real cost, scale, viol, rho_bd, rho_obs, s_final, contest_margin, max_abs_d;
    real x_final[6];
    int flags;
    real U[2 * REF_MAX_N];
} sample_res;

/* One candidate: perturb, clip, roll out, score, check (Sec. III-A, III-B). */
static void evaluate_sample(const ref_track *T, const ref_params *p, const ref_br_in *in, int k, sample_res *res,
                            float *noise_out)
{
    const int N = p->N;
    float z[2 * REF_MAX_N];
    ref_noise_seq(in->seed, in->plan_step, in->agent, in->phase, k, N, z);
    if (noise_out) memcpy(noise_out, z, sizeof(float) * 2 * N);

    real x[6];
    for (int i = 0; i < 6; ++i) x[i] = in->x0[i];
    long seg = in->seg0;
    real J = 0.0, rho_bd = INFINITY, dsum = 0.0, max_abs_d = 0.0;
    real g2[REF_MAX_OPP]; /* squared footprint distances; d_min of eq. (Dmin) is the root of their minimum */
    for (int j = 0; j < in->n_opp; ++j) g2[j] = INFINITY;
    real up[2] = {0.0, 0.0};
    real s = in->s0;
    int any_limit = 0;

    /* learned proposal: samples k < K_prop are drawn about the proposal mean with its
     * scales, the others about the nominal with the plain scales */
    const int use_prop = in->prop && k < in->K_prop;
    for (int tau = 0; tau < N; ++tau) {
        real u[2];
        const real za = (double)z[2 * tau], zd = (double)z[2 * tau + 1];
        if (use_prop) {
            const double *q = in->prop + 4 * tau;
            u[0] = clampd(q[0] + q[2] * za, p->a_min, p->a_max);
            u[1] = clampd(q[1] + q[3] * zd, p->d_min, p->d_max);
        } else {
            u[0] = clampd(in->ubar[2 * tau] + p->sigma_a * za, p->a_min, p->a_max);
            u[1] = clampd(in->ubar[2 * tau + 1] + p->sigma_d * zd, p->d_min, p->d_max);
        }
        res->U[2 * tau] = u[0];
        res->U[2 * tau + 1] = u[1];
        ref_step(p, x, u);

        int limit;
        seg = walk(T, p->max_moves, x, seg, &limit);
        any_limit |= limit;
        foot_t f = foot_on_segment(T, seg, x);
        s = f.s;
        if (fabs(f.d) > max_abs_d) max_abs_d = fabs(f.d);

        /* tracking and control cost, eq. (ctrack) */
        const double *xr = in->xr + 4 * tau;
        real ex = x[0] - xr[0], ey = x[1] - xr[1];
        real epsi = remainder(x[2] - xr[2], 2.0 * M_PI);
        real ev = x[3] - xr[3];
        J += p->Q[0] * ex * ex + p->Q[1] * ey * ey + p->Q[2] * epsi * epsi + p->Q[3] * ev * ev;
        J += p->R[0] * u[0] * u[0] + p->R[1] * u[1] * u[1];
        if (tau >= 1) {
            real da = u[0] - up[0], dd = u[1] - up[1];
            J += p->S[0] * da * da + p->S[1] * dd * dd;
        }
        up[0] = u[0];
        up[1] = u[1];

        /* boundary clearance, eq. (selection-boundary) */
        real rb = fmin(f.wR + f.d, f.wL - f.d);
        if (rb < rho_bd || rb != rb) rho_bd = rb;

        /* time-aligned footprint distance to each opponent, eq. (Dmin): the smallest
         * disc-centre distance over disc pairs and steps, taken as the root of the smallest
         * squared distance (the root is monotone, so both give the same value) */
        real ch = cos(x[2]), sh = sin(x[2]);
        real cax[4], cay[4]; /* own disc centres */
        for (int a = 0; a < p->n_disc; ++a) {
            cax[a] = x[0] + p->disc_off[a] * ch;
            cay[a] = x[1] + p->disc_off[a] * sh;
        }
        for (int j = 0; j < in->n_opp; ++j) {
            const double *o = in->opp_traj + 8 * ((size_t)j * (N + 1) + tau + 1);
            double och = cos(o[2]), osh = sin(o[2]);
            for (int a = 0; a < p->n_disc; ++a) {
                for (int b = 0; b < p->n_disc; ++b) {
                    double cbx = o[0] + p->disc_off[b] * och, cby = o[1] + p->disc_off[b] * osh;
                    real ddx = cax[a] - cbx, ddy = cay[a] - cby;
                    real dist2 = ddx * ddx + ddy * ddy;
                    if (dist2 < g2[j] || dist2 != dist2) g2[j] = dist2;
                }
            }
        }

        /* tail lateral offsets, T_tail = {N - n_tail + 1, ..., N} */
        if (tau + 1 > N - p->n_tail) dsum += f.d;
    }

    /* game-aware cost, eqs. (game_cost), (c_contest), (c_long), (c_block), (c_safety) */
    real g[REF_MAX_OPP];
    for (int j = 0; j < in->n_opp; ++j) g[j] = sqrt(g2[j]);
    real cgame = 0.0, cgame_abs = 0.0, rho_obs = INFINITY, cmargin = INFINITY;
    real dbar_i = dsum / (double)p->n_tail;
    for (int j = 0; j < in->n_opp; ++j) {
        const double *oj = in->opp_traj + 8 * ((size_t)j * (N + 1));
        double sN_j = oj[8 * N + 6];
        double dbar_j = 0.0;
        for (int tau = N - p->n_tail + 1; tau <= N; ++tau) dbar_j += oj[8 * tau + 7];
        dbar_j /= (double)p->n_tail;
        real dsN = s - sN_j;           /* terminal progress gap */
        double ds0 = in->s0 - in->opp_s0[j]; /* current progress gap */
        double alpha = 1.0 / (1.0 + fabs(ds0) / (p->s_contest + p->eps_alpha));
        double gamma = (ds0 > p->s_role && ds0 < p->s_contest) ? p->w_block : 0.0;
        real c_contest = (fabs(dsN) < p->s_contest) ? (real)-p->w_contest : (real)0.0;
        real c_long = -p->w_long * alpha * dsN;
        real c_block = -gamma / (1.0 + fabs(dbar_i - dbar_j));
        real sh = fmax(0.0, p->g_safe - g[j]);
        real c_safety = p->w_safety * sh * sh;
        cgame += c_contest + c_long + c_block + c_safety;
        cgame_abs += fabs(c_contest) + fabs(c_long) + fabs(c_block) + fabs(c_safety);
        if (g[j] < rho_obs || g[j] != g[j]) rho_obs = g[j];
        real cm = fabs(fabs(dsN) - p->s_contest);
        if (cm < cmargin) cmargin = cm;
    }
    real c = J + in->w_game * cgame; /* eq. (allc) */

    int flags = 0;
    int finite = isfinite(c) && !isnan(rho_bd) && !isnan(rho_obs);
    for (int i = 0; i < 6; ++i) finite = finite && isfinite(x[i]);
    if (rho_bd >= p->m_bd) flags |= F_B;
    if (rho_obs >= p->d_col) flags |= F_O;
    if (any_limit) flags |= F_LIMIT;
    real viol = fmax(0.0, p->m_bd - rho_bd) + fmax(0.0, p->d_col - rho_obs);
    if (!finite) {
        flags |= F_NONFINITE;
        flags &= ~(F_B | F_O);
        viol = INFINITY;
    }
    if ((flags & F_B) && (flags & F_O)) flags |= F_H;

    res->cost = c;
    res->scale = J + fabs(in->w_game) * cgame_abs;
    res->viol = viol;
    res->rho_bd = rho_bd;
    res->rho_obs = rho_obs;
    res->s_final = s;
    res->contest_margin = cmargin;
    res->max_abs_d = max_abs_d;
    for (int i = 0; i < 6; ++i) res->x_final[i] = x[i];
    res->flags = flags;
}

/* Selection, eq. (selection) with the least-violation fallback: lowest cost among
 * feasible samples, else lowest violation; ties go to the lowest index. */
static void select_sample(int K, const double *cost, const double *viol, const int *flags, ref_choice *ch)
{
    int kbest = -1, nfeas = 0;
    double cbest = INFINITY, c2 = INFINITY;
    for (int k = 0; k < K; ++k) {
        if (!(flags[k] & F_H)) continue;
        ++nfeas;
        if (kbest < 0 || cost[k] < cbest) {
            c2 = cbest;
            cbest = cost[k];
            kbest = k;
        } else if (cost[k] < c2) {
            c2 = cost[k];
        }
    }
    ch->n_feasible = nfeas;
    ch->cost2 = c2;
    if (kbest >= 0) {
        ch->k = kbest;
        ch->fallback = 0;
        ch->cost = cost[kbest];
        ch->viol = viol[kbest];
        return;
    }
    int kv = 0;
    for (int k = 1; k < K; ++k)
        if (viol[k] < viol[kv]) kv = k;
    ch->k = kv;
    ch->fallback = 1;
    ch->cost = cost[kv];
    ch->viol = viol[kv];
}

/* Path-integral update (the GA-IBR-MPPI ablation of Sec. IV-A; the weighting is the
 * standard MPPI one, the paper gives no temperature): every sample with a finite
 * score S_k = c_k + w_viol nu_k gets the weight exp(-(S_k - S_min) / lambda); the
 * new nominal is the weighted mean of the sampled (clipped) control sequences.  No
 * feasibility selection: constraints enter only through the soft terms of S.  The
 * record holds the lowest-score sample k, S_min as cost, and the number of feasible
 * samples; with no finite score the nominal is kept (fallback = 1). */
static void path_integral(const ref_params *p, int K, int N, const double *cost, const double *viol,
                          const int *flags, const double *Uall, const double *ubar, ref_choice *ch, double *U_out)
{
    int kmin = -1, nfeas = 0;
    double Smin = INFINITY;
    for (int k = 0; k < K; ++k) {
        if (flags[k] & F_H) ++nfeas;
        const double S = cost[k] + p->mppi_w_viol * viol[k];
        if (isfinite(S) && S < Smin) {
            Smin = S;
            kmin = k;
        }
    }
    ch->n_feasible = nfeas;
    ch->cost2 = INFINITY;
    ch->fallback = kmin < 0;
    ch->k = kmin < 0 ? 0 : kmin;
    ch->cost = kmin < 0 ? INFINITY : Smin;
    ch->viol = 0.0;
    ch->k_used = ch->k;
    ch->cost_used = ch->cost;
    ch->scale_used = 0.0;
    ch->viol_used = 0.0;
    ch->flags_used = kmin < 0 ? 0 : flags[kmin];
    if (!U_out) return;
    if (kmin < 0) {
        memcpy(U_out, ubar, sizeof(double) * 2 * N);
        return;
    }
    double wsum = 0.0;
    for (int t = 0; t < 2 * N; ++t) U_out[t] = 0.0;
    for (int k = 0; k < K; ++k) {
        const double S = cost[k] + p->mppi_w_viol * viol[k];
        if (!isfinite(S)) continue;
        const double w = exp(-(S - Smin) / p->mppi_lambda);
        wsum += w;
        for (int t = 0; t < 2 * N; ++t) U_out[t] += w * Uall[(size_t)k * 2 * N + t];
    }
    for (int t = 0; t < 2 * N; ++t) U_out[t] /= wsum;
}

/* One best response: all K samples, optional per-sample outputs, selection.
 * `k_force` >= 0 adopts that sample instead of the selected one (lock-step
 * comparison with another implementation); U_out receives the adopted controls. */
int ref_best_response(const ref_track *T, const ref_params *p, const ref_br_in *in, int k_force,
                      const ref_sample_out *out, ref_choice *ch, double *U_out)
{
    const int K = in->K, N = p->N;
    if (N > REF_MAX_N || in->n_opp > REF_MAX_OPP || K < 1 || p->n_disc < 1 || p->n_disc > 4) return -1;
    double *cost = (double *)malloc(sizeof(double) * K);
    double *viol = (double *)malloc(sizeof(double) * K);
    int *flags = (int *)malloc(sizeof(int) * K);
    double *scale = (double *)malloc(sizeof(double) * K);
    const int pi_update = p->update == 1;
    if (pi_update && !(p->mppi_lambda > 0.0)) {
        free(cost); free(viol); free(flags); free(scale);
        return -1;
    }
    double *Uall = pi_update ? (double *)malloc(sizeof(double) * (size_t)K * 2 * N) : NULL;
    if (!cost || !viol || !flags || !scale || (pi_update && !Uall)) {
        free(cost); free(viol); free(flags); free(scale); free(Uall);
        return -2;
    }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < K; ++k) {
        sample_res r;
        evaluate_sample(T, p, in, k, &r, (out && out->noise) ? out->noise + (size_t)k * 2 * N : NULL);
        cost[k] = REF_D(r.cost);
        viol[k] = REF_D(r.viol);
        flags[k] = r.flags;
        scale[k] = REF_D(r.scale);
        if (Uall)
            for (int t = 0; t < 2 * N; ++t) Uall[(size_t)k * 2 * N + t] = REF_D(r.U[t]);
        if (out) {
            if (out->cost) out->cost[k] = REF_D(r.cost);
            if (out->scale) out->scale[k] = REF_D(r.scale);
            if (out->viol) out->viol[k] = REF_D(r.viol);
            if (out->rho_bd) out->rho_bd[k] = REF_D(r.rho_bd);
            if (out->rho_obs) out->rho_obs[k] = REF_D(r.rho_obs);
            if (out->s_final) out->s_final[k] = REF_D(r.s_final);
            if (out->contest_margin) out->contest_margin[k] = REF_D(r.contest_margin);
            if (out->max_abs_d) out->max_abs_d[k] = REF_D(r.max_abs_d);
            if (out->flags) out->flags[k] = r.flags;
            if (out->x_final)
                for (int i = 0; i < 6; ++i) out->x_final[6 * (size_t)k + i] = REF_D(r.x_final[i]);
        }
    }
    if (pi_update) {
        path_integral(p, K, N, cost, viol, flags, Uall, in->ubar, ch, U_out);
        free(cost); free(viol); free(flags); free(scale); free(Uall);
        return 0;
    }
    select_sample(K, cost, viol, flags, ch);
    int ku = (k_force >= 0 && k_force < K) ? k_force : ch->k;
    ch->k_used = ku;
    ch->cost_used = cost[ku];
    ch->scale_used = scale[ku];
    ch->viol_used = viol[ku];
    ch->flags_used = flags[ku];
    if (U_out) {
        sample_res r;
        evaluate_sample(T, p, in, ku, &r, NULL);
        for (int t = 0; t < 2 * N; ++t) U_out[t] = REF_D(r.U[t]);
    }
    free(cost); free(viol); free(flags); free(scale);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1: one planning step                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    long seg;
    double s, d;
    double xr[4 * REF_MAX_N];
} agent_state;

static void agent_setup(const ref_track *T, const ref_params *p, const ref_race *R, int i, agent_state *A)
{
    double o3[3];
    long seg = ref_project_global(T, R->x + 6 * i, o3);
    double s = o3[0];
    if (T->closed && R->s_prev && isfinite(R->s_prev[i])) {
        double lap = nearbyint((R->s_prev[i] - s) / T->length);
        seg += (long)lap * T->n;
        s += lap * T->length;
    }
    A->seg = seg;
    A->s = s;
    A->d = o3[1];
    ref_reference(T, p, seg, s, R->v_scale[i], A->xr);
}

/* Perturbed opponent prediction (robustness to prediction uncertainty, Sec. IV-F, Table
 * II; the paper cites its perturbation model without details).  Reading: every predicted
 * position tau = 1..N of opponent j, as seen by `observer` in `phase`, moves by
 * sigma_lon z0 along the predicted heading and sigma_lat z1 across it, with (z0, z1) the
 * Gaussian pair of the first two words of Philox(counter = (2^31 | j, tau,
 * observer | phase << 16, plan_step), key = seed); headings, progress and lateral offsets
 * of the prediction are kept.  traj: [N+1][8] world rows (x, y, psi, ...). */
void ref_perturb_prediction(const ref_params *p, unsigned long long seed, unsigned int plan_step, int observer,
                            int phase, int j, int N, double *traj)
{
    if (!(p->pred_sig_lon > 0.0) && !(p->pred_sig_lat > 0.0)) return;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int tau = 1; tau <= N; ++tau) {
        const uint32_t ctr[4] = {0x80000000u | (uint32_t)j, (uint32_t)tau,
                                 (uint32_t)observer | ((uint32_t)phase << 16), plan_step};
        uint32_t r[4];
        float z[2];
        ref_philox4x32_10(ctr, key, r);
        ref_gauss_pair(r[0], r[1], z);
        double *row = traj + 8 * (size_t)tau;
        const double dl = p->pred_sig_lon * (double)z[0], dn = p->pred_sig_lat * (double)z[1];
        const double c = cos(row[2]), sn = sin(row[2]);
        row[0] += dl * c - dn * sn;
        row[1] += dl * sn + dn * c;
    }
}

static void build_br_in(const ref_params *p, const ref_race *R, const agent_state *A, int i, int phase,
                        const double *ubar_all, const double *traj_all, double *opp_buf, double *opp_s0,
                        ref_br_in *in)
{
    const int N = p->N, n = R->n_agents;
    int no = 0;
    for (int j = 0; j < n; ++j) {
        if (j == i) continue;
        memcpy(opp_buf + (size_t)no * (N + 1) * 8, traj_all + (size_t)j * (N + 1) * 8, sizeof(double) * (N + 1) * 8);
        ref_perturb_prediction(p, R->seed, R->plan_step, R->agent_id ? R->agent_id[i] : i, phase,
                               R->agent_id ? R->agent_id[j] : j, N, opp_buf + (size_t)no * (N + 1) * 8);
        opp_s0[no] = A[j].s;
        ++no;
    }
    in->agent = R->agent_id ? R->agent_id[i] : i;
    in->phase = phase;
    in->n_opp = no;
    in->K = R->K;
    in->seg0 = A[i].seg;
    in->s0 = A[i].s;
    in->w_game = (phase == 0) ? 0.0 : p->w_game;
    in->seed = R->seed;
    in->plan_step = R->plan_step;
    in->x0 = R->x + 6 * i;
    in->xr = A[i].xr;
    in->ubar = ubar_all + (size_t)i * N * 2;
    in->opp_traj = opp_buf;
    in->opp_s0 = opp_s0;
    in->prop = R->prop ? R->prop + (size_t)i * N * 4 : NULL;
    in->K_prop = R->K_prop;
}

/* Setup only: projections (s, d, seg) and reference states of every agent. */
int ref_agent_setup(const ref_track *T, const ref_params *p, const ref_race *R, double *s_out, double *d_out,
                    long *seg_out, double *xr_out /*[n][N][4]*/)
{
    if (p->N > REF_MAX_N) return -1;
    for (int i = 0; i < R->n_agents; ++i) {
        agent_state A;
        agent_setup(T, p, R, i, &A);
        if (s_out) s_out[i] = A.s;
        if (d_out) d_out[i] = A.d;
        if (seg_out) seg_out[i] = A.seg;
        if (xr_out) memcpy(xr_out + (size_t)i * p->N * 4, A.xr, sizeof(double) * 4 * p->N);
    }
    return 0;
}

/* One best response of `agent` in `phase` at the planning instant R, with every
 * opponent predicted by the noise-free rollout of its nominal sequence (the
 * state at the start of any sweep of Alg. 1).  U_out [N][2] (or NULL) receives the
 * adopted sequence: the selected sample's controls, or the path-integral mean. */
int ref_rollout_cost(const ref_track *T, const ref_params *p, const ref_race *R, int agent, int phase,
                     const ref_sample_out *out, ref_choice *ch, double *U_out)
{
    const int n = R->n_agents, N = p->N;
    if (N > REF_MAX_N || n - 1 > REF_MAX_OPP || agent < 0 || agent >= n) return -1;
    agent_state *A = (agent_state *)malloc(sizeof(agent_state) * n);
    double *ubar = (double *)malloc(sizeof(double) * n * N * 2);
    double *traj = (double *)malloc(sizeof(double) * n * (N + 1) * 8);
    double *opp = (double *)malloc(sizeof(double) * n * (N + 1) * 8);
    double opp_s0[REF_MAX_OPP + 1];
    for (int i = 0; i < n; ++i) agent_setup(T, p, R, i, &A[i]);
    memcpy(ubar, R->u_nom, sizeof(double) * n * N * 2);
    for (int i = 0; i < n; ++i)
        ref_rollout_controls(T, p, R->x + 6 * i, A[i].seg, A[i].s, A[i].d, ubar + (size_t)i * N * 2,
                             traj + (size_t)i * (N + 1) * 8);
    ref_br_in in;
    build_br_in(p, R, A, agent, phase, ubar, traj, opp, opp_s0, &in);
    int rc = ref_best_response(T, p, &in, -1, out, ch, U_out);
    free(A); free(ubar); free(traj); free(opp);
    return rc;
}

/* Alg. 1.  Phase 0 initialises every agent without the game-aware cost (feasibility,
 * including the distance-based collision check, still applies) against the
 * noise-free rollouts of the nominal sequences; phases 1..L are Jacobi sweeps in
 * which every agent answers the previous phase's trajectories; phase L+1 is the
 * extra ego response.  After each phase an agent's nominal becomes its adopted
 * controls and its prediction the rollout of those controls.
 *
 * forced:  [(L+2)][n] sample indices to adopt (-1 = own selection), or NULL.
 * trace:   [(L+2)][n] selections (k = -1 for agents not in the phase).
 * traj:    [n][N+1][8] final predictions; u_apply: [n][2] first controls;
 * u_next:  [n][N][2] warm start for the next step (shifted, last repeated);
 * s_abs:   [n] unwrapped progress of the current states. */
int ref_plan_step(const ref_track *T, const ref_params *p, const ref_race *R, int L_ibr, const int *forced,
                  ref_choice *trace, double *traj_out, double *u_apply, double *u_next, double *s_abs)
{
    const int n = R->n_agents, N = p->N;
    if (N > REF_MAX_N || n - 1 > REF_MAX_OPP || L_ibr < 0 || R->ego < 0 || R->ego >= n) return -1;
    agent_state *A = (agent_state *)malloc(sizeof(agent_state) * n);
    double *ubar = (double *)malloc(sizeof(double) * n * N * 2);
    double *ubar_new = (double *)malloc(sizeof(double) * n * N * 2);
    double *traj = (double *)malloc(sizeof(double) * n * (N + 1) * 8);
    double *opp = (double *)malloc(sizeof(double) * n * (N + 1) * 8);
    double opp_s0[REF_MAX_OPP + 1];
    int rc = 0;
    for (int i = 0; i < n; ++i) agent_setup(T, p, R, i, &A[i]);
    memcpy(ubar, R->u_nom, sizeof(double) * n * N * 2);
    for (int i = 0; i < n; ++i)
        ref_rollout_controls(T, p, R->x + 6 * i, A[i].seg, A[i].s, A[i].d, ubar + (size_t)i * N * 2,
                             traj + (size_t)i * (N + 1) * 8);
    for (int phase = 0; phase <= L_ibr + 1 && rc == 0; ++phase) {
        memcpy(ubar_new, ubar, sizeof(double) * n * N * 2);
        for (int i = 0; i < n; ++i) {
            ref_choice *ch = trace ? &trace[phase * n + i] : NULL;
            if (phase == L_ibr + 1 && i != R->ego) {
                if (ch) {
                    memset(ch, 0, sizeof *ch);
                    ch->k = ch->k_used = -1;
                }
                continue;
            }
            ref_br_in in;
            build_br_in(p, R, A, i, phase, ubar, traj, opp, opp_s0, &in);
            ref_choice local;
            int kf = forced ? forced[phase * n + i] : -1;
            rc = ref_best_response(T, p, &in, kf, NULL, ch ? ch : &local, ubar_new + (size_t)i * N * 2);
            if (rc) break;
        }
        /* Jacobi update: adopt all new nominals, then re-predict those agents */
        for (int i = 0; i < n && rc == 0; ++i) {
            if (phase == L_ibr + 1 && i != R->ego) continue;
            memcpy(ubar + (size_t)i * N * 2, ubar_new + (size_t)i * N * 2, sizeof(double) * N * 2);
            ref_rollout_controls(T, p, R->x + 6 * i, A[i].seg, A[i].s, A[i].d, ubar + (size_t)i * N * 2,
                                 traj + (size_t)i * (N + 1) * 8);
        }
    }
    if (rc == 0) {
        if (traj_out) memcpy(traj_out, traj, sizeof(double) * n * (N + 1) * 8);
        for (int i = 0; i < n; ++i) {
            const double *U = ubar + (size_t)i * N * 2;
            if (u_apply) {
                u_apply[2 * i] = U[0];
                u_apply[2 * i + 1] = U[1];
            }
            if (u_next) {
                double *W = u_next + (size_t)i * N * 2;
                for (int t = 0; t < N; ++t) {
                    int src = (t + 1 < N) ? t + 1 : N - 1;
                    W[2 * t] = U[2 * src];
                    W[2 * t + 1] = U[2 * src + 1];
                }
            }
            if (s_abs) s_abs[i] = A[i].s;
        }
    }
    free(A); free(ubar); free(ubar_new); free(traj); free(opp);
    return rc;
}

/* Closed loop: every agent applies its first control for one interval. */
void ref_advance(const ref_params *p, int n, double *x, const double *u)
{
    for (int i = 0; i < n; ++i) {
        real xi[6], ui[2] = {u[2 * i], u[2 * i + 1]};
        for (int j = 0; j < 6; ++j) xi[j] = x[6 * i + j];
        ref_step(p, xi, ui);
        for (int j = 0; j < 6; ++j) x[6 * i + j] = REF_D(xi[j]);
    }
}

/* ------------------------------------------------------------------------ */
/* Learned proposal: features, MLP, Gaussian negative log-likelihood        */
/* (an extension of this project, not in the paper; the oracle checks the    */
/* GPU kernels).                                                             */
/* ------------------------------------------------------------------------ */

#define FEAT_DIM 50
#define FEAT_OPP 4
#define FEAT_CURV 20
#define FEAT_CURV_DS 5.0

/* Features of vehicle i (50 values):
 *   ego (6): d / w, heading error to the raceline (wrapped), v_x / 30, v_y / 5, omega,
 *            (v_x - v_ref(s)) / 10
 *   4 nearest opponents by |s_j - s_i| (6 each, zeros when absent): (s_j - s_i) / 20,
 *            (d_j - d_i) / w, heading difference (wrapped), (v_x,j - v_x,i) / 10, v_y,j / 5, 1
 *   curvature ahead (20): 20 kappa(s_i + 5 m * m), m = 1..20 (linear interpolation)
 * w is the half width at the vehicle. */
static double wrap_pi(double a) { return remainder(a, 2.0 * M_PI); }

static double kappa_at(const ref_track *T, double s, long *hint)
{
    long i = *hint;
    for (int it = 0; it < 1000000; ++it) {
        node_t a = node_at(T, i), b = node_at(T, i + 1);
        if (s < a.s && can_retreat(T, i)) { --i; continue; }
        if (s >= b.s && can_advance(T, i)) { ++i; continue; }
        break;
    }
    *hint = i;
    node_t a = node_at(T, i), b = node_at(T, i + 1);
    long ia = T->closed ? ((i % T->n) + T->n) % T->n : (i < 0 ? 0 : (i > T->n - 1 ? T->n - 1 : i));
    long ib = T->closed ? (((i + 1) % T->n) + T->n) % T->n : (i + 1 > T->n - 1 ? T->n - 1 : i + 1);
    double t = (s - a.s) / (b.s - a.s);
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    return T->nodes[8 * ia + 3] + t * (T->nodes[8 * ib + 3] - T->nodes[8 * ia + 3]);
}

int ref_features(const ref_track *T, const ref_params *p, const ref_race *R, double *X /*[n][50]*/)
{
    const int n = R->n_agents;
    agent_state *A = (agent_state *)malloc(sizeof(agent_state) * n);
    double *psi_r = (double *)malloc(sizeof(double) * n);
    double *vref = (double *)malloc(sizeof(double) * n);
    double *half = (double *)malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) {
        agent_setup(T, p, R, i, &A[i]);
        long h = A[i].seg;
        double x, y, ps, v;
        interp_at_s(T, A[i].s, &h, &x, &y, &ps, &v);
        psi_r[i] = ps;
        vref[i] = v;
        double o6[6];
        ref_project_walk(T, p->max_moves, R->x + 6 * i, A[i].seg, o6);
        half[i] = 0.5 * (o6[3] + o6[4]);
    }
    for (int i = 0; i < n; ++i) {
        double *f = X + (size_t)i * FEAT_DIM;
        const double *xi = R->x + 6 * i;
        for (int c = 0; c < FEAT_DIM; ++c) f[c] = 0.0;
        f[0] = A[i].d / half[i];
        f[1] = wrap_pi(xi[2] - psi_r[i]);
        f[2] = xi[3] / 30.0;
        f[3] = xi[4] / 5.0;
        f[4] = xi[5];
        f[5] = (xi[3] - vref[i]) / 10.0;
        /* nearest opponents: smallest |s_j - s_i|, ties by index */
        int used[REF_MAX_OPP + 1] = {0};
        for (int m = 0; m < FEAT_OPP; ++m) {
            int best = -1;
            double bd = INFINITY;
            for (int j = 0; j < n; ++j) {
                if (j == i || used[j]) continue;
                double dd = fabs(A[j].s - A[i].s);
                if (dd < bd) { bd = dd; best = j; }
            }
            if (best < 0) break;
            used[best] = 1;
            const double *xj = R->x + 6 * best;
            double *g = f + 6 + 6 * m;
            g[0] = (A[best].s - A[i].s) / 20.0;
            g[1] = (A[best].d - A[i].d) / half[i];
            g[2] = wrap_pi(xj[2] - xi[2]);
            g[3] = (xj[3] - xi[3]) / 10.0;
            g[4] = xj[4] / 5.0;
            g[5] = 1.0;
        }
        long h = A[i].seg;
        for (int m = 1; m <= FEAT_CURV; ++m)
            f[6 + 6 * FEAT_OPP + m - 1] = 20.0 * kappa_at(T, A[i].s + FEAT_CURV_DS * m, &h);
    }
    free(A); free(psi_r); free(vref); free(half);
    return 0;
}

/* MLP d_in -> H -> H -> d_out with tanh-form GELU; W[l] stored [fan_in][fan_out].
 * Output per horizon step tau (4 values): mu_a = A_SCALE o0, mu_d = D_SCALE o1,
 * log sigma_a = log sigma_a,plain + clamp(o2), log sigma_d = log sigma_d,plain + clamp(o3),
 * clamp to [LS_MIN, LS_MAX]. */
#define MLP_A_SCALE 4.0
#define MLP_D_SCALE 0.2
#define MLP_LS_MIN (-4.0)
#define MLP_LS_MAX 1.0

/* bf16 != 0: every matrix-product operand (inputs, weights, hidden activations, and in
 * the backward pass the output gradient and both hidden-layer gradients) is rounded to
 * bfloat16 first, as the learned-proposal workload specifies (BF16 operands, FP32
 * accumulation; a product of two bfloat16 values is exact in float32, so only the
 * accumulation order and its rounding remain between this and an FP32 accumulator). */
typedef struct {
    int d_in, d_h, d_out, bf16;
    const double *W1, *b1, *W2, *b2, *W3, *b3;
} ref_mlp;

/* Round to float32 (nearest), then to bfloat16 (nearest, ties to even). */
static double to_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) != 0x7f800000u) u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}
static double q_op(const ref_mlp *M, double x) { return M->bf16 ? to_bf16(x) : x; }

static double gelu(double x)
{
    const double c = 0.7978845608028654; /* sqrt(2/pi) */
    return 0.5 * x * (1.0 + tanh(c * (x + 0.044715 * x * x * x)));
}
static double gelu_grad(double x)
{
    const double c = 0.7978845608028654;
    double u = c * (x + 0.044715 * x * x * x);
    double t = tanh(u);
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * c * (1.0 + 3.0 * 0.044715 * x * x);
}

/* Forward of B rows; optional intermediates: pre1/h1/pre2/h2 [B][d_h].  h1_in / h2_in
 * (optional, [B][d_h]): hidden activations to continue from in place of the network's
 * own roundings of GELU(pre1) / GELU(pre2) (a lockstep comparison adopts another
 * implementation's rounding decisions after checking them); pre1 / pre2 are computed
 * from the layer inputs either way. */
void ref_mlp_forward_ex(const ref_mlp *M, int B, const double *X, const double *h1_in, const double *h2_in,
                        double *out, double *pre1, double *h1, double *pre2, double *h2)
{
    const int di = M->d_in, dh = M->d_h, dn = M->d_out;
    double *a1 = (double *)malloc(sizeof(double) * dh), *z1 = (double *)malloc(sizeof(double) * dh);
    double *a2 = (double *)malloc(sizeof(double) * dh), *z2 = (double *)malloc(sizeof(double) * dh);
    for (int b = 0; b < B; ++b) {
        const double *x = X + (size_t)b * di;
        for (int j = 0; j < dh; ++j) {
            double acc = M->b1[j];
            for (int k = 0; k < di; ++k) acc += q_op(M, x[k]) * q_op(M, M->W1[(size_t)k * dh + j]);
            z1[j] = acc;
            a1[j] = h1_in ? h1_in[(size_t)b * dh + j] : q_op(M, gelu(acc));
        }
        for (int j = 0; j < dh; ++j) {
            double acc = M->b2[j];
            for (int k = 0; k < dh; ++k) acc += a1[k] * q_op(M, M->W2[(size_t)k * dh + j]);
            z2[j] = acc;
            a2[j] = h2_in ? h2_in[(size_t)b * dh + j] : q_op(M, gelu(acc));
        }
        for (int j = 0; j < dn; ++j) {
            double acc = M->b3[j];
            for (int k = 0; k < dh; ++k) acc += a2[k] * q_op(M, M->W3[(size_t)k * dn + j]);
            out[(size_t)b * dn + j] = acc;
        }
        if (pre1) memcpy(pre1 + (size_t)b * dh, z1, sizeof(double) * dh);
        if (h1) memcpy(h1 + (size_t)b * dh, a1, sizeof(double) * dh);
        if (pre2) memcpy(pre2 + (size_t)b * dh, z2, sizeof(double) * dh);
        if (h2) memcpy(h2 + (size_t)b * dh, a2, sizeof(double) * dh);
    }
    free(a1); free(z1); free(a2); free(z2);
}

void ref_mlp_forward(const ref_mlp *M, int B, const double *X, double *out, double *pre1, double *h1, double *pre2,
                     double *h2)
{
    ref_mlp_forward_ex(M, B, X, NULL, NULL, out, pre1, h1, pre2, h2);
}

/* Proposal of one row of network outputs (N steps): (mu_a, mu_d, sigma_a, sigma_d).
 * With ubar [N][2] (residual form) the means are offsets from the nominal sequence. */
void ref_mlp_proposal(const double *o, int N, double sig_a, double sig_d, const double *ubar, double *prop)
{
    for (int t = 0; t < N; ++t) {
        double o2 = o[4 * t + 2], o3 = o[4 * t + 3];
        o2 = o2 < MLP_LS_MIN ? MLP_LS_MIN : (o2 > MLP_LS_MAX ? MLP_LS_MAX : o2);
        o3 = o3 < MLP_LS_MIN ? MLP_LS_MIN : (o3 > MLP_LS_MAX ? MLP_LS_MAX : o3);
        prop[4 * t + 0] = (ubar ? ubar[2 * t] : 0.0) + MLP_A_SCALE * o[4 * t + 0];
        prop[4 * t + 1] = (ubar ? ubar[2 * t + 1] : 0.0) + MLP_D_SCALE * o[4 * t + 1];
        prop[4 * t + 2] = sig_a * exp(o2);
        prop[4 * t + 3] = sig_d * exp(o3);
    }
}

/* Mean over the batch of the Gaussian negative log-likelihood of the targets U [B][N][2]
 * (constant 0.5 log 2 pi dropped), and its gradient d_out [B][d_out] w.r.t. the outputs. */
double ref_mlp_nll(const double *out, int B, int N, int d_out, double sig_a, double sig_d, const double *U,
                   double *d_out_grad)
{
    double L = 0.0;
    const double ls_plain[2] = {log(sig_a), log(sig_d)};
    const double scale[2] = {MLP_A_SCALE, MLP_D_SCALE};
    for (int b = 0; b < B; ++b) {
        const double *o = out + (size_t)b * d_out;
        double *g = d_out_grad ? d_out_grad + (size_t)b * d_out : NULL;
        if (g) for (int j = 0; j < d_out; ++j) g[j] = 0.0;
        for (int t = 0; t < N; ++t) {
            for (int c = 0; c < 2; ++c) {
                double mu = scale[c] * o[4 * t + c];
                double raw = o[4 * t + 2 + c];
                double cl = raw < MLP_LS_MIN ? MLP_LS_MIN : (raw > MLP_LS_MAX ? MLP_LS_MAX : raw);
                double ls = ls_plain[c] + cl;
                double sg2 = exp(2.0 * ls);
                double r = U[((size_t)b * N + t) * 2 + c] - mu;
                L += 0.5 * r * r / sg2 + ls;
                if (g) {
                    g[4 * t + c] = -scale[c] * r / sg2 / B;
                    g[4 * t + 2 + c] = (raw > MLP_LS_MIN && raw < MLP_LS_MAX) ? (1.0 - r * r / sg2) / B : 0.0;
                }
            }
        }
    }
    return L / B;
}

/* Back-propagation of d_out through the MLP: gradients of W1..b3 (same layouts).
 * Optional lockstep inputs ([B][d_h]): h1_in / h2_in as in ref_mlp_forward_ex, and d2_in /
 * d1_in in place of the network's own roundings of the pre-activation gradients of layers
 * 2 and 1; d2_pre / d1_pre (optional outputs, [B][d_h]) receive those gradients before
 * rounding. */
void ref_mlp_backward_ex(const ref_mlp *M, int B, const double *X, const double *h1_in, const double *h2_in,
                         const double *d_out, const double *d2_in, const double *d1_in, double *d2_pre,
                         double *d1_pre, double *gW1, double *gb1, double *gW2, double *gb2, double *gW3,
                         double *gb3)
{
    const int di = M->d_in, dh = M->d_h, dn = M->d_out;
    double *pre1 = (double *)malloc(sizeof(double) * (size_t)B * dh), *h1 = (double *)malloc(sizeof(double) * (size_t)B * dh);
    double *pre2 = (double *)malloc(sizeof(double) * (size_t)B * dh), *h2 = (double *)malloc(sizeof(double) * (size_t)B * dh);
    double *out = (double *)malloc(sizeof(double) * (size_t)B * dn);
    double *d2 = (double *)malloc(sizeof(double) * dh), *d1 = (double *)malloc(sizeof(double) * dh);
    ref_mlp_forward_ex(M, B, X, h1_in, h2_in, out, pre1, h1, pre2, h2);
    memset(gW1, 0, sizeof(double) * di * dh); memset(gb1, 0, sizeof(double) * dh);
    memset(gW2, 0, sizeof(double) * dh * dh); memset(gb2, 0, sizeof(double) * dh);
    memset(gW3, 0, sizeof(double) * dh * dn); memset(gb3, 0, sizeof(double) * dn);
    double *g = (double *)malloc(sizeof(double) * dn);
    for (int b = 0; b < B; ++b) {
        for (int j = 0; j < dn; ++j) g[j] = q_op(M, d_out[(size_t)b * dn + j]);
        const double *a2 = h2 + (size_t)b * dh, *a1 = h1 + (size_t)b * dh, *x = X + (size_t)b * di;
        for (int j = 0; j < dn; ++j) {
            gb3[j] += g[j];
            for (int k = 0; k < dh; ++k) gW3[(size_t)k * dn + j] += a2[k] * g[j];
        }
        for (int k = 0; k < dh; ++k) {
            double acc = 0.0;
            for (int j = 0; j < dn; ++j) acc += q_op(M, M->W3[(size_t)k * dn + j]) * g[j];
            const double v = acc * gelu_grad(pre2[(size_t)b * dh + k]);
            if (d2_pre) d2_pre[(size_t)b * dh + k] = v;
            d2[k] = d2_in ? d2_in[(size_t)b * dh + k] : q_op(M, v);
        }
        for (int j = 0; j < dh; ++j) {
            gb2[j] += d2[j];
            for (int k = 0; k < dh; ++k) gW2[(size_t)k * dh + j] += a1[k] * d2[j];
        }
        for (int k = 0; k < dh; ++k) {
            double acc = 0.0;
            for (int j = 0; j < dh; ++j) acc += q_op(M, M->W2[(size_t)k * dh + j]) * d2[j];
            const double v = acc * gelu_grad(pre1[(size_t)b * dh + k]);
            if (d1_pre) d1_pre[(size_t)b * dh + k] = v;
            d1[k] = d1_in ? d1_in[(size_t)b * dh + k] : q_op(M, v);
        }
        for (int j = 0; j < dh; ++j) {
            gb1[j] += d1[j];
            for (int k = 0; k < di; ++k) gW1[(size_t)k * dh + j] += q_op(M, x[k]) * d1[j];
        }
    }
    free(g);
    free(pre1); free(h1); free(pre2); free(h2); free(out); free(d2); free(d1);
}

void ref_mlp_backward(const ref_mlp *M, int B, const double *X, const double *d_out, double *gW1, double *gb1,
                      double *gW2, double *gb2, double *gW3, double *gb3)
{
    ref_mlp_backward_ex(M, B, X, NULL, NULL, d_out, NULL, NULL, NULL, NULL, gW1, gb1, gW2, gb2, gW3, gb3);
}

int ref_abi_version(void) { return 2; }
