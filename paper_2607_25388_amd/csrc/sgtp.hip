// sgtp.hip -- MI355X (gfx950) implementation of the SGTP planning step.
//
// Hot path: one Jacobi sweep of sampled best responses (Alg. 1, Sec. III).  One
// lane owns one sample for the whole horizon: its vehicle state, cost
// accumulators, boundary clearance and per-opponent clearances live in VGPRs;
// the nominal sequence, reference states, the opponents' footprint trajectories
// and a window of the raceline are staged in LDS per workgroup; perturbations
// come from an in-register Philox4x32-10 stream; the argmin over samples is a
// 64-bit key reduced with DPP row operations and readlane, then one global
// atomic per wave.  No sample trajectory is written: the selected sample is
// re-rolled by one lane (same device code, same inputs, same bits).
//
// Kernels of one planning step:
//   k_setup   one workgroup per vehicle: global Frenet projection, unwrapped
//             progress, local frame, raceline window, reference states, and the
//             noise-free rollout of the nominal sequence (initial predictions).
//   k_sweep   every sample of every participating vehicle -> selection keys; the
//             last workgroup of each vehicle re-rolls k* (new nominal,
//             prediction, trajectory, choice; first control and warm start in
//             the vehicle's final phase).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <array>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "sgtp.h"

namespace {

constexpr int BLOCK = 256;
constexpr int MAX_TRACKS = 64;
constexpr int WIN_BACK = 48;    // raceline nodes kept behind the current segment
constexpr int WIN_MAX = 1536;   // window nodes per vehicle (workspace bound)
constexpr int PRED_STRIDE = 8;  // x, y, cos psi, sin psi, s_rel, d, -, - in the owner's frame
constexpr int NODE_STRIDE = 10; // device node row: x, y, psi, nx, ny, wL, wR, vref, s, kappa
constexpr unsigned long long KEY_NONE = ~0ull;
constexpr long long LPS2_MAX_SAMPLES = 32768;  // pair variant up to 1024 waves
// Split variant (launches of about one wave per SIMD or fewer): each sample runs on two
// waves, dynamics on one and projection and scoring on the other, its states passing
// through an LDS ring of SPLIT_RING steps.
constexpr long long SPLIT_MAX_SAMPLES = 65536;  // up to 2048 waves
constexpr int SPLIT_RING = 4;
constexpr int SPLIT_AHEAD = 2;  // controls published ahead of the state being scored (2 and a
                                // ring of 4 measured faster than 1, 3, 4 or 6 and a ring of 8)
constexpr int SPLIT_FIN = 8;    // floats per sample handed from the dynamics to the scoring lane
// The split variant's roles by wave: even waves integrate the dynamics, odd waves score,
// wave 2j + 1 partnering wave 2j.  A workgroup's four waves occupy the CU's four SIMDs in
// a fixed cyclic order, and the next workgroup resident on the same CU starts one SIMD
// further along it (measured); with the roles in halves, two resident workgroups put two
// dynamics chains on one SIMD, with alternating roles every SIMD holds one chain and one
// scoring wave.  Virtual thread index: role x 128 + wave pair x 64 + lane.
__device__ __forceinline__ int split_vt(int t) { return ((t >> 6) & 1) * (BLOCK / 2) + ((t >> 7) << 6) + (t & 63); }
constexpr int NQ = 8;           // tile queues of the persistent sweep (one per XCD under round-robin dispatch)
// Re-roll chunks: each lane keeps its state after every ceil(N / chunks) steps, so the
// selected sample is re-rolled in that many pieces at once.  Latency variants (about
// one wave per SIMD, registers to spare) keep 10, throughput variants 4.
constexpr int NCP_MAX = 10;
template <int NPF>
constexpr int ncp_of() { return NPF > 0 ? 10 : 4; }
constexpr int CP_FLOATS = 72;   // export slot per group: up to 9 checkpoints x (6 states + segment), cost, violation
constexpr int CP_COST = 70, CP_VIOL = 71;

enum Mode { SWEEP = 0, WINNER = 1, NOMINAL = 2 };

// ------------------------------------------------------------------------------
// Kernel-side parameters (float32 with derived constants folded in)
// ------------------------------------------------------------------------------
struct KParams {
    // read in the sample loop (kept together: their scalar loads and registers stay compact)
    float dt, half_dt, dt6;
    // dynamic single-track: the axles' peak forces mu F_z enter the rates only through
    // kf_m = mu F_zf / m, kf_Iz = mu F_zf l_f / I_z, kr_m = mu F_zr / m, kr_Iz = mu F_zr l_r / I_z
    float lf, lr, kf_m, kf_Iz, kr_m, kr_Iz, B, C, v_eps, C_rev;
    float lr_over_L, inv_lr;                                 // kinematic bicycle
    float a_min, a_max, d_min, d_max, sigma_a, sigma_d;
    float Q0, Q1, Q2, Q3, R0, R1, S0, S1;
    float cap2, skip2;
    float off[4];
    int max_moves;
    // read once per sample or outside the loop
    int model, n_disc, update;  // update: 0 selection, 1 path-integral
    float w_game, w_contest, w_long, w_block, w_safety, s_contest, s_role, eps_alpha;
    float g_safe, m_bd, d_col;
    float inv_lambda, w_viol;                                // path-integral update
    float pred_sig_lon, pred_sig_lat;                        // opponent-prediction perturbation
    int spin_limit;  // polls of a bounded LDS wait (split variant, winner re-roll) before it gives up
};

struct TrackDev {
    const double *nodes;  // [n][NODE_STRIDE]
    int n, closed;
    double length, psi_lap, ds_min, inner_factor, vmax;
};

struct RaceDev {
    int n_agents, ego, N, n_tail, track, slot0, K, pad0;
    unsigned long long seed;
    unsigned int plan_step, pad1;
    double *x;
    double *s_abs;
    const float *v_scale;
    float *u_nom;
    double *traj;
    const float4 *prop;  // [n][N] proposal (mu_a, mu_d, sigma_a, sigma_d), or NULL
    int K_prop, pad2;
};

struct ItemDev {  // one best response (race, vehicle) of a launch
    int race, agent, slot, tile0;
    int group0, pad0;  // first 64-sample group of the vehicle in the checkpoint slots
};

struct AgentRec {  // per vehicle, written by k_setup
    double ox, oy, psi0, c0, s0, s_abs, d0;
    double half_w, psi_ref, v_ref;  // at the foot of the current state (features)
    long long seg_abs, win0;
    int win_n, seg_loc;
    float vx, vy, om, lam;
};

struct LdsLayout {  // byte offsets of the staged tables, identical for every block of a launch
    int ubar, xref, oppT, oppc, opp, nodes, prop;
    int rr_u, rr_st, rr_f, rr_t;  // re-roll scratch (rr_t: setup's reference recursion)
    int rr_sync;                  // re-roll: states written per piece (NCP_MAX ints)
    int sp_ring, sp_uring, sp_sync, sp_fin;  // split variant: state and control rings, counters, final state
    int total;
    int n_opp_max, w_max, N_max;
};

struct LaunchArgs {
    KParams P;
    LdsLayout L;
    const TrackDev *tracks;
    const RaceDev *races;
    const ItemDev *items;
    int n_items, n_tiles, spl, phase;
    int lps;               // lanes per sample (2: the pair variant of small launches)
    int split;             // 1: the split variant (two waves per sample)
    AgentRec *agents;
    const float4 *win;     // [slot][WIN_MAX][2]
    const float4 *xref;    // [slot][N_max]
    const float *pred_in;  // [slot][N_max+1][PRED_STRIDE]
    float *pred_out;
    unsigned long long *keys;
    int *nfeas;
    int *counters;         // finished workgroups per vehicle
    // outputs of the re-roll of the selected sample
    sgtp_choice *choice;   // indexed by slot - choice_base, or NULL
    int choice_base;
    int adopt;             // write u_nom / traj
    int final_mode;        // 0 none, 1 every vehicle but the ego, 2 every vehicle: first control + warm start
    float2 *u_apply;       // [slot] first controls, or NULL
    // persistent sweep: per-queue tile ranges and fetch counters
    int chunk;             // tiles taken per fetch
    int q_begin[NQ], q_len[NQ];
    int *qctr;             // [NQ] fetch counters of this sweep
    int *qreset;           // counters zeroed by k_setup (all sweeps of a planning step), or NULL
    int n_qreset;
    // debug outputs of k_sweep (indexed by sample), or NULL
    float *dbg_cost;
    unsigned char *dbg_flags;
    float *dbg_viol;
    double *dbg_xfinal;
    float *dbg_noise;
    float *cp_slots;       // [group][CP_FLOATS] checkpoints of each wave's best sample
    float *pi_part;        // [tile][2 N_max + 2] path-integral partial sums, or NULL
    int *status;           // context status word: bits SGTP_STATUS_* set when a bounded wait gave up
};

// ------------------------------------------------------------------------------
// Noise: Philox4x32-10 and the float32 Box-Muller transform
// ------------------------------------------------------------------------------
// a ^ b ^ k with k wave-uniform (a scalar register), one v_bitop3 (truth table 0x96); the
// compiler keeps two separate xors when one operand is scalar
__device__ __forceinline__ uint32_t xor3_uniform(uint32_t a, uint32_t b, uint32_t k) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

// Philox4x32-10 (Salmon et al., SC'11).  BITOP3: each round's two three-way xors as one
// instruction each (the keys are wave-uniform: every caller passes the race's seed); the
// throughput kernels take it, the latency variants measured faster with plain xors.  Same
// values either way.
template <bool BITOP3 = false>
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
            // the round keys are bumped in place at every call (scalar adds): kept for the
            // whole sample loop, twenty of them were spilled and reloaded with v_readlane
            asm volatile("" : "+s"(k0), "+s"(k1));
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        if constexpr (BITOP3)
            c = make_uint4(xor3_uniform((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1,
                           xor3_uniform((uint32_t)(p0 >> 32), c.w, k1), (uint32_t)p0);
        else
            c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
                           (uint32_t)p0);
    }
    return c;
}

// IEEE division and square root for the operand ranges of the transform below (normal,
// finite, no zero divisor, square roots of positive normal values only): the hardware
// estimate refined by the same fused steps as the general correctly rounded sequences,
// without their scaling and special-value steps, which never act in these ranges -- the
// results are the IEEE ones bit for bit.
__device__ __forceinline__ float div_rn_normal(float n, float d) {
    float r = __builtin_amdgcn_rcpf(d);
    r = __builtin_fmaf(__builtin_fmaf(-d, r, 1.0f), r, r);
    float q = n * r;
    q = __builtin_fmaf(__builtin_fmaf(-d, q, n), r, q);
    return __builtin_fmaf(__builtin_fmaf(-d, q, n), r, q);
}
__device__ __forceinline__ float sqrt_rn_normal(float x) {
    const float s = __builtin_amdgcn_sqrtf(x);  // within 1 ulp
    const float s_dn = __uint_as_float(__float_as_uint(s) - 1u), s_up = __uint_as_float(__float_as_uint(s) + 1u);
    float r = __builtin_fmaf(-s_dn, s, x) <= 0.0f ? s_dn : s;
    return __builtin_fmaf(-s_up, s, x) > 0.0f ? s_up : r;
}

// Gaussian pair from two 32-bit words.  The float32 operation sequence is fixed
// (IEEE round-to-nearest add, mul, fma, div, sqrt; no contraction), so the
// perturbations are reproducible bit for bit on any IEEE-conforming device.
__device__ __forceinline__ float2 gauss_pair(uint32_t r_even, uint32_t r_odd) {
#pragma clang fp contract(off)
    const float L3 = 0x1.555556p-1f, L5 = 0x1.99999ap-2f, L7 = 0x1.24924ap-2f;
    const float L9 = 0x1.c71c72p-3f, L11 = 0x1.745d18p-3f, L13 = 0x1.3b13b2p-3f;
    const float LN2_HI = 0x1.62e4p-1f, LN2_LO = 0x1.7f7d1cp-20f;
    const float S1 = 0x1.921fb6p+2f, S3 = -0x1.4abbcep+5f, S5 = 0x1.466bc6p+6f;
    const float S7 = -0x1.32d2ccp+6f, S9 = 0x1.507834p+5f;
    const float C2 = -0x1.3bd3ccp+4f, C4 = 0x1.03c1f0p+6f, C6 = -0x1.55d3c8p+6f;
    const float C8 = 0x1.e1f506p+5f, C10 = -0x1.a6d1f2p+4f;
    // radius sqrt(-2 ln u1), u1 = (2*(r_even >> 9) + 1) 2^-24, ln by exponent split + atanh series
    const float u1 = (float)(2u * (r_even >> 9) + 1u) * 0x1p-24f;
    // u1 = m 2^e with m in [sqrt(1/2), sqrt 2]: m > SQRT2 (the float just below sqrt 2) is
    // halved.  In integer form: adding 2^23 - 0x3504f4 to the bits carries into the
    // exponent exactly when the mantissa field exceeds that of SQRT2, and the mantissa of
    // m is then the low 23 bits plus the bits of the float above sqrt(1/2).
    const uint32_t b = __float_as_uint(u1) + 0x4afb0cu;
    const int e = (int)(b >> 23) - 127;
    const float m = __uint_as_float((b & 0x7fffffu) + 0x3f3504f4u);
    const float f = m - 1.0f;
    const float z = div_rn_normal(f, m + 1.0f);  // f in [-0.293, 0.415], m + 1 in [1.707, 2.415]
    const float w = z * z;
    float p = __builtin_fmaf(L13, w, L11);
    p = __builtin_fmaf(p, w, L9);
    p = __builtin_fmaf(p, w, L7);
    p = __builtin_fmaf(p, w, L5);
    p = __builtin_fmaf(p, w, L3);
    p = p * w;
    const float lnm = __builtin_fmaf(z, p, z + z);
    const float ef = (float)e;
    const float lnu = __builtin_fmaf(ef, LN2_HI, __builtin_fmaf(ef, LN2_LO, lnm));
    const float rho = sqrt_rn_normal(-2.0f * lnu);  // -2 ln u1 in [1.1e-7, 33.3]
    // angle 2 pi u2, u2 = (r_odd >> 8) 2^-24: exact quarter-turn split, Taylor polynomials
    const uint32_t j = r_odd >> 8;
    const uint32_t q = (j + (1u << 21)) >> 22;
    const int32_t ri = (int32_t)j - (int32_t)(q << 22);
    const float r = (float)ri * 0x1p-24f;
    const float r2 = r * r;
    float ps = __builtin_fmaf(S9, r2, S7);
    ps = __builtin_fmaf(ps, r2, S5);
    ps = __builtin_fmaf(ps, r2, S3);
    ps = __builtin_fmaf(ps, r2, S1);
    const float sn = ps * r;
    float pc = __builtin_fmaf(C10, r2, C8);
    pc = __builtin_fmaf(pc, r2, C6);
    pc = __builtin_fmaf(pc, r2, C4);
    pc = __builtin_fmaf(pc, r2, C2);
    const float cs = __builtin_fmaf(pc, r2, 1.0f);
    // quarter turns: (sin, cos) = (sn, cs), (cs, -sn), (-sn, -cs), (-cs, sn) for qq = 0..3;
    // the signs as sign-bit flips (exact), no branches
    const uint32_t qq = q & 3u;
    const bool odd = (qq & 1u) != 0u;
    const float sa = odd ? cs : sn, ca = odd ? sn : cs;
    const float sin_t = __uint_as_float(__float_as_uint(sa) ^ ((qq & 2u) << 30));
    const float cos_t = __uint_as_float(__float_as_uint(ca) ^ (((qq + 1u) & 2u) << 30));
    return make_float2(rho * cos_t, rho * sin_t);
}

// ------------------------------------------------------------------------------
// Elementary functions for the vehicle model
// ------------------------------------------------------------------------------
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// atan: odd polynomial of degree 13 on [0, 1], reflected via pi/2 - atan(1/x).  Its
// coefficients are a minimax (equal-ripple) fit of the absolute error on [0, 1], rounded to
// float32: 2.55e-7 in exact arithmetic, 3.1e-7 evaluated in float32 (4e-7 with the reflection).
// (A 6-term fit with 1.8e-6 error moved chaotic sliding samples past the 1e-3 state tolerance.)
__device__ __forceinline__ float atan_poly(float t, float t2) {
    float p = 0x1.be6b36p-8f;
    p = __builtin_fmaf(p, t2, -0x1.134946p-5f);
    p = __builtin_fmaf(p, t2, 0x1.46238ap-4f);
    p = __builtin_fmaf(p, t2, -0x1.0f04d8p-3f);
    p = __builtin_fmaf(p, t2, 0x1.95aa02p-3f);
    p = __builtin_fmaf(p, t2, -0x1.552b7cp-2f);
    p = __builtin_fmaf(p, t2, 0x1.ffff7ep-1f);
    return p * t;
}
// UNIFORM: when no lane of the wave has |x| > 1, the odd polynomial of x itself (no range
// reduction, no sign handling: p(x^2) x equals copysign(p(|x|^2) |x|, x) bit for bit), taken
// as a real branch -- saves issue slots where several waves share a SIMD; a wave alone on its
// SIMD takes the branch-free form instead.  Both forms give the same value.
template <bool UNIFORM = false>
__device__ __forceinline__ float fast_atan(float x) {
    const float ax = fabsf(x);
    const bool inv = ax > 1.0f;
    if (UNIFORM && __builtin_expect(__builtin_amdgcn_ballot_w64(inv) == 0, 1)) return atan_poly(x, x * x);
    const float t = inv ? fast_rcp(ax) : ax;
    float r = atan_poly(t, t * t);
    r = inv ? (1.57079637f - r) : r;
    return copysignf(r, x);
}

// atan of a slip angle's argument (v_y + l om) / v_x, which stays within 1/4 in all but a
// few samples: there an odd quintic whose coefficients are a minimax (equal-ripple) fit of
// the absolute error on [0, 1/4] rounded to float32 (1.2e-7 exact, 1.4e-7 evaluated in
// float32), beyond it the general atan.  The choice is per lane, so a sample's value never
// depends on the other lanes of its wave: a branch that diverges only in waves holding both
// cases, or (UNIFORM) a wave-uniform test for the common case of a wave with no argument
// beyond 1/4 and both forms selected per lane otherwise.
__device__ __forceinline__ float atan_quintic(float x) {
    const float x2 = x * x;
    float p = __builtin_fmaf(0x1.7b89a0p-3f, x2, -0x1.54dfd2p-2f);
    p = __builtin_fmaf(p, x2, 0x1.ffff8cp-1f);
    return p * x;
}
template <bool UNIFORM = false>
__device__ __forceinline__ float atan_slip(float x) {
    const bool small = fabsf(x) <= 0.25f;
    if (UNIFORM) {
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(!small) == 0, 1)) return atan_quintic(x);
        const float q = atan_quintic(x), g = fast_atan<true>(x);
        return small ? q : g;
    }
    if (__builtin_expect(small, 1)) return atan_quintic(x);
    return fast_atan<UNIFORM>(x);
}

// sin/cos through the transcendental unit (argument in revolutions)
__device__ __forceinline__ float fast_sin(float x) { return __builtin_amdgcn_sinf(x * 0.159154943f); }
__device__ __forceinline__ float fast_cos(float x) { return __builtin_amdgcn_cosf(x * 0.159154943f); }

// Elementary functions of the vehicle model.  Angles handed to sin_rev/cos_rev are
// pre-scaled by to_rev (revolutions for the float32 transcendental unit, radians in float64).
struct MathF32 {
    using T = float;
    static __device__ __forceinline__ T atan_(T x) { return fast_atan<false>(x); }
    static __device__ __forceinline__ T atan_slip_(T x) { return atan_slip<false>(x); }
    static __device__ __forceinline__ T sin_(T x) { return fast_sin(x); }
    static __device__ __forceinline__ T cos_(T x) { return fast_cos(x); }
    static __device__ __forceinline__ T rcp_(T x) { return fast_rcp(x); }
    static __device__ __forceinline__ T to_rev(T x) { return x * 0.159154943f; }
    static __device__ __forceinline__ T sin_rev(T x) { return __builtin_amdgcn_sinf(x); }
    static __device__ __forceinline__ T cos_rev(T x) { return __builtin_amdgcn_cosf(x); }
    static __device__ __forceinline__ T fma_(T a, T b, T c) { return __builtin_fmaf(a, b, c); }
    // max(x, 0) as one median (0 for a NaN, like x > 0 ? x : 0; +inf becomes the largest
    // finite value, which only a state that is already non-finite reaches)
    static __device__ __forceinline__ T pos_(T x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 3.40282347e38f); }
    // max(x, lo) of a value pos_ returned (never NaN)
    static __device__ __forceinline__ T floor_(T x, T lo) { return fmaxf(x, lo); }
};

// MathF32 with the wave-uniform atan range reduction (throughput kernels)
struct MathF32U : MathF32 {
    static __device__ __forceinline__ T atan_(T x) { return fast_atan<true>(x); }
    static __device__ __forceinline__ T atan_slip_(T x) { return atan_slip<true>(x); }
};

struct MathF64 {
    using T = double;
    static __device__ __forceinline__ T atan_(T x) { return ::atan(x); }
    static __device__ __forceinline__ T atan_slip_(T x) { return ::atan(x); }
    static __device__ __forceinline__ T sin_(T x) { return ::sin(x); }
    static __device__ __forceinline__ T cos_(T x) { return ::cos(x); }
    static __device__ __forceinline__ T rcp_(T x) { return 1.0 / x; }
    static __device__ __forceinline__ T to_rev(T x) { return x; }
    static __device__ __forceinline__ T sin_rev(T x) { return ::sin(x); }
    static __device__ __forceinline__ T cos_rev(T x) { return ::cos(x); }
    static __device__ __forceinline__ T fma_(T a, T b, T c) { return ::fma(a, b, c); }
    static __device__ __forceinline__ T pos_(T x) { return x > 0.0 ? x : 0.0; }
    static __device__ __forceinline__ T floor_(T x, T lo) { return x > lo ? x : lo; }
};

template <typename T>
struct VehConst {
    T lf, lr, kf_m, kf_Iz, kr_m, kr_Iz, B, C, v_eps, lr_over_L, inv_lr;
    T Cs;  // C scaled to the angle unit of M::sin_rev
};

// Per control interval: functions of the held control (a, delta).
template <typename T>
struct StepConst {
    T a, delta;
    T kf3, kf4, kf5;  // dynamic: kf_m sin delta, kf_m cos delta, kf_Iz cos delta
    T kc, ks, kw;     // kinematic: cos beta, sin beta, sin(beta)/l_r
};

template <int MODEL, class M>
__device__ __forceinline__ StepConst<typename M::T> step_const(const VehConst<typename M::T> &V, typename M::T a,
                                                                 typename M::T delta) {
    using T = typename M::T;
    StepConst<T> c;
    c.a = a;
    c.delta = delta;
    if (MODEL == 0) {
        const T sd = M::sin_(delta), cd = M::cos_(delta);
        c.kf3 = V.kf_m * sd;
        c.kf4 = V.kf_m * cd;
        c.kf5 = V.kf_Iz * cd;
        c.kc = c.ks = c.kw = T(0);
    } else {
        const T beta = M::atan_(V.lr_over_L * (M::sin_(delta) * M::rcp_(M::cos_(delta))));
        c.kc = M::cos_(beta);
        c.ks = M::sin_(beta);
        c.kw = c.ks * V.inv_lr;
        c.kf3 = c.kf4 = c.kf5 = T(0);
    }
    return c;
}

// Lateral force of one axle over its peak mu F_z: slip angle alpha = delta_axle -
// atan((v_y + l om) / v_hat) (l = l_f for the front axle, -l_r for the rear one, whose
// steering angle is 0) and F_y / (mu F_z) = sin(C atan(B alpha)).  Both axles go through
// this one expression, so the two-lane evaluation below gives the same bits as the
// one-lane one.
template <class M>
__device__ __forceinline__ typename M::T tyre_force(const VehConst<typename M::T> &V, typename M::T l,
                                                     typename M::T delta_axle, typename M::T vy, typename M::T om,
                                                     typename M::T inv_vh) {
    using T = typename M::T;
    const T alpha = delta_axle - M::atan_slip_((vy + l * om) * inv_vh);
    return M::sin_rev(V.Cs * M::atan_(V.B * alpha));
}

// Vehicle model f (Sec. II).  MODEL 0: dynamic single-track with
// F_y = mu F_z sin(C atan(B alpha)); MODEL 1: kinematic bicycle at the CoG.
// Position rates use max(v_x, 0), so no stage of RK4 moves the car backwards.
// Sf, Sr: the axles' forces over their peaks (tyre_force); v_x' = a - F_yf sin(delta) / m
// + v_y om, v_y' = (F_yr + F_yf cos(delta)) / m - v_x om, om' = (l_f F_yf cos(delta) -
// l_r F_yr) / I_z with the force scales folded into kf3..kf5, kr_m and kr_Iz.
template <class M>
__device__ __forceinline__ void deriv_rates(const VehConst<typename M::T> &V, const StepConst<typename M::T> &c,
                                            typename M::T vx, typename M::T vy, typename M::T om, typename M::T cp,
                                            typename M::T sp, typename M::T Sf, typename M::T Sr,
                                            typename M::T d[6]) {
    d[0] = vx * cp - vy * sp;
    d[1] = vx * sp + vy * cp;
    d[2] = om;
    d[3] = M::fma_(vy, om, M::fma_(-Sf, c.kf3, c.a));
    d[4] = M::fma_(Sf, c.kf4, M::fma_(Sr, V.kr_m, -(vx * om)));
    d[5] = M::fma_(Sf, c.kf5, -(Sr * V.kr_Iz));
}

// f at a state whose heading cosine and sine (cp, sp) are given
template <int MODEL, class M>
__device__ __forceinline__ void deriv_cs(const VehConst<typename M::T> &V, const StepConst<typename M::T> &c,
                                         typename M::T cp, typename M::T sp, typename M::T vx_, typename M::T vy,
                                         typename M::T om, typename M::T d[6]) {
    using T = typename M::T;
    const T vx = M::pos_(vx_);
    if (MODEL == 0) {
        const T inv_vh = M::rcp_(M::floor_(vx, V.v_eps));
        const T Fyf = tyre_force<M>(V, V.lf, c.delta, vy, om, inv_vh);
        const T Fyr = tyre_force<M>(V, -V.lr, T(0), vy, om, inv_vh);
        deriv_rates<M>(V, c, vx, vy, om, cp, sp, Fyf, Fyr, d);
    } else {
        d[0] = vx * (cp * c.kc - sp * c.ks);
        d[1] = vx * (sp * c.kc + cp * c.ks);
        d[2] = vx * c.kw;
        d[3] = c.a;
        d[4] = T(0);
        d[5] = T(0);
    }
}

template <int MODEL, class M>
__device__ __forceinline__ void deriv(const VehConst<typename M::T> &V, const StepConst<typename M::T> &c,
                                      typename M::T psi, typename M::T vx_, typename M::T vy, typename M::T om,
                                      typename M::T d[6]) {
    const typename M::T pr = M::to_rev(psi);
    deriv_cs<MODEL, M>(V, c, M::cos_rev(pr), M::sin_rev(pr), vx_, vy, om, d);
}

// Value of the neighbouring lane of a pair (quad permute [1, 0, 3, 2]).
__device__ __forceinline__ float dpp_swap_f32(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xf, 0xf, false));
}

// The dynamic model's derivative on a pair of neighbouring lanes: each lane evaluates
// one axle (rear = odd lane) and the two forces are swapped with a DPP quad permute;
// everything else is computed by both lanes alike.  Same values as deriv<0, MathF32>.
__device__ __forceinline__ void deriv_pair(const VehConst<float> &V, const StepConst<float> &c, float psi, float vx_,
                                           float vy, float om, bool rear, float d[6]) {
    const float vx = MathF32::pos_(vx_);
    const float pr = MathF32::to_rev(psi);
    const float cp = MathF32::cos_rev(pr), sp = MathF32::sin_rev(pr);
    const float inv_vh = MathF32::rcp_(MathF32::floor_(vx, V.v_eps));
    const float F = tyre_force<MathF32>(V, rear ? -V.lr : V.lf, rear ? 0.0f : c.delta, vy, om, inv_vh);
    const float Fo = dpp_swap_f32(F);
    deriv_rates<MathF32>(V, c, vx, vy, om, cp, sp, rear ? Fo : F, rear ? F : Fo, d);
}

// Classic RK4 over one interval with the control held, then v_x <- max(v_x, 0).
// CS: the heading's cosine and sine at the start of the interval are given (cp0, sp0: the
// values M::cos_rev / M::sin_rev give for s[2], so the result does not change)
template <int MODEL, class M, bool CS = false>
__device__ __forceinline__ void rk4(const VehConst<typename M::T> &V, const StepConst<typename M::T> &c,
                                    typename M::T h, typename M::T s[6], typename M::T cp0 = typename M::T(0),
                                    typename M::T sp0 = typename M::T(0)) {
    using T = typename M::T;
    T k1[6], k2[6], k3[6], k4[6];
    const T hh = T(0.5) * h;
    if constexpr (CS) deriv_cs<MODEL, M>(V, c, cp0, sp0, s[3], s[4], s[5], k1);
    else deriv<MODEL, M>(V, c, s[2], s[3], s[4], s[5], k1);
    deriv<MODEL, M>(V, c, s[2] + hh * k1[2], s[3] + hh * k1[3], s[4] + hh * k1[4], s[5] + hh * k1[5], k2);
    deriv<MODEL, M>(V, c, s[2] + hh * k2[2], s[3] + hh * k2[3], s[4] + hh * k2[4], s[5] + hh * k2[5], k3);
    deriv<MODEL, M>(V, c, s[2] + h * k3[2], s[3] + h * k3[3], s[4] + h * k3[4], s[5] + h * k3[5], k4);
    const T h6 = h / T(6);
#pragma unroll
    for (int i = 0; i < 6; ++i) s[i] = s[i] + h6 * (k1[i] + T(2) * k2[i] + T(2) * k3[i] + k4[i]);
    if (!(s[3] > T(0)) && s[3] == s[3]) s[3] = T(0);
}

// rk4<0, MathF32> on a pair of lanes (deriv_pair); same expressions, same bits.
__device__ __forceinline__ void rk4_pair(const VehConst<float> &V, const StepConst<float> &c, float h, float s[6],
                                         bool rear) {
    float k1[6], k2[6], k3[6], k4[6];
    const float hh = 0.5f * h;
    deriv_pair(V, c, s[2], s[3], s[4], s[5], rear, k1);
    deriv_pair(V, c, s[2] + hh * k1[2], s[3] + hh * k1[3], s[4] + hh * k1[4], s[5] + hh * k1[5], rear, k2);
    deriv_pair(V, c, s[2] + hh * k2[2], s[3] + hh * k2[3], s[4] + hh * k2[4], s[5] + hh * k2[5], rear, k3);
    deriv_pair(V, c, s[2] + h * k3[2], s[3] + h * k3[3], s[4] + h * k3[4], s[5] + h * k3[5], rear, k4);
    const float h6 = h / 6.0f;
#pragma unroll
    for (int i = 0; i < 6; ++i) s[i] = s[i] + h6 * (k1[i] + 2.0f * k2[i] + 2.0f * k3[i] + k4[i]);
    if (!(s[3] > 0.0f) && s[3] == s[3]) s[3] = 0.0f;
}

// A uniform 32-bit value moved into a scalar register of its own (an opaque copy): the
// sample loop then holds single registers instead of the wide tuples that kernel
// arguments are loaded into, and a spilled value is reloaded alone.
template <class T>
__device__ __forceinline__ T sreg(T v) {
    static_assert(sizeof(T) == 4, "32-bit values only");
    asm("" : "+s"(v));
    return v;
}

// The fields of the parameters read inside the sample loop, each in its own register.
__device__ __forceinline__ KParams loop_params(const KParams &P_in) {
    KParams P = P_in;
    P.dt = sreg(P.dt); P.half_dt = sreg(P.half_dt); P.dt6 = sreg(P.dt6);
    P.lf = sreg(P.lf); P.lr = sreg(P.lr); P.kf_m = sreg(P.kf_m); P.kf_Iz = sreg(P.kf_Iz);
    P.kr_m = sreg(P.kr_m); P.kr_Iz = sreg(P.kr_Iz); P.B = sreg(P.B); P.C = sreg(P.C);
    P.v_eps = sreg(P.v_eps); P.C_rev = sreg(P.C_rev); P.lr_over_L = sreg(P.lr_over_L); P.inv_lr = sreg(P.inv_lr);
    P.a_min = sreg(P.a_min); P.a_max = sreg(P.a_max); P.d_min = sreg(P.d_min); P.d_max = sreg(P.d_max);
    P.sigma_a = sreg(P.sigma_a); P.sigma_d = sreg(P.sigma_d);
    P.Q0 = sreg(P.Q0); P.Q1 = sreg(P.Q1); P.Q2 = sreg(P.Q2); P.Q3 = sreg(P.Q3);
    P.R0 = sreg(P.R0); P.R1 = sreg(P.R1); P.S0 = sreg(P.S0); P.S1 = sreg(P.S1);
    P.cap2 = sreg(P.cap2); P.skip2 = sreg(P.skip2);
    P.off[0] = sreg(P.off[0]); P.off[1] = sreg(P.off[1]); P.off[2] = sreg(P.off[2]); P.off[3] = sreg(P.off[3]);
    P.max_moves = sreg(P.max_moves);
    return P;
}

// A uniform value copied into a vector register (an opaque copy).  On this hardware an
// instruction that reads a scalar register is never issued in the same cycle as another
// wave's instruction, while float add, multiply and fma with vector, literal or inline
// operands are (measured with the issue counters), so the few constants the dynamics
// read many times per step are held in vector registers where registers allow.
template <class T>
__device__ __forceinline__ T vreg(T v) {
    static_assert(sizeof(T) == 4, "32-bit values only");
    asm volatile("" : "+v"(v));
    return v;
}

__device__ __forceinline__ VehConst<float> veh_f32(const KParams &P) {
    VehConst<float> V;
    V.lf = P.lf; V.lr = P.lr; V.kf_m = P.kf_m; V.kf_Iz = P.kf_Iz; V.kr_m = P.kr_m; V.kr_Iz = P.kr_Iz;
    V.B = P.B; V.C = P.C; V.v_eps = P.v_eps; V.lr_over_L = P.lr_over_L; V.inv_lr = P.inv_lr;
    V.Cs = P.C_rev;
    return V;
}

// Pi_U: box clip; a NaN stays NaN so that the sample is flagged non-finite
__device__ __forceinline__ float clip_keep_nan(float v, float lo, float hi) {
    const float c = __builtin_amdgcn_fmed3f(v, lo, hi);
    return v != v ? v : c;
}

// ------------------------------------------------------------------------------
// Frenet projection on the staged raceline window (normal-interpolated polyline)
// ------------------------------------------------------------------------------
// Node in LDS: A = (x, y, nx, ny), B = (wL, wR, s_rel, 0), local frame.
__device__ __forceinline__ float ahead_of(const float4 A, float X, float Y) { return (X - A.x) * A.w - (Y - A.y) * A.z; }

struct Foot {
    float s, d, wL, wR;
    int seg;
    bool limit;
};

// Foot on segment `seg` between the geometry rows A0, A1 (g0, g1: the point's signed
// distances ahead of their normal lines): t solves cross(p - c(t), n(t)) = 0 with the
// stable quadratic root; s, w_L, w_R interpolated from the segment's second rows.
__device__ __forceinline__ Foot foot_on(const float4 *__restrict__ nodes, float X, float Y, int seg, float4 A0,
                                        float4 A1, float g0, float g1) {
    Foot f;
    f.seg = seg;
    f.limit = !(g0 >= 0.0f && g1 <= 0.0f);
    const float4 B0 = nodes[2 * seg + 1], B1 = nodes[2 * seg + 3];
    const float rx = X - A0.x, ry = Y - A0.y;
    const float Dx = A1.x - A0.x, Dy = A1.y - A0.y;
    const float dnx = A1.z - A0.z, dny = A1.w - A0.w;
    const float Cc = g0;
    const float Bc = (rx * dny - ry * dnx) - (Dx * A0.w - Dy * A0.z);
    const float Ac = -(Dx * dny - Dy * dnx);
    const float disc = fmaxf(Bc * Bc - 4.0f * Ac * Cc, 0.0f);
    const float den = -Bc - copysignf(__builtin_amdgcn_sqrtf(disc), Bc);
    float t = (den != 0.0f) ? (2.0f * Cc) * fast_rcp(den) : 0.0f;
    t = fminf(fmaxf(t, 0.0f), 1.0f);
    const float cx = __builtin_fmaf(t, Dx, A0.x), cy = __builtin_fmaf(t, Dy, A0.y);
    const float nx = __builtin_fmaf(t, dnx, A0.z), ny = __builtin_fmaf(t, dny, A0.w);
    f.d = ((X - cx) * nx + (Y - cy) * ny) * __builtin_amdgcn_rsqf(nx * nx + ny * ny);
    f.s = __builtin_fmaf(t, B1.z - B0.z, B0.z);
    f.wL = __builtin_fmaf(t, B1.x - B0.x, B0.x);
    f.wR = __builtin_fmaf(t, B1.y - B0.y, B0.y);
    return f;
}

// Segment search from `seg` (at most max_moves moves, inside the window), then the foot.
// The search carries only the signed distances; the geometry rows of the final segment
// are read again together with its second rows.
// (The move budget and the window's ends are folded into one bound on the row address per
// direction, so a move costs the row read, the normal-line test, two compares and one add.)
__device__ __forceinline__ Foot project(const float4 *__restrict__ nodes, int W, int max_moves, float X, float Y,
                                        int seg) {
    const int seg0 = seg;
    const float4 *q = nodes + 2 * seg + 2;  // geometry row of node seg + 1
    const float4 *const q_hi = nodes + 2 * min(seg0 + max_moves, W - 2) + 2;
    float g1 = ahead_of(*q, X, Y);
    float g0;
    bool fwd = false;
    while (q < q_hi && g1 > 0.0f) {
        q += 2;
        g0 = g1;
        g1 = ahead_of(*q, X, Y);
        fwd = true;
    }
    seg = (int)(q - nodes) / 2 - 1;
    q -= 2;  // geometry row of node seg
    if (!fwd) g0 = ahead_of(*q, X, Y);
    const float4 *const q_lo = nodes + 2 * max(0, seg - (max_moves - (seg - seg0)));
    while (q > q_lo && g0 < 0.0f) {
        q -= 2;
        g1 = g0;
        g0 = ahead_of(*q, X, Y);
    }
    seg = (int)(q - nodes) / 2;
    return foot_on(nodes, X, Y, seg, q[0], q[2], g0, g1);
}

// The same search with the geometry rows of segments seg .. seg + NPF - 1 read ahead
// (before the step's dynamics, so their LDS latency is hidden): the first NPF - 2
// forward moves are decided on registers, further moves read LDS.  Same result.
template <int NPF>
struct NodeAhead {
    float4 q[NPF];
};
template <int NPF>
__device__ __forceinline__ NodeAhead<NPF> read_ahead(const float4 *__restrict__ nodes, int W, int seg) {
    NodeAhead<NPF> a;
#pragma unroll
    for (int i = 0; i < NPF; ++i) a.q[i] = nodes[2 * min(seg + i, W - 1)];
    return a;
}
template <int NPF>
__device__ __forceinline__ Foot project_ahead(const float4 *__restrict__ nodes, int W, int max_moves, float X,
                                              float Y, int seg, const NodeAhead<NPF> &a) {
    float g[NPF];
#pragma unroll
    for (int i = 0; i < NPF; ++i) g[i] = ahead_of(a.q[i], X, Y);
    int moves = 0;
    float g0 = g[0], g1 = g[1];
    bool go = true;
#pragma unroll
    for (int i = 1; i < NPF - 1; ++i) {
        go = go && moves < max_moves && seg + 1 <= W - 2 && g1 > 0.0f;
        seg += go ? 1 : 0;
        moves += go ? 1 : 0;
        g0 = go ? g1 : g0;
        g1 = go ? g[i + 1] : g1;
    }
    while (go && moves < max_moves && seg + 1 <= W - 2 && g1 > 0.0f) {
        ++seg;
        ++moves;
        g0 = g1;
        g1 = ahead_of(nodes[2 * seg + 2], X, Y);
    }
    while (moves < max_moves && seg > 0 && g0 < 0.0f) {
        --seg;
        ++moves;
        g1 = g0;
        g0 = ahead_of(nodes[2 * seg], X, Y);
    }
    return foot_on(nodes, X, Y, seg, nodes[2 * seg], nodes[2 * seg + 2], g0, g1);
}

// ------------------------------------------------------------------------------
// Selection key: lexicographic (infeasible, value, k); value = cost if feasible,
// total violation otherwise; float order mapped onto unsigned order.
// ------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t float_order(float v) {
    const uint32_t b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ unsigned long long make_key(bool h, float v, uint32_t k) {
    return ((unsigned long long)(h ? 0u : 1u) << 63) | ((unsigned long long)float_order(v) << 31) |
           (unsigned long long)(k & 0x7fffffffu);
}

// Wave-wide minimum of a 64-bit key: DPP butterflies inside each row of 16 lanes
// (quad permutes, half-row and row mirrors), then the four row minima by readlane.
template <int CTRL>
__device__ __forceinline__ void dpp_min_step(uint32_t &lo, uint32_t &hi) {
    const uint32_t olo = (uint32_t)__builtin_amdgcn_update_dpp((int)0xffffffff, (int)lo, CTRL, 0xf, 0xf, false);
    const uint32_t ohi = (uint32_t)__builtin_amdgcn_update_dpp((int)0xffffffff, (int)hi, CTRL, 0xf, 0xf, false);
    const bool take = (ohi < hi) || (ohi == hi && olo < lo);
    lo = take ? olo : lo;
    hi = take ? ohi : hi;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    dpp_min_step<0xB1>(lo, hi);   // quad_perm [1,0,3,2]
    dpp_min_step<0x4E>(lo, hi);   // quad_perm [2,3,0,1]
    dpp_min_step<0x141>(lo, hi);  // row_half_mirror
    dpp_min_step<0x140>(lo, hi);  // row_mirror
    unsigned long long best = KEY_NONE;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t rlo = (uint32_t)__builtin_amdgcn_readlane((int)lo, 16 * r);
        const uint32_t rhi = (uint32_t)__builtin_amdgcn_readlane((int)hi, 16 * r);
        const unsigned long long rv = ((unsigned long long)rhi << 32) | rlo;
        best = rv < best ? rv : best;
    }
    return best;
}

// Sum / minimum over the 64 lanes (every lane active), returned to every lane: DPP
// butterflies inside each row of 16, then the four row results in a fixed order.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float rows_f32(float v, int r) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16 * r)); }
__device__ __forceinline__ float wave_sum_f32(float v) {
    v += dpp_f32<0xB1>(v);
    v += dpp_f32<0x4E>(v);
    v += dpp_f32<0x141>(v);
    v += dpp_f32<0x140>(v);
    return (rows_f32(v, 0) + rows_f32(v, 1)) + (rows_f32(v, 2) + rows_f32(v, 3));
}
__device__ __forceinline__ float wave_min_f32(float v) {
    v = fminf(v, dpp_f32<0xB1>(v));
    v = fminf(v, dpp_f32<0x4E>(v));
    v = fminf(v, dpp_f32<0x141>(v));
    v = fminf(v, dpp_f32<0x140>(v));
    return fminf(fminf(rows_f32(v, 0), rows_f32(v, 1)), fminf(rows_f32(v, 2), rows_f32(v, 3)));
}

// ------------------------------------------------------------------------------
// Per-block staging into LDS (every sweep workgroup of a vehicle stages the same tables)
// ------------------------------------------------------------------------------
struct BlockState {
    int slot, race, agent, N, n_tail, n_opp, W, seg0, K, K_prop;
    float vx0, vy0, om0, inv_n_tail, w_game;
    uint32_t key0, key1, ctr2, ctr3;
};

template <int NDISC>
__device__ void stage_block(const LaunchArgs &A, int item_idx, BlockState &bs, char *lds) {
    const KParams &P = A.P;
    const LdsLayout &L = A.L;
    const ItemDev it = A.items[item_idx];
    const RaceDev R = A.races[it.race];
    const AgentRec me = A.agents[it.slot];
    bs.slot = it.slot;
    bs.race = it.race;
    bs.agent = it.agent;
    bs.N = R.N;
    bs.n_tail = R.n_tail;
    bs.K = R.K;
    bs.K_prop = R.prop ? R.K_prop : 0;
    bs.n_opp = R.n_agents - 1;
    bs.W = me.win_n;
    bs.seg0 = me.seg_loc;
    bs.vx0 = me.vx;
    bs.vy0 = me.vy;
    bs.om0 = me.om;
    bs.inv_n_tail = 1.0f / (float)R.n_tail;
    bs.w_game = (A.phase == 0) ? 0.0f : P.w_game;
    bs.key0 = (uint32_t)R.seed;
    bs.key1 = (uint32_t)(R.seed >> 32);
    bs.ctr2 = (uint32_t)it.agent | ((uint32_t)A.phase << 16);
    bs.ctr3 = R.plan_step;

    const int tid = threadIdx.x, nth = blockDim.x;
    const int pstride = (L.N_max + 1) * PRED_STRIDE;
    float2 *ubar = (float2 *)(lds + L.ubar);
    float4 *xref = (float4 *)(lds + L.xref);
    float4 *nodes = (float4 *)(lds + L.nodes);
    // window and reference rows: whole buffers (w_max, N_max rows), so these reads do not
    // wait for the vehicle record; rows past the vehicle's own are never read
    const float4 *wn = A.win + (size_t)it.slot * WIN_MAX * 2;
    for (int t = tid; t < 2 * L.w_max; t += nth) nodes[t] = wn[t];
    const float4 *xr = A.xref + (size_t)it.slot * L.N_max;
    for (int t = tid; t < L.N_max; t += nth) xref[t] = xr[t];
    const float2 *un = (const float2 *)(R.u_nom) + (size_t)it.agent * R.N;
    for (int t = tid; t < R.N; t += nth) ubar[t] = un[t];
    if (R.prop) {
        float4 *pq = (float4 *)(lds + L.prop);
        const float4 *src = R.prop + (size_t)it.agent * R.N;
        for (int t = tid; t < R.N; t += nth) pq[t] = src[t];
    }

    if (bs.n_opp > 0) {
        float4 *oppT = (float4 *)(lds + L.oppT);
        float4 *oppc = (float4 *)(lds + L.oppc);
        float2 *opp = (float2 *)(lds + L.opp);
        const int total = R.N * bs.n_opp;
        // the first footprint row of this thread, read before the frames are known
        float4 pre = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (tid < total) {
            const int t = tid / bs.n_opp + 1;
            const int jo = tid - (t - 1) * bs.n_opp;
            const int j = jo < it.agent ? jo : jo + 1;
            pre = *(const float4 *)(A.pred_in + (size_t)(R.slot0 + j) * pstride + t * PRED_STRIDE);
        }
        if (tid < bs.n_opp) {
            const int j = tid < it.agent ? tid : tid + 1;
            const int sj = R.slot0 + j;
            const AgentRec o = A.agents[sj];
            // frame j -> frame i: p_i = Rot(psi_j - psi_i) p_j + Rot(-psi_i) (O_j - O_i)
            const double dpsi = o.psi0 - me.psi0;
            const double dx = o.ox - me.ox, dy = o.oy - me.oy;
            oppT[tid] = make_float4((float)cos(dpsi), (float)sin(dpsi), (float)(me.c0 * dx + me.s0 * dy),
                                    (float)(-me.s0 * dx + me.c0 * dy));
            const float *pj = A.pred_in + (size_t)sj * pstride;
            float dsum = 0.0f;
            for (int t = R.N - R.n_tail + 1; t <= R.N; ++t) dsum += pj[t * PRED_STRIDE + 5];
            const double ds0 = me.s_abs - o.s_abs;
            const double alpha = 1.0 / (1.0 + fabs(ds0) / ((double)P.s_contest + (double)P.eps_alpha));
            const float gam = (ds0 > (double)P.s_role && ds0 < (double)P.s_contest) ? P.w_block : 0.0f;
            const float sN = (float)((o.s_abs - me.s_abs) + (double)pj[R.N * PRED_STRIDE + 4]);
            oppc[tid] = make_float4(sN, dsum / (float)R.n_tail, (float)((double)P.w_long * alpha), gam);
        }
        __syncthreads();
        // footprint rows of opponent j at step t in this vehicle's frame
        auto footprint = [&](int t, int jo, int j, float4 pr) {
            const float4 T = oppT[jo];
            float px = pr.x, py = pr.y;
            const float pc = pr.z, psn = pr.w;
            if (P.pred_sig_lon > 0.0f || P.pred_sig_lat > 0.0f) {
                // perturbed prediction (robustness experiment): a Gaussian pair of its own
                // Philox counter moves the position along / across the predicted heading
                const uint4 r = philox4x32_10(make_uint4(0x80000000u | (uint32_t)j, (uint32_t)t, bs.ctr2, bs.ctr3),
                                              bs.key0, bs.key1);
                const float2 z = gauss_pair(r.x, r.y);
                const float dl = P.pred_sig_lon * z.x, dn = P.pred_sig_lat * z.y;
                px += dl * pc - dn * psn;
                py += dl * psn + dn * pc;
            }
            float2 *dst = opp + ((size_t)(t - 1) * L.n_opp_max + jo) * (NDISC + 1);
            dst[0] = make_float2(T.x * px - T.y * py + T.z, T.y * px + T.x * py + T.w);
#pragma unroll
            for (int b = 0; b < NDISC; ++b) {
                const float cxj = __builtin_fmaf(P.off[b], pc, px), cyj = __builtin_fmaf(P.off[b], psn, py);
                dst[1 + b] = make_float2(T.x * cxj - T.y * cyj + T.z, T.y * cxj + T.x * cyj + T.w);
            }
        };
        if (tid < total) {
            const int t = tid / bs.n_opp + 1;
            const int jo = tid - (t - 1) * bs.n_opp;
            footprint(t, jo, jo < it.agent ? jo : jo + 1, pre);
        }
        for (int e = tid + nth; e < total; e += nth) {
            const int t = e / bs.n_opp + 1;  // tau = 1..N
            const int jo = e - (t - 1) * bs.n_opp;
            const int j = jo < it.agent ? jo : jo + 1;
            footprint(t, jo, j, *(const float4 *)(A.pred_in + (size_t)(R.slot0 + j) * pstride + t * PRED_STRIDE));
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------------------------
// Per-step terms.  The sweep lanes and the cooperative re-roll call the same
// functions on the same values and accumulate in the same order, so the
// re-rolled sample reproduces its lane bit for bit.
// ------------------------------------------------------------------------------
__device__ __forceinline__ float2 controls(const KParams &P, float2 ub, float za, float zd) {
    return make_float2(clip_keep_nan(__builtin_fmaf(P.sigma_a, za, ub.x), P.a_min, P.a_max),
                       clip_keep_nan(__builtin_fmaf(P.sigma_d, zd, ub.y), P.d_min, P.d_max));
}
// sample k < K_prop of a vehicle with a learned proposal: mean and scale from the proposal table
__device__ __forceinline__ float2 controls_k(const KParams &P, const BlockState &bs, const char *lds,
                                            const LdsLayout &L, uint32_t k, int tau, float2 ub, float za, float zd) {
    if ((int)k < bs.K_prop) {
        const float4 q = ((const float4 *)(lds + L.prop))[tau];
        return make_float2(clip_keep_nan(__builtin_fmaf(q.z, za, q.x), P.a_min, P.a_max),
                           clip_keep_nan(__builtin_fmaf(q.w, zd, q.y), P.d_min, P.d_max));
    }
    return controls(P, ub, za, zd);
}

// tracking term of eq. (ctrack) at one step; heading error wrapped to [-pi, pi]
__device__ __forceinline__ float track_term(const KParams &P, const float *st, float4 xr) {
    const float ex = st[0] - xr.x, ey = st[1] - xr.y, ev = st[3] - xr.w;
    float ep = st[2] - xr.z;
    ep = ep - 6.28318531f * rintf(ep * 0.159154943f);
    return P.Q0 * ex * ex + P.Q1 * ey * ey + P.Q2 * ep * ep + P.Q3 * ev * ev;
}
__device__ __forceinline__ float ctrl_term(const KParams &P, float2 u) { return P.R0 * u.x * u.x + P.R1 * u.y * u.y; }
__device__ __forceinline__ float rate_term(const KParams &P, float2 u, float2 up) {
    const float da = u.x - up.x, dd = u.y - up.y;
    return P.S0 * da * da + P.S1 * dd * dd;
}
// boundary clearance of eq. (selection-boundary) at one step
__device__ __forceinline__ float bound_term(const Foot &f) { return fminf(f.wR + f.d, f.wL - f.d); }

// Squared footprint distance to one opponent at one step (eq. Dmin over disc pairs),
// folded into `cur` (values are capped at cap^2: only smaller ones change any result;
// a pair is skipped when the centres are too far apart for any disc pair to go below it).
// UNIFORM: one wave-wide test skips the pairs when no lane is close (the common case);
// otherwise every lane computes them and the close lanes keep the result, so each lane
// gets the value of the per-lane form.
template <int NDISC, bool UNIFORM = false>
__device__ __forceinline__ float opp_min2(const KParams &P, const float2 *e, float2 cg, float X, float Y,
                                          const float *ax, const float *ay, float cur) {
    const float dx = X - cg.x, dy = Y - cg.y;
    const bool close = dx * dx + dy * dy < P.skip2;
    auto pairs = [&](float m) {
#pragma unroll
        for (int a = 0; a < NDISC; ++a) {
#pragma unroll
            for (int b = 0; b < NDISC; ++b) {
                const float2 c = e[1 + b];
                const float qx = ax[a] - c.x, qy = ay[a] - c.y;
                m = fminf(m, qx * qx + qy * qy);
            }
        }
        return m;
    };
    if (UNIFORM) {
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(close) == 0, 1)) return cur;
        const float m = pairs(cur);
        return close ? m : cur;
    }
    if (close) cur = pairs(cur);
    return cur;
}

// Disc centres of the own footprint at (X, Y) with heading cosine / sine (ch, sh).
template <int NDISC>
__device__ __forceinline__ void disc_centres(const KParams &P, float X, float Y, float ch, float sh, float *ax,
                                             float *ay) {
#pragma unroll
    for (int a = 0; a < NDISC; ++a) {
        ax[a] = __builtin_fmaf(P.off[a], ch, X);
        ay[a] = __builtin_fmaf(P.off[a], sh, Y);
    }
}

struct SampleResult {
    float cost, viol;
    bool h;
    unsigned char flags;
    float st[6];
    float cp[NCP_MAX - 1][7];  // state and segment after steps C, 2C, ... (C = ceil(N / chunks))
};

// Terminal scoring: game-aware cost (eqs. game_cost, c_contest, c_long, c_block,
// c_safety), total cost (eq. allc), flags b, o, h and the violation nu.
template <int MAXOPP>
__device__ __forceinline__ SampleResult terminal(const KParams &P, const BlockState &bs, const char *lds,
                                                 const LdsLayout &L, float J, float rho_bd, float dsum, float s,
                                                 const float *g2, bool limit, const float *st) {
    const float4 *oppc = (const float4 *)(lds + L.oppc);
    float cgame = 0.0f, rho_obs = INFINITY;
    const float dbar_i = dsum * bs.inv_n_tail;
#pragma unroll
    for (int j = 0; j < MAXOPP; ++j) {
        if (j < bs.n_opp) {
            const float4 c = oppc[j];  // (s_hat_N - s_i, dbar_j, w_long alpha_ij, gamma_ij)
            const float dsN = s - c.x;
            const float cc = (fabsf(dsN) < P.s_contest) ? -P.w_contest : 0.0f;
            const float cl = -c.z * dsN;
            const float cb = -c.w / (1.0f + fabsf(dbar_i - c.y));
            const float gj = __builtin_sqrtf(g2[j]);
            const float shv = fmaxf(0.0f, P.g_safe - gj);
            cgame += cc + cl + cb + P.w_safety * shv * shv;
            rho_obs = fminf(rho_obs, gj);
        }
    }
    const float c = J + bs.w_game * cgame;
    bool finite = isfinite(c) && !isnan(rho_bd) && !isnan(rho_obs);
#pragma unroll
    for (int i = 0; i < 6; ++i) finite = finite && isfinite(st[i]);
    const bool b = finite && rho_bd >= P.m_bd;
    const bool o = finite && rho_obs >= P.d_col;
    SampleResult res;
    res.h = b && o;
    res.cost = c;
    res.viol = finite ? fmaxf(0.0f, P.m_bd - rho_bd) + fmaxf(0.0f, P.d_col - rho_obs) : INFINITY;
    res.flags = (unsigned char)((b ? 1 : 0) | (o ? 2 : 0) | (res.h ? 4 : 0) | (limit ? 8 : 0) | (finite ? 0 : 16));
#pragma unroll
    for (int i = 0; i < 6; ++i) res.st[i] = st[i];
    return res;
}

// ------------------------------------------------------------------------------
// One sample in one lane: perturb, clip, roll out, score, check (Sec. III)
// ------------------------------------------------------------------------------
// NPF > 0 (launches with about one wave per SIMD, where nothing hides LDS latency):
// the raceline rows of the next NPF segments are read ahead of each step's dynamics.
// LPS = 2 (dynamic model, launches far below one wave per SIMD): a pair of lanes runs
// one sample; each lane draws one of the two Gaussian pairs of a Philox call and
// evaluates one axle, the halves are swapped by DPP, and both lanes hold the same state.
template <int MODEL, int NDISC, int MAXOPP, int NPF = 0, int LPS = 1>
__device__ __forceinline__ SampleResult lane_sample(const KParams &P_in, const BlockState &bs, const char *lds,
                                                   const LdsLayout &L, uint32_t k, float *noise_out,
                                                   bool rear = false) {
    // parameters in single scalar registers, except in the one-lane latency variant
    // (about one wave per SIMD), which measured faster with the compiler's own allocation
    const KParams P = (NPF > 0 && LPS == 1) ? P_in : loop_params(P_in);
    const float2 *ubar = (const float2 *)(lds + L.ubar);
    const float4 *xref = (const float4 *)(lds + L.xref);
    const float2 *opp = (const float2 *)(lds + L.opp);
    const float4 *nodes = (const float4 *)(lds + L.nodes);
    VehConst<float> V = veh_f32(P);
    float h = P.dt;
    if constexpr (NPF == 0 && LPS == 1) {  // throughput variants: the dynamics' hot constants
        V.B = vreg(V.B); V.Cs = vreg(V.Cs); V.lf = vreg(V.lf); V.lr = vreg(V.lr);
        V.kr_m = vreg(V.kr_m); V.kr_Iz = vreg(V.kr_Iz); h = vreg(h);
    }

    float st[6] = {0.0f, 0.0f, 0.0f, bs.vx0, bs.vy0, bs.om0};
    int seg = bs.seg0;
    float J = 0.0f, rho_bd = INFINITY, dsum = 0.0f, s = 0.0f;
    float g2[MAXOPP];
#pragma unroll
    for (int j = 0; j < MAXOPP; ++j) g2[j] = P.cap2;
    float2 up = make_float2(0.0f, 0.0f);
    bool limit = false;
    constexpr int NC = ncp_of<NPF>();
    float cp[NC - 1][7];
#pragma unroll
    for (int c = 0; c < NC - 1; ++c)
#pragma unroll
        for (int i = 0; i < 7; ++i) cp[c][i] = 0.0f;
    const int C = (bs.N + NC - 1) / NC;

    float2 zn = make_float2(0.0f, 0.0f);  // perturbation of the odd step of a Philox call
    // throughput variants: the heading's cosine and sine after a step (the footprint's) are
    // the first RK4 stage's of the next step, computed once
    constexpr bool HCS = NPF == 0 && LPS == 1;
    float hc = 0.0f, hs = 0.0f;
    if constexpr (HCS) {
        hc = fast_cos(st[2]);
        hs = fast_sin(st[2]);
    }
    for (int tau = 0; tau < bs.N; ++tau) {
        float2 z;
        if ((tau & 1) == 0) {
            const uint4 r = philox4x32_10<NPF == 0 && LPS == 1>(make_uint4(k, (uint32_t)(tau >> 1), bs.ctr2, bs.ctr3),
                                                                bs.key0, bs.key1);
            if constexpr (LPS == 2) {
                const float2 g = gauss_pair(rear ? r.z : r.x, rear ? r.w : r.y);
                const float2 go = make_float2(dpp_swap_f32(g.x), dpp_swap_f32(g.y));
                z = rear ? go : g;
                zn = rear ? g : go;
            } else {
                z = gauss_pair(r.x, r.y);
                zn = gauss_pair(r.z, r.w);
            }
        } else {
            z = zn;
        }
        // LDS reads that do not depend on this step's dynamics go first
        const float2 ub = ubar[tau];
        const float4 xr = xref[tau];
        NodeAhead<(NPF > 0 ? NPF : 1)> ahead;
        if constexpr (NPF > 0) ahead = read_ahead<NPF>(nodes, bs.W, seg);
        // the opponents' rows of this step; the latency variants read them whole here
        const float2 *ot = opp + tau * (L.n_opp_max * (NDISC + 1));
        constexpr bool PRE_ALL = NPF > 0 && MAXOPP <= 3;
        float2 orow[PRE_ALL ? MAXOPP * (NDISC + 1) : 1];
        if constexpr (PRE_ALL) {
#pragma unroll
            for (int i = 0; i < MAXOPP * (NDISC + 1); ++i) orow[i] = ot[i];
        }
        if (noise_out) {
            noise_out[2 * tau] = z.x;
            noise_out[2 * tau + 1] = z.y;
        }
        const float2 u = controls_k(P, bs, lds, L, k, tau, ub, z.x, z.y);
        // latency variants (NPF > 0) branch-free, throughput variants with the uniform atan
        using MS = typename std::conditional<NPF == 0, MathF32U, MathF32>::type;
        const StepConst<float> sc = step_const<MODEL, MS>(V, u.x, u.y);
        if constexpr (LPS == 2 && MODEL == 0) rk4_pair(V, sc, P.dt, st, rear);
        else if constexpr (HCS) rk4<MODEL, MS, true>(V, sc, h, st, hc, hs);
        else rk4<MODEL, MS>(V, sc, h, st);
        Foot f;
        if constexpr (NPF > 0) f = project_ahead<NPF>(nodes, bs.W, P.max_moves, st[0], st[1], seg, ahead);
        else f = project(nodes, bs.W, P.max_moves, st[0], st[1], seg);
        seg = f.seg;
        limit |= f.limit;
        s = f.s;
        J += track_term(P, st, xr);
        J += ctrl_term(P, u);
        if (tau >= 1) J += rate_term(P, u, up);
        up = u;
        rho_bd = fminf(rho_bd, bound_term(f));
        float ch = 1.0f, sh = 0.0f;
        if constexpr (HCS) {
            hc = fast_cos(st[2]);
            hs = fast_sin(st[2]);
            ch = hc;
            sh = hs;
        } else if (NDISC > 1) {
            ch = fast_cos(st[2]);
            sh = fast_sin(st[2]);
        }
        // (other variants with up to 3 opponents read every centre before the first test,
        // all within the table; more would hold too many registers)
        constexpr int NPRE = (!PRE_ALL && MAXOPP <= 3) ? MAXOPP : 1;
        float2 cg[NPRE];
        if constexpr (!PRE_ALL && MAXOPP <= 3) {
#pragma unroll
            for (int j = 0; j < NPRE; ++j) cg[j] = ot[j * (NDISC + 1)];
        }
        float ax[NDISC], ay[NDISC];
        disc_centres<NDISC>(P, st[0], st[1], ch, sh, ax, ay);
        // opponent count compared on the scalar unit at every step (held as one compare mask
        // per opponent, the masks were spilled and reloaded with v_readlane)
        int n_opp = bs.n_opp;
        asm volatile("" : "+s"(n_opp));
#pragma unroll
        for (int j = 0; j < MAXOPP; ++j) {
            if (j < n_opp) {
                if constexpr (PRE_ALL) {
                    g2[j] = opp_min2<NDISC>(P, orow + j * (NDISC + 1), orow[j * (NDISC + 1)], st[0], st[1], ax, ay,
                                            g2[j]);
                } else {
                    const float2 c0 = MAXOPP <= 3 ? cg[j < NPRE ? j : 0] : ot[j * (NDISC + 1)];
                    g2[j] = opp_min2<NDISC, NPF == 0 && LPS == 1>(P, ot + j * (NDISC + 1), c0, st[0], st[1], ax,
                                                                  ay, g2[j]);
                }
            }
        }
        if (tau + 1 > bs.N - bs.n_tail) dsum += f.d;
        // (C re-read at every step: the step counts (c + 1) C are not kept in registers)
        int Cv = C;
        asm volatile("" : "+s"(Cv));
#pragma unroll
        for (int c = 0; c < NC - 1; ++c) {
            if (tau + 1 == (c + 1) * Cv) {
#pragma unroll
                for (int i = 0; i < 6; ++i) cp[c][i] = st[i];
                cp[c][6] = __int_as_float(seg);
            }
        }
    }
    SampleResult res = terminal<MAXOPP>(P, bs, lds, L, J, rho_bd, dsum, s, g2, limit, st);
#pragma unroll
    for (int c = 0; c < NC - 1; ++c)
#pragma unroll
        for (int i = 0; i < 7; ++i) res.cp[c][i] = cp[c][i];
    return res;
}

// ------------------------------------------------------------------------------
// One sample on two waves (the split variant).  A lane of an even wave integrates the
// dynamics, the longest dependent chain of a step.  Its partner lane in the next (odd)
// wave does the rest: it draws the perturbation and clips the controls
// SPLIT_AHEAD steps ahead, projects every state onto the raceline and scores it
// (tracking, control and rate terms, boundary, footprint distances, tail offsets), then
// takes the terminal scoring.  Controls and states pass through LDS rings of SPLIT_RING
// steps; uprod / prod count the controls and states written, cons the states consumed,
// per wave pair, and each side re-reads a count only when its ring runs empty (or full).
// The scoring side publishes the controls of step tau + SPLIT_AHEAD before it waits for
// state tau, and a control slot is rewritten only after its state was published, so
// both waits end; their bounds are guards only (a wait polls every 256 cycles: shorter
// sleeps took issue slots from the wave sharing the SIMD, longer ones woke late).  Checkpoints: states on the dynamics
// lane, segments on the scoring lane.  Arithmetic and summation order as in lane_sample:
// the two variants give the same bits.
// ------------------------------------------------------------------------------
template <int MODEL, int NDISC, int MAXOPP, int NPF>
__device__ __forceinline__ SampleResult lane_sample_split(const KParams &P, const BlockState &bs, char *lds,
                                                         const LdsLayout &L, uint32_t k, float *noise_out, bool dyn,
                                                         int *status) {
    constexpr int TS = BLOCK / 2;
    constexpr int NC = ncp_of<NPF>();
    static_assert(SPLIT_AHEAD + 1 <= SPLIT_RING, "a control slot is rewritten only after its state was published");
    const int vt = split_vt(threadIdx.x);
    const int i = vt & (TS - 1);
    const int w = (vt >> 6) & 1;  // wave pair
    const int lane = threadIdx.x & 63;
    float4 *ring = (float4 *)(lds + L.sp_ring);    // [SPLIT_RING][TS]: X, Y, PSI, VX after the step
    float2 *uring = (float2 *)(lds + L.sp_uring);  // [SPLIT_RING][TS]: controls of the step
    volatile int *prod = (volatile int *)(lds + L.sp_sync);
    volatile int *cons = prod + 2;
    volatile int *uprod = prod + 6;
    float *fin = (float *)(lds + L.sp_fin);  // [TS][SPLIT_FIN]: final state
    const int C = (bs.N + NC - 1) / NC;
    if (threadIdx.x < 8) prod[threadIdx.x] = 0;
    __syncthreads();
    // each side's values, set and used only on that side (one barrier, outside both)
    float cp[NC - 1][6];                                   // dynamics: checkpointed states
    float J, rho_bd, dsum, s, g2[MAXOPP];                  // scoring
    bool limit;
    int cseg[NC - 1];
    // a wait that gave up (its partner did not advance within P.spin_limit polls): the
    // sample's values are then unreliable, so it is scored non-finite (never selected)
    bool stalled = false;
    if (dyn) {
        const VehConst<float> V = veh_f32(P);
        float st[6] = {0.0f, 0.0f, 0.0f, bs.vx0, bs.vy0, bs.om0};
#pragma unroll
        for (int c = 0; c < NC - 1; ++c)
#pragma unroll
            for (int j = 0; j < 6; ++j) cp[c][j] = 0.0f;
        int useen = 0, seen = 0;  // the scoring side's counts as last read
        for (int tau = 0; tau < bs.N; ++tau) {
            if (useen <= tau) {
                for (int spin = 0; spin < P.spin_limit; ++spin) {
                    useen = uprod[w];
                    if (useen > tau) break;
                    __builtin_amdgcn_s_sleep(4);
                }
                stalled |= useen <= tau;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
            const float2 u = uring[(tau % SPLIT_RING) * TS + i];
            const StepConst<float> sc = step_const<MODEL, MathF32>(V, u.x, u.y);
            rk4<MODEL, MathF32>(V, sc, P.dt, st);
            if (tau - seen >= SPLIT_RING) {
                for (int spin = 0; spin < P.spin_limit; ++spin) {
                    seen = cons[w];
                    if (tau - seen < SPLIT_RING) break;
                    __builtin_amdgcn_s_sleep(4);
                }
                stalled |= tau - seen >= SPLIT_RING;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
            ring[(tau % SPLIT_RING) * TS + i] = make_float4(st[0], st[1], st[2], st[3]);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0) prod[w] = tau + 1;
            int Cv = C;
            asm volatile("" : "+s"(Cv));
#pragma unroll
            for (int c = 0; c < NC - 1; ++c) {
                if (tau + 1 == (c + 1) * Cv) {
#pragma unroll
                    for (int j = 0; j < 6; ++j) cp[c][j] = st[j];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) fin[i * SPLIT_FIN + j] = st[j];
        fin[i * SPLIT_FIN + 6] = stalled ? 1.0f : 0.0f;
    } else {
        const float2 *ubar = (const float2 *)(lds + L.ubar);
        const float4 *xref = (const float4 *)(lds + L.xref);
        const float2 *opp = (const float2 *)(lds + L.opp);
        const float4 *nodes = (const float4 *)(lds + L.nodes);
        int seg = bs.seg0;
        J = 0.0f;
        rho_bd = INFINITY;
        dsum = 0.0f;
        s = 0.0f;
#pragma unroll
        for (int j = 0; j < MAXOPP; ++j) g2[j] = P.cap2;
        limit = false;
#pragma unroll
        for (int c = 0; c < NC - 1; ++c) cseg[c] = 0;
        // controls of step t, in step order (one Philox call per pair of steps), published
        float2 zn = make_float2(0.0f, 0.0f);
        int t_u = 0;
        auto control = [&]() {
            const int t = t_u++;
            float2 z;
            if ((t & 1) == 0) {
                const uint4 r = philox4x32_10(make_uint4(k, (uint32_t)(t >> 1), bs.ctr2, bs.ctr3), bs.key0, bs.key1);
                z = gauss_pair(r.x, r.y);
                zn = gauss_pair(r.z, r.w);
            } else {
                z = zn;
            }
            uring[(t % SPLIT_RING) * TS + i] = controls_k(P, bs, lds, L, k, t, ubar[t], z.x, z.y);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0) uprod[w] = t + 1;
        };
        const int ahead0 = bs.N < SPLIT_AHEAD ? bs.N : SPLIT_AHEAD;
        for (int t = 0; t < ahead0; ++t) control();
        int seen = 0;  // the dynamics side's count as last read
        float2 up = make_float2(0.0f, 0.0f);
        for (int tau = 0; tau < bs.N; ++tau) {
            if (tau + SPLIT_AHEAD < bs.N) control();
            // reads that do not depend on this step's state go first (the step's control is
            // still in its slot: it is rewritten SPLIT_RING - SPLIT_AHEAD iterations later)
            const float2 u = uring[(tau % SPLIT_RING) * TS + i];
            const float4 xr = xref[tau];
            NodeAhead<NPF> ahead = read_ahead<NPF>(nodes, bs.W, seg);
            const float2 *ot = opp + tau * (L.n_opp_max * (NDISC + 1));
            float2 orow[MAXOPP * (NDISC + 1)];
#pragma unroll
            for (int j = 0; j < MAXOPP * (NDISC + 1); ++j) orow[j] = ot[j];
            if (seen <= tau) {
                for (int spin = 0; spin < P.spin_limit; ++spin) {
                    seen = prod[w];
                    if (seen > tau) break;
                    __builtin_amdgcn_s_sleep(4);
                }
                stalled |= seen <= tau;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
            const float4 sv = ring[(tau % SPLIT_RING) * TS + i];
            const float st4[4] = {sv.x, sv.y, sv.z, sv.w};
            const Foot f = project_ahead<NPF>(nodes, bs.W, P.max_moves, sv.x, sv.y, seg, ahead);
            seg = f.seg;
            limit |= f.limit;
            s = f.s;
            // the terms summed in the one-lane order, so that both variants give the same bits
            J += track_term(P, st4, xr);
            J += ctrl_term(P, u);
            if (tau >= 1) J += rate_term(P, u, up);
            up = u;
            rho_bd = fminf(rho_bd, bound_term(f));
            float ch = 1.0f, sh = 0.0f;
            if (NDISC > 1) {
                ch = fast_cos(sv.z);
                sh = fast_sin(sv.z);
            }
            float ax[NDISC], ay[NDISC];
            disc_centres<NDISC>(P, sv.x, sv.y, ch, sh, ax, ay);
            int n_opp = bs.n_opp;
            asm volatile("" : "+s"(n_opp));
#pragma unroll
            for (int j = 0; j < MAXOPP; ++j) {
                if (j < n_opp)
                    g2[j] = opp_min2<NDISC>(P, orow + j * (NDISC + 1), orow[j * (NDISC + 1)], sv.x, sv.y, ax, ay,
                                            g2[j]);
            }
            if (tau + 1 > bs.N - bs.n_tail) dsum += f.d;
            int Cv = C;
            asm volatile("" : "+s"(Cv));
#pragma unroll
            for (int c = 0; c < NC - 1; ++c) {
                if (tau + 1 == (c + 1) * Cv) cseg[c] = seg;
            }
            // the state is used: its ring entry may be overwritten
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0) cons[w] = tau + 1;
        }
        if (noise_out) {  // debug output only: the perturbations drawn again, outside the loop
            for (int m = 0; 2 * m < bs.N; ++m) {
                const uint4 r = philox4x32_10(make_uint4(k, (uint32_t)m, bs.ctr2, bs.ctr3), bs.key0, bs.key1);
                const float2 z0 = gauss_pair(r.x, r.y), z1 = gauss_pair(r.z, r.w);
                noise_out[4 * m] = z0.x;
                noise_out[4 * m + 1] = z0.y;
                if (2 * m + 1 < bs.N) {
                    noise_out[4 * m + 2] = z1.x;
                    noise_out[4 * m + 3] = z1.y;
                }
            }
        }
    }
    __syncthreads();
    // one result object for both sides, written field by field
    SampleResult res;
    const float *fo = fin + i * SPLIT_FIN;  // the final state, read where it lies
    if (dyn) {
        res.cost = 0.0f;
        res.viol = 0.0f;
        res.h = false;
        res.flags = 0;
#pragma unroll
        for (int j = 0; j < 6; ++j) res.st[j] = fo[j];
#pragma unroll
        for (int c = 0; c < NC - 1; ++c) {
#pragma unroll
            for (int j = 0; j < 6; ++j) res.cp[c][j] = cp[c][j];
            res.cp[c][6] = 0.0f;
        }
    } else {
        const SampleResult t = terminal<MAXOPP>(P, bs, lds, L, J, rho_bd, dsum, s, g2, limit, fo);
        res.cost = t.cost;
        res.viol = t.viol;
        res.h = t.h;
        res.flags = t.flags;
        if (stalled || fo[6] != 0.0f) {  // either side gave up a wait
            res.cost = __builtin_nanf("");
            res.viol = INFINITY;
            res.h = false;
            res.flags = (unsigned char)((t.flags & 8) | 16);
            atomicOr(status, SGTP_STATUS_WAIT_GAVE_UP);
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) res.st[j] = t.st[j];
#pragma unroll
        for (int c = 0; c < NC - 1; ++c) {
#pragma unroll
            for (int j = 0; j < 6; ++j) res.cp[c][j] = 0.0f;
            res.cp[c][6] = __int_as_float(cseg[c]);
        }
    }
    return res;
}

template <int MODEL, int NDISC, int MAXOPP, int NPF, int LPS, int SPL>
__device__ __forceinline__ SampleResult run_sample(const KParams &P, const BlockState &bs, char *lds,
                                                  const LdsLayout &L, uint32_t k, float *noise_out, bool rear,
                                                  bool dyn, int *status) {
    if constexpr (SPL != 0) return lane_sample_split<MODEL, NDISC, MAXOPP, NPF>(P, bs, lds, L, k, noise_out, dyn, status);
    else return lane_sample<MODEL, NDISC, MAXOPP, NPF, LPS>(P, bs, lds, L, k, noise_out, rear);
}

// ------------------------------------------------------------------------------
// One sample re-rolled by a whole workgroup for its outputs: controls and output
// writes in parallel over the horizon, the dynamics and the projection serially (in
// ncp_of<NPF>() pieces at once when the sample's checkpoints are given).  MODE WINNER
// re-rolls the selected sample, whose cost and violation its own lane exported;
// NOMINAL rolls out the unperturbed nominal (predictions only).
// ------------------------------------------------------------------------------
struct RerollOut {
    float *pred;        // [N+1][PRED_STRIDE] owner's frame
    float2 *u;          // [N] adopted controls (WINNER with adopt), or NULL
    double *traj;       // [N+1][8] world, or NULL
    float2 *u_apply;    // first control (final phase), or NULL
    bool final_shift;   // write the warm start (shifted) instead of the adopted sequence
};

template <int MODEL, int MODE, int NPF = 0>
__device__ void reroll_block(const KParams &P, const LdsLayout &L, const BlockState &bs, char *lds,
                             const AgentRec &rec, uint32_t k, const RerollOut &out, int *status,
                             const float *cps = nullptr) {
    const int tid = threadIdx.x, nth = blockDim.x, N = bs.N;
    const float2 *ubar = (const float2 *)(lds + L.ubar);
    const float4 *nodes = (const float4 *)(lds + L.nodes);
    float2 *wu = (float2 *)(lds + L.rr_u);
    float4 *wst = (float4 *)(lds + L.rr_st);  // [N][2]: (X, Y, PSI, VX), (VY, OM, -, -)
    float4 *wf = (float4 *)(lds + L.rr_f);    // [N]: (s, d, wL, wR)
    const VehConst<float> V = veh_f32(P);

    // the pieces of the horizon and their starting states (checkpoints are read before
    // the controls are drawn); the dynamic model puts each piece on two lanes, one axle each
    constexpr int NC = ncp_of<NPF>();
    const int nch = cps ? NC : 1;
    const int C = cps ? (N + NC - 1) / NC : N;
    constexpr int LPC = MODEL == 0 ? 2 : 1;  // lanes per piece
    const bool chunk_lane = tid < LPC * nch;
    const int ch = tid / LPC;
    const bool rear = LPC == 2 && (tid & 1);
    // the projection of each piece runs on a lane of the second wave, one step behind
    // its dynamics (which do not need it); prog[piece] counts the states written
    const bool proj_lane = tid >= 64 && tid < 64 + nch;
    const int pch = tid - 64;
    volatile int *prog = (volatile int *)(lds + L.rr_sync);
    float st[6] = {0.0f, 0.0f, 0.0f, bs.vx0, bs.vy0, bs.om0};
    int seg = bs.seg0;
    if (chunk_lane && ch > 0) {
        const float *c = cps + 7 * (ch - 1);
#pragma unroll
        for (int i = 0; i < 6; ++i) st[i] = c[i];
    }
    if (proj_lane && pch > 0) seg = __float_as_int(cps[7 * (pch - 1) + 6]);
    if (tid < nch) prog[tid] = tid * C;

    // A. controls of every step (one Philox call per pair of steps)
    for (int m = tid; 2 * m < N; m += nth) {
        float2 z0 = make_float2(0.0f, 0.0f), z1 = z0;
        if (MODE != NOMINAL) {
            const uint4 r = philox4x32_10(make_uint4(k, (uint32_t)m, bs.ctr2, bs.ctr3), bs.key0, bs.key1);
            z0 = gauss_pair(r.x, r.y);
            z1 = gauss_pair(r.z, r.w);
        }
        if (MODE == NOMINAL) {
            wu[2 * m] = controls(P, ubar[2 * m], z0.x, z0.y);
            if (2 * m + 1 < N) wu[2 * m + 1] = controls(P, ubar[2 * m + 1], z1.x, z1.y);
        } else {
            wu[2 * m] = controls_k(P, bs, lds, L, k, 2 * m, ubar[2 * m], z0.x, z0.y);
            if (2 * m + 1 < N) wu[2 * m + 1] = controls_k(P, bs, lds, L, k, 2 * m + 1, ubar[2 * m + 1], z1.x, z1.y);
        }
    }
    __syncthreads();
    // B. dynamics (first wave) and projection (second wave), serial within each piece
    if (chunk_lane) {
        const int t_end = min((ch + 1) * C, N);
        for (int tau = ch * C; tau < t_end; ++tau) {
            const float2 u = wu[tau];
            const StepConst<float> sc = step_const<MODEL, MathF32>(V, u.x, u.y);
            if constexpr (MODEL == 0) rk4_pair(V, sc, P.dt, st, rear);
            else rk4<MODEL, MathF32>(V, sc, P.dt, st);
            if (!rear) {
                wst[2 * tau] = make_float4(st[0], st[1], st[2], st[3]);
                wst[2 * tau + 1] = make_float4(st[4], st[5], 0.0f, 0.0f);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                prog[ch] = tau + 1;
            }
        }
    } else if (proj_lane) {
        const int t_end = min((pch + 1) * C, N);
        for (int tau = pch * C; tau < t_end; ++tau) {
            NodeAhead<(NPF > 0 ? NPF : 1)> ahead;
            if constexpr (NPF > 0) ahead = read_ahead<NPF>(nodes, bs.W, seg);
            // the dynamics lanes never wait, so this wait ends; if it gives up all the same
            // (bound P.spin_limit) the outputs are unreliable and the status word says so
            for (int spin = 0; prog[pch] <= tau && spin < P.spin_limit; ++spin) __builtin_amdgcn_s_sleep(1);
            if (prog[pch] <= tau) atomicOr(status, SGTP_STATUS_REROLL_GAVE_UP);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            const float4 xy = wst[2 * tau];
            Foot f;
            if constexpr (NPF > 0) f = project_ahead<NPF>(nodes, bs.W, P.max_moves, xy.x, xy.y, seg, ahead);
            else f = project(nodes, bs.W, P.max_moves, xy.x, xy.y, seg);
            seg = f.seg;
            wf[tau] = make_float4(f.s, f.d, f.wL, f.wR);
        }
    }
    __syncthreads();
    // C. outputs, parallel over the horizon
    for (int tau = tid; tau < N; tau += nth) {
        const float4 a = wst[2 * tau], b = wst[2 * tau + 1];
        const float st[6] = {a.x, a.y, a.z, a.w, b.x, b.y};
        const float4 fv = wf[tau];
        const float2 u = wu[tau];
        float *pr = out.pred + (tau + 1) * PRED_STRIDE;
        pr[0] = st[0]; pr[1] = st[1]; pr[2] = fast_cos(st[2]); pr[3] = fast_sin(st[2]);
        pr[4] = fv.x; pr[5] = fv.y; pr[6] = 0.0f; pr[7] = 0.0f;
        if (out.u) out.u[tau] = out.final_shift ? wu[tau + 1 < N ? tau + 1 : N - 1] : u;
        if (out.traj) {
            double *o = out.traj + (size_t)(tau + 1) * 8;
            const double X = st[0], Y = st[1];
            o[0] = rec.ox + rec.c0 * X - rec.s0 * Y;
            o[1] = rec.oy + rec.s0 * X + rec.c0 * Y;
            o[2] = rec.psi0 + (double)st[2];
            o[3] = st[3]; o[4] = st[4]; o[5] = st[5];
            o[6] = rec.s_abs + (double)fv.x;
            o[7] = fv.y;
        }
    }
    if (tid == 0) {
        float *pr = out.pred;
        pr[0] = 0.0f; pr[1] = 0.0f; pr[2] = 1.0f; pr[3] = 0.0f; pr[4] = 0.0f; pr[5] = (float)rec.d0;
        pr[6] = 0.0f; pr[7] = 0.0f;
        if (out.traj) {
            double *o = out.traj;
            o[0] = rec.ox; o[1] = rec.oy; o[2] = rec.psi0; o[3] = bs.vx0; o[4] = bs.vy0; o[5] = bs.om0;
            o[6] = rec.s_abs; o[7] = rec.d0;
        }
        if (out.u_apply) *out.u_apply = wu[0];
    }
    __syncthreads();
}

// ------------------------------------------------------------------------------
// Kernels
// ------------------------------------------------------------------------------
__device__ __forceinline__ int find_item(const ItemDev *items, int n, int tile) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Path-integral accumulation of one wave's samples (update = 1): score S = c + w_viol nu
// (non-finite scores get no weight), weights exp(-(S - S_ref) / lambda) against the
// wave's running reference S_ref, and the weighted sums of the sampled controls,
// regenerated from the same Philox counters.  Lane l holds columns l and l + 64 of
// (a_0, delta_0, a_1, delta_1, ...).
struct PiAcc {
    float S, w, c0, c1;
};

__device__ __forceinline__ void pi_accumulate(const KParams &P, const BlockState &bs, const char *lds,
                                              const LdsLayout &L, uint32_t k, bool valid, const SampleResult &res,
                                              PiAcc &a) {
    const int lane = threadIdx.x & 63;
    float S = res.cost + P.w_viol * res.viol;
    const bool fin = valid && isfinite(S);
    S = fin ? S : INFINITY;
    const float Sw = wave_min_f32(S);
    if (!(Sw < INFINITY)) return;  // uniform over the wave
    const float w = fin ? expf((Sw - S) * P.inv_lambda) : 0.0f;
    const float Sn = fminf(a.S, Sw);
    const float fa = (a.S < INFINITY) ? expf((Sn - a.S) * P.inv_lambda) : 0.0f;
    const float fb = expf((Sn - Sw) * P.inv_lambda);
    a.S = Sn;
    a.w = a.w * fa + wave_sum_f32(w) * fb;
    a.c0 *= fa;
    a.c1 *= fa;
    const float2 *ubar = (const float2 *)(lds + L.ubar);
    for (int m = 0; 2 * m < bs.N; ++m) {
        const uint4 r = philox4x32_10(make_uint4(k, (uint32_t)m, bs.ctr2, bs.ctr3), bs.key0, bs.key1);
        const float2 z0 = gauss_pair(r.x, r.y), z1 = gauss_pair(r.z, r.w);
        const float2 u0 = controls(P, ubar[2 * m], z0.x, z0.y);
        const float2 u1 = (2 * m + 1 < bs.N) ? controls(P, ubar[2 * m + 1], z1.x, z1.y) : make_float2(0.0f, 0.0f);
        const float v[4] = {wave_sum_f32(w * u0.x) * fb, wave_sum_f32(w * u0.y) * fb, wave_sum_f32(w * u1.x) * fb,
                            wave_sum_f32(w * u1.y) * fb};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = 4 * m + j;
            if (lane == (c & 63)) {
                if (c < 64) a.c0 += v[j];
                else a.c1 += v[j];
            }
        }
    }
}

// One tile (spl x BLOCK consecutive samples) of a staged vehicle, then the hand-off:
// the workgroup that finishes the vehicle's last tile (device-scope counter) reads
// the selection and re-rolls it with the tables it holds in LDS.  With the
// path-integral update every tile leaves its weighted partial sums instead, and the
// last workgroup combines them in tile order, adopts the weighted mean sequence and
// rolls it out noise-free.
template <int MODEL, int NDISC, int MAXOPP, int NPF = 0, int LPS = 1, int SPL = 0>
__device__ __forceinline__ void sweep_tile(const LaunchArgs &A, int tile, int item, const BlockState &bs, char *lds,
                                           int *s_last) {
    constexpr int G = SPL ? 64 : 64 / LPS;  // samples per wave (per wave pair when split) = checkpoint group
    constexpr int TS = SPL ? BLOCK / 2 : BLOCK;  // samples per pass of the workgroup (one lane each: LPS = 1)
    const bool rear = LPS == 2 && (threadIdx.x & 1);
    const int vt = SPL ? split_vt(threadIdx.x) : (int)threadIdx.x;
    const bool dyn = SPL && vt < BLOCK / 2;  // the split variant's dynamics lanes
    const int lane = threadIdx.x & 63;
    const bool pi = A.P.update == 1;
    const int t0 = A.items[item].tile0;
    const int n_tiles_item = (item + 1 < A.n_items ? A.items[item + 1].tile0 : A.n_tiles) - t0;
    const int local_tile = tile - t0;
    const int pstride = 2 * A.L.N_max + 2;
    PiAcc pa{INFINITY, 0.0f, 0.0f, 0.0f};
    for (int r = 0; r < A.spl; ++r) {
        const uint32_t k = LPS == 1 ? (uint32_t)((local_tile * A.spl + r) * TS + (vt & (TS - 1)))
                                    : (uint32_t)(local_tile * (BLOCK / 2) + (threadIdx.x >> 1));
        const bool valid = k < (uint32_t)bs.K;
        // (the split variant draws the perturbation on the scoring lane)
        float *nz = (A.dbg_noise && valid && !rear && !dyn) ? A.dbg_noise + (size_t)k * bs.N * 2 : nullptr;
        const SampleResult res =
            run_sample<MODEL, NDISC, MAXOPP, NPF, LPS, SPL>(A.P, bs, lds, A.L, valid ? k : 0u, nz, rear, dyn, A.status);
        unsigned long long key;
        if (dyn) {
            key = KEY_NONE;  // scored by the partner lane
        } else if (pi) {
            const float S = res.cost + A.P.w_viol * res.viol;
            key = valid ? make_key(isfinite(S), isfinite(S) ? S : 0.0f, k) : KEY_NONE;
        } else {
            key = valid ? make_key(res.h, res.h ? res.cost : res.viol, k) : KEY_NONE;
        }
        const unsigned long long wmin = wave_min_u64(key);
        const unsigned long long feas = __ballot(valid && res.h && !rear && !dyn);
        if (lane == 0) {
            if (wmin != KEY_NONE) atomicMin(A.keys + bs.slot, wmin);
            const int cnt = __popcll(feas);
            if (cnt) atomicAdd(A.nfeas + bs.slot, cnt);
        }
        if (pi) {
            pi_accumulate(A.P, bs, lds, A.L, valid ? k : 0u, valid && !dyn, res, pa);
        } else if (SPL) {
            // the scoring wave names its best lane; the two partner lanes export their parts
            int *best = (int *)(lds + A.L.sp_sync) + 4;
            if (!dyn) {
                const unsigned long long b = __ballot(valid && key == wmin);
                if (lane == 0) best[(vt >> 6) & 1] = (wmin != KEY_NONE && b) ? __builtin_ctzll(b) : -1;
            }
            __syncthreads();
            if (valid && lane == best[(vt >> 6) & 1]) {
                float *slot = A.cp_slots + ((size_t)A.items[item].group0 + k / G) * CP_FLOATS;
                if (dyn) {  // states on the dynamics lane; segments and score on the scoring lane
#pragma unroll
                    for (int c = 0; c < ncp_of<NPF>() - 1; ++c)
#pragma unroll
                        for (int i = 0; i < 6; ++i) slot[7 * c + i] = res.cp[c][i];
                } else {
#pragma unroll
                    for (int c = 0; c < ncp_of<NPF>() - 1; ++c) slot[7 * c + 6] = res.cp[c][6];
                    slot[CP_COST] = res.cost;
                    slot[CP_VIOL] = res.viol;
                }
            }
        } else if (valid && key == wmin && !rear) {  // the wave's best sample exports checkpoints and score
            float *slot = A.cp_slots + ((size_t)A.items[item].group0 + k / G) * CP_FLOATS;
#pragma unroll
            for (int c = 0; c < ncp_of<NPF>() - 1; ++c)
#pragma unroll
                for (int i = 0; i < 7; ++i) slot[7 * c + i] = res.cp[c][i];
            slot[CP_COST] = res.cost;
            slot[CP_VIOL] = res.viol;
        }
        if (valid && !rear && !dyn) {
            if (A.dbg_cost) A.dbg_cost[k] = res.cost;
            if (A.dbg_viol) A.dbg_viol[k] = res.viol;
            if (A.dbg_flags) A.dbg_flags[k] = res.flags;
            if (A.dbg_xfinal) {
                const AgentRec &a = A.agents[bs.slot];
                double *o = A.dbg_xfinal + (size_t)k * 6;
                const double X = res.st[0], Y = res.st[1];
                o[0] = a.ox + a.c0 * X - a.s0 * Y;
                o[1] = a.oy + a.s0 * X + a.c0 * Y;
                o[2] = a.psi0 + (double)res.st[2];
                o[3] = res.st[3]; o[4] = res.st[4]; o[5] = res.st[5];
            }
        }
    }
    if (pi) {  // the tile's partial: combine the four waves in order
        float *pw = (float *)(lds + A.L.rr_u);  // [4][2N + 2] (re-roll scratch, free here)
        const int ws = 2 * bs.N + 2, wv = threadIdx.x >> 6;
        if (lane == 0) {
            pw[wv * ws] = pa.S;
            pw[wv * ws + 1] = pa.w;
        }
        if (lane < 2 * bs.N) pw[wv * ws + 2 + lane] = pa.c0;
        if (lane + 64 < 2 * bs.N) pw[wv * ws + 2 + lane + 64] = pa.c1;
        __syncthreads();
        if ((int)threadIdx.x < ws) {
            float Sb = INFINITY;
            for (int w = 0; w < BLOCK / 64; ++w) Sb = fminf(Sb, pw[w * ws]);
            float v = Sb;
            if (threadIdx.x > 0) {
                v = 0.0f;
                for (int w = 0; w < BLOCK / 64; ++w) {
                    const float Sw = pw[w * ws];
                    if (Sw < INFINITY) v += pw[w * ws + threadIdx.x] * expf((Sb - Sw) * A.P.inv_lambda);
                }
            }
            A.pi_part[(size_t)tile * pstride + threadIdx.x] = v;
        }
    }
    // descriptors the hand-off needs, read by every workgroup before the counter
    const ItemDev it = A.items[item];
    const RaceDev R = A.races[it.race];
    const AgentRec rec = A.agents[bs.slot];
    __syncthreads();
    if (threadIdx.x == 0) {
        // release: the workgroup's key, count, slot and partial writes before its count
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        *s_last = atomicAdd(A.counters + bs.slot, 1) == n_tiles_item - 1;
    }
    __syncthreads();
    if (!*s_last) return;
    // acquire: every other workgroup's writes of this vehicle are visible from here
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const unsigned long long key = atomicMin(A.keys + bs.slot, KEY_NONE);  // current value
    const int nfeas = atomicAdd(A.nfeas + bs.slot, 0);
    uint32_t k = (uint32_t)(key & 0x7fffffffu);
    if (k >= (uint32_t)bs.K) k = 0;
    RerollOut out{};
    out.pred = A.pred_out + (size_t)bs.slot * (A.L.N_max + 1) * PRED_STRIDE;
    const bool final_phase = A.final_mode == 2 || (A.final_mode == 1 && it.agent != R.ego);
    if (A.adopt) {
        out.u = (float2 *)(R.u_nom) + (size_t)it.agent * R.N;
        out.traj = R.traj ? R.traj + (size_t)it.agent * (R.N + 1) * 8 : nullptr;
        out.final_shift = final_phase;
        out.u_apply = (final_phase && A.u_apply) ? A.u_apply + bs.slot : nullptr;
    }
    SampleResult res{};
    float pi_min = INFINITY;
    if (pi) {
        // combine the tiles' partials in tile order; the weighted mean replaces the nominal
        float *sums = (float *)(lds + A.L.rr_u);  // [2N + 1]: sum of weights, weighted controls
        const float *pp = A.pi_part + (size_t)t0 * pstride;
        float Smin = INFINITY;
        for (int t = 0; t < n_tiles_item; ++t) Smin = fminf(Smin, pp[(size_t)t * pstride]);
        pi_min = Smin;
        if (Smin < INFINITY) {
            if ((int)threadIdx.x < 2 * bs.N + 1) {
                float v = 0.0f;
                for (int t = 0; t < n_tiles_item; ++t) {
                    const float St = pp[(size_t)t * pstride];
                    if (St < INFINITY) v += pp[(size_t)t * pstride + 1 + threadIdx.x] * expf((Smin - St) * A.P.inv_lambda);
                }
                sums[threadIdx.x] = v;
            }
            __syncthreads();
            float *ub = (float *)(lds + A.L.ubar);
            if ((int)threadIdx.x < 2 * bs.N) ub[threadIdx.x] = sums[1 + threadIdx.x] / sums[0];
        }
        __syncthreads();
        reroll_block<MODEL, NOMINAL, NPF>(A.P, A.L, bs, lds, rec, 0u, out, A.status);
    } else {
        const float *cps = A.cp_slots + ((size_t)it.group0 + k / G) * CP_FLOATS;  // k's lane exported them
        reroll_block<MODEL, WINNER, NPF>(A.P, A.L, bs, lds, rec, k, out, A.status, cps);
        res.cost = cps[CP_COST];
        res.viol = cps[CP_VIOL];
    }
    if (threadIdx.x == 0) {
        if (A.choice) {
            sgtp_choice c;
            c.k = (int)k;
            c.fallback = (key >> 63) ? 1 : 0;
            c.n_feasible = nfeas;
            c.cost = pi ? pi_min : res.cost;
            c.viol = pi ? 0.0f : res.viol;
            A.choice[bs.slot - A.choice_base] = c;
        }
        A.keys[bs.slot] = KEY_NONE;
        A.nfeas[bs.slot] = 0;
        A.counters[bs.slot] = 0;
    }
    __syncthreads();
}

// Tile of workgroup b when workgroups go to the NQ XCDs round-robin (b mod NQ): each XCD
// takes one contiguous range of tiles, so the tiles of a vehicle -- which stage the same
// tables -- mostly share one XCD's L2 instead of all eight.  A bijection on [0, n).
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int x = b % NQ, i = b / NQ, per = n / NQ, rem = n % NQ;
    return x * per + min(x, rem) + i;
}

// Sweep with one workgroup per tile.
template <int MODEL, int NDISC, int MAXOPP, int NPF = 0, int LPS = 1, int SPL = 0>
__global__ void __launch_bounds__(BLOCK, (NPF == 0 && LPS == 1 && SPL == 0) ? 4 : 1) k_sweep(LaunchArgs A) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int s_last;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int item = find_item(A.items, A.n_items, tile);
    BlockState bs;
    stage_block<NDISC>(A, item, bs, lds);
    sweep_tile<MODEL, NDISC, MAXOPP, NPF, LPS, SPL>(A, tile, item, bs, lds, &s_last);
}

// Persistent sweep: a fixed grid of workgroups pulls chunks of tiles from NQ queues
// (its own first, then the others), restaging LDS only when the vehicle changes.
// Every workgroup leaves once all queues are exhausted.
template <int MODEL, int NDISC, int MAXOPP>
// (at least four waves per SIMD, as the one-workgroup-per-tile throughput kernels reach by
// themselves: left alone the queue state takes it to ~200 registers and half that
// occupancy; capped, its spills stay outside the sample loop -- measured +2 % on the
// 256-race batch, where the tuner then prefers it)
__global__ void __launch_bounds__(BLOCK, 4) k_sweep_persistent(LaunchArgs A) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int s_last;
    __shared__ int s_fetch[2];
    BlockState bs;
    int staged = -1;
    const int q0 = blockIdx.x % NQ;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            int first = -1, cnt = 0;
            for (int a = 0; a < NQ; ++a) {
                const int q = (q0 + a) % NQ;
                if (A.q_len[q] == 0) continue;
                const int t = atomicAdd(A.qctr + q, A.chunk);
                if (t < A.q_len[q]) {
                    first = A.q_begin[q] + t;
                    cnt = min(A.chunk, A.q_len[q] - t);
                    break;
                }
            }
            s_fetch[0] = first;
            s_fetch[1] = cnt;
        }
        __syncthreads();
        const int first = s_fetch[0], cnt = s_fetch[1];
        if (first < 0) break;
        for (int t = first; t < first + cnt; ++t) {
            const int item = find_item(A.items, A.n_items, t);
            if (item != staged) {
                __syncthreads();
                stage_block<NDISC>(A, item, bs, lds);
                staged = item;
            }
            sweep_tile<MODEL, NDISC, MAXOPP>(A, t, item, bs, lds, &s_last);
        }
    }
}

// Setup of every vehicle: global Frenet projection of the current state,
// unwrapped progress, local frame, raceline window, reference states
// (Sec. III-A: s^r recursion over v^r) and the noise-free rollout of the
// nominal sequence (initial prediction).  Two workgroups per vehicle run at once
// (grid 2 x n_items): the first writes the vehicle record, the window and the
// reference states, the second rolls out the nominal; both compute the projection
// and the frame, with the same bits.  The second may read the unwrapped progress
// before or after the first has updated it; both give the same lap count.
template <int MODEL>
__global__ void __launch_bounds__(BLOCK) k_setup(LaunchArgs A, int w_limit) {
    extern __shared__ __align__(16) char lds[];
    __shared__ double red_v[BLOCK];
    __shared__ long long red_i[BLOCK];
    __shared__ double sh[8];
    __shared__ long long shl[4];
    __shared__ AgentRec s_rec;
    const bool roller = (int)blockIdx.x >= A.n_items;
    const ItemDev it = A.items[roller ? blockIdx.x - A.n_items : blockIdx.x];
    const RaceDev R = A.races[it.race];
    const TrackDev T = A.tracks[R.track];
    const double *xs = R.x + (size_t)it.agent * 6;
    const double px = xs[0], py = xs[1];
    const int tid = threadIdx.x;
    const long long n = T.n;
    const long long nseg = T.closed ? n : n - 1;
    if (blockIdx.x == 0 && A.qreset)  // (a first workgroup)
        for (int i = tid; i < A.n_qreset; i += BLOCK) A.qreset[i] = 0;

    auto node = [&](long long i, double *o) {  // unwrapped node access (float64 row)
        long long lap = 0, b = i;
        if (T.closed) {
            lap = i / n;
            if (i - lap * n < 0) --lap;
            b = i - lap * n;
        } else {
            b = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
        }
        const double *r = T.nodes + (size_t)b * NODE_STRIDE;
#pragma unroll
        for (int c = 0; c < NODE_STRIDE; ++c) o[c] = r[c];
        o[2] += (double)lap * T.psi_lap;
        o[8] += (double)lap * T.length;
    };
    auto ahead = [&](long long i) {
        double nd[NODE_STRIDE];
        node(i, nd);
        return (px - nd[0]) * nd[4] - (py - nd[1]) * nd[3];
    };
    auto foot = [&](long long i, double *o /* s, d, t, half width, psi_ref, v_ref */) {
        double a[NODE_STRIDE], b[NODE_STRIDE];
        node(i, a);
        node(i + 1, b);
        const double rx = px - a[0], ry = py - a[1];
        const double Dx = b[0] - a[0], Dy = b[1] - a[1];
        const double dnx = b[3] - a[3], dny = b[4] - a[4];
        const double Cc = rx * a[4] - ry * a[3];
        const double Bc = (rx * dny - ry * dnx) - (Dx * a[4] - Dy * a[3]);
        const double Ac = -(Dx * dny - Dy * dnx);
        double disc = Bc * Bc - 4.0 * Ac * Cc;
        if (disc < 0.0) disc = 0.0;
        const double den = -Bc - copysign(sqrt(disc), Bc);
        double t = (den != 0.0) ? 2.0 * Cc / den : 0.0;
        if (!(t >= 0.0)) t = 0.0;
        if (t > 1.0) t = 1.0;
        const double cx = a[0] + t * Dx, cy = a[1] + t * Dy;
        const double nx = a[3] + t * dnx, ny = a[4] + t * dny;
        o[0] = a[8] + t * (b[8] - a[8]);
        o[1] = ((px - cx) * nx + (py - cy) * ny) / sqrt(nx * nx + ny * ny);
        o[2] = t;
        o[3] = 0.5 * ((a[5] + t * (b[5] - a[5])) + (a[6] + t * (b[6] - a[6])));
        o[4] = a[2] + t * (b[2] - a[2]);
        o[5] = a[7] + t * (b[7] - a[7]);
    };
    auto block_argmin = [&](double v, long long i) {  // smallest v, lowest index on ties (i < 0: none)
        red_v[tid] = v;
        red_i[tid] = i;
        __syncthreads();
        for (int w = BLOCK / 2; w > 0; w >>= 1) {
            if (tid < w) {
                const double v2 = red_v[tid + w];
                const long long i2 = red_i[tid + w];
                if (i2 >= 0 && (red_i[tid] < 0 || v2 < red_v[tid] || (v2 == red_v[tid] && i2 < red_i[tid]))) {
                    red_v[tid] = v2;
                    red_i[tid] = i2;
                }
            }
            __syncthreads();
        }
        const long long r = red_i[0];
        __syncthreads();
        return r;
    };

    // 1. global projection: smallest |d| among enclosing segments, lowest index on ties.
    //    Each thread takes a run of consecutive segments (its node reads, one more than
    //    its segments, are issued UNR at a time); runs ascend with the thread index.
    double best = INFINITY;
    long long bi = -1;
    {
        constexpr int UNR = 16;
        const long long per = (nseg + BLOCK - 1) / BLOCK;
        const long long i_lo = (long long)tid * per;
        const long long i_hi = i_lo + per < nseg ? i_lo + per : nseg;
        double gprev = i_lo < i_hi ? ahead(i_lo) : 0.0;
        for (long long i0 = i_lo; i0 < i_hi; i0 += UNR) {
            double g[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) g[u] = i0 + u < i_hi ? ahead(i0 + u + 1) : 0.0;
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const long long i = i0 + u;
                const double g0 = u == 0 ? gprev : g[u - 1];
                if (i < i_hi && g0 >= 0.0 && g[u] <= 0.0) {
                    double o[6];
                    foot(i, o);
                    const double ad = fabs(o[1]);
                    if (ad < best) {
                        best = ad;
                        bi = i;
                    }
                }
            }
            gprev = g[UNR - 1];
        }
    }
    long long seg = block_argmin(best, bi);
    if (seg < 0) {  // no enclosing segment: the one starting at the nearest node
        best = INFINITY;
        bi = -1;
        for (long long i = tid; i < nseg; i += BLOCK) {
            double nd[NODE_STRIDE];
            node(i, nd);
            const double dd = (px - nd[0]) * (px - nd[0]) + (py - nd[1]) * (py - nd[1]);
            if (dd < best) {
                best = dd;
                bi = i;
            }
        }
        seg = block_argmin(best, bi);
    }

    // 2. unwrapped progress, frame and window extent
    if (tid == 0) {
        double o[6];
        foot(seg, o);
        double s = o[0];
        const double sp = R.s_abs[it.agent];
        if (T.closed && isfinite(sp)) {
            const double lap = rint((sp - s) / T.length);
            seg += (long long)lap * n;
            s += lap * T.length;
        }
        const double psi0 = xs[2];
        const double c0 = cos(psi0), s0 = sin(psi0);
        const double vx = xs[3] > 0.0 ? xs[3] : 0.0, vy = xs[4];
        const double v = sqrt(vx * vx + vy * vy);
        const double Th = (double)R.N * (double)A.P.dt;
        const double lam = (double)R.v_scale[it.agent];
        const double reach_samples = v * Th + 0.5 * (double)(A.P.a_max > 0.f ? A.P.a_max : 0.f) * Th * Th;
        const double reach_ref = (lam > 1.0 ? lam : 1.0) * T.vmax * Th;
        const double reach = (reach_samples > reach_ref ? reach_samples : reach_ref) + 10.0;
        long long W = WIN_BACK + (long long)ceil(T.inner_factor * reach / T.ds_min) + 8;
        if (W > w_limit) W = w_limit;
        long long win0 = seg - WIN_BACK;
        if (!T.closed) {
            if (win0 < 0) win0 = 0;
            if (W > n - win0) W = n - win0;
        }
        AgentRec rec;
        rec.ox = px; rec.oy = py; rec.psi0 = psi0; rec.c0 = c0; rec.s0 = s0;
        rec.s_abs = s; rec.d0 = o[1];
        rec.half_w = o[3]; rec.psi_ref = o[4]; rec.v_ref = o[5];
        rec.seg_abs = seg; rec.win0 = win0;
        rec.win_n = (int)W; rec.seg_loc = (int)(seg - win0);
        rec.vx = (float)xs[3]; rec.vy = (float)xs[4]; rec.om = (float)xs[5];
        rec.lam = R.v_scale[it.agent];
        s_rec = rec;
        sh[0] = c0; sh[1] = s0; sh[2] = psi0; sh[3] = s; sh[4] = lam;
        shl[0] = win0; shl[1] = W; shl[2] = seg - win0;
        if (!roller) {
            R.s_abs[it.agent] = s;
            A.agents[it.slot] = rec;
            A.keys[it.slot] = KEY_NONE;
            A.nfeas[it.slot] = 0;
            A.counters[it.slot] = 0;
        }
    }
    __syncthreads();
    const double c0 = sh[0], s0 = sh[1], psi0 = sh[2], sa = sh[3], lam = sh[4];
    const long long win0 = shl[0], W = shl[1], segl = shl[2];
    if (roller) {
        // stage the float32 window and the nominal, roll the nominal out (predictions)
        float4 *nodes_l = (float4 *)(lds + A.L.nodes);
        for (long long w = tid; w < W; w += BLOCK) {
            double nd[NODE_STRIDE];
            node(win0 + w, nd);
            const double dx = nd[0] - px, dy = nd[1] - py;
            const double nxl = c0 * nd[3] + s0 * nd[4], nyl = -s0 * nd[3] + c0 * nd[4];
            nodes_l[2 * w] = make_float4((float)(c0 * dx + s0 * dy), (float)(-s0 * dx + c0 * dy), (float)nxl, (float)nyl);
            nodes_l[2 * w + 1] = make_float4((float)nd[5], (float)nd[6], (float)(nd[8] - sa), 0.0f);
        }
        float2 *ubar = (float2 *)(lds + A.L.ubar);
        const float2 *un = (const float2 *)(R.u_nom) + (size_t)it.agent * R.N;
        for (int t = tid; t < R.N; t += BLOCK) ubar[t] = un[t];
        __syncthreads();
        BlockState bs{};
        bs.slot = it.slot; bs.race = it.race; bs.agent = it.agent; bs.N = R.N; bs.n_tail = R.n_tail; bs.K = R.K;
        bs.n_opp = 0; bs.W = (int)W; bs.seg0 = (int)segl;
        bs.vx0 = (float)xs[3]; bs.vy0 = (float)xs[4]; bs.om0 = (float)xs[5];
        bs.inv_n_tail = 1.0f / (float)R.n_tail; bs.w_game = 0.0f;
        const AgentRec rec = s_rec;
        RerollOut out{};
        out.pred = A.pred_out + (size_t)it.slot * (A.L.N_max + 1) * PRED_STRIDE;
        reroll_block<MODEL, NOMINAL, 6>(A.P, A.L, bs, lds, rec, 0u, out, A.status);
        return;
    }

    // 3. raceline window in the local frame to HBM: A = (x, y, nx, ny), B = (wL, wR, s - s_abs, 0);
    //    arc length and reference speed of the window nodes to LDS (float64) for the recursion
    float4 *dst = (float4 *)(A.win + (size_t)it.slot * WIN_MAX * 2);
    double2 *sv = (double2 *)(lds + A.L.nodes);  // reused below for the float32 window
    for (long long w = tid; w < W; w += BLOCK) {
        double nd[NODE_STRIDE];
        node(win0 + w, nd);
        const double dx = nd[0] - px, dy = nd[1] - py;
        const double nxl = c0 * nd[3] + s0 * nd[4], nyl = -s0 * nd[3] + c0 * nd[4];
        dst[2 * w] = make_float4((float)(c0 * dx + s0 * dy), (float)(-s0 * dx + c0 * dy), (float)nxl, (float)nyl);
        dst[2 * w + 1] = make_float4((float)nd[5], (float)nd[6], (float)(nd[8] - sa), 0.0f);
        sv[w] = make_double2(nd[8], nd[7]);
    }
    __syncthreads();
    // 4. s^r recursion (thread 0, LDS only): s^r_{t+1} = s^r_t + dt lam v^r(s^r_t)
    double *srs = (double *)(lds + A.L.rr_st);  // N values
    long long *segs = (long long *)(lds + A.L.rr_t);
    if (tid == 0) {
        long long h = segl;
        double sr = sa;
        const double dt = (double)A.P.dt;
        auto seek = [&](double q) {  // segment of the window holding q (clamped to the window)
            while (q < sv[h].x && h > 0) --h;
            while (h + 2 < W && q >= sv[h + 1].x) ++h;
        };
        for (int t = 0; t < R.N; ++t) {
            seek(sr);
            double tt = (sr - sv[h].x) / (sv[h + 1].x - sv[h].x);
            tt = tt < 0.0 ? 0.0 : (tt > 1.0 ? 1.0 : tt);
            const double v = sv[h].y + tt * (sv[h + 1].y - sv[h].y);
            sr = sr + dt * lam * v;
            seek(sr);
            srs[t] = sr;
            segs[t] = h;
        }
    }
    __syncthreads();
    // 5. reference states x^r(s^r_t), t = 1..N, in the local frame (heading shifted by a
    //    multiple of 2 pi so it starts near the vehicle's heading)
    float4 *xr = (float4 *)(A.xref + (size_t)it.slot * A.L.N_max);
    for (int t = tid; t < R.N; t += BLOCK) {
        const long long h = segs[t];
        double a[NODE_STRIDE], b[NODE_STRIDE];
        node(win0 + h, a);
        node(win0 + h + 1, b);
        double tt = (srs[t] - a[8]) / (b[8] - a[8]);
        tt = tt < 0.0 ? 0.0 : (tt > 1.0 ? 1.0 : tt);
        const double x = a[0] + tt * (b[0] - a[0]), y = a[1] + tt * (b[1] - a[1]);
        const double ps = a[2] + tt * (b[2] - a[2]), v = a[7] + tt * (b[7] - a[7]);
        double a0[NODE_STRIDE], b0[NODE_STRIDE];
        node(win0 + segs[0], a0);
        node(win0 + segs[0] + 1, b0);
        double t0 = (srs[0] - a0[8]) / (b0[8] - a0[8]);
        t0 = t0 < 0.0 ? 0.0 : (t0 > 1.0 ? 1.0 : t0);
        const double ps0 = a0[2] + t0 * (b0[2] - a0[2]);
        const double shift = 6.283185307179586 * rint((ps0 - psi0) / 6.283185307179586);
        const double dx = x - px, dy = y - py;
        const float4 q = make_float4((float)(c0 * dx + s0 * dy), (float)(-s0 * dx + c0 * dy),
                                     (float)(ps - psi0 - shift), (float)(lam * v));
        xr[t] = q;
    }
}

// ------------------------------------------------------------------------------
// Learned proposal: features of every vehicle and the proposal tables from the
// network outputs (the network itself is in mlp.hip)
// ------------------------------------------------------------------------------
constexpr int FEAT_DIM = 50;
constexpr int FEAT_OPP = 4;
constexpr int FEAT_CURV = 20;
constexpr double FEAT_CURV_DS = 5.0;
constexpr float MLP_A_SCALE = 4.0f, MLP_D_SCALE = 0.2f, MLP_LS_MIN = -4.0f, MLP_LS_MAX = 1.0f;

// Unwrapped arc length and curvature of node i (laps add the track length).
__device__ __forceinline__ void node_s_kappa(const TrackDev &T, long long i, double &s, double &kappa) {
    const long long n = T.n;
    long long lap = 0, b = i;
    if (T.closed) {
        lap = i / n;
        if (i - lap * n < 0) --lap;
        b = i - lap * n;
    } else {
        b = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
    }
    const double *r = T.nodes + (size_t)b * NODE_STRIDE;
    s = r[8] + (double)lap * T.length;
    kappa = r[9];
}

__device__ void node_row(const TrackDev &T, long long i, double *o) {  // unwrapped node access
    const long long n = T.n;
    long long lap = 0, b = i;
    if (T.closed) {
        lap = i / n;
        if (i - lap * n < 0) --lap;
        b = i - lap * n;
    } else {
        b = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
    }
    const double *r = T.nodes + (size_t)b * NODE_STRIDE;
#pragma unroll
    for (int c = 0; c < NODE_STRIDE; ++c) o[c] = r[c];
    o[2] += (double)lap * T.psi_lap;
    o[8] += (double)lap * T.length;
}

// One 64-thread block per vehicle: thread 0 writes the ego (6) and the 4 nearest
// opponents by |s_j - s_i| (6 each, zero when absent); threads 1..20 the curvature
// 5..100 m ahead (20), each locating its segment (the one whose node arc lengths
// bracket the query) by bisection.  Same definitions as the oracle's features.
__global__ void __launch_bounds__(64) k_features(LaunchArgs A, float *X) {
    const int i = blockIdx.x;
    if (i >= A.n_items) return;
    const int tid = threadIdx.x;
    const ItemDev it = A.items[i];
    const RaceDev R = A.races[it.race];
    const AgentRec me = A.agents[it.slot];
    const TrackDev T = A.tracks[R.track];
    const double *xi = R.x + (size_t)it.agent * 6;
    float *f = X + (size_t)it.slot * FEAT_DIM;
    if (tid == 0) {
        for (int c = 0; c < 6 + 6 * FEAT_OPP; ++c) f[c] = 0.0f;
        f[0] = (float)(me.d0 / me.half_w);
        f[1] = (float)remainder(xi[2] - me.psi_ref, 6.283185307179586);
        f[2] = (float)(xi[3] / 30.0);
        f[3] = (float)(xi[4] / 5.0);
        f[4] = (float)xi[5];
        f[5] = (float)((xi[3] - me.v_ref) / 10.0);
        unsigned used = 0;
        for (int m = 0; m < FEAT_OPP; ++m) {
            int best = -1;
            double bd = INFINITY;
            for (int j = 0; j < R.n_agents; ++j) {
                if (j == it.agent || (used >> j) & 1u) continue;
                const double dd = fabs(A.agents[R.slot0 + j].s_abs - me.s_abs);
                if (dd < bd) {
                    bd = dd;
                    best = j;
                }
            }
            if (best < 0) break;
            used |= 1u << best;
            const AgentRec o = A.agents[R.slot0 + best];
            const double *xj = R.x + (size_t)best * 6;
            float *g = f + 6 + 6 * m;
            g[0] = (float)((o.s_abs - me.s_abs) / 20.0);
            g[1] = (float)((o.d0 - me.d0) / me.half_w);
            g[2] = (float)remainder(xj[2] - xi[2], 6.283185307179586);
            g[3] = (float)((xj[3] - xi[3]) / 10.0);
            g[4] = (float)(xj[4] / 5.0);
            g[5] = 1.0f;
        }
    } else if (tid <= FEAT_CURV) {
        const double sq = me.s_abs + FEAT_CURV_DS * tid;
        // bracket: the vehicle's segment up to its index plus the reach over the shortest segment
        long long lo = me.seg_abs;
        long long hi = lo + (long long)ceil(FEAT_CURV_DS * FEAT_CURV / T.ds_min) + 2;
        if (!T.closed) {
            lo = lo < 0 ? 0 : (lo > T.n - 2 ? T.n - 2 : lo);
            hi = hi > T.n - 2 ? T.n - 2 : hi;
        }
        double s_lo, k_lo;
        node_s_kappa(T, lo, s_lo, k_lo);
        // largest h in [lo, hi] with s(h) <= sq (lo itself when sq < s(lo))
        while (lo < hi) {
            const long long mid = (lo + hi + 1) >> 1;
            double s_m, k_m;
            node_s_kappa(T, mid, s_m, k_m);
            if (s_m <= sq) lo = mid;
            else hi = mid - 1;
        }
        double sa, ka, sb, kb;
        node_s_kappa(T, lo, sa, ka);
        node_s_kappa(T, lo + 1, sb, kb);
        double t = (sq - sa) / (sb - sa);
        t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        f[6 + 6 * FEAT_OPP + tid - 1] = (float)(20.0 * (ka + t * (kb - ka)));
    }
}

// Network outputs (rows = vehicles in slot order, ld floats each, 4 per horizon step)
// -> proposal table of every race: mu = scale o (plus the nominal control when
// residual), sigma = sigma_plain exp(clamp(o)).
__global__ void k_proposal(const RaceDev *races, const ItemDev *items, int n_items, const float *out, int ld,
                           float sig_a, float sig_d, int residual) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = e / SGTP_MAX_N, tau = e % SGTP_MAX_N;
    if (i >= n_items) return;
    const ItemDev it = items[i];
    const RaceDev R = races[it.race];
    if (tau >= R.N || !R.prop) return;
    const float *o = out + (size_t)it.slot * ld + 4 * tau;
    const float o2 = fminf(fmaxf(o[2], MLP_LS_MIN), MLP_LS_MAX), o3 = fminf(fmaxf(o[3], MLP_LS_MIN), MLP_LS_MAX);
    float4 *dst = (float4 *)R.prop + (size_t)it.agent * R.N + tau;
    float2 base = make_float2(0.0f, 0.0f);
    if (residual) base = ((const float2 *)R.u_nom)[(size_t)it.agent * R.N + tau];
    *dst = make_float4(base.x + MLP_A_SCALE * o[0], base.y + MLP_D_SCALE * o[1], sig_a * expf(o2), sig_d * expf(o3));
}

// Advance the Philox counter word of every race (planning-step index).
// The Gaussian transform on given words (instrumentation: checks of the float32 spec).
__global__ void k_gauss_pairs(const uint32_t *re, const uint32_t *ro, float2 *out, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = gauss_pair(re[i], ro[i]);
}

// Descriptor image of a one-vehicle call passed by value and written to device memory
// (the allocation-free entry point: no host staging buffer, no copy from the host).
constexpr int NOALLOC_MAX_ITEMS = SGTP_MAX_AGENTS;
struct DescImage {
    RaceDev race;
    ItemDev all[NOALLOC_MAX_ITEMS];
    ItemDev one;
    int n_all;
};
__global__ void k_write_desc(DescImage img, RaceDev *races, ItemDev *all, ItemDev *one) {
    const int t = threadIdx.x;
    if (t == 0) races[0] = img.race;
    if (t < img.n_all) all[t] = img.all[t];
    if (t == 0) one[0] = img.one;
}

__global__ void k_bump_step(RaceDev *races, int n_races) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_races) races[i].plan_step += 1u;
}

// Closed loop: one float64 RK4 interval per vehicle.  With bump != NULL (a plan's step)
// the thread of each race's first vehicle also advances the race's planning-step counter.
template <int MODEL>
__global__ void k_advance(const RaceDev *races, const ItemDev *items, int n_items, const float2 *u, VehConst<double> V,
                          double dt, RaceDev *bump) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    const ItemDev it = items[i];
    const RaceDev R = races[it.race];
    if (bump && it.agent == 0) bump[it.race].plan_step = R.plan_step + 1u;
    double *x = R.x + (size_t)it.agent * 6;
    double s[6];
    for (int c = 0; c < 6; ++c) s[c] = x[c];
    const float2 ui = u[it.slot];
    const StepConst<double> sc = step_const<MODEL, MathF64>(V, (double)ui.x, (double)ui.y);
    rk4<MODEL, MathF64>(V, sc, dt, s);
    for (int c = 0; c < 6; ++c) x[c] = s[c];
}

}  // namespace

// ==============================================================================
// Allocation-free best response (sgtp_rollout_cost_noalloc): every scratch buffer of
// its kernels -- vehicle records, raceline windows, reference states, predictions,
// selection keys and counters, checkpoint slots and the call's descriptors -- lies in
// one static device array, at most SGTP_NOALLOC_MAX_K samples and SGTP_MAX_AGENTS
// vehicles, about 1.5 MB per GPU.  Host code never uses the array's name as an
// address: the address of each device's copy is taken once per device, when a context
// is created there (map_scratch), and that pointer is what the kernels receive.
// ==============================================================================
namespace {
struct NoallocLayout {
    size_t agents, win, xref, pred0, pred1, keys, nfeas, counters, cp, races, all, one, total;
};
constexpr size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr NoallocLayout noalloc_layout() {
    NoallocLayout S{};
    size_t o = 0;
    auto take = [&o](size_t bytes) {
        const size_t r = o;
        o += al256(bytes);
        return r;
    };
    S.agents = take(sizeof(AgentRec) * SGTP_MAX_AGENTS);
    S.win = take(sizeof(float4) * 2 * WIN_MAX * SGTP_MAX_AGENTS);
    S.xref = take(sizeof(float4) * SGTP_MAX_N * SGTP_MAX_AGENTS);
    S.pred0 = take(sizeof(float) * PRED_STRIDE * (SGTP_MAX_N + 1) * SGTP_MAX_AGENTS);
    S.pred1 = take(sizeof(float) * PRED_STRIDE * (SGTP_MAX_N + 1) * SGTP_MAX_AGENTS);
    S.keys = take(sizeof(unsigned long long) * SGTP_MAX_AGENTS);
    S.nfeas = take(sizeof(int) * SGTP_MAX_AGENTS);
    S.counters = take(sizeof(int) * SGTP_MAX_AGENTS);
    // checkpoint slots of one vehicle's samples in groups of 32 (the pair variant's groups)
    S.cp = take(sizeof(float) * CP_FLOATS * (SGTP_NOALLOC_MAX_K / 32));
    S.races = take(sizeof(RaceDev));
    S.all = take(sizeof(ItemDev) * NOALLOC_MAX_ITEMS);
    S.one = take(sizeof(ItemDev));
    S.total = o;
    return S;
}
}  // namespace

static __device__ __align__(256) char scratch[noalloc_layout().total];

// ==============================================================================
// Host side: context, validation, launches, C ABI
// ==============================================================================
struct TrackHost {
    double *d_nodes = nullptr;
    int n = 0, closed = 0;
    double length = 0, psi_lap = 0, ds_min = 0, vmax = 0, inner_factor = 1;
};

// Autotuner cache key: model, discs, opponent bucket, longest horizon, log2 of the total
// samples, log2 of the race count, update rule, IBR sweeps (the device is the context's
// own).
using TuneKey = std::array<long long, 8>;
struct TuneEntry {
    sgtp_plan_options opt;
    double ms;
};

struct sgtp_ctx {
    int device = 0;
    std::map<TuneKey, TuneEntry> tune_cache;  // schedules found by sgtp_autotune
    int max_agents = 0, max_N = 0, max_races = 0, max_nodes = 0;
    std::string err;
    TrackHost tracks[MAX_TRACKS];
    TrackDev *d_tracks = nullptr;
    AgentRec *d_agents = nullptr;
    float4 *d_win = nullptr;
    float4 *d_xref = nullptr;
    float *d_pred[2] = {nullptr, nullptr};
    unsigned long long *d_keys = nullptr;
    int *d_nfeas = nullptr;
    int *d_counters = nullptr;
    float *d_cp = nullptr;     // checkpoint slots, CP_FLOATS per 64-sample group
    long long max_groups = 0;
    float *d_pi = nullptr;     // path-integral partial sums per tile (sgtp_ctx_enable_path_integral)
    long long pi_tiles = 0;
    int *d_status = nullptr;   // SGTP_STATUS_* bits raised by the kernels (read by sgtp_ctx_status)
    int spin_limit = 1 << 22;  // polls of a bounded LDS wait before it gives up
    // descriptor uploads: pinned ring, each slot guarded by an event
    static constexpr int RING = 8;
    char *h_stage[RING] = {};
    hipEvent_t stage_ev[RING] = {};
    bool stage_used[RING] = {};
    int ring_pos = 0;
    char *d_desc = nullptr;  // [RING][desc_bytes]
    size_t desc_bytes = 0;
    // instrumentation
    bool timing = false;
    std::vector<hipEvent_t> ev_pairs;
    std::vector<long long> ev_work;
    double total_ms = 0;
    long long launches = 0, sample_steps = 0;
};

namespace {

// The address of each device's copy of `scratch`, taken once per device with that device
// current (at context creation); host code passes these pointers, never the array's name.
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

int map_scratch(int dev) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return SGTP_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return SGTP_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SGTP_EDEVICE;
    g_scratch_ptr[dev] = (char *)ptr;
    return SGTP_OK;
}

char *scratch_of(int dev) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[dev];
}

int fail(sgtp_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) return fail(ctx, SGTP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

KParams make_kparams(const sgtp_params *p) {
    KParams k{};
    k.model = p->model;
    k.n_disc = p->n_disc;
    k.max_moves = p->max_moves;
    k.dt = p->dt;
    k.half_dt = 0.5f * p->dt;
    k.dt6 = p->dt / 6.0f;
    k.a_min = p->a_min; k.a_max = p->a_max; k.d_min = p->d_min; k.d_max = p->d_max;
    k.sigma_a = p->sigma_a; k.sigma_d = p->sigma_d;
    k.Q0 = p->Q[0]; k.Q1 = p->Q[1]; k.Q2 = p->Q[2]; k.Q3 = p->Q[3];
    k.R0 = p->R[0]; k.R1 = p->R[1]; k.S0 = p->S[0]; k.S1 = p->S[1];
    k.w_game = p->w_game; k.w_contest = p->w_contest; k.w_long = p->w_long; k.w_block = p->w_block;
    k.w_safety = p->w_safety; k.s_contest = p->s_contest; k.s_role = p->s_role; k.eps_alpha = p->eps_alpha;
    k.g_safe = p->g_safe; k.m_bd = p->m_bd; k.d_col = p->d_col;
    const double cap = std::max((double)p->g_safe, (double)p->d_col);
    k.cap2 = (float)(cap * cap);
    double offmax = 0;
    for (int i = 0; i < 4; ++i) {
        k.off[i] = (i < p->n_disc) ? p->disc_off[i] : 0.0f;
        if (i < p->n_disc) offmax = std::max(offmax, (double)std::fabs(p->disc_off[i]));
    }
    // a pair of discs can only come closer than cap when the CoGs are within cap + 2 max|offset|
    const double sk = cap + 2.0 * offmax + 1e-3;
    k.skip2 = (float)(sk * sk);
    const double L = (double)p->lf + (double)p->lr;
    k.lf = p->lf; k.lr = p->lr;
    const double muFzf = (double)p->mu * p->m * p->g * p->lr / L, muFzr = (double)p->mu * p->m * p->g * p->lf / L;
    k.kf_m = (float)(muFzf / p->m);
    k.kf_Iz = (float)(muFzf * p->lf / p->Iz);
    k.kr_m = (float)(muFzr / p->m);
    k.kr_Iz = (float)(muFzr * p->lr / p->Iz);
    k.B = p->B; k.C = p->C; k.v_eps = p->v_eps;
    k.C_rev = (float)((double)p->C / (2.0 * M_PI));
    k.lr_over_L = (float)(p->lr / L);
    k.inv_lr = (float)(1.0 / p->lr);
    k.update = p->update;
    k.inv_lambda = p->update == 1 ? (float)(1.0 / (double)p->mppi_lambda) : 0.0f;
    k.w_viol = p->mppi_w_viol;
    k.pred_sig_lon = p->pred_sig_lon;
    k.pred_sig_lat = p->pred_sig_lat;
    return k;
}

VehConst<double> make_veh64(const sgtp_params *p) {
    VehConst<double> V;
    const double L = (double)p->lf + (double)p->lr;
    V.lf = p->lf; V.lr = p->lr;
    const double muFzf = (double)p->mu * p->m * p->g * p->lr / L, muFzr = (double)p->mu * p->m * p->g * p->lf / L;
    V.kf_m = muFzf / p->m;
    V.kf_Iz = muFzf * p->lf / p->Iz;
    V.kr_m = muFzr / p->m;
    V.kr_Iz = muFzr * p->lr / p->Iz;
    V.B = p->B; V.C = p->C; V.v_eps = p->v_eps; V.lr_over_L = p->lr / L; V.inv_lr = 1.0 / p->lr;
    V.Cs = p->C;
    return V;
}

int check_params(sgtp_ctx *c, const sgtp_params *p) {
    if (!p) return fail(c, SGTP_EINVAL, "params is NULL");
    if (p->model != 0 && p->model != 1) return fail(c, SGTP_EINVAL, "model must be 0 or 1");
    if (p->n_disc != 1 && p->n_disc != 3) return fail(c, SGTP_EINVAL, "n_disc must be 1 or 3");
    if (!(p->dt > 0.f) || !(p->a_min <= p->a_max) || !(p->d_min <= p->d_max))
        return fail(c, SGTP_EINVAL, "bad dt or control bounds");
    if (p->max_moves < 1 || p->max_moves > 1024) return fail(c, SGTP_EINVAL, "max_moves out of range");
    if (!(p->m > 0.f) || !(p->Iz > 0.f) || !(p->lf > 0.f) || !(p->lr > 0.f) || !(p->v_eps > 0.f))
        return fail(c, SGTP_EINVAL, "vehicle constants must be positive");
    if (!(p->pred_sig_lon >= 0.f) || !(p->pred_sig_lat >= 0.f) || !std::isfinite(p->pred_sig_lon) ||
        !std::isfinite(p->pred_sig_lat))
        return fail(c, SGTP_EINVAL, "prediction perturbation scales must be finite and >= 0");
    if (p->update != 0 && p->update != 1) return fail(c, SGTP_EINVAL, "update must be 0 or 1");
    if (p->update == 1) {
        if (!(p->mppi_lambda > 0.f) || !std::isfinite(p->mppi_lambda) || !(p->mppi_w_viol >= 0.f) ||
            !std::isfinite(p->mppi_w_viol))
            return fail(c, SGTP_EINVAL, "path-integral temperature must be positive, violation weight >= 0");
        if (!c->d_pi) return fail(c, SGTP_EINVAL, "path-integral update not enabled on this context");
    }
    return SGTP_OK;
}

struct Plan {  // host image of one launch sequence's descriptors
    std::vector<RaceDev> races;
    std::vector<ItemDev> all, ego, one;
    int N_max = 0, n_opp_max = 0, w_max = 0, agents_total = 0;
    int tiles_all = 0, tiles_ego = 0;
    int lps = 1;          // lanes per sample
    int split = 0;        // two waves per sample
    int tile_samples = 0;  // samples per tile: BLOCK x samples per lane / lanes per sample
};

LdsLayout make_layout(const Plan &pl, int maxopp, int ndisc);
int maxopp_bucket(int n_opp);
constexpr int LDS_BUDGET = 58 * 1024;

int build_plan_once(sgtp_ctx *c, const sgtp_params *p, const sgtp_race *races, int n_races, int spl, Plan &pl,
                    int one_agent, bool allow_split, bool ctx_limits) {
    if (!races || n_races < 1) return fail(c, SGTP_EINVAL, "no races");
    if (ctx_limits && n_races > c->max_races) return fail(c, SGTP_ESHAPE, "n_races exceeds the context");
    // launches of about one wave per SIMD or fewer (at most 3 opponents, one sample per
    // lane): the split variant where its rings fit in LDS, else the pair variant (dynamic
    // model, feasibility selection); both measured faster than one lane per sample there,
    // the split one the faster of the two
    {
        long long samples = 0;
        int nopp = 0;
        for (int r = 0; r < n_races; ++r) {
            samples += (long long)std::max(races[r].K, 0) * std::max(races[r].n_agents, 0);
            nopp = std::max(nopp, races[r].n_agents - 1);
        }
        pl.split = (allow_split && spl == 1 && nopp <= 3 && samples <= SPLIT_MAX_SAMPLES) ? 1 : 0;
        pl.lps = (!pl.split && spl == 1 && p->model == 0 && p->update == 0 && nopp <= 3 &&
                  samples <= LPS2_MAX_SAMPLES) ? 2 : 1;
        pl.tile_samples = BLOCK * spl / (pl.split ? 2 : pl.lps);
    }
    const int gsz = 64 / pl.lps;  // samples per wave (per wave pair when split) = checkpoint group
    int slot = 0;
    long long group_total = 0;
    double wneed = 0;
    for (int r = 0; r < n_races; ++r) {
        const sgtp_race &s = races[r];
        if (s.n_agents < 1 || s.n_agents > SGTP_MAX_AGENTS) return fail(c, SGTP_EINVAL, "n_agents out of range");
        if (s.ego < 0 || s.ego >= s.n_agents) return fail(c, SGTP_EINVAL, "ego out of range");
        if (s.N < 1 || s.N > SGTP_MAX_N) return fail(c, SGTP_EINVAL, "N out of range");
        if (ctx_limits && s.N > c->max_N) return fail(c, SGTP_ESHAPE, "N exceeds the context");
        if (s.n_tail < 1 || s.n_tail > s.N) return fail(c, SGTP_EINVAL, "n_tail out of range");
        if (s.K < 1 || s.K > SGTP_MAX_K) return fail(c, SGTP_EINVAL, "K out of range");
        if (!s.x || !s.s_abs || !s.v_scale || !s.u_nom) return fail(c, SGTP_EINVAL, "null race array");
        if (s.track_id < 0 || s.track_id >= MAX_TRACKS || !c->tracks[s.track_id].d_nodes)
            return fail(c, SGTP_ETRACK, "unknown track id");
        const TrackHost &T = c->tracks[s.track_id];
        RaceDev d{};
        d.n_agents = s.n_agents; d.ego = s.ego; d.N = s.N; d.n_tail = s.n_tail; d.track = s.track_id;
        d.slot0 = slot; d.K = s.K; d.seed = s.seed; d.plan_step = s.plan_step;
        d.x = s.x; d.s_abs = s.s_abs; d.v_scale = s.v_scale; d.u_nom = s.u_nom; d.traj = s.traj;
        d.prop = (const float4 *)s.prop;
        d.K_prop = s.prop ? std::min(std::max(s.K_prop, 0), s.K) : 0;
        if (p->update == 1 && s.prop && s.K_prop > 0)
            return fail(c, SGTP_EINVAL, "a learned proposal cannot be combined with the path-integral update");
        pl.races.push_back(d);
        const int tiles = (s.K + pl.tile_samples - 1) / pl.tile_samples;
        const long long groups = (s.K + gsz - 1) / gsz;
        for (int i = 0; i < s.n_agents; ++i) {
            ItemDev it{r, i, slot + i, pl.tiles_all, (int)(group_total + i * groups), 0};
            pl.tiles_all += tiles;
            pl.all.push_back(it);
            if (r == 0 && i == one_agent) {
                ItemDev o = it;
                o.tile0 = 0;
                pl.one.push_back(o);
            }
            if (i == s.ego) {
                ItemDev e = it;
                e.tile0 = pl.tiles_ego;
                pl.tiles_ego += tiles;
                pl.ego.push_back(e);
            }
        }
        slot += s.n_agents;
        group_total += (long long)s.n_agents * groups;
        pl.N_max = std::max(pl.N_max, s.N);
        pl.n_opp_max = std::max(pl.n_opp_max, s.n_agents - 1);
        // window: reachable arc length at up to 1.2 v_ref,max + 5 m/s, inner-side factor, margins
        const double Th = s.N * (double)p->dt;
        const double vb = 1.2 * T.vmax + 5.0;
        const double reach = vb * Th + 0.5 * std::max(0.0, (double)p->a_max) * Th * Th + 10.0;
        wneed = std::max(wneed, WIN_BACK + std::ceil(T.inner_factor * reach / T.ds_min) + 8.0);
    }
    if (ctx_limits && slot > c->max_agents) return fail(c, SGTP_ESHAPE, "total vehicles exceed the context");
    if (ctx_limits && group_total > c->max_groups * pl.lps)
        return fail(c, SGTP_ESHAPE, "total samples exceed the context (max_K)");
    if (p->update == 1 && (long long)pl.tiles_all > c->pi_tiles)
        return fail(c, SGTP_ESHAPE, "tiles exceed the path-integral buffer");
    pl.agents_total = slot;
    pl.w_max = (int)std::min<double>(WIN_MAX, wneed);
    return SGTP_OK;
}

// The plan of one launch sequence; the split variant only where its LDS ring fits.
int build_plan(sgtp_ctx *c, const sgtp_params *p, const sgtp_race *races, int n_races, int spl, Plan &pl,
               int one_agent = -1, bool ctx_limits = true) {
    int rc = build_plan_once(c, p, races, n_races, spl, pl, one_agent, true, ctx_limits);
    if (rc || !pl.split || make_layout(pl, maxopp_bucket(pl.n_opp_max), p->n_disc).total <= LDS_BUDGET) return rc;
    pl = Plan();
    return build_plan_once(c, p, races, n_races, spl, pl, one_agent, false, ctx_limits);
}

LdsLayout make_layout(const Plan &pl, int maxopp, int ndisc) {
    LdsLayout L{};
    int off = 0;
    auto take = [&](int bytes) {
        const int o = off;
        off += (bytes + 15) & ~15;
        return o;
    };
    L.N_max = pl.N_max;
    L.n_opp_max = std::max(1, maxopp);
    L.w_max = pl.w_max;
    L.ubar = take(pl.N_max * 8);
    L.xref = take(pl.N_max * 16);
    L.oppT = take(L.n_opp_max * 16);
    L.oppc = take(L.n_opp_max * 16);
    L.opp = take(pl.N_max * L.n_opp_max * (ndisc + 1) * 8);
    L.nodes = take(pl.w_max * 32);
    L.prop = take(pl.N_max * 16);
    // rr_u..rr_f also hold the path-integral partials of a tile's four waves,
    // 4 x (2N + 2) floats, which fit for every N >= 1
    L.rr_u = take(pl.N_max * 8);
    L.rr_st = take(pl.N_max * 32);
    L.rr_f = take(pl.N_max * 16);
    L.rr_t = take(pl.N_max * 16);
    L.rr_sync = take(NCP_MAX * 4);
    if (pl.split) {
        L.sp_ring = take(SPLIT_RING * (BLOCK / 2) * 16);
        L.sp_uring = take(SPLIT_RING * (BLOCK / 2) * 8);
        L.sp_sync = take(8 * 4);            // prod[2], cons[2], best lane[2], uprod[2]
        L.sp_fin = take((BLOCK / 2) * SPLIT_FIN * 4);  // per sample: final state
    }
    L.total = off;
    return L;
}

int maxopp_bucket(int n_opp) {
    if (n_opp <= 1) return 1;
    if (n_opp <= 3) return 3;
    if (n_opp <= 9) return 9;
    return 15;
}

// Upload the descriptor image of a plan into a ring slot; returns device pointers.
int upload_plan(sgtp_ctx *c, const Plan &pl, hipStream_t st, RaceDev **d_races, ItemDev **d_all, ItemDev **d_ego,
                ItemDev **d_one = nullptr) {
    const size_t nr = pl.races.size() * sizeof(RaceDev);
    const size_t na = pl.all.size() * sizeof(ItemDev);
    const size_t ne = pl.ego.size() * sizeof(ItemDev);
    const size_t no = pl.one.size() * sizeof(ItemDev);
    const size_t a0 = 0, a1 = (nr + 255) & ~size_t(255), a2 = a1 + ((na + 255) & ~size_t(255));
    const size_t a3 = a2 + ((ne + 255) & ~size_t(255));
    const size_t tot = a3 + no;
    if (tot > c->desc_bytes) return fail(c, SGTP_ESHAPE, "descriptor image too large");
    const int slot = c->ring_pos;
    c->ring_pos = (c->ring_pos + 1) % sgtp_ctx::RING;
    if (c->stage_used[slot]) HIPCHK(c, hipEventSynchronize(c->stage_ev[slot]));
    char *h = c->h_stage[slot];
    std::memcpy(h + a0, pl.races.data(), nr);
    std::memcpy(h + a1, pl.all.data(), na);
    if (ne) std::memcpy(h + a2, pl.ego.data(), ne);
    if (no) std::memcpy(h + a3, pl.one.data(), no);
    char *d = c->d_desc + (size_t)slot * c->desc_bytes;
    HIPCHK(c, hipMemcpyAsync(d, h, tot, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipEventRecord(c->stage_ev[slot], st));
    c->stage_used[slot] = true;
    *d_races = (RaceDev *)(d + a0);
    *d_all = (ItemDev *)(d + a1);
    *d_ego = (ItemDev *)(d + a2);
    if (d_one) *d_one = (ItemDev *)(d + a3);
    return SGTP_OK;
}

// grid = 0: one workgroup per tile; grid > 0: persistent sweep with that many workgroups;
// grid < 0: query the occupancy (workgroups per CU) of the persistent kernel into *occ.
template <int MODEL, int NDISC, int MAXOPP>
void launch_sweep_t(const LaunchArgs &A, int grid, hipStream_t st, int *occ) {
    if (grid < 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_sweep_persistent<MODEL, NDISC, MAXOPP>, BLOCK,
                                                         A.L.total) != hipSuccess)
            n = 1;
        *occ = n;
    } else if (grid == 0) {
        // about one wave per SIMD or fewer (small games): the latency variant reads ahead
        constexpr int LAT_WAVES = 1536;
        if (MAXOPP <= 3 && A.split)
            hipLaunchKernelGGL((k_sweep<MODEL, NDISC, MAXOPP <= 3 ? MAXOPP : 3, 6, 1, 1>), dim3(A.n_tiles),
                               dim3(BLOCK), A.L.total, st, A);
        else if (MODEL == 0 && MAXOPP <= 3 && A.lps == 2)
            hipLaunchKernelGGL((k_sweep<0, NDISC, MAXOPP <= 3 ? MAXOPP : 3, 6, 2>), dim3(A.n_tiles), dim3(BLOCK),
                               A.L.total, st, A);
        else if (MAXOPP <= 3 && A.n_tiles * (BLOCK / 64) <= LAT_WAVES)
            hipLaunchKernelGGL((k_sweep<MODEL, NDISC, MAXOPP <= 3 ? MAXOPP : 3, 6>), dim3(A.n_tiles), dim3(BLOCK),
                               A.L.total, st, A);
        else
            hipLaunchKernelGGL((k_sweep<MODEL, NDISC, MAXOPP>), dim3(A.n_tiles), dim3(BLOCK), A.L.total, st, A);
    } else {
        hipLaunchKernelGGL((k_sweep_persistent<MODEL, NDISC, MAXOPP>), dim3(grid), dim3(BLOCK), A.L.total, st, A);
    }
}

template <int MODEL, int NDISC>
void dispatch_opp(int mo, const LaunchArgs &A, int grid, hipStream_t st, int *occ) {
    if (mo == 1) launch_sweep_t<MODEL, NDISC, 1>(A, grid, st, occ);
    else if (mo == 3) launch_sweep_t<MODEL, NDISC, 3>(A, grid, st, occ);
    else if (mo == 9) launch_sweep_t<MODEL, NDISC, 9>(A, grid, st, occ);
    else launch_sweep_t<MODEL, NDISC, 15>(A, grid, st, occ);
}

void dispatch_sweep(int model, int ndisc, int mo, const LaunchArgs &A, hipStream_t st, int grid = 0,
                    int *occ = nullptr) {
    if (model == 0) {
        if (ndisc == 1) dispatch_opp<0, 1>(mo, A, grid, st, occ);
        else dispatch_opp<0, 3>(mo, A, grid, st, occ);
    } else {
        if (ndisc == 1) dispatch_opp<1, 1>(mo, A, grid, st, occ);
        else dispatch_opp<1, 3>(mo, A, grid, st, occ);
    }
}

// Order the items of a sweep for the persistent kernel: vehicles go to NQ queues
// by longest-processing-time first (work = K N), each queue is a contiguous run of
// tiles, heaviest vehicles first inside a queue.
void layout_queues(const Plan &pl, std::vector<ItemDev> &items, int q_begin[NQ], int q_len[NQ]) {
    std::vector<int> order(items.size());
    for (size_t i = 0; i < items.size(); ++i) order[i] = (int)i;
    auto work = [&](const ItemDev &it) {
        const RaceDev &r = pl.races[it.race];
        return (double)r.K * r.N * (1.0 + 0.02 * (r.n_agents - 1));
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(items[a]) > work(items[b]); });
    double load[NQ] = {0};
    std::vector<int> qof(items.size());
    for (int i : order) {
        int q = 0;
        for (int j = 1; j < NQ; ++j)
            if (load[j] < load[q]) q = j;
        qof[i] = q;
        load[q] += work(items[i]);
    }
    std::vector<ItemDev> out;
    int tile = 0;
    for (int q = 0; q < NQ; ++q) {
        q_begin[q] = tile;
        for (int i : order) {
            if (qof[i] != q) continue;
            ItemDev it = items[i];
            it.tile0 = tile;
            const RaceDev &r = pl.races[it.race];
            tile += (r.K + pl.tile_samples - 1) / pl.tile_samples;
            out.push_back(it);
        }
        q_len[q] = tile - q_begin[q];
    }
    items = out;
}

struct Runner {
    sgtp_ctx *c;
    const sgtp_params *p;
    hipStream_t st;
    Plan pl;
    LaunchArgs A{};
    RaceDev *d_races = nullptr;
    ItemDev *d_all = nullptr, *d_ego = nullptr, *d_one = nullptr;
    float *pred[2] = {nullptr, nullptr};  // prediction buffers read / written by the sweeps
    bool allow_timing = true;             // sgtp_set_timing events (not for the allocation-free call)
    int mo = 1;

    int init(const sgtp_race *races, int n_races, int one_agent = -1) {
        int rc = check_params(c, p);
        if (rc) return rc;
        rc = build_plan(c, p, races, n_races, 1, pl, one_agent);
        if (rc) return rc;
        mo = maxopp_bucket(pl.n_opp_max);
        A.P = make_kparams(p);
        A.P.spin_limit = c->spin_limit;
        A.L = make_layout(pl, mo, p->n_disc);
        if (A.L.total > LDS_BUDGET) return fail(c, SGTP_ESHAPE, "staged tables exceed the LDS budget");
        rc = upload_plan(c, pl, st, &d_races, &d_all, &d_ego, &d_one);
        if (rc) return rc;
        A.tracks = c->d_tracks;
        A.races = d_races;
        A.agents = c->d_agents;
        A.win = c->d_win;
        A.xref = c->d_xref;
        A.keys = c->d_keys;
        A.nfeas = c->d_nfeas;
        A.counters = c->d_counters;
        A.cp_slots = c->d_cp;
        A.pi_part = c->d_pi;
        A.status = c->d_status;
        A.spl = 1;
        A.lps = pl.lps;
        A.split = pl.split;
        pred[0] = c->d_pred[0];
        pred[1] = c->d_pred[1];
        return SGTP_OK;
    }
    // One vehicle's best response with every scratch buffer in the static device array at
    // `base` (noalloc_layout); the descriptors are written there by a kernel.
    int init_static(const sgtp_race *race, int agent, char *base) {
        int rc = check_params(c, p);
        if (rc) return rc;
        if (p->update != 0) return fail(c, SGTP_EINVAL, "the allocation-free entry point takes update = 0 only");
        rc = build_plan(c, p, race, 1, 1, pl, agent, false);
        if (rc) return rc;
        if (pl.all.size() > (size_t)NOALLOC_MAX_ITEMS || pl.one.size() != 1)
            return fail(c, SGTP_EINVAL, "bad vehicle count for the allocation-free entry point");
        mo = maxopp_bucket(pl.n_opp_max);
        A.P = make_kparams(p);
        A.P.spin_limit = c->spin_limit;
        A.L = make_layout(pl, mo, p->n_disc);
        if (A.L.total > LDS_BUDGET) return fail(c, SGTP_ESHAPE, "staged tables exceed the LDS budget");
        const NoallocLayout S = noalloc_layout();
        DescImage img{};
        img.race = pl.races[0];
        img.n_all = (int)pl.all.size();
        for (int i = 0; i < img.n_all; ++i) img.all[i] = pl.all[i];
        img.one = pl.one[0];
        img.one.group0 = 0;  // only this vehicle samples: its checkpoint groups start the array
        d_races = (RaceDev *)(base + S.races);
        d_all = (ItemDev *)(base + S.all);
        d_one = (ItemDev *)(base + S.one);
        d_ego = nullptr;
        hipLaunchKernelGGL(k_write_desc, dim3(1), dim3(64), 0, st, img, d_races, d_all, d_one);
        HIPCHK(c, hipGetLastError());
        A.tracks = c->d_tracks;
        A.races = d_races;
        A.agents = (AgentRec *)(base + S.agents);
        A.win = (float4 *)(base + S.win);
        A.xref = (float4 *)(base + S.xref);
        A.keys = (unsigned long long *)(base + S.keys);
        A.nfeas = (int *)(base + S.nfeas);
        A.counters = (int *)(base + S.counters);
        A.cp_slots = (float *)(base + S.cp);
        A.pi_part = nullptr;
        A.status = c->d_status;
        A.spl = 1;
        A.lps = pl.lps;
        A.split = pl.split;
        pred[0] = (float *)(base + S.pred0);
        pred[1] = (float *)(base + S.pred1);
        allow_timing = false;
        return SGTP_OK;
    }
    // projection, frames, windows, references, initial predictions (into pred[0])
    int setup_all() {
        LaunchArgs a = A;
        a.items = d_all;
        a.n_items = (int)pl.all.size();
        a.pred_out = pred[0];
        if (p->model == 0)
            hipLaunchKernelGGL(k_setup<0>, dim3(2 * a.n_items), dim3(BLOCK), A.L.total, st, a, pl.w_max);
        else
            hipLaunchKernelGGL(k_setup<1>, dim3(2 * a.n_items), dim3(BLOCK), A.L.total, st, a, pl.w_max);
        HIPCHK(c, hipGetLastError());
        return SGTP_OK;
    }
    // one sweep over `items` reading predictions pred[par]; the selected samples are
    // re-rolled in the same launch and write pred[par ^ 1]
    int sweep(const ItemDev *items, const std::vector<ItemDev> &host_items, int n_tiles, int phase, int par,
              sgtp_choice *choice, int choice_base, int adopt, int final_mode, float *u_apply,
              const LaunchArgs *dbg = nullptr) {
        LaunchArgs a = dbg ? *dbg : A;
        a.items = items;
        a.n_items = (int)host_items.size();
        a.n_tiles = n_tiles;
        a.phase = phase;
        a.pred_in = pred[par];
        a.pred_out = pred[par ^ 1];
        a.choice = choice;
        a.choice_base = choice_base;
        a.adopt = adopt;
        a.final_mode = final_mode;
        a.u_apply = (float2 *)u_apply;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const bool timed = c->timing && allow_timing;
        if (timed) {
            HIPCHK(c, hipEventCreate(&e0));
            HIPCHK(c, hipEventCreate(&e1));
            HIPCHK(c, hipEventRecord(e0, st));
        }
        dispatch_sweep(p->model, p->n_disc, mo, a, st);
        HIPCHK(c, hipGetLastError());
        if (timed) {
            HIPCHK(c, hipEventRecord(e1, st));
            c->ev_pairs.push_back(e0);
            c->ev_pairs.push_back(e1);
            long long ss = 0;
            for (const ItemDev &it : host_items) ss += (long long)pl.races[it.race].K * pl.races[it.race].N;
            c->ev_work.push_back(ss);
        }
        return SGTP_OK;
    }
};

}  // namespace

struct sgtp_plan {
    sgtp_ctx *c = nullptr;
    sgtp_params p{};
    int L = 0;
    Plan pl;
    LaunchArgs base{};
    int mo = 1;
    char *d_mem = nullptr;  // descriptors + queue counters, owned by the plan
    RaceDev *d_races = nullptr;
    ItemDev *d_all = nullptr, *d_ego = nullptr;
    int *d_qctr = nullptr;  // [(L+2)][NQ]
    int qb_all[NQ], ql_all[NQ], qb_ego[NQ], ql_ego[NQ];
    float *u_apply = nullptr;
    sgtp_choice *trace = nullptr;
    sgtp_plan_options opt{};
    int grid_all = 0, grid_ego = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool capturing = false;
    sgtp_mlp *mlp = nullptr;  // learned proposal computed inside the step, or NULL
    int residual = 0;
    float *d_feat = nullptr, *d_mlp_out = nullptr;  // [vehicles][50], [vehicles][200]
};

namespace {

// Enqueue one planning step of a plan (also used while capturing its graph).
int plan_enqueue(sgtp_plan *P, hipStream_t st) {
    sgtp_ctx *c = P->c;
    LaunchArgs a = P->base;
    a.items = P->d_all;
    a.n_items = (int)P->pl.all.size();
    a.pred_out = c->d_pred[0];
    a.qreset = P->d_qctr;
    a.n_qreset = (P->L + 2) * NQ;
    if (P->p.model == 0)
        hipLaunchKernelGGL(k_setup<0>, dim3(2 * a.n_items), dim3(BLOCK), a.L.total, st, a, P->pl.w_max);
    else
        hipLaunchKernelGGL(k_setup<1>, dim3(2 * a.n_items), dim3(BLOCK), a.L.total, st, a, P->pl.w_max);
    HIPCHK(c, hipGetLastError());
    const int nt = P->pl.agents_total;
    if (P->mlp) {  // learned proposal: features -> network -> tables, before the first sweep
        hipLaunchKernelGGL(k_features, dim3(a.n_items), dim3(64), 0, st, a, P->d_feat);
        HIPCHK(c, hipGetLastError());
        const int mrc = sgtp_mlp_forward(P->mlp, P->d_feat, nt, P->d_mlp_out, SGTP_MLP_OUT, st);
        if (mrc) return fail(c, mrc, std::string("proposal network: ") + sgtp_mlp_last_error(P->mlp));
        const int n = nt * SGTP_MAX_N;
        hipLaunchKernelGGL(k_proposal, dim3((n + 255) / 256), dim3(256), 0, st, P->d_races, P->d_all, nt,
                           P->d_mlp_out, SGTP_MLP_OUT, P->p.sigma_a, P->p.sigma_d, P->residual);
        HIPCHK(c, hipGetLastError());
    }
    for (int ph = 0; ph <= P->L + 1; ++ph) {
        const bool ego = ph == P->L + 1;
        LaunchArgs w = P->base;
        w.items = ego ? P->d_ego : P->d_all;
        w.n_items = (int)(ego ? P->pl.ego.size() : P->pl.all.size());
        w.n_tiles = ego ? P->pl.tiles_ego : P->pl.tiles_all;
        w.phase = ph;
        w.pred_in = c->d_pred[ph & 1];
        w.pred_out = c->d_pred[(ph & 1) ^ 1];
        w.choice = P->trace ? P->trace + (size_t)ph * nt : nullptr;
        w.choice_base = 0;
        w.adopt = 1;
        w.final_mode = ego ? 2 : (ph == P->L ? 1 : 0);
        w.u_apply = (float2 *)P->u_apply;
        w.qctr = P->d_qctr + ph * NQ;
        for (int q = 0; q < NQ; ++q) {
            w.q_begin[q] = ego ? P->qb_ego[q] : P->qb_all[q];
            w.q_len[q] = ego ? P->ql_ego[q] : P->ql_all[q];
        }
        const int grid = P->opt.persistent ? (ego ? P->grid_ego : P->grid_all) : 0;
        const bool timed = c->timing && !P->capturing;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timed) {
            HIPCHK(c, hipEventCreate(&e0));
            HIPCHK(c, hipEventCreate(&e1));
            HIPCHK(c, hipEventRecord(e0, st));
        }
        dispatch_sweep(P->p.model, P->p.n_disc, P->mo, w, st, grid);
        HIPCHK(c, hipGetLastError());
        if (timed) {
            HIPCHK(c, hipEventRecord(e1, st));
            c->ev_pairs.push_back(e0);
            c->ev_pairs.push_back(e1);
            long long ss = 0;
            for (const ItemDev &it : (ego ? P->pl.ego : P->pl.all))
                ss += (long long)P->pl.races[it.race].K * P->pl.races[it.race].N;
            c->ev_work.push_back(ss);
        }
    }
    const int nr = (int)P->pl.races.size();
    if (P->opt.include_advance) {  // closed-loop step and the step counters in one launch
        if (P->p.model == 0)
            hipLaunchKernelGGL(k_advance<0>, dim3((nt + 63) / 64), dim3(64), 0, st, P->d_races, P->d_all, nt,
                               (const float2 *)P->u_apply, make_veh64(&P->p), (double)P->p.dt, P->d_races);
        else
            hipLaunchKernelGGL(k_advance<1>, dim3((nt + 63) / 64), dim3(64), 0, st, P->d_races, P->d_all, nt,
                               (const float2 *)P->u_apply, make_veh64(&P->p), (double)P->p.dt, P->d_races);
    } else {
        hipLaunchKernelGGL(k_bump_step, dim3((nr + 63) / 64), dim3(64), 0, st, P->d_races, nr);
    }
    HIPCHK(c, hipGetLastError());
    return SGTP_OK;
}

// Capture one planning step into the plan's graph (on a private stream).
bool capture_plan(sgtp_plan *P) {
    hipStream_t cap = nullptr;
    bool ok = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
    P->capturing = true;
    int erc = ok ? plan_enqueue(P, cap) : SGTP_EDEVICE;
    P->capturing = false;
    hipGraph_t g = nullptr;
    if (ok) ok = hipStreamEndCapture(cap, &g) == hipSuccess;
    ok = ok && erc == SGTP_OK && hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0) == hipSuccess;
    P->graph = g;
    if (cap) (void)hipStreamDestroy(cap);
    return ok;
}

}  // namespace

extern "C" {

int sgtp_abi_version(void) { return 1; }

int sgtp_ctx_create(sgtp_ctx **out, int max_agents_total, int max_N, int max_races, int max_track_nodes,
                    int max_K) {
    if (!out) return SGTP_EINVAL;
    *out = nullptr;
    if (max_agents_total < 1 || max_N < 1 || max_N > SGTP_MAX_N || max_races < 1 || max_track_nodes < 2 ||
        max_K < 1 || max_K > SGTP_MAX_K)
        return SGTP_EINVAL;
    sgtp_ctx *c = new sgtp_ctx();
    c->max_agents = max_agents_total;
    c->max_N = max_N;
    c->max_races = max_races;
    c->max_nodes = max_track_nodes;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1 || hipGetDevice(&c->device) != hipSuccess ||
        map_scratch(c->device) != SGTP_OK) {
        delete c;
        return SGTP_EDEVICE;
    }
    bool ok = true;
    auto al = [&](void **p, size_t bytes) {
        if (ok && hipMalloc(p, bytes) != hipSuccess) ok = false;
        if (ok && hipMemset(*p, 0, bytes) != hipSuccess) ok = false;
    };
    al((void **)&c->d_tracks, sizeof(TrackDev) * MAX_TRACKS);
    al((void **)&c->d_agents, sizeof(AgentRec) * max_agents_total);
    al((void **)&c->d_win, sizeof(float4) * 2 * WIN_MAX * (size_t)max_agents_total);
    al((void **)&c->d_xref, sizeof(float4) * (size_t)max_N * max_agents_total);
    for (int i = 0; i < 2; ++i) al((void **)&c->d_pred[i], sizeof(float) * PRED_STRIDE * (max_N + 1) * (size_t)max_agents_total);
    al((void **)&c->d_keys, sizeof(unsigned long long) * max_agents_total);
    al((void **)&c->d_nfeas, sizeof(int) * max_agents_total);
    al((void **)&c->d_counters, sizeof(int) * max_agents_total);
    al((void **)&c->d_status, sizeof(int));
    c->max_groups = (long long)max_agents_total * ((max_K + 63) / 64);
    al((void **)&c->d_cp, sizeof(float) * CP_FLOATS * 2 * (size_t)c->max_groups);  // 2: pair variant groups of 32
    c->desc_bytes = ((sizeof(RaceDev) * max_races + 255) & ~size_t(255)) +
                    3 * ((sizeof(ItemDev) * max_agents_total + 255) & ~size_t(255)) + 256;
    al((void **)&c->d_desc, c->desc_bytes * sgtp_ctx::RING);
    for (int i = 0; i < sgtp_ctx::RING && ok; ++i) {
        if (hipHostMalloc((void **)&c->h_stage[i], c->desc_bytes, hipHostMallocDefault) != hipSuccess) ok = false;
        if (ok && hipEventCreateWithFlags(&c->stage_ev[i], hipEventDisableTiming) != hipSuccess) ok = false;
    }
    if (!ok) {
        sgtp_ctx_destroy(c);
        return SGTP_ENOMEM;
    }
    *out = c;
    return SGTP_OK;
}

int sgtp_ctx_destroy(sgtp_ctx *c) {
    if (!c) return SGTP_EINVAL;
    (void)hipDeviceSynchronize();
    for (auto &t : c->tracks)
        if (t.d_nodes) (void)hipFree(t.d_nodes);
    void *bufs[] = {c->d_tracks, c->d_agents,   c->d_win, c->d_xref, c->d_pred[0], c->d_pred[1], c->d_keys,
                    c->d_nfeas,  c->d_counters, c->d_cp,  c->d_desc, c->d_pi,      c->d_status};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    for (int i = 0; i < sgtp_ctx::RING; ++i) {
        if (c->h_stage[i]) (void)hipHostFree(c->h_stage[i]);
        if (c->stage_ev[i]) (void)hipEventDestroy(c->stage_ev[i]);
    }
    for (auto e : c->ev_pairs) (void)hipEventDestroy(e);
    delete c;
    return SGTP_OK;
}

const char *sgtp_last_error(const sgtp_ctx *c) { return c ? c->err.c_str() : "null context"; }

int sgtp_ctx_status(sgtp_ctx *c, int *flags, int clear, void *stream) {
    if (!c || !flags) return SGTP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    int v = 0;
    HIPCHK(c, hipMemcpyAsync(&v, c->d_status, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (clear && v) {
        const int zero = 0;
        HIPCHK(c, hipMemcpy(c->d_status, &zero, sizeof(int), hipMemcpyHostToDevice));
    }
    *flags = v;
    if (v) {
        std::string m = "kernel status:";
        if (v & SGTP_STATUS_WAIT_GAVE_UP)
            m += " a sample's bounded LDS wait gave up (the sample was scored non-finite)";
        if (v & SGTP_STATUS_REROLL_GAVE_UP) m += " a winner re-roll's bounded LDS wait gave up (outputs unreliable)";
        c->err = m;
    }
    return SGTP_OK;
}

int sgtp_ctx_set_poll_limit(sgtp_ctx *c, int polls) {
    if (!c || polls < 1) return SGTP_EINVAL;
    c->spin_limit = polls;
    return SGTP_OK;
}

int sgtp_ctx_enable_path_integral(sgtp_ctx *c) {
    if (!c) return SGTP_EINVAL;
    if (c->d_pi) return SGTP_OK;
    // tiles of BLOCK / 2 samples (the split variant), one partial tile per vehicle
    const long long tiles = c->max_groups / (BLOCK / 128) + c->max_agents;
    const size_t bytes = sizeof(float) * (size_t)tiles * (size_t)(2 * c->max_N + 2);
    if (hipMalloc((void **)&c->d_pi, bytes) != hipSuccess) {
        c->d_pi = nullptr;
        return fail(c, SGTP_ENOMEM, "path-integral buffer");
    }
    c->pi_tiles = tiles;
    return SGTP_OK;
}

int sgtp_track_upload(sgtp_ctx *c, int id, const double *nodes, int n, int closed, double length, double psi_lap) {
    if (!c) return SGTP_EINVAL;
    if (id < 0 || id >= MAX_TRACKS) return fail(c, SGTP_ETRACK, "track id out of range");
    if (!nodes || n < 2 || n > c->max_nodes) return fail(c, SGTP_ESHAPE, "bad node count");
    if (closed && !(length > 0)) return fail(c, SGTP_EINVAL, "closed track needs a positive length");
    std::vector<double> h((size_t)n * NODE_STRIDE);
    double ds_min = INFINITY, vmax = 0, kmax = 0, wmax = 0;
    for (int i = 0; i < n; ++i) {
        const double *r = nodes + (size_t)i * 8;
        double *o = h.data() + (size_t)i * NODE_STRIDE;
        o[0] = r[0]; o[1] = r[1]; o[2] = r[2];
        o[3] = -std::sin(r[2]);
        o[4] = std::cos(r[2]);
        o[5] = r[4]; o[6] = r[5]; o[7] = r[6]; o[8] = r[7]; o[9] = r[3];
        if (i + 1 < n) ds_min = std::min(ds_min, nodes[(size_t)(i + 1) * 8 + 7] - r[7]);
        vmax = std::max(vmax, r[6]);
        kmax = std::max(kmax, std::fabs(r[3]));
        wmax = std::max(wmax, std::max(r[4], r[5]));
        if (!std::isfinite(r[0]) || !std::isfinite(r[1]) || !std::isfinite(r[2]) || !std::isfinite(r[7]))
            return fail(c, SGTP_ETRACK, "non-finite node");
    }
    if (closed) ds_min = std::min(ds_min, length + nodes[7] - nodes[(size_t)(n - 1) * 8 + 7]);
    if (!(ds_min > 0)) return fail(c, SGTP_ETRACK, "node arc lengths must increase");
    TrackHost &T = c->tracks[id];
    if (T.d_nodes) {
        HIPCHK(c, hipDeviceSynchronize());
        HIPCHK(c, hipFree(T.d_nodes));
        T.d_nodes = nullptr;
    }
    HIPCHK(c, hipMalloc((void **)&T.d_nodes, h.size() * sizeof(double)));
    HIPCHK(c, hipMemcpy(T.d_nodes, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
    T.n = n;
    T.closed = closed ? 1 : 0;
    T.length = length;
    T.psi_lap = closed ? psi_lap : 0.0;
    T.ds_min = ds_min;
    T.vmax = vmax;
    T.inner_factor = 1.0 / std::max(0.25, 1.0 - kmax * (wmax + 2.0));
    TrackDev d{T.d_nodes, T.n, T.closed, T.length, T.psi_lap, T.ds_min, T.inner_factor, T.vmax};
    HIPCHK(c, hipMemcpy(c->d_tracks + id, &d, sizeof d, hipMemcpyHostToDevice));
    return SGTP_OK;
}

int sgtp_rollout_cost(sgtp_ctx *c, const sgtp_params *p, const sgtp_race *race, int agent, int phase, float *cost,
                      unsigned char *flags, float *viol, double *x_final, float *noise, sgtp_choice *out,
                      void *stream) {
    if (!c) return SGTP_EINVAL;
    if (!race) return fail(c, SGTP_EINVAL, "race is NULL");
    if (agent < 0 || agent >= race->n_agents) return fail(c, SGTP_EINVAL, "agent out of range");
    if (phase < 0 || phase > 0xffff) return fail(c, SGTP_EINVAL, "phase out of range");
    Runner r{c, p, (hipStream_t)stream};
    int rc = r.init(race, 1, agent);
    if (rc) return rc;
    rc = r.setup_all();
    if (rc) return rc;
    LaunchArgs dbg = r.A;
    dbg.dbg_cost = cost;
    dbg.dbg_flags = flags;
    dbg.dbg_viol = viol;
    dbg.dbg_xfinal = x_final;
    dbg.dbg_noise = noise;
    const int tiles = (race->K + r.pl.tile_samples - 1) / r.pl.tile_samples;
    return r.sweep(r.d_one, r.pl.one, tiles, phase, 0, out, r.pl.all[agent].slot, 0, 0, nullptr, &dbg);
}

int sgtp_rollout_cost_noalloc(sgtp_ctx *c, const sgtp_params *p, const sgtp_race *race, int agent, int phase,
                              float *cost, unsigned char *flags, float *viol, double *x_final, float *noise,
                              sgtp_choice *out, void *stream) {
    if (!c) return SGTP_EINVAL;
    if (!race) return fail(c, SGTP_EINVAL, "race is NULL");
    if (agent < 0 || agent >= race->n_agents) return fail(c, SGTP_EINVAL, "agent out of range");
    if (phase < 0 || phase > 0xffff) return fail(c, SGTP_EINVAL, "phase out of range");
    if (race->K > SGTP_NOALLOC_MAX_K)
        return fail(c, SGTP_ESHAPE, "K exceeds the allocation-free entry point's maximum (SGTP_NOALLOC_MAX_K)");
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev != c->device) return fail(c, SGTP_EDEVICE, "the context's device is not the current device");
    char *base = scratch_of(dev);
    if (!base) return fail(c, SGTP_EDEVICE, "static scratch not mapped on this device");
    Runner r{c, p, (hipStream_t)stream};
    int rc = r.init_static(race, agent, base);
    if (rc) return rc;
    rc = r.setup_all();
    if (rc) return rc;
    LaunchArgs dbg = r.A;
    dbg.dbg_cost = cost;
    dbg.dbg_flags = flags;
    dbg.dbg_viol = viol;
    dbg.dbg_xfinal = x_final;
    dbg.dbg_noise = noise;
    const int tiles = (race->K + r.pl.tile_samples - 1) / r.pl.tile_samples;
    return r.sweep(r.d_one, r.pl.one, tiles, phase, 0, out, r.pl.all[agent].slot, 0, 0, nullptr, &dbg);
}

int sgtp_gauss_pairs(const unsigned int *r_even, const unsigned int *r_odd, float *out, int n, void *stream) {
    if (!r_even || !r_odd || !out || n < 0) return SGTP_EINVAL;
    if (n == 0) return SGTP_OK;
    hipLaunchKernelGGL(k_gauss_pairs, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       (const uint32_t *)r_even, (const uint32_t *)r_odd, (float2 *)out, n);
    return hipGetLastError() == hipSuccess ? SGTP_OK : SGTP_EDEVICE;
}

int sgtp_ibr_sweep(sgtp_ctx *c, const sgtp_params *p, const sgtp_race *races, int n_races, int phase, int ego_only,
                   sgtp_choice *out, void *stream) {
    if (!c) return SGTP_EINVAL;
    if (phase < 0 || phase > 0xffff) return fail(c, SGTP_EINVAL, "phase out of range");
    Runner r{c, p, (hipStream_t)stream};
    int rc = r.init(races, n_races);
    if (rc) return rc;
    rc = r.setup_all();
    if (rc) return rc;
    if (ego_only) return r.sweep(r.d_ego, r.pl.ego, r.pl.tiles_ego, phase, 0, out, 0, 1, 0, nullptr);
    return r.sweep(r.d_all, r.pl.all, r.pl.tiles_all, phase, 0, out, 0, 1, 0, nullptr);
}

int sgtp_plan_step(sgtp_ctx *c, const sgtp_params *p, const sgtp_race *races, int n_races, int L_ibr, float *u_apply,
                   sgtp_choice *trace, void *stream) {
    if (!c) return SGTP_EINVAL;
    if (L_ibr < 0 || L_ibr + 1 > 0xffff) return fail(c, SGTP_EINVAL, "L_ibr out of range");
    if (!u_apply) return fail(c, SGTP_EINVAL, "u_apply is NULL");
    Runner r{c, p, (hipStream_t)stream};
    int rc = r.init(races, n_races);
    if (rc) return rc;
    rc = r.setup_all();
    if (rc) return rc;
    const int nt = r.pl.agents_total;
    for (int ph = 0; ph <= L_ibr + 1; ++ph) {
        const bool ego = ph == L_ibr + 1;
        const int final_mode = ego ? 2 : (ph == L_ibr ? 1 : 0);
        sgtp_choice *tr = trace ? trace + (size_t)ph * nt : nullptr;
        if (ego)
            rc = r.sweep(r.d_ego, r.pl.ego, r.pl.tiles_ego, ph, ph & 1, tr, 0, 1, final_mode, u_apply);
        else
            rc = r.sweep(r.d_all, r.pl.all, r.pl.tiles_all, ph, ph & 1, tr, 0, 1, final_mode, u_apply);
        if (rc) return rc;
    }
    return SGTP_OK;
}

int sgtp_advance(sgtp_ctx *c, const sgtp_params *p, const sgtp_race *races, int n_races, const float *u, void *stream) {
    if (!c) return SGTP_EINVAL;
    if (!u) return fail(c, SGTP_EINVAL, "u is NULL");
    int rc = check_params(c, p);
    if (rc) return rc;
    Plan pl;
    rc = build_plan(c, p, races, n_races, 1, pl);
    if (rc) return rc;
    RaceDev *dr;
    ItemDev *da, *de;
    hipStream_t st = (hipStream_t)stream;
    rc = upload_plan(c, pl, st, &dr, &da, &de);
    if (rc) return rc;
    const int nt = pl.agents_total;
    const VehConst<double> V = make_veh64(p);
    if (p->model == 0)
        hipLaunchKernelGGL(k_advance<0>, dim3((nt + 63) / 64), dim3(64), 0, st, dr, da, nt, (const float2 *)u, V, (double)p->dt, nullptr);
    else
        hipLaunchKernelGGL(k_advance<1>, dim3((nt + 63) / 64), dim3(64), 0, st, dr, da, nt, (const float2 *)u, V, (double)p->dt, nullptr);
    HIPCHK(c, hipGetLastError());
    return SGTP_OK;
}

int sgtp_plan_create(sgtp_ctx *c, const sgtp_params *p, const sgtp_race *races, int n_races, int L_ibr,
                     float *u_apply, sgtp_choice *trace, const sgtp_plan_options *opt, sgtp_plan **out,
                     void *stream) {
    if (!c) return SGTP_EINVAL;
    if (!out) return fail(c, SGTP_EINVAL, "out is NULL");
    *out = nullptr;
    if (L_ibr < 0 || L_ibr + 1 > 0xffff) return fail(c, SGTP_EINVAL, "L_ibr out of range");
    if (!u_apply) return fail(c, SGTP_EINVAL, "u_apply is NULL");
    int rc = check_params(c, p);
    if (rc) return rc;
    sgtp_plan_options o{};
    o.persistent = 1;
    o.blocks_per_cu = 0;
    o.tiles_per_fetch = 1;
    o.samples_per_lane = 1;
    o.use_graph = 1;
    o.include_advance = 0;
    if (opt) o = *opt;
    if (o.samples_per_lane < 1 || o.samples_per_lane > 16 || o.tiles_per_fetch < 1 || o.tiles_per_fetch > 64 ||
        o.blocks_per_cu < 0 || o.blocks_per_cu > 64)
        return fail(c, SGTP_EINVAL, "plan options out of range");
    sgtp_plan *P = new sgtp_plan();
    P->c = c;
    P->p = *p;
    P->L = L_ibr;
    P->opt = o;
    P->u_apply = u_apply;
    P->trace = trace;
    rc = build_plan(c, p, races, n_races, o.samples_per_lane, P->pl);
    if (rc) {
        delete P;
        return rc;
    }
    // the pair and split variants run one workgroup per tile
    if (P->pl.lps == 2 || P->pl.split) P->opt.persistent = o.persistent = 0;
    layout_queues(P->pl, P->pl.all, P->qb_all, P->ql_all);
    layout_queues(P->pl, P->pl.ego, P->qb_ego, P->ql_ego);
    P->pl.tiles_all = P->ql_all[NQ - 1] + P->qb_all[NQ - 1];
    P->pl.tiles_ego = P->ql_ego[NQ - 1] + P->qb_ego[NQ - 1];
    P->mo = maxopp_bucket(P->pl.n_opp_max);
    LaunchArgs &A = P->base;
    A.P = make_kparams(p);
    A.P.spin_limit = c->spin_limit;
    A.L = make_layout(P->pl, P->mo, p->n_disc);
    if (A.L.total > LDS_BUDGET) {
        delete P;
        return fail(c, SGTP_ESHAPE, "staged tables exceed the LDS budget");
    }
    const size_t nr = P->pl.races.size() * sizeof(RaceDev), na = P->pl.all.size() * sizeof(ItemDev),
                 ne = P->pl.ego.size() * sizeof(ItemDev), nq = (size_t)(L_ibr + 2) * NQ * sizeof(int);
    const size_t o1 = (nr + 255) & ~size_t(255), o2 = o1 + ((na + 255) & ~size_t(255)),
                 o3 = o2 + ((ne + 255) & ~size_t(255));
    bool ok = hipMalloc((void **)&P->d_mem, o3 + nq) == hipSuccess;
    ok = ok && hipMemcpy(P->d_mem, P->pl.races.data(), nr, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(P->d_mem + o1, P->pl.all.data(), na, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(P->d_mem + o2, P->pl.ego.data(), ne, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemset(P->d_mem + o3, 0, nq) == hipSuccess;
    if (!ok) {
        if (P->d_mem) (void)hipFree(P->d_mem);
        delete P;
        return fail(c, SGTP_ENOMEM, "plan descriptors");
    }
    P->d_races = (RaceDev *)P->d_mem;
    P->d_all = (ItemDev *)(P->d_mem + o1);
    P->d_ego = (ItemDev *)(P->d_mem + o2);
    P->d_qctr = (int *)(P->d_mem + o3);
    A.tracks = c->d_tracks;
    A.races = P->d_races;
    A.agents = c->d_agents;
    A.win = c->d_win;
    A.xref = c->d_xref;
    A.keys = c->d_keys;
    A.nfeas = c->d_nfeas;
    A.counters = c->d_counters;
    A.cp_slots = c->d_cp;
    A.pi_part = c->d_pi;
    A.status = c->d_status;
    A.spl = o.samples_per_lane;
    A.lps = P->pl.lps;
    A.split = P->pl.split;
    A.chunk = o.tiles_per_fetch;
    if (o.persistent) {
        int occ = 1, dev = 0, cus = 0;
        dispatch_sweep(p->model, p->n_disc, P->mo, A, nullptr, -1, &occ);
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const int bpc = o.blocks_per_cu > 0 ? std::min(o.blocks_per_cu, std::max(1, occ)) : std::max(1, occ);
        const int g = std::max(1, cus) * bpc;
        P->grid_all = std::max(1, std::min(g, P->pl.tiles_all));
        P->grid_ego = std::max(1, std::min(g, P->pl.tiles_ego));
    }
    (void)stream;
    if (o.use_graph && !capture_plan(P)) {
        sgtp_plan_destroy(P);
        return fail(c, SGTP_EDEVICE, "graph capture of the planning step failed");
    }
    *out = P;
    return SGTP_OK;
}

int sgtp_plan_set_proposal(sgtp_plan *P, sgtp_mlp *m, int residual) {
    if (!P) return SGTP_EINVAL;
    sgtp_ctx *c = P->c;
    if (m) {
        bool any = false;
        for (const RaceDev &r : P->pl.races)
            if (r.prop) {
                any = true;
                if (4 * r.N > SGTP_MLP_OUT) return fail(c, SGTP_ESHAPE, "horizon longer than the network's output");
            }
        if (!any) return fail(c, SGTP_EINVAL, "no race of the plan has a proposal table");
        if (sgtp_mlp_batch_max(m) < P->pl.agents_total)
            return fail(c, SGTP_ESHAPE, "network batch smaller than the plan's vehicle count");
    }
    HIPCHK(c, hipDeviceSynchronize());
    if (m && !P->d_feat) {
        const size_t nt = (size_t)P->pl.agents_total;
        if (hipMalloc((void **)&P->d_feat, nt * SGTP_FEAT_DIM * 4) != hipSuccess ||
            hipMalloc((void **)&P->d_mlp_out, nt * SGTP_MLP_OUT * 4) != hipSuccess)
            return fail(c, SGTP_ENOMEM, "proposal buffers");
    }
    P->mlp = m;
    P->residual = residual ? 1 : 0;
    if (P->opt.use_graph) {
        if (P->exec) (void)hipGraphExecDestroy(P->exec);
        if (P->graph) (void)hipGraphDestroy(P->graph);
        P->exec = nullptr;
        P->graph = nullptr;
        if (!capture_plan(P)) return fail(c, SGTP_EDEVICE, "graph capture of the planning step failed");
    }
    return SGTP_OK;
}

int sgtp_plan_run(sgtp_plan *P, void *stream) {
    if (!P) return SGTP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (P->exec) {
        HIPCHK(P->c, hipGraphLaunch(P->exec, st));
        return SGTP_OK;
    }
    return plan_enqueue(P, st);
}

int sgtp_plan_set_step(sgtp_plan *P, unsigned int plan_step) {
    if (!P) return SGTP_EINVAL;
    HIPCHK(P->c, hipDeviceSynchronize());
    for (size_t r = 0; r < P->pl.races.size(); ++r) {
        P->pl.races[r].plan_step = plan_step;
        HIPCHK(P->c, hipMemcpy(&P->d_races[r].plan_step, &plan_step, sizeof plan_step, hipMemcpyHostToDevice));
    }
    return SGTP_OK;
}

int sgtp_plan_info(const sgtp_plan *P, int *grid_sweep, int *tiles_sweep, int *lds_bytes) {
    if (!P) return SGTP_EINVAL;
    if (grid_sweep) *grid_sweep = P->opt.persistent ? P->grid_all : P->pl.tiles_all;
    if (tiles_sweep) *tiles_sweep = P->pl.tiles_all;
    if (lds_bytes) *lds_bytes = P->base.L.total;
    return SGTP_OK;
}

int sgtp_plan_destroy(sgtp_plan *P) {
    if (!P) return SGTP_EINVAL;
    (void)hipDeviceSynchronize();
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->d_mem) (void)hipFree(P->d_mem);
    if (P->d_feat) (void)hipFree(P->d_feat);
    if (P->d_mlp_out) (void)hipFree(P->d_mlp_out);
    delete P;
    return SGTP_OK;
}

int sgtp_autotune(sgtp_ctx *c, const sgtp_params *p, const sgtp_race *races, int n_races, int L_ibr,
                  float *u_apply, sgtp_plan_options *best, double *best_ms, void *stream) {
    if (!c) return SGTP_EINVAL;
    if (!best) return fail(c, SGTP_EINVAL, "best is NULL");
    if (!races || n_races < 1) return fail(c, SGTP_EINVAL, "no races");
    // a schedule found before for this kind of workload is returned without timing
    TuneKey key{};
    {
        long long samples = 0;
        int N = 0, nopp = 0;
        for (int r = 0; r < n_races; ++r) {
            samples += (long long)std::max(races[r].K, 0) * std::max(races[r].n_agents, 0);
            N = std::max(N, races[r].N);
            nopp = std::max(nopp, races[r].n_agents - 1);
        }
        auto lg = [](long long v) {
            long long b = 0;
            while (v > 1) {
                v >>= 1;
                ++b;
            }
            return b;
        };
        key = TuneKey{p->model, p->n_disc, maxopp_bucket(nopp), N, lg(samples), lg(n_races), p->update, L_ibr};
        const auto hit = c->tune_cache.find(key);
        if (hit != c->tune_cache.end()) {
            *best = hit->second.opt;
            if (best_ms) *best_ms = hit->second.ms;
            return SGTP_OK;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    // the search runs real planning steps: save and restore the mutable race state (the
    // state is restored and the buffers freed on every exit path, failed candidates included)
    std::vector<size_t> sizes;
    for (int r = 0; r < n_races; ++r) {
        sizes.push_back((size_t)races[r].n_agents * races[r].N * 2 * sizeof(float));
        sizes.push_back((size_t)races[r].n_agents * sizeof(double));
    }
    std::vector<void *> saved(sizes.size(), nullptr);
    int rc = SGTP_OK;
    for (size_t i = 0; i < sizes.size() && !rc; ++i)
        if (hipMalloc(&saved[i], sizes[i]) != hipSuccess) rc = fail(c, SGTP_ENOMEM, "autotune: save buffers");
    auto save_restore = [&](bool save) -> int {
        for (int r = 0; r < n_races; ++r) {
            void *un = races[r].u_nom, *sa = races[r].s_abs;
            HIPCHK(c, hipMemcpyAsync(save ? saved[2 * r] : un, save ? un : saved[2 * r], sizes[2 * r],
                                     hipMemcpyDeviceToDevice, st));
            HIPCHK(c, hipMemcpyAsync(save ? saved[2 * r + 1] : sa, save ? sa : saved[2 * r + 1], sizes[2 * r + 1],
                                     hipMemcpyDeviceToDevice, st));
        }
        return SGTP_OK;
    };
    bool have_saved = false;
    if (!rc) {
        rc = save_restore(true);
        have_saved = rc == SGTP_OK;
    }
    std::vector<sgtp_plan_options> cand;
    for (int spl : {1, 2}) {
        sgtp_plan_options o{};
        o.persistent = 0;
        o.samples_per_lane = spl;
        o.tiles_per_fetch = 1;
        cand.push_back(o);
    }
    for (int chunk : {1, 2, 4})
        for (int bpc : {0, 2}) {
            sgtp_plan_options o{};
            o.persistent = 1;
            o.samples_per_lane = 1;
            o.tiles_per_fetch = chunk;
            o.blocks_per_cu = bpc;
            cand.push_back(o);
        }
    double best_t = INFINITY;
    sgtp_plan_options best_o = cand[0];
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(c, SGTP_EDEVICE, "autotune: events");
    for (const sgtp_plan_options &o : cand) {
        if (rc) break;
        sgtp_plan *P = nullptr;
        rc = sgtp_plan_create(c, p, races, n_races, L_ibr, u_apply, nullptr, &o, &P, stream);
        if (rc) break;
        // median of 5 timed steps after one warm-up step
        std::vector<double> ts;
        for (int rep = 0; rep < 6 && rc == 0; ++rep) {
            rc = save_restore(false);
            if (!rc) (void)hipEventRecord(e0, st);
            if (!rc) rc = sgtp_plan_run(P, stream);
            if (!rc) (void)hipEventRecord(e1, st);
            if (!rc && hipEventSynchronize(e1) == hipSuccess) {
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0) ts.push_back((double)ms);
            }
        }
        sgtp_plan_destroy(P);
        double t = INFINITY;
        if (!ts.empty()) {
            std::sort(ts.begin(), ts.end());
            t = ts[ts.size() / 2];
        }
        // a later candidate must be clearly faster (earlier ones are the simpler schedules)
        if (t < 0.98 * best_t) {
            best_t = t;
            best_o = o;
        }
    }
    if (have_saved) {
        const int rr = save_restore(false);
        if (!rc) rc = rr;
    }
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (void *b : saved)
        if (b) (void)hipFree(b);
    if (rc) return rc;
    best_o.use_graph = 1;
    *best = best_o;
    if (best_ms) *best_ms = best_t;
    c->tune_cache[key] = TuneEntry{best_o, best_t};
    return SGTP_OK;
}

int sgtp_autotune_forget(sgtp_ctx *c) {
    if (!c) return SGTP_EINVAL;
    c->tune_cache.clear();
    return SGTP_OK;
}

int sgtp_features(sgtp_ctx *c, const sgtp_params *p, const sgtp_race *races, int n_races, float *X, void *stream) {
    if (!c) return SGTP_EINVAL;
    if (!X) return fail(c, SGTP_EINVAL, "X is NULL");
    Runner r{c, p, (hipStream_t)stream};
    int rc = r.init(races, n_races);
    if (rc) return rc;
    rc = r.setup_all();
    if (rc) return rc;
    LaunchArgs a = r.A;
    a.items = r.d_all;
    a.n_items = (int)r.pl.all.size();
    hipLaunchKernelGGL(k_features, dim3(a.n_items), dim3(64), 0, r.st, a, X);
    HIPCHK(c, hipGetLastError());
    return SGTP_OK;
}

int sgtp_proposal_from_outputs(sgtp_ctx *c, const sgtp_params *p, const sgtp_race *races, int n_races,
                               const float *out, int ld_out, int residual, void *stream) {
    if (!c) return SGTP_EINVAL;
    if (!out || ld_out < 4) return fail(c, SGTP_EINVAL, "bad network outputs");
    int rc = check_params(c, p);
    if (rc) return rc;
    Plan pl;
    rc = build_plan(c, p, races, n_races, 1, pl);
    if (rc) return rc;
    for (int r = 0; r < n_races; ++r)
        if (races[r].prop && 4 * races[r].N > ld_out) return fail(c, SGTP_ESHAPE, "horizon longer than the outputs");
    RaceDev *dr;
    ItemDev *da, *de;
    hipStream_t st = (hipStream_t)stream;
    rc = upload_plan(c, pl, st, &dr, &da, &de);
    if (rc) return rc;
    const int n = pl.agents_total * SGTP_MAX_N;
    hipLaunchKernelGGL(k_proposal, dim3((n + 255) / 256), dim3(256), 0, st, dr, da, pl.agents_total, out, ld_out,
                       p->sigma_a, p->sigma_d, residual ? 1 : 0);
    HIPCHK(c, hipGetLastError());
    return SGTP_OK;
}

int sgtp_set_timing(sgtp_ctx *c, int on) {
    if (!c) return SGTP_EINVAL;
    c->timing = on != 0;
    return SGTP_OK;
}

int sgtp_sweep_stats(sgtp_ctx *c, double *total_ms, long long *launches, long long *sample_steps, int reset) {
    if (!c) return SGTP_EINVAL;
    for (size_t i = 0; i + 1 < c->ev_pairs.size(); i += 2) {
        HIPCHK(c, hipEventSynchronize(c->ev_pairs[i + 1]));
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pairs[i], c->ev_pairs[i + 1]));
        c->total_ms += ms;
        c->launches += 1;
        c->sample_steps += c->ev_work[i / 2];
        (void)hipEventDestroy(c->ev_pairs[i]);
        (void)hipEventDestroy(c->ev_pairs[i + 1]);
    }
    c->ev_pairs.clear();
    c->ev_work.clear();
    if (total_ms) *total_ms = c->total_ms;
    if (launches) *launches = c->launches;
    if (sample_steps) *sample_steps = c->sample_steps;
    if (reset) {
        c->total_ms = 0;
        c->launches = 0;
        c->sample_steps = 0;
    }
    return SGTP_OK;
}

}  // extern "C"
