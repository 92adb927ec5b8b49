// opcount.cpp -- operation counts of the oracle's per-sample work.
//
// TEST AND MEASUREMENT INFRASTRUCTURE, like the rest of this directory: it counts the
// work the method defines per sample and horizon step, the numerator of the achieved
// FLOP rate.  The oracle source (sgtp_ref.c) is compiled here as C++ with counting types
// in place of its per-sample scalar types `real` (double) and `real32` (float, the
// Box-Muller specification): every arithmetic operation on a value that depends on the
// sample is counted by kind and precision.  Values that do not depend on the sample
// (parameters, raceline rows, opponent predictions, the vehicle's current state) stay
// double in the oracle and are not counted.  Integer work (the Philox rounds) is not a
// floating-point operation and is not counted either.
//
// Kinds: add (and subtract), mul, fma (2 operations), cmp (compare, min, max), and the
// elementary operations listed on their own: div, sqrt, sin, cos, tan, atan, remainder.
// Sign operations (negation, fabs, copysign) and classification (isfinite, isnan) are
// not arithmetic and are not counted.
#include <cmath>
#include <cstdint>
#include <cstring>

namespace opc {
enum Kind { ADD, MUL, FMA, CMP, DIV, SQRT, SIN, COS, TAN, ATAN, REM, NKIND };
long long n64[NKIND], n32[NKIND];
}  // namespace opc

struct CReal {
    double v;
    CReal() : v(0.0) {}
    CReal(double x) : v(x) {}
};
struct CF32 {
    float v;
    CF32() : v(0.0f) {}
    CF32(float x) : v(x) {}
};

#define OPC_BIN(T, CNT, OP, KIND)                                                          \
    inline T operator OP(T a, T b) {                                                      \
        ++opc::CNT[opc::KIND];                                                             \
        return T(a.v OP b.v);                                                              \
    }                                                                                      \
    inline T &operator OP##=(T &a, T b) {                                                  \
        ++opc::CNT[opc::KIND];                                                             \
        a.v = a.v OP b.v;                                                                  \
        return a;                                                                          \
    }
#define OPC_CMP(T, CNT, OP)                                                                \
    inline bool operator OP(T a, T b) {                                                   \
        ++opc::CNT[opc::CMP];                                                              \
        return a.v OP b.v;                                                                 \
    }
#define OPC_TYPE(T, CNT)                                                                   \
    OPC_BIN(T, CNT, +, ADD)                                                                \
    OPC_BIN(T, CNT, -, ADD)                                                                \
    OPC_BIN(T, CNT, *, MUL)                                                                \
    OPC_BIN(T, CNT, /, DIV)                                                                \
    OPC_CMP(T, CNT, <)                                                                     \
    OPC_CMP(T, CNT, <=)                                                                    \
    OPC_CMP(T, CNT, >)                                                                     \
    OPC_CMP(T, CNT, >=)                                                                    \
    OPC_CMP(T, CNT, ==)                                                                    \
    OPC_CMP(T, CNT, !=)                                                                    \
    inline T operator-(T a) { return T(-a.v); }

OPC_TYPE(CReal, n64)
OPC_TYPE(CF32, n32)

// float64 elementary functions and min / max
inline CReal fmax(CReal a, CReal b) { ++opc::n64[opc::CMP]; return CReal(std::fmax(a.v, b.v)); }
inline CReal fmin(CReal a, CReal b) { ++opc::n64[opc::CMP]; return CReal(std::fmin(a.v, b.v)); }
inline CReal fabs(CReal a) { return CReal(std::fabs(a.v)); }
inline CReal copysign(CReal a, CReal b) { return CReal(std::copysign(a.v, b.v)); }
inline CReal sqrt(CReal a) { ++opc::n64[opc::SQRT]; return CReal(std::sqrt(a.v)); }
inline CReal sin(CReal a) { ++opc::n64[opc::SIN]; return CReal(std::sin(a.v)); }
inline CReal cos(CReal a) { ++opc::n64[opc::COS]; return CReal(std::cos(a.v)); }
inline CReal tan(CReal a) { ++opc::n64[opc::TAN]; return CReal(std::tan(a.v)); }
inline CReal atan(CReal a) { ++opc::n64[opc::ATAN]; return CReal(std::atan(a.v)); }
inline CReal remainder(CReal a, CReal b) { ++opc::n64[opc::REM]; return CReal(std::remainder(a.v, b.v)); }
inline bool isfinite(CReal a) { return std::isfinite(a.v); }
inline bool isnan(CReal a) { return std::isnan(a.v); }
// float32 (the Box-Muller specification)
inline CF32 fmaf(CF32 a, CF32 b, CF32 c) { ++opc::n32[opc::FMA]; return CF32(std::fma(a.v, b.v, c.v)); }
inline CF32 sqrtf(CF32 a) { ++opc::n32[opc::SQRT]; return CF32(std::sqrt(a.v)); }

#define REF_COUNTING 1
typedef CReal real;
typedef CF32 real32;
#define REF_D(x) ((x).v)
#define REF_F(x) ((x).v)

#include "sgtp_ref.c"

// One best response of `agent` (ref_rollout_cost) with the counters reset first;
// counts[0..NKIND) receive the float64 counts, counts[NKIND..2 NKIND) the float32 ones.
extern "C" int ref_opcount_kinds(void) { return opc::NKIND; }
extern "C" int ref_opcount_rollout_cost(const ref_track *T, const ref_params *p, const ref_race *R, int agent,
                                        int phase, long long *counts) {
    std::memset(opc::n64, 0, sizeof opc::n64);
    std::memset(opc::n32, 0, sizeof opc::n32);
    ref_choice ch;
    const int rc = ref_rollout_cost(T, p, R, agent, phase, nullptr, &ch, nullptr);
    for (int i = 0; i < opc::NKIND; ++i) {
        counts[i] = opc::n64[i];
        counts[opc::NKIND + i] = opc::n32[i];
    }
    return rc;
}
