// opcount.cpp -- op-counting build of the FP64 oracle (test and measurement
// infrastructure, like the oracle itself; never linked into libctu).
//
// ctu_oracle.c is compiled unchanged as C++ with every `double` replaced by
// Real, a double that counts the arithmetic done on it: additions and
// subtractions, multiplications, divisions, square roots, transcendental
// calls (exp, log, pow, cbrt), and separately comparisons and min / max /
// abs / copysign.  ORC_STAGE(k) in orc_step snapshots the counters at the
// end of each stage, so the counts split into primitive recovery (1), the
// t^n fluxes and their increments (2), the normal predictors and corner
// coupling (3), the time-centred Riemann solves (4), with parabolic terms the
// half-step state V^{n+1/2} (5) and its fluxes (6), and the update, split
// sources and CFL rate (7).  The numerical
// inversion of the right-eigenvector matrix, which stands in for the
// closed-form left eigenvectors, and the relativistic conserved-to-primitive
// bisections are booked apart (ORC_SIDE_*, ORC_ROOT_*).
// The library is single-threaded (built without OpenMP).  Used by
// oracle/opcount.py.
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

namespace opc {
enum { ADD, MUL, DIV, SQRT, TRANS, CMP, MINMAX, NCAT };
static uint64_t cnt[NCAT];
static uint64_t stage[8][NCAT];  // [1..7]: snapshots at the stage ends
static uint64_t side[NCAT];   // operations of the numerical eigenvector inversions
static uint64_t root[NCAT];   // operations of the relativistic inversions (bisection)
static uint64_t nroot = 0;    // relativistic inversions done
static uint64_t saved[NCAT];
inline void side_begin() { std::memcpy(saved, cnt, sizeof(cnt)); }
inline void side_end(uint64_t *into)
{
    for (int c = 0; c < NCAT; c++) into[c] += cnt[c] - saved[c];
    std::memcpy(cnt, saved, sizeof(cnt));
}
}  // namespace opc

struct Real {
    double v;
    Real() = default;
    constexpr Real(double x) : v(x) {}
    explicit operator double() const { return v; }
    Real &operator+=(Real b) { opc::cnt[opc::ADD]++; v += b.v; return *this; }
    Real &operator-=(Real b) { opc::cnt[opc::ADD]++; v -= b.v; return *this; }
    Real &operator*=(Real b) { opc::cnt[opc::MUL]++; v *= b.v; return *this; }
    Real &operator/=(Real b) { opc::cnt[opc::DIV]++; v /= b.v; return *this; }
    Real &operator++() { opc::cnt[opc::ADD]++; v += 1.0; return *this; }
};

#define OPC_BIN(op, cat)                                                              \
    inline Real operator op(Real a, Real b) { opc::cnt[opc::cat]++; return Real(a.v op b.v); } \
    inline Real operator op(Real a, double b) { opc::cnt[opc::cat]++; return Real(a.v op b); } \
    inline Real operator op(double a, Real b) { opc::cnt[opc::cat]++; return Real(a op b.v); } \
    inline Real operator op(Real a, int b) { opc::cnt[opc::cat]++; return Real(a.v op b); }    \
    inline Real operator op(int a, Real b) { opc::cnt[opc::cat]++; return Real(a op b.v); }
OPC_BIN(+, ADD)
OPC_BIN(-, ADD)
OPC_BIN(*, MUL)
OPC_BIN(/, DIV)
#undef OPC_BIN
inline Real operator-(Real a) { return Real(-a.v); }  // a sign flip, not counted
inline Real operator+(Real a) { return a; }

#define OPC_CMP(op)                                                                   \
    inline bool operator op(Real a, Real b) { opc::cnt[opc::CMP]++; return a.v op b.v; } \
    inline bool operator op(Real a, double b) { opc::cnt[opc::CMP]++; return a.v op b; } \
    inline bool operator op(double a, Real b) { opc::cnt[opc::CMP]++; return a op b.v; } \
    inline bool operator op(Real a, int b) { opc::cnt[opc::CMP]++; return a.v op b; }    \
    inline bool operator op(int a, Real b) { opc::cnt[opc::CMP]++; return a op b.v; }
OPC_CMP(<)
OPC_CMP(>)
OPC_CMP(<=)
OPC_CMP(>=)
OPC_CMP(==)
OPC_CMP(!=)
#undef OPC_CMP

inline Real sqrt(Real a) { opc::cnt[opc::SQRT]++; return Real(std::sqrt(a.v)); }
inline Real exp(Real a) { opc::cnt[opc::TRANS]++; return Real(std::exp(a.v)); }
inline Real log(Real a) { opc::cnt[opc::TRANS]++; return Real(std::log(a.v)); }
inline Real cbrt(Real a) { opc::cnt[opc::TRANS]++; return Real(std::cbrt(a.v)); }
inline Real pow(Real a, Real b) { opc::cnt[opc::TRANS]++; return Real(std::pow(a.v, b.v)); }
inline Real pow(Real a, double b) { opc::cnt[opc::TRANS]++; return Real(std::pow(a.v, b)); }
inline Real pow(double a, Real b) { opc::cnt[opc::TRANS]++; return Real(std::pow(a, b.v)); }
inline Real fabs(Real a) { opc::cnt[opc::MINMAX]++; return Real(std::fabs(a.v)); }
inline Real fmax(Real a, Real b) { opc::cnt[opc::MINMAX]++; return Real(std::fmax(a.v, b.v)); }
inline Real fmin(Real a, Real b) { opc::cnt[opc::MINMAX]++; return Real(std::fmin(a.v, b.v)); }
inline Real fmax(Real a, double b) { opc::cnt[opc::MINMAX]++; return Real(std::fmax(a.v, b)); }
inline Real fmin(Real a, double b) { opc::cnt[opc::MINMAX]++; return Real(std::fmin(a.v, b)); }
inline Real fmax(double a, Real b) { opc::cnt[opc::MINMAX]++; return Real(std::fmax(a, b.v)); }
inline Real fmin(double a, Real b) { opc::cnt[opc::MINMAX]++; return Real(std::fmin(a, b.v)); }
inline Real copysign(Real a, Real b) { opc::cnt[opc::MINMAX]++; return Real(std::copysign(a.v, b.v)); }
inline Real floor(Real a) { return Real(std::floor(a.v)); }
inline bool isnan(Real a) { return std::isnan(a.v); }
inline bool isfinite(Real a) { return std::isfinite(a.v); }

#define ORC_STAGE(k) std::memcpy(opc::stage[k], opc::cnt, sizeof(opc::cnt))
#define ORC_SIDE_BEGIN opc::side_begin()
#define ORC_SIDE_END opc::side_end(opc::side)
#define ORC_ROOT_BEGIN (opc::side_begin(), opc::nroot++)
#define ORC_ROOT_END opc::side_end(opc::root)
#define double Real
extern "C" {
#include "ctu_oracle.c"
}
#undef double

extern "C" {

// clear the counters and the stage snapshots
void opc_reset(void)
{
    std::memset(opc::cnt, 0, sizeof(opc::cnt));
    std::memset(opc::stage, 0, sizeof(opc::stage));
    std::memset(opc::side, 0, sizeof(opc::side));
    std::memset(opc::root, 0, sizeof(opc::root));
    opc::nroot = 0;
}

// out[11][NCAT] + 1: counter snapshots at the end of stages 1..7 of the
// last orc_step (row 0 unused; a stage the option set skips keeps a zero
// row), row 8 the counters now, row 9 the operations of the numerical
// eigenvector inversions, row 10 those of the relativistic inversions (both
// kept out of the other rows), then the number of relativistic inversions;
// returns NCAT
int opc_read(uint64_t *out)
{
    std::memcpy(out, opc::stage, sizeof(opc::stage));
    std::memcpy(out + 8 * opc::NCAT, opc::cnt, sizeof(opc::cnt));
    std::memcpy(out + 9 * opc::NCAT, opc::side, sizeof(opc::side));
    std::memcpy(out + 10 * opc::NCAT, opc::root, sizeof(opc::root));
    out[11 * opc::NCAT] = opc::nroot;
    return opc::NCAT;
}

}  // extern "C"
