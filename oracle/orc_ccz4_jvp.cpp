/*
 * Oracle: exact Jacobian-vector product of the CCZ4 right-hand side,
 *   R'(U) V = d/de R(U + e V) at e = 0,
 * by forward-mode differentiation of the oracle itself: the stencils
 * (orc_stencil.c) and the CCZ4 right-hand side (orc_ccz4.c) are compiled a
 * second time with every double replaced by a dual number (value,
 * derivative).  The value part repeats the oracle's arithmetic operation by
 * operation, so it equals orc_ccz4_rhs bitwise; the derivative part is the
 * JVP up to rounding (no difference quotient).  The transpose of this map,
 * assembled column by column in oracle.py, is the reference for the discrete
 * adjoint.  The sign branch of the lop-sided stencils is taken on the value
 * part, so it is frozen at U, as the adjoint requires.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

namespace orc_dual {

struct Dual {
    double v, d;
    Dual(double a = 0.0, double b = 0.0) : v(a), d(b) {}
    Dual& operator+=(const Dual& o) { d += o.d; v += o.v; return *this; }
    Dual& operator-=(const Dual& o) { d -= o.d; v -= o.v; return *this; }
};
inline Dual operator-(const Dual& a) { return Dual(-a.v, -a.d); }
inline Dual operator+(const Dual& a, const Dual& b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(const Dual& a, const Dual& b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator*(const Dual& a, const Dual& b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(const Dual& a, const Dual& b)
{
    const double q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual operator+(const Dual& a, double b) { return Dual(a.v + b, a.d); }
inline Dual operator+(double a, const Dual& b) { return Dual(a + b.v, b.d); }
inline Dual operator-(const Dual& a, double b) { return Dual(a.v - b, a.d); }
inline Dual operator-(double a, const Dual& b) { return Dual(a - b.v, -b.d); }
inline Dual operator*(const Dual& a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator*(double a, const Dual& b) { return Dual(a * b.v, a * b.d); }
inline Dual operator/(const Dual& a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual operator/(double a, const Dual& b)
{
    const double q = a / b.v;
    return Dual(q, -q * b.d / b.v);
}
inline bool operator>=(const Dual& a, double b) { return a.v >= b; }
inline Dual log1p(const Dual& a) { return Dual(::log1p(a.v), a.d / (1.0 + a.v)); }

#define double Dual
#include "orc_stencil.c"
#include "orc_ccz4.c"
#undef double

}  // namespace orc_dual

extern "C" void orc_ccz4_rhs_jvp(const double* U, const double* V, double* R, double* RV, int nx, int ny, int nz,
                                 const double h[3], const orc_params* p)
{
    const long n = 25L * (nx + 2 * ORC_G) * (ny + 2 * ORC_G) * (nz + 2 * ORC_G);
    orc_dual::Dual* X = (orc_dual::Dual*)calloc(n, sizeof(orc_dual::Dual));
    orc_dual::Dual* Y = (orc_dual::Dual*)calloc(n, sizeof(orc_dual::Dual));
    for (long i = 0; i < n; ++i) X[i] = orc_dual::Dual(U[i], V[i]);
    const orc_dual::Dual hh[3] = {h[0], h[1], h[2]};
    orc_dual::orc_ccz4_rhs(X, Y, nx, ny, nz, hh, p);
    for (long i = 0; i < n; ++i) {
        R[i] = Y[i].v;
        RV[i] = Y[i].d;
    }
    free(X);
    free(Y);
}
