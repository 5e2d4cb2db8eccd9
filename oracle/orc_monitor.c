/*
 * Oracle: magnitude of the Kreiss-Oliger dissipation term (Sec. II.B.1,
 * eq. semidiscrete: Q_d added to the right-hand side of every field) at every
 * interior point.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include "oracle.h"

void orc_ko_monitor(int system, const double* U, double* M, int nx, int ny, int nz,
                    const double h[3], const orc_params* p)
{
    long NX = nx + 2 * ORC_G, NY = ny + 2 * ORC_G, NZ = nz + 2 * ORC_G;
    long vol = NX * NY * NZ;
    long st[3] = {1, NX, NX * NY};
    int nf = orc_nfields(system);
    for (int kk = ORC_G; kk < nz + ORC_G; ++kk)
        for (int jj = ORC_G; jj < ny + ORC_G; ++jj)
            for (int ii = ORC_G; ii < nx + ORC_G; ++ii) {
                long c = (kk * NY + jj) * NX + ii;
                double s = 0.0;
                for (int f = 0; f < nf; ++f) {
                    /* summed over the axes in the order the right-hand sides use */
                    double q = 0.0;
                    for (int d = 0; d < 3; ++d) q += orc_ko(U + (long)f * vol + c, st[d], h[d], p->sigma);
                    s += q * q;
                }
                M[c] = s;
            }
}
