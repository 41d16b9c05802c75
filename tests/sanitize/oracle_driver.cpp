// Sanitizer driver for the oracle: built with -fsanitize=address,undefined
// by tests/test_sanitizers.py and run on the CPU.  Exercises the step, the
// traced step, the binary32 run, the loss, its tangent and its gradient on a
// small rough state with every boundary kind, thin films and dry cells.
#include "../../oracle/swe_oracle.cpp"

#include <stdio.h>

int main() {
    const int nx = 23, ny = 17;
    const size_t N = (size_t)nx * ny;
    std::vector<double> z(N), n(N), eta(N), qx(N), qy(N);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t s = (size_t)j * nx + i;
            z[s] = 0.3 * sin(0.7 * i) * cos(0.5 * j) + 0.02 * i;
            const double h = (i + j) % 7 == 0 ? 0.0 : ((i * j) % 5 == 0 ? 5e-4 : 0.4 + 0.1 * cos(i + 2.0 * j));
            eta[s] = z[s] + h;
            qx[s] = h > 1e-3 ? 0.1 * sin(0.3 * j) : 0.0;
            qy[s] = h > 1e-3 ? -0.05 * cos(0.2 * i) : 0.0;
            n[s] = 0.03 + 0.01 * sin(0.1 * (i + j));
        }
    const double ht[3] = {0.0, 1.0, 3.0}, hq[3] = {0.0, 0.8, 0.2};
    orc_cfg c;
    memset(&c, 0, sizeof c);
    c.nx = nx; c.ny = ny;
    c.bc[0] = BC_INFLOW; c.bc[1] = BC_OPEN; c.bc[2] = BC_WALL; c.bc[3] = BC_OPEN;
    for (int k = 0; k < 4; ++k) { c.in_lo[k] = 2; c.in_hi[k] = 12; }
    c.hydro_len = 3; c.hydro_t = ht; c.hydro_q = hq;
    c.dx = 1.0; c.dy = 1.5; c.g = 9.81; c.cfl = 0.5; c.h_dry = 1e-3; c.kappa = 0.5;
    c.eps_max = 0.25; c.dt_max = 1.0; c.dt_fixed = 0.0; c.h_film = 0.05;
    int rc = 0;
    // plain and traced steps
    {
        std::vector<double> e = eta, a = qx, b = qy;
        double t = 0.0, dt = 0.0;
        int64_t step = 0;
        orc_stats st;
        rc |= orc_run(&c, e.data(), a.data(), b.data(), z.data(), n.data(), &t, &step, &dt, 12,
                      INFINITY, &st) < 0;
        std::vector<double> arrays((size_t)ORC_NTRACE * (nx + 2) * (ny + 2)), sc(ORC_NSCALAR);
        rc |= orc_trace(&c, e.data(), a.data(), b.data(), z.data(), n.data(), t, step, dt,
                        arrays.data(), sc.data()) < 0;
        std::vector<double> e2 = eta, a2 = qx, b2 = qy;
        double t2 = 0.0, dt2 = 0.0;
        int64_t s2 = 0;
        rc |= orc_run_f32(&c, e2.data(), a2.data(), b2.data(), z.data(), n.data(), &t2, &s2,
                          &dt2, 12, INFINITY, &st) < 0;
    }
    // the loss, its tangent and its gradient
    {
        const int64_t nsteps = 10;
        std::vector<double> dts(nsteps);
        std::vector<double> e = eta, a = qx, b = qy;
        double t = 0.0, dt = 0.0;
        int64_t step = 0;
        orc_stats st;
        rc |= orc_run_record(&c, e.data(), a.data(), b.data(), z.data(), n.data(), &t, &step,
                             &dt, nsteps, INFINITY, &st, dts.data()) < 0;
        const int64_t gauges[4] = {30, 77, 150, 301};
        std::vector<double> hobs(5 * 4, 0.2);
        double J = 0.0, dJ = 0.0;
        std::vector<double> dn(N, 1e-3), gn(N), gz(N);
        rc |= orc_loss_tangent(&c, eta.data(), qx.data(), qy.data(), z.data(), n.data(), 0.0, 0,
                               nsteps, dts.data(), 4, gauges, 2, hobs.data(), dn.data(), nullptr,
                               &J, &dJ) < 0;
        rc |= orc_loss_gradient(&c, eta.data(), qx.data(), qy.data(), z.data(), n.data(), 0.0, 0,
                                nsteps, dts.data(), 4, gauges, 2, hobs.data(), &J, gn.data(),
                                gz.data()) < 0;
        double dot = 0.0;
        for (size_t s = 0; s < N; ++s) dot += gn[s] * dn[s];
        printf("J %.6e  tangent %.6e  <grad, dn> %.6e\n", J, dJ, dot);
    }
    printf(rc ? "oracle driver: a call failed\n" : "oracle driver: ok\n");
    return rc;
}
