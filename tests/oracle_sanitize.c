/* Drives the oracle's entry points once each on small problems so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer can check its memory accesses and arithmetic
 * (test infrastructure: built and run by tests/test_oracle_sanitize.py).  Exits non-zero if a
 * result that must be finite is not. */
#include "../oracle/afm_oracle.c"

#include <stdio.h>

static int bad = 0;
static void need(int ok, const char *what) {
    if (!ok) {
        fprintf(stderr, "not finite or failed: %s\n", what);
        bad = 1;
    }
}

static orc_model point_mass(int law, int N, int nc, int lock, int ic) {
    orc_model m;
    memset(&m, 0, sizeof(m));
    m.n_modes = 1;
    m.law = law;
    m.steps_per_cycle = N;
    m.n_cycles = nc;
    m.lockin_cycles = lock;
    m.ic = ic;
    m.k = 40.0;
    m.f0 = 300e3;
    m.drive_freq = 300e3;
    m.free_amplitude = 20e-9;
    m.div_limit = 100.0;
    m.q[0] = 400.0;
    m.ratio[0] = 1.0;
    m.gain[0] = 1.0;
    m.drive_mode = ORC_DRIVE_TABLE;
    return m;
}

int main(void) {
    /* DMT point mass: forward with trace and misfit against it, gradient, points, steady exit */
    orc_model m = point_mass(ORC_LAW_DMT, 64, 30, 4, ORC_IC_FREE_STEADY);
    double p[ORC_MAX_PARAMS] = {14.6e-9, 6.4e-20, 1e9, 0.3e-9, 10e-9};
    const int W = 4 * 64;
    double U[4 * 64], tr[4 * 64], A, phi, J, g[ORC_MAX_PARAMS];
    need(orc_forward(&m, p, m.n_cycles, NULL, &A, &phi, &J, U) == 0 && isfinite(A), "forward");
    for (int i = 0; i < W; i++) U[i] *= 0.98;
    need(orc_forward(&m, p, m.n_cycles, U, &A, &phi, &J, tr) == 0 && isfinite(J), "misfit");
    need(orc_misfit_grad(&m, p, m.n_cycles, U, &J, g) == 0 && isfinite(g[1]), "gradient dmt");
    double wts[2] = {1.0, 0.5}, Ap[2], php[2], trp[2 * 4 * 64];
    need(orc_forward_points(&m, p, m.n_cycles, 2, wts, Ap, php, trp) == 0 && isfinite(Ap[1]),
         "points");
    int32_t used = 0;
    need(orc_forward_steady(&m, p, m.n_cycles, 1e-4, U, &A, &phi, &J, tr, &used) == 0 &&
             isfinite(A),
         "steady exit");
    int32_t cyc = 0;
    need(isfinite(orc_steady_amplitude(&m, p, 200, 1e-6, &cyc)), "steady amplitude");
    need(isfinite(orc_zc_from_setpoint(&m, p, 0.8, 200, 1e-6, 1e-6)), "set-point search");

    /* PSO and L-BFGS on (H, E*) */
    int32_t idx[2] = {1, 2}, logs[2] = {0, 1}, gen = -1;
    double lo[2] = {1e-20, 0.1e9}, hi[2] = {1e-19, 10e9}, bz[2], bJ, hist[3];
    orc_pso_invert(&m, p, 2, idx, lo, hi, logs, U, 6, 3, 7, 0.0, 0.7298, 1.49618, 1.49618, 1.0,
                   bz, &bJ, &gen, hist);
    need(isfinite(bJ), "pso");
    need(isfinite(orc_lbfgs(&m, p, 2, idx, lo, hi, logs, U, bz, 2)), "lbfgs");

    /* LJ from rest, 3-mode Kelvin-Voigt, spring-damper, the parameter-driven base */
    orc_model lj = point_mass(ORC_LAW_LJ, 64, 20, 2, ORC_IC_REST);
    double pl[ORC_MAX_PARAMS] = {16.3e-9, 1.25e-19, 0.35e-9, 10.0, 5.5};
    double Ul[2 * 64];
    need(orc_forward(&lj, pl, lj.n_cycles, NULL, &A, &phi, &J, Ul) == 0, "forward lj");
    need(orc_misfit_grad(&lj, pl, lj.n_cycles, Ul, &J, g) == 0 && isfinite(g[2]), "gradient lj");
    orc_model kv = point_mass(ORC_LAW_KV, 128, 12, 2, ORC_IC_FREE_STEADY);
    kv.n_modes = 3;
    double bL[3], ratio[3], mass[3], gain[3];
    orc_eb_modes(3, 101, bL, ratio, mass, gain);
    for (int i = 0; i < 3; i++) {
        kv.q[i] = 400.0;
        kv.ratio[i] = ratio[i];
        kv.gain[i] = gain[i];
    }
    double pk[ORC_MAX_PARAMS] = {11e-9, 6.4e-20, 0.5e9, 0.3e-9, 10e-9, 20.0};
    double Uk[2 * 128];
    need(orc_forward(&kv, pk, kv.n_cycles, NULL, &A, &phi, &J, Uk) == 0, "forward kv3");
    need(orc_misfit_grad(&kv, pk, kv.n_cycles, Uk, &J, g) == 0 && isfinite(g[5]), "gradient kv3");
    orc_model sd = point_mass(ORC_LAW_SD, 64, 10, 2, ORC_IC_REST);
    double ps[ORC_MAX_PARAMS] = {15e-9, 4.0, 0.1e-6};
    need(orc_forward(&sd, ps, sd.n_cycles, NULL, &A, &phi, &J, NULL) == 0, "forward sd");
    orc_model ch = point_mass(ORC_LAW_NONE, 64, 3, 3, ORC_IC_REST);
    ch.drive_mode = ORC_DRIVE_PARAMS;
    double pc[ORC_MAX_PARAMS] = {0.0};
    pc[ORC_P_A] = 0.05e-9;
    pc[ORC_P_F] = 290e3;
    pc[ORC_P_G] = 1e9;
    double Uc[3 * 64];
    need(orc_forward(&ch, pc, ch.n_cycles, NULL, &A, &phi, &J, Uc) == 0, "forward chirp");
    need(orc_misfit_grad(&ch, pc, ch.n_cycles, Uc, &J, g) == 0, "gradient chirp");

    /* random numbers */
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    orc_philox4x32_10(ctr, key, out);
    need(orc_u53(out[0], out[1]) < 1.0, "philox");
    if (!bad) printf("oracle sanitizer run: all entry points exercised\n");
    return bad;
}
