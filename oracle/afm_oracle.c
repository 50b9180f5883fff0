/*
 * afm_oracle.c -- reference computation for the dynamic-AFM tip-sample force inversion.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, single-threaded FP64 CPU statement of
 * what the GPU library computes.  It exists so the GPU path can be checked against something
 * written directly from the paper (Busch, Zou, Ganapathysubramanian, "A near real-time framework
 * for extracting tip-sample forces in dynamic atomic force microscopy", arXiv 1109.0334).  Only
 * the test suite, the package smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never does, and this file shares no source with the GPU library.
 *
 * Units are SI throughout (metres, seconds, newtons).  No blocking, fusion or reordering: every
 * function follows the definition it cites, in the order the paper states it.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared afm_oracle.c -lm
 *
 * Model (paper Sec. 2.2, Eq. 1-2; modal reduction Appendix B Eq. 13-14):
 *   u(t)   = sum_i q_i(t)                tip deflection relative to the base, tip-normalised modes
 *   d      = z_c + u                     tip-sample gap (u positive away from the sample)
 *   q_i'' + (w_i/Q_i) q_i' + w_i^2 q_i = F(d, d')/M + gamma_i * a * wd^2 * sin(wd t)
 * Eq. 2 writes the damping as 2 zeta w_i; here zeta_i = 1/(2 Q_i).  The last term is -Y_i of
 * Eq. 2: the base acceleration -y_b'' of the sinusoidal base motion y_b = a sin(2 pi f t) (Eq. 9)
 * projected on mode i.  F > 0 is repulsive (pushes the tip away from the sample).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_MODES 8
#define ORC_MAX_PARAMS 12

/* Force laws.  Parameter vector p[] always holds the separation z_c at index 0. */
enum {
    ORC_LAW_DMT = 0,   /* p = {z_c, H, E*, a0, R}          */
    ORC_LAW_LJ = 1,    /* p = {z_c, eps, r0, n, m}         */
    ORC_LAW_KV = 2,    /* p = {z_c, H, E*, a0, R, eta}     */
    ORC_LAW_HOOKE = 3, /* p = {z_c, k_s}          Eq. 3     */
    ORC_LAW_SD = 4,    /* p = {z_c, k_s, zeta_s}  Eq. 4, 12 */
    ORC_LAW_NONE = 5   /* p = {z_c}  (tip force switched off) */
};
static const int orc_law_nparams[6] = {5, 5, 6, 2, 3, 1};

enum { ORC_IC_FREE_STEADY = 0, ORC_IC_REST = 1 };
enum { ORC_ST_NONFINITE = 1, ORC_ST_DIVERGED = 2 };

typedef struct {
    int32_t n_modes;         /* 1 = point mass                                      */
    int32_t law;             /* ORC_LAW_*                                           */
    int32_t steps_per_cycle; /* N: RK4 steps per drive period                       */
    int32_t n_cycles;        /* Nc: drive periods integrated                        */
    int32_t lockin_cycles;   /* periods at the end used for lock-in and misfit      */
    int32_t ic;              /* ORC_IC_*                                            */
    double k;                /* first-mode stiffness, N/m                           */
    double f0;               /* first-mode natural frequency, Hz                    */
    double drive_freq;       /* base drive frequency, Hz                            */
    double free_amplitude;   /* A0: free tip amplitude, m (sets the base amplitude) */
    double div_limit;        /* |u| > div_limit * A0 at a period end => diverged    */
    double q[ORC_MAX_MODES];     /* quality factor per mode                         */
    double ratio[ORC_MAX_MODES]; /* w_i / w_0                                        */
    double gain[ORC_MAX_MODES];  /* gamma_i: base-drive participation of mode i      */
    int32_t drive_mode;          /* ORC_DRIVE_*                                      */
} orc_model;

/* Base motion.  TABLE: y_b = a sin(wd t) with a set from the free amplitude A0 (the force
 * inversions).  PARAMS: the chirp of Eq. 10, y_b = a sin(2 pi (f + g t) t), with a = p[8] (m),
 * f = p[9] (Hz) and g = p[10] (Hz/s) per trajectory (g = 0: the sinusoid of Eq. 9), the
 * base-motion and chirp inversions of Sec. 4; the time step stays 1 / (drive_freq N). */
enum { ORC_DRIVE_TABLE = 0, ORC_DRIVE_PARAMS = 1 };
enum { ORC_P_A = 8, ORC_P_F = 9, ORC_P_G = 10 };

int orc_law_param_count(int law) { return (law >= 0 && law <= 5) ? orc_law_nparams[law] : -1; }

/* Entries of p that describe one trajectory: the law's, plus the base motion's with PARAMS. */
static int param_count(const orc_model *mo) {
    return mo->drive_mode == ORC_DRIVE_PARAMS ? ORC_MAX_PARAMS : orc_law_param_count(mo->law);
}

/* ------------------------------------------------------------------------------------------ */
/* Derived constants                                                                          */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    int m;            /* modes                               */
    double wd;        /* drive angular frequency             */
    double w[ORC_MAX_MODES];
    double c[ORC_MAX_MODES]; /* w_i / Q_i                    */
    double M;         /* modal mass k / w_0^2 (same for every tip-normalised mode) */
    double a;         /* base amplitude                      */
    double h;         /* time step 1/(f_d N)                 */
} orc_derived;

/* Free linear response of mode i per unit base amplitude, complex amplitude of q_i for
 * y_b = Im(e^{i wd t}):  H_i = gamma_i wd^2 / (w_i^2 - wd^2 + i w_i wd / Q_i). */
static double complex free_response(const orc_model *mo, const orc_derived *dv, int i) {
    double wd = dv->wd, wi = dv->w[i];
    return mo->gain[i] * wd * wd / ((wi * wi - wd * wd) + I * (wi * wd / mo->q[i]));
}

static void derive(const orc_model *mo, orc_derived *dv) {
    dv->m = mo->n_modes;
    dv->wd = 2.0 * M_PI * mo->drive_freq;
    double w0 = 2.0 * M_PI * mo->f0;
    for (int i = 0; i < dv->m; i++) {
        dv->w[i] = w0 * mo->ratio[i];
        dv->c[i] = dv->w[i] / mo->q[i];
    }
    dv->M = mo->k / (w0 * w0);
    /* Base amplitude a chosen so that the free (tip force off) steady tip amplitude is A0. */
    double complex s = 0.0;
    for (int i = 0; i < dv->m; i++) s += free_response(mo, dv, i);
    dv->a = mo->free_amplitude / cabs(s);
    dv->h = 1.0 / (mo->drive_freq * (double)mo->steps_per_cycle);
}

double orc_base_amplitude(const orc_model *mo) {
    orc_derived dv;
    derive(mo, &dv);
    return dv.a;
}

/* Initial state y = (q_1..q_m, q_1'..q_m').  FREE_STEADY: the linear free steady state at t = 0,
 * q_i = Im(a H_i), q_i' = wd Re(a H_i).  REST: zero. */
void orc_initial_state(const orc_model *mo, double *y) {
    orc_derived dv;
    derive(mo, &dv);
    int m = dv.m;
    for (int i = 0; i < m; i++) {
        if (mo->ic == ORC_IC_FREE_STEADY) {
            double complex Hi = dv.a * free_response(mo, &dv, i);
            y[i] = cimag(Hi);
            y[m + i] = dv.wd * creal(Hi);
        } else {
            y[i] = 0.0;
            y[m + i] = 0.0;
        }
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Tip-sample force laws F(d, d'; p) and their partial derivatives                             */
/* ------------------------------------------------------------------------------------------ */

/* DMT: van der Waals sphere-plane attraction -H R / (6 d^2) out of contact; in contact
 * (d <= a0) the attraction saturates at its a0 value and Hertz repulsion (4/3) E* sqrt(R)
 * (a0 - d)^{3/2} is added.  The paper names Hertz and van der Waals forces as the richer
 * models beyond Eq. 3-4 (Sec. 2.2) and adhesion / van der Waals as an extension (Sec. 5). */
static double f_dmt(double H, double E, double a0, double R, double d) {
    if (d > a0) return -H * R / (6.0 * d * d);
    double del = a0 - d;
    return -H * R / (6.0 * a0 * a0) + (4.0 / 3.0) * E * sqrt(R) * del * sqrt(del);
}

/* Lennard-Jones-type (Mie) force from U = eps [m/(n-m) (r0/d)^n - n/(n-m) (r0/d)^m]:
 * F = -dU/dd = eps n m / (n - m) / d * [(r0/d)^n - (r0/d)^m]; minimum -eps at d = r0. */
static double f_lj(double eps, double r0, double n, double m, double d) {
    double s = r0 / d;
    return eps * (n * m / (n - m)) / d * (pow(s, n) - pow(s, m));
}

/* F(d, dd) for the law; dd is the gap velocity. d <= 0 is unphysical for LJ (returns NaN). */
double orc_force(int law, const double *p, double d, double dd) {
    switch (law) {
    case ORC_LAW_DMT:
        return f_dmt(p[1], p[2], p[3], p[4], d);
    case ORC_LAW_LJ:
        if (!(d > 0.0)) return NAN;
        return f_lj(p[1], p[2], p[3], p[4], d);
    case ORC_LAW_KV: {
        /* DMT plus Kelvin-Voigt dissipation in contact: -eta * (contact radius sqrt(R delta)) * d'
         * (the spring-damper idea of Eq. 4 / Eq. 12 applied to a Hertzian contact). */
        double F = f_dmt(p[1], p[2], p[3], p[4], d);
        if (d <= p[3]) F += -p[5] * sqrt(p[4] * (p[3] - d)) * dd;
        return F;
    }
    case ORC_LAW_HOOKE: /* Eq. 3: elastic sample, acting while the tip presses in (d < 0) */
        return d < 0.0 ? -p[1] * d : 0.0;
    case ORC_LAW_SD: /* Eq. 4 / Eq. 12: spring-damper sample while in contact */
        return d < 0.0 ? -p[1] * d - p[2] * dd : 0.0;
    case ORC_LAW_NONE:
        return 0.0;
    }
    return NAN;
}

/* Partial derivatives: Fd = dF/dd, Fdd = dF/d(d'), Fp[j] = dF/dp_j holding d, d' fixed
 * (Fp[0], the z_c slot, is left 0: z_c enters only through d). */
static void force_partials(int law, const double *p, double d, double dd, double *Fd, double *Fdd,
                           double *Fp) {
    for (int j = 0; j < ORC_MAX_PARAMS; j++) Fp[j] = 0.0;
    *Fd = 0.0;
    *Fdd = 0.0;
    switch (law) {
    case ORC_LAW_DMT:
    case ORC_LAW_KV: {
        double H = p[1], E = p[2], a0 = p[3], R = p[4];
        if (d > a0) {
            *Fd = H * R / (3.0 * d * d * d);
            Fp[1] = -R / (6.0 * d * d);
            Fp[4] = -H / (6.0 * d * d);
        } else {
            double del = a0 - d, sd = sqrt(del), sR = sqrt(R);
            *Fd = -2.0 * E * sR * sd;
            Fp[1] = -R / (6.0 * a0 * a0);
            Fp[2] = (4.0 / 3.0) * sR * del * sd;
            Fp[3] = H * R / (3.0 * a0 * a0 * a0) + 2.0 * E * sR * sd;
            Fp[4] = -H / (6.0 * a0 * a0) + (2.0 / 3.0) * E / sR * del * sd;
            if (law == ORC_LAW_KV) {
                double eta = p[5];
                *Fdd = -eta * sR * sd;
                Fp[5] = -sR * sd * dd;
                if (del > 0.0) {
                    double g = eta * dd * sR / (2.0 * sd); /* d/d(delta) of eta sqrt(R delta) d' */
                    *Fd += g;
                    Fp[3] += -g;
                }
                Fp[4] += -eta * dd * sd / (2.0 * sR);
            }
        }
        break;
    }
    case ORC_LAW_LJ: {
        double eps = p[1], r0 = p[2], n = p[3], m = p[4];
        double s = r0 / d, sn = pow(s, n), sm = pow(s, m), ls = log(s);
        double c = n * m / (n - m);
        *Fd = eps * c / (d * d) * (-(n + 1.0) * sn + (m + 1.0) * sm);
        Fp[1] = c / d * (sn - sm);
        Fp[2] = eps * c / (d * r0) * (n * sn - m * sm);
        double cn = -m * m / ((n - m) * (n - m)), cm = n * n / ((n - m) * (n - m));
        Fp[3] = eps / d * (cn * (sn - sm) + c * sn * ls);
        Fp[4] = eps / d * (cm * (sn - sm) - c * sm * ls);
        break;
    }
    case ORC_LAW_HOOKE:
        if (d < 0.0) {
            *Fd = -p[1];
            Fp[1] = -d;
        }
        break;
    case ORC_LAW_SD:
        if (d < 0.0) {
            *Fd = -p[1];
            *Fdd = -p[2];
            Fp[1] = -d;
            Fp[2] = -dd;
        }
        break;
    default:
        break;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Right-hand side and the classical RK4 step (paper Sec. 3.2)                                */
/* ------------------------------------------------------------------------------------------ */

static void rhs(const orc_model *mo, const orc_derived *dv, const double *p, double t,
                const double *y, double *dy) {
    int m = dv->m;
    double u = 0.0, ud = 0.0;
    for (int i = 0; i < m; i++) {
        u += y[i];
        ud += y[m + i];
    }
    double F = orc_force(mo->law, p, p[0] + u, ud);
    double base_acc; /* -y_b''(t) */
    if (mo->drive_mode == ORC_DRIVE_PARAMS) {
        /* y_b = a sin(phi), phi = 2 pi (f + g t) t, phi' = 2 pi (f + 2 g t), phi'' = 4 pi g:
         * -y_b'' = a (phi'^2 sin(phi) - phi'' cos(phi)) */
        double a = p[ORC_P_A], f = p[ORC_P_F], g = p[ORC_P_G];
        double phi = 2.0 * M_PI * (f + g * t) * t, om = 2.0 * M_PI * (f + 2.0 * g * t);
        base_acc = a * (om * om * sin(phi) - 4.0 * M_PI * g * cos(phi));
    } else {
        base_acc = dv->a * dv->wd * dv->wd * sin(dv->wd * t);
    }
    for (int i = 0; i < m; i++) {
        dy[i] = y[m + i];
        dy[m + i] = -dv->w[i] * dv->w[i] * y[i] - dv->c[i] * y[m + i] + F / dv->M +
                    mo->gain[i] * base_acc;
    }
}

/* One classical RK4 step from t: c = (0, 1/2, 1/2, 1), b = (1/6, 1/3, 1/3, 1/6). */
static void rk4_step(const orc_model *mo, const orc_derived *dv, const double *p, double t,
                     double *y) {
    int n = 2 * dv->m;
    double h = dv->h, k1[2 * ORC_MAX_MODES], k2[2 * ORC_MAX_MODES], k3[2 * ORC_MAX_MODES],
           k4[2 * ORC_MAX_MODES], Y[2 * ORC_MAX_MODES];
    rhs(mo, dv, p, t, y, k1);
    for (int i = 0; i < n; i++) Y[i] = y[i] + 0.5 * h * k1[i];
    rhs(mo, dv, p, t + 0.5 * h, Y, k2);
    for (int i = 0; i < n; i++) Y[i] = y[i] + 0.5 * h * k2[i];
    rhs(mo, dv, p, t + 0.5 * h, Y, k3);
    for (int i = 0; i < n; i++) Y[i] = y[i] + h * k3[i];
    rhs(mo, dv, p, t + h, Y, k4);
    for (int i = 0; i < n; i++) y[i] = y[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

static double tip(const orc_derived *dv, const double *y) {
    double u = 0.0;
    for (int i = 0; i < dv->m; i++) u += y[i];
    return u;
}

/* ------------------------------------------------------------------------------------------ */
/* Trajectory                                                                                 */
/* ------------------------------------------------------------------------------------------ */

/* Deflection at n_pts points along the beam from the tip-normalised modal coordinates (App. B,
 * Eq. 13): u(x_k) = sum_i w[k][i] y_i with w[k][i] = Phi_i(x_k) / Phi_i(L). */
static double point(const orc_derived *dv, const double *w, const double *y) {
    double u = 0.0;
    for (int i = 0; i < dv->m; i++) u += w[i] * y[i];
    return u;
}

/* Integrate n_cycles drive periods (N_tot = n_cycles * N steps) from y0 (NULL: the model's
 * initial condition).  States are y_n, n = 0..N_tot, y_n at t_n = n h.  Writes the tip deflection
 * u_n (and its rate into ud_out if non-NULL) for n = N_tot - n_out + 1 .. N_tot, and, for each of
 * n_pts points with weights w ([n_pts][m]), the deflection there into pts_out ([n_pts][n_out]).
 * At the end of every period the state is checked: non-finite => NONFINITE,
 * |u| > div_limit * A0 => DIVERGED; integration stops there and every output sample is NaN.
 * Returns the status bits. */
static int trajectory(const orc_model *mo, const double *p, int32_t n_cycles, const double *y0,
                      int64_t n_out, double *u_out, double *ud_out, double *y_end, int n_pts,
                      const double *w, double *pts_out) {
    orc_derived dv;
    derive(mo, &dv);
    int m = dv.m, N = mo->steps_per_cycle;
    int64_t Ntot = (int64_t)n_cycles * N, first = Ntot - n_out + 1;
    double y[2 * ORC_MAX_MODES];
    if (y0)
        memcpy(y, y0, sizeof(double) * 2 * m);
    else
        orc_initial_state(mo, y);
    for (int64_t k = 0; k < n_out; k++) {
        if (u_out) u_out[k] = NAN;
        if (ud_out) ud_out[k] = NAN;
        for (int q = 0; q < n_pts; q++) pts_out[q * n_out + k] = NAN;
    }
    if (first <= 0) { /* the initial state is inside the output range */
        int64_t k = 0 - first;
        if (u_out) u_out[k] = tip(&dv, y);
        if (ud_out) {
            double v = 0.0;
            for (int i = 0; i < m; i++) v += y[m + i];
            ud_out[k] = v;
        }
        for (int q = 0; q < n_pts; q++) pts_out[q * n_out + k] = point(&dv, w + q * m, y);
    }
    int status = 0;
    for (int64_t n = 0; n < Ntot; n++) {
        rk4_step(mo, &dv, p, (double)n * dv.h, y);
        int64_t idx = n + 1 - first;
        if (idx >= 0 && idx < n_out) {
            if (u_out) u_out[idx] = tip(&dv, y);
            if (ud_out) {
                double v = 0.0;
                for (int i = 0; i < m; i++) v += y[m + i];
                ud_out[idx] = v;
            }
            for (int q = 0; q < n_pts; q++) pts_out[q * n_out + idx] = point(&dv, w + q * m, y);
        }
        if ((n + 1) % N == 0) {
            double u = tip(&dv, y);
            int bad = 0;
            for (int i = 0; i < 2 * m; i++)
                if (!isfinite(y[i])) bad = 1;
            if (bad) status |= ORC_ST_NONFINITE;
            else if (fabs(u) > mo->div_limit * mo->free_amplitude) status |= ORC_ST_DIVERGED;
            if (status) {
                for (int64_t k = 0; k < n_out; k++) {
                    if (u_out) u_out[k] = NAN;
                    if (ud_out) ud_out[k] = NAN;
                    for (int q = 0; q < n_pts; q++) pts_out[q * n_out + k] = NAN;
                }
                break;
            }
        }
    }
    if (y_end) memcpy(y_end, y, sizeof(double) * 2 * m);
    return status;
}

int orc_trajectory(const orc_model *mo, const double *p, int32_t n_cycles, const double *y0,
                   int64_t n_out, double *u_out, double *ud_out, double *y_end) {
    return trajectory(mo, p, n_cycles, y0, n_out, u_out, ud_out, y_end, 0, NULL, NULL);
}

/* ------------------------------------------------------------------------------------------ */
/* Lock-in projection and misfit                                                              */
/* ------------------------------------------------------------------------------------------ */

/* Lock-in amplitude and phase of W samples u[k] taken at drive-phase index p_k = (p0 + k) mod N
 * (sample at t_n = n h has phase 2 pi n / N).  X = 2/W sum u cos, Y = 2/W sum u sin,
 * A = sqrt(X^2 + Y^2), phi = atan2(-X, Y), so that u ~ A sin(wd t - phi).  The dynamic AFM
 * measures exactly this amplitude and phase and holds the amplitude at a set-point (Sec. 1). */
void orc_lockin(const double *u, int64_t W, int32_t N, int64_t p0, double *A, double *phi) {
    double X = 0.0, Y = 0.0;
    for (int64_t k = 0; k < W; k++) {
        double ang = 2.0 * M_PI * (double)((p0 + k) % N) / (double)N;
        X += u[k] * cos(ang);
        Y += u[k] * sin(ang);
    }
    X *= 2.0 / (double)W;
    Y *= 2.0 / (double)W;
    *A = sqrt(X * X + Y * Y);
    *phi = atan2(-X, Y);
}

/* Misfit over the window: J = sum (U - u)^2 / sum U^2 -- the squared L2 cost of Eq. 5 restricted
 * to the steady-state window and normalised like the relative L2 error of Sec. 3.3, so that
 * sqrt(J) is that relative error.  Non-finite results become +inf. */
double orc_misfit(const double *U, const double *u, int64_t W) {
    double num = 0.0, den = 0.0;
    for (int64_t k = 0; k < W; k++) {
        double e = U[k] - u[k];
        num += e * e;
        den += U[k] * U[k];
    }
    double J = num / den;
    return isfinite(J) ? J : INFINITY;
}

/* One forward problem (FP, Sec. 2.2): trajectory, lock-in amplitude/phase over the last
 * lockin_cycles periods, and the misfit against target U (NULL: no misfit, J = NaN).
 * trace (W doubles, may be NULL) receives the window deflection.  Returns status bits; on a
 * non-zero status A = phi = NaN and J = +inf. */
int orc_forward(const orc_model *mo, const double *p, int32_t n_cycles, const double *U,
                double *A, double *phi, double *J, double *trace) {
    int64_t N = mo->steps_per_cycle, W = (int64_t)mo->lockin_cycles * N;
    double *u = (double *)malloc(sizeof(double) * W);
    int st = orc_trajectory(mo, p, n_cycles, NULL, W, u, NULL, NULL);
    /* first window sample is n = N_tot - W + 1, whose phase index is 1 mod N */
    if (st == 0) {
        orc_lockin(u, W, (int32_t)N, 1, A, phi);
        *J = U ? orc_misfit(U, u, W) : NAN;
    } else {
        *A = NAN;
        *phi = NAN;
        *J = INFINITY;
    }
    if (trace) memcpy(trace, u, sizeof(double) * W);
    free(u);
    return st;
}

/* Deflection at n_pts points along the beam (the paper's deflection points, n_dp, Sec. 3.2):
 * weights w [n_pts][m] with w[k][i] = Phi_i(x_k) / Phi_i(L); per point the lock-in amplitude A
 * and phase phi over the window and, if trace is non-NULL, the window deflection
 * ([n_pts][W], m).  Failed trajectories give NaN.  Returns the status bits. */
int orc_forward_points(const orc_model *mo, const double *p, int32_t n_cycles, int32_t n_pts,
                       const double *w, double *A, double *phi, double *trace) {
    int64_t N = mo->steps_per_cycle, W = (int64_t)mo->lockin_cycles * N;
    double *u = (double *)malloc(sizeof(double) * W * (n_pts > 0 ? n_pts : 1));
    int st = trajectory(mo, p, n_cycles, NULL, W, NULL, NULL, NULL, n_pts, w, u);
    for (int q = 0; q < n_pts; q++) {
        if (st == 0) orc_lockin(u + q * W, W, (int32_t)N, 1, A + q, phi + q);
        else A[q] = phi[q] = NAN;
    }
    if (trace) memcpy(trace, u, sizeof(double) * W * n_pts);
    free(u);
    return st;
}

/* Forward solve with an adaptive steady-state exit (the uneven-pixel workload's period counts
 * "until the steady-state tolerance is met"): from the initial condition, period by period, the
 * stroboscopic point of the orbit -- deflection u and rate u' / wd at the end of each period,
 * the same drive phase every time -- is compared with the previous period's (the initial state
 * before the first period): the transient ends after the first period c with
 * |P_c - P_{c-1}| < rtol |P_c|, P = (u, u' / wd) (for a steady sinusoid |P| is its amplitude, and
 * the change covers amplitude and phase), and at the latest after n_cycles - lockin periods; the
 * lock-in window is the following lockin periods.  *periods receives the periods integrated
 * (transient + window).  Outputs, health checks and failure rules as orc_forward (a failed
 * trajectory reports the periods it reached). */
static void strobe(const orc_derived *dv, const double *y, double *P) {
    double ud = 0.0;
    for (int i = 0; i < dv->m; i++) ud += y[dv->m + i];
    P[0] = tip(dv, y);
    P[1] = ud / dv->wd;
}

int orc_forward_steady(const orc_model *mo, const double *p, int32_t n_cycles, double rtol,
                       const double *U, double *A, double *phi, double *J, double *trace,
                       int32_t *periods) {
    orc_derived dv;
    derive(mo, &dv);
    int m = dv.m, N = mo->steps_per_cycle, L = mo->lockin_cycles;
    int64_t W = (int64_t)L * N;
    double y[2 * ORC_MAX_MODES], *win = (double *)malloc(sizeof(double) * W);
    orc_initial_state(mo, y);
    int status = 0, T = n_cycles - L, c = 0;
    int64_t n = 0;
    double Pprev[2], P[2];
    strobe(&dv, y, Pprev);
    for (int k = 0; k < W; k++) win[k] = NAN;
    for (c = 0; c < T + L && !status; c++) {
        int in_window = c >= T;
        for (int s = 0; s < N; s++, n++) {
            rk4_step(mo, &dv, p, (double)n * dv.h, y);
            if (in_window) win[(int64_t)(c - T) * N + s] = tip(&dv, y);
        }
        int bad = 0;
        for (int i = 0; i < 2 * m; i++)
            if (!isfinite(y[i])) bad = 1;
        if (bad) status |= ORC_ST_NONFINITE;
        else if (fabs(tip(&dv, y)) > mo->div_limit * mo->free_amplitude) status |= ORC_ST_DIVERGED;
        if (status || in_window) continue;
        strobe(&dv, y, P);
        if (hypot(P[0] - Pprev[0], P[1] - Pprev[1]) < rtol * hypot(P[0], P[1])) T = c + 1;
        Pprev[0] = P[0];
        Pprev[1] = P[1];
    }
    if (periods) *periods = c;
    if (status == 0) {
        orc_lockin(win, W, N, 1, A, phi);
        *J = U ? orc_misfit(U, win, W) : NAN;
    } else {
        for (int64_t k = 0; k < W; k++) win[k] = NAN;
        *A = NAN;
        *phi = NAN;
        *J = INFINITY;
    }
    if (trace) memcpy(trace, win, sizeof(double) * W);
    free(win);
    return status;
}

/* ------------------------------------------------------------------------------------------ */
/* Set-point -> separation (AFM amplitude feedback, Sec. 1)                                   */
/* ------------------------------------------------------------------------------------------ */

/* Steady amplitude at the parameters p: integrate period by period from the model's initial
 * condition; after each period take the stroboscopic point P = (u, u'/wd) at the period's end
 * (the same drive phase every time) and stop after the first period c with
 * |P_c - P_{c-1}| < rtol |P_c|, or after max_cycles.  Returns the lock-in amplitude of the last
 * period.  (A test on the one-period amplitude alone stops too early: the transient rings, and
 * at an extremum of its envelope the amplitude stands still while the phase still moves.) */
double orc_steady_amplitude(const orc_model *mo, const double *p, int32_t max_cycles, double rtol,
                            int32_t *cycles_used) {
    orc_derived dv;
    derive(mo, &dv);
    int N = mo->steps_per_cycle;
    double y[2 * ORC_MAX_MODES], *u = (double *)malloc(sizeof(double) * N);
    orc_initial_state(mo, y);
    double A = NAN, phi, Pprev[2], P[2];
    strobe(&dv, y, Pprev);
    int64_t n = 0;
    int c;
    for (c = 0; c < max_cycles; c++) {
        for (int s = 0; s < N; s++, n++) {
            rk4_step(mo, &dv, p, (double)n * dv.h, y);
            u[s] = tip(&dv, y);
        }
        orc_lockin(u, N, N, 1, &A, &phi);
        if (!isfinite(A)) break;
        strobe(&dv, y, P);
        if (hypot(P[0] - Pprev[0], P[1] - Pprev[1]) < rtol * hypot(P[0], P[1])) {
            c++;
            break;
        }
        Pprev[0] = P[0];
        Pprev[1] = P[1];
    }
    if (cycles_used) *cycles_used = c;
    free(u);
    return A;
}

/* Separation z_c at which the steady amplitude equals setpoint * A0.  An approach curve: z_c
 * steps down from A0 + 2 nm in 0.25 nm steps until the amplitude first falls below the
 * set-point, then bisection on that bracket until |A - s A0| < tol * A0.  p[0] is overwritten
 * during the search; returns z_c (NaN if no crossing down to z_c = 0). */
double orc_zc_from_setpoint(const orc_model *mo, const double *p_in, double setpoint,
                            int32_t max_cycles, double rtol, double tol) {
    int np = param_count(mo);
    double p[ORC_MAX_PARAMS];
    memcpy(p, p_in, sizeof(double) * np);
    double A0 = mo->free_amplitude, target = setpoint * A0;
    double hi = A0 + 2e-9, lo = NAN;
    p[0] = hi;
    double Ahi = orc_steady_amplitude(mo, p, max_cycles, rtol, NULL);
    if (!(Ahi > target)) return NAN;
    for (double z = hi - 0.25e-9; z > 0.0; z -= 0.25e-9) {
        p[0] = z;
        double Az = orc_steady_amplitude(mo, p, max_cycles, rtol, NULL);
        if (Az < target) {
            lo = z;
            break;
        }
        hi = z;
    }
    if (isnan(lo)) return NAN;
    for (int it = 0; it < 200; it++) {
        double mid = 0.5 * (lo + hi);
        p[0] = mid;
        double Am = orc_steady_amplitude(mo, p, max_cycles, rtol, NULL);
        if (fabs(Am - target) < tol * A0) return mid;
        if (Am < target) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* ------------------------------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)            */
/* ------------------------------------------------------------------------------------------ */

/* Ten rounds of the Philox-4x32 bijection.  Each round multiplies words 0 and 2 by the two
 * round multipliers, swaps the halves and mixes in the round key; the key is advanced by the
 * two Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    const uint32_t MA = 0xD2511F53u, MB = 0xCD9E8D57u, WA = 0x9E3779B9u, WB = 0xBB67AE85u;
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        uint64_t pa = (uint64_t)MA * x0, pb = (uint64_t)MB * x2;
        uint32_t hia = (uint32_t)(pa >> 32), loa = (uint32_t)pa;
        uint32_t hib = (uint32_t)(pb >> 32), lob = (uint32_t)pb;
        uint32_t n0 = hib ^ x1 ^ k0, n1 = lob, n2 = hia ^ x3 ^ k1, n3 = loa;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
        k0 += WA;
        k1 += WB;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 53-bit uniform in [0, 1) from two 32-bit words: top 27 bits of a, top 26 bits of b. */
double orc_u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

/* Stream layout: key = (low 32 bits of seed, swarm), counter = (iter, particle,
 * dim << 8 | purpose, high 32 bits of seed).  purpose 0 = move, 1 = initial position,
 * 2 = initial velocity. */
static void draw(uint64_t seed, int32_t swarm, int32_t iter, int32_t particle, int32_t dim,
                 int32_t purpose, uint32_t out[4]) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)swarm};
    uint32_t ctr[4] = {(uint32_t)iter, (uint32_t)particle, ((uint32_t)dim << 8) | (uint32_t)purpose,
                       (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

void orc_draw(uint64_t seed, int32_t swarm, int32_t iter, int32_t particle, int32_t dim,
              int32_t purpose, uint32_t *out) {
    draw(seed, swarm, iter, particle, dim, purpose, out);
}

/* ------------------------------------------------------------------------------------------ */
/* Particle swarm optimisation (paper Sec. 3.4, Eq. 8)                                        */
/* ------------------------------------------------------------------------------------------ */

/* Arrays are structure-of-arrays: z, v, pbest_z are [D][S*P] (dimension-major, particle index
 * g = s*P + p), pbest_J is [S*P], gbest_z is [D][S], gbest_J and gen_to_cutoff are [S].
 * Positions live in normalised coordinates z in [0,1]^D. */

/* Positions and velocities drawn uniformly over the search space (Sec. 3.4): z ~ U[0,1),
 * v = U[0,1) - z.  pbest_J = gbest_J = +inf, gen_to_cutoff = -1. */
void orc_pso_init(int32_t D, int32_t P, int32_t S, uint64_t seed, double *z, double *v,
                  double *pbest_z, double *pbest_J, double *gbest_z, double *gbest_J,
                  int32_t *gen_to_cutoff) {
    int64_t n = (int64_t)S * P;
    for (int32_t s = 0; s < S; s++)
        for (int32_t p = 0; p < P; p++) {
            int64_t g = (int64_t)s * P + p;
            for (int32_t j = 0; j < D; j++) {
                uint32_t rz[4], rv[4];
                draw(seed, s, 0, p, j, 1, rz);
                draw(seed, s, 0, p, j, 2, rv);
                double z0 = orc_u53(rz[0], rz[1]);
                z[(int64_t)j * n + g] = z0;
                v[(int64_t)j * n + g] = orc_u53(rv[0], rv[1]) - z0;
                pbest_z[(int64_t)j * n + g] = z0;
            }
            pbest_J[g] = INFINITY;
        }
    for (int32_t s = 0; s < S; s++) {
        gbest_J[s] = INFINITY;
        gen_to_cutoff[s] = -1;
        for (int32_t j = 0; j < D; j++) gbest_z[(int64_t)j * S + s] = 0.0;
    }
}

/* One PSO generation given the misfits J of the current positions:
 *   1. personal best: if J < pbest_J (strict; non-finite J counts as +inf) take the position;
 *   2. global best: the swarm's lowest pbest_J, ties to the lowest particle index;
 *   3. gen_to_cutoff: first iteration whose sqrt(gbest_J) <= cutoff;
 *   4. unless is_last: Eq. 8 velocity update with r1, r2 ~ U[0,1) per particle and dimension,
 *      v = w v + c1 r1 (pbest - z) + c2 r2 (gbest - z), clamp v to [-vmax, vmax], z = z + v, and a
 *      dimension that leaves [0,1] is put back on the boundary with zero velocity.
 * The floating-point expression order is fixed so that any IEEE FP64 implementation that
 * evaluates it the same way, without contraction, reproduces it bit for bit. */
void orc_pso_update(int32_t D, int32_t P, int32_t S, const double *J, int32_t iter,
                    int32_t is_last, uint64_t seed, double cutoff, double w, double c1, double c2,
                    double vmax, double *z, double *v, double *pbest_z, double *pbest_J,
                    double *gbest_z, double *gbest_J, int32_t *gen_to_cutoff) {
    int64_t n = (int64_t)S * P;
    for (int32_t s = 0; s < S; s++) {
        for (int32_t p = 0; p < P; p++) {
            int64_t g = (int64_t)s * P + p;
            double Jg = isfinite(J[g]) ? J[g] : INFINITY;
            if (Jg < pbest_J[g]) {
                pbest_J[g] = Jg;
                for (int32_t j = 0; j < D; j++) pbest_z[(int64_t)j * n + g] = z[(int64_t)j * n + g];
            }
        }
        int32_t best = 0;
        for (int32_t p = 1; p < P; p++)
            if (pbest_J[(int64_t)s * P + p] < pbest_J[(int64_t)s * P + best]) best = p;
        int64_t gb = (int64_t)s * P + best;
        gbest_J[s] = pbest_J[gb];
        for (int32_t j = 0; j < D; j++) gbest_z[(int64_t)j * S + s] = pbest_z[(int64_t)j * n + gb];
        if (gen_to_cutoff[s] < 0 && sqrt(gbest_J[s]) <= cutoff) gen_to_cutoff[s] = iter;
        if (is_last) continue;
        for (int32_t p = 0; p < P; p++) {
            int64_t g = (int64_t)s * P + p;
            for (int32_t j = 0; j < D; j++) {
                uint32_t r[4];
                draw(seed, s, iter, p, j, 0, r);
                double r1 = orc_u53(r[0], r[1]), r2 = orc_u53(r[2], r[3]);
                int64_t ij = (int64_t)j * n + g;
                double zj = z[ij];
                double t1 = w * v[ij];
                double t2 = (c1 * r1) * (pbest_z[ij] - zj);
                double t3 = (c2 * r2) * (gbest_z[(int64_t)j * S + s] - zj);
                double vn = (t1 + t2) + t3;
                if (vn > vmax) vn = vmax;
                if (vn < -vmax) vn = -vmax;
                double zn = zj + vn;
                if (zn < 0.0) {
                    zn = 0.0;
                    vn = 0.0;
                }
                if (zn > 1.0) {
                    zn = 1.0;
                    vn = 0.0;
                }
                z[ij] = zn;
                v[ij] = vn;
            }
        }
    }
}

/* Normalised coordinate -> physical parameter: lo + z (hi - lo), or geometric
 * lo (hi/lo)^z = exp(log lo + z (log hi - log lo)) for log-scaled parameters. */
double orc_z_to_theta(double z, double lo, double hi, int32_t log_scale) {
    if (log_scale) return exp(log(lo) + z * (log(hi) - log(lo)));
    return lo + z * (hi - lo);
}

/* d theta / d z of the map above. */
double orc_dtheta_dz(double z, double lo, double hi, int32_t log_scale) {
    if (log_scale) return orc_z_to_theta(z, lo, hi, 1) * (log(hi) - log(lo));
    return hi - lo;
}

/* ------------------------------------------------------------------------------------------ */
/* Discrete adjoint of RK4 + window misfit                                                    */
/* ------------------------------------------------------------------------------------------ */

/* ybar += (df/dy)^T kbar and pbar += (df/dp)^T kbar for the model right-hand side at state Y. */
/* Derivatives of the parameter-driven base term -y_b''(t) = a (w^2 sin(phi) - 4 pi g cos(phi)),
 * phi = 2 pi (f + g t) t, w = 2 pi (f + 2 g t), with respect to a, f and g (Eq. 10). */
static void base_acc_grad(const double *p, double t, double *da) {
    double a = p[ORC_P_A], f = p[ORC_P_F], g = p[ORC_P_G];
    double phi = 2.0 * M_PI * (f + g * t) * t, w = 2.0 * M_PI * (f + 2.0 * g * t);
    double sn = sin(phi), cs = cos(phi);
    da[0] = w * w * sn - 4.0 * M_PI * g * cs;
    /* dphi/df = 2 pi t, dw/df = 2 pi; dphi/dg = 2 pi t^2, dw/dg = 4 pi t */
    da[1] = a * (2.0 * w * 2.0 * M_PI * sn + w * w * cs * 2.0 * M_PI * t +
                 4.0 * M_PI * g * sn * 2.0 * M_PI * t);
    da[2] = a * (2.0 * w * 4.0 * M_PI * t * sn + w * w * cs * 2.0 * M_PI * t * t -
                 4.0 * M_PI * cs + 4.0 * M_PI * g * sn * 2.0 * M_PI * t * t);
}

static void rhs_vjp(const orc_model *mo, const orc_derived *dv, const double *p, double t,
                    const double *Y, const double *kbar, double *ybar, double *pbar) {
    int m = dv->m;
    double u = 0.0, ud = 0.0, sp = 0.0;
    for (int i = 0; i < m; i++) {
        u += Y[i];
        ud += Y[m + i];
        sp += kbar[m + i];
    }
    double Fd, Fdd, Fp[ORC_MAX_PARAMS];
    force_partials(mo->law, p, p[0] + u, ud, &Fd, &Fdd, Fp);
    for (int i = 0; i < m; i++) {
        ybar[i] += -dv->w[i] * dv->w[i] * kbar[m + i] + Fd / dv->M * sp;
        ybar[m + i] += kbar[i] - dv->c[i] * kbar[m + i] + Fdd / dv->M * sp;
    }
    int np = orc_law_param_count(mo->law);
    pbar[0] += Fd / dv->M * sp; /* z_c enters through d = z_c + u */
    for (int j = 1; j < np; j++) pbar[j] += Fp[j] / dv->M * sp;
    if (mo->drive_mode == ORC_DRIVE_PARAMS) { /* gamma_i (-y_b'') enters every velocity slope */
        double sg = 0.0, da[3];
        for (int i = 0; i < m; i++) sg += mo->gain[i] * kbar[m + i];
        base_acc_grad(p, t, da);
        pbar[ORC_P_A] += sg * da[0];
        pbar[ORC_P_F] += sg * da[1];
        pbar[ORC_P_G] += sg * da[2];
    }
}

/* Misfit J and its exact gradient with respect to every entry of p (SI), by reverse-mode
 * differentiation of the RK4 steps and the window misfit.  The whole trajectory y_0..y_Ntot is
 * stored (no checkpointing).  For a step with stages Y_i and slopes k_i = f(t_i, Y_i):
 *   kbar_i = h (b_i ybar_{n+1} + sum_{j>i} a_ji Ybar_j), i = 4..1,
 *   Ybar_i = (df/dy)^T kbar_i,  pbar += (df/dp)^T kbar_i,
 *   ybar_n = ybar_{n+1} + sum_i Ybar_i + dJ/dy_n.
 * The initial condition does not depend on p.  Returns status bits (gradient NaN if non-zero). */
int orc_misfit_grad(const orc_model *mo, const double *p, int32_t n_cycles, const double *U,
                    double *J_out, double *grad) {
    orc_derived dv;
    derive(mo, &dv);
    int m = dv.m, ns = 2 * m, np = param_count(mo);
    int64_t N = mo->steps_per_cycle, Ntot = (int64_t)n_cycles * N, W = (int64_t)mo->lockin_cycles * N;
    double *ys = (double *)malloc(sizeof(double) * ns * (Ntot + 1));
    orc_initial_state(mo, ys);
    int status = 0;
    for (int64_t n = 0; n < Ntot; n++) {
        memcpy(ys + (n + 1) * ns, ys + n * ns, sizeof(double) * ns);
        rk4_step(mo, &dv, p, (double)n * dv.h, ys + (n + 1) * ns);
        if ((n + 1) % N == 0) {
            double *y = ys + (n + 1) * ns;
            for (int i = 0; i < ns; i++)
                if (!isfinite(y[i])) status |= ORC_ST_NONFINITE;
            if (!status && fabs(tip(&dv, y)) > mo->div_limit * mo->free_amplitude)
                status |= ORC_ST_DIVERGED;
            if (status) break;
        }
    }
    for (int j = 0; j < np; j++) grad[j] = NAN;
    if (status) {
        *J_out = INFINITY;
        free(ys);
        return status;
    }
    /* window: n = Ntot - W + 1 .. Ntot, sample k = n - (Ntot - W + 1) */
    double num = 0.0, den = 0.0;
    for (int64_t k = 0; k < W; k++) {
        double u = tip(&dv, ys + (Ntot - W + 1 + k) * ns), e = U[k] - u;
        num += e * e;
        den += U[k] * U[k];
    }
    *J_out = num / den;
    double ybar[2 * ORC_MAX_MODES], pbar[ORC_MAX_PARAMS];
    for (int j = 0; j < ORC_MAX_PARAMS; j++) pbar[j] = 0.0;
    for (int i = 0; i < ns; i++) ybar[i] = 0.0;
    double h = dv.h, b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    for (int64_t n = Ntot; n >= 1; n--) {
        /* dJ/dy_n from the window term (only the q components enter u = sum q_i) */
        int64_t k = n - (Ntot - W + 1);
        if (k >= 0) {
            double u = tip(&dv, ys + n * ns);
            double g = -2.0 * (U[k] - u) / den;
            for (int i = 0; i < m; i++) ybar[i] += g;
        }
        /* reverse the step y_{n-1} -> y_n */
        const double *y = ys + (n - 1) * ns;
        double t = (double)(n - 1) * h;
        double Ys[4][2 * ORC_MAX_MODES], ks[4][2 * ORC_MAX_MODES];
        memcpy(Ys[0], y, sizeof(double) * ns);
        rhs(mo, &dv, p, t, Ys[0], ks[0]);
        for (int i = 0; i < ns; i++) Ys[1][i] = y[i] + 0.5 * h * ks[0][i];
        rhs(mo, &dv, p, t + 0.5 * h, Ys[1], ks[1]);
        for (int i = 0; i < ns; i++) Ys[2][i] = y[i] + 0.5 * h * ks[1][i];
        rhs(mo, &dv, p, t + 0.5 * h, Ys[2], ks[2]);
        for (int i = 0; i < ns; i++) Ys[3][i] = y[i] + h * ks[2][i];
        double Ybar[4][2 * ORC_MAX_MODES], kbar[2 * ORC_MAX_MODES];
        const double a_next[4] = {0.5, 0.5, 1.0, 0.0}; /* a_{i+1,i} */
        const double c_st[4] = {0.0, 0.5, 0.5, 1.0};   /* stage times, in steps */
        for (int st = 3; st >= 0; st--) {
            for (int i = 0; i < ns; i++) {
                kbar[i] = h * b[st] * ybar[i];
                if (st < 3) kbar[i] += h * a_next[st] * Ybar[st + 1][i];
            }
            for (int i = 0; i < ns; i++) Ybar[st][i] = 0.0;
            rhs_vjp(mo, &dv, p, t + c_st[st] * h, Ys[st], kbar, Ybar[st], pbar);
        }
        for (int i = 0; i < ns; i++) ybar[i] += Ybar[0][i] + Ybar[1][i] + Ybar[2][i] + Ybar[3][i];
    }
    for (int j = 0; j < np; j++) grad[j] = pbar[j];
    free(ys);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Inversion drivers (IP, Sec. 2.3)                                                           */
/* ------------------------------------------------------------------------------------------ */

static void theta_from_z(const double *p_fixed, int32_t np, int32_t n_free, const int32_t *idx,
                         const double *lo, const double *hi, const int32_t *logs, const double *z,
                         double *p) {
    memcpy(p, p_fixed, sizeof(double) * np);
    for (int32_t j = 0; j < n_free; j++) p[idx[j]] = orc_z_to_theta(z[j], lo[j], hi[j], logs[j]);
}

/* PSO inversion of one target (single swarm, swarm index 0): T generations of P particles,
 * each generation evaluates J at every position and then calls orc_pso_update.  Outputs the
 * best normalised position, its J, the generation at which sqrt(J) first fell below cutoff
 * (-1: never) and, if hist is non-NULL, gbest_J after every generation. */
void orc_pso_invert(const orc_model *mo, const double *p_fixed, int32_t n_free, const int32_t *idx,
                    const double *lo, const double *hi, const int32_t *logs, const double *U,
                    int32_t P, int32_t T, uint64_t seed, double cutoff, double w, double c1,
                    double c2, double vmax, double *best_z, double *best_J, int32_t *gen,
                    double *hist) {
    int32_t D = n_free, np = param_count(mo);
    double *z = malloc(sizeof(double) * D * P), *v = malloc(sizeof(double) * D * P);
    double *pz = malloc(sizeof(double) * D * P), *pJ = malloc(sizeof(double) * P);
    double *J = malloc(sizeof(double) * P), gz[ORC_MAX_PARAMS], gJ;
    int32_t g2c;
    orc_pso_init(D, P, 1, seed, z, v, pz, pJ, gz, &gJ, &g2c);
    for (int32_t t = 0; t < T; t++) {
        for (int32_t q = 0; q < P; q++) {
            double zq[ORC_MAX_PARAMS], p[ORC_MAX_PARAMS], A, phi;
            for (int32_t j = 0; j < D; j++) zq[j] = z[(int64_t)j * P + q];
            theta_from_z(p_fixed, np, n_free, idx, lo, hi, logs, zq, p);
            orc_forward(mo, p, mo->n_cycles, U, &A, &phi, &J[q], NULL);
        }
        orc_pso_update(D, P, 1, J, t, t == T - 1, seed, cutoff, w, c1, c2, vmax, z, v, pz, pJ, gz,
                       &gJ, &g2c);
        if (hist) hist[t] = gJ;
    }
    for (int32_t j = 0; j < D; j++) best_z[j] = gz[j];
    *best_J = gJ;
    *gen = g2c;
    free(z); free(v); free(pz); free(pJ); free(J);
}

/* J and dJ/dz at normalised position z (gradient through the adjoint, chain rule through the
 * coordinate map). */
static double misfit_z(const orc_model *mo, const double *p_fixed, int32_t n_free,
                       const int32_t *idx, const double *lo, const double *hi, const int32_t *logs,
                       const double *U, const double *z, double *gz) {
    int32_t np = param_count(mo);
    double p[ORC_MAX_PARAMS], g[ORC_MAX_PARAMS], J;
    theta_from_z(p_fixed, np, n_free, idx, lo, hi, logs, z, p);
    if (gz) {
        orc_misfit_grad(mo, p, mo->n_cycles, U, &J, g);
        for (int32_t j = 0; j < n_free; j++) gz[j] = g[idx[j]] * orc_dtheta_dz(z[j], lo[j], hi[j], logs[j]);
    } else {
        double A, phi;
        orc_forward(mo, p, mo->n_cycles, U, &A, &phi, &J, NULL);
    }
    return J;
}

/* Projected L-BFGS in normalised coordinates: history 5, H0 = s'y / y'y, backtracking Armijo
 * (c = 1e-4, alpha from 1, halving at most 20 times) on the clamped path z(alpha) =
 * clamp(z + alpha d, 0, 1); a pair with s'y <= 1e-12 |s| |y| is not stored.  Runs `steps`
 * iterations (stopping early when no descent step is found) and returns the final J. */
double orc_lbfgs(const orc_model *mo, const double *p_fixed, int32_t n_free, const int32_t *idx,
                 const double *lo, const double *hi, const int32_t *logs, const double *U,
                 double *z, int32_t steps) {
    enum { HM = 5 };
    int32_t D = n_free;
    double S[HM][ORC_MAX_PARAMS], Y[HM][ORC_MAX_PARAMS], rho[HM], g[ORC_MAX_PARAMS];
    int hn = 0, head = 0;
    double J = misfit_z(mo, p_fixed, n_free, idx, lo, hi, logs, U, z, g);
    for (int32_t it = 0; it < steps; it++) {
        /* two-loop recursion: d = -H g */
        double q[ORC_MAX_PARAMS], al[HM], d[ORC_MAX_PARAMS];
        for (int j = 0; j < D; j++) q[j] = g[j];
        for (int k = 0; k < hn; k++) {
            int i = (head - 1 - k + HM) % HM;
            double sq = 0.0;
            for (int j = 0; j < D; j++) sq += S[i][j] * q[j];
            al[i] = rho[i] * sq;
            for (int j = 0; j < D; j++) q[j] -= al[i] * Y[i][j];
        }
        double gamma = 1.0;
        if (hn > 0) {
            int i = (head - 1 + HM) % HM;
            double sy = 0.0, yy = 0.0;
            for (int j = 0; j < D; j++) {
                sy += S[i][j] * Y[i][j];
                yy += Y[i][j] * Y[i][j];
            }
            gamma = sy / yy;
        }
        for (int j = 0; j < D; j++) d[j] = gamma * q[j];
        for (int k = hn - 1; k >= 0; k--) {
            int i = (head - 1 - k + HM) % HM;
            double yd = 0.0;
            for (int j = 0; j < D; j++) yd += Y[i][j] * d[j];
            double be = rho[i] * yd;
            for (int j = 0; j < D; j++) d[j] += S[i][j] * (al[i] - be);
        }
        for (int j = 0; j < D; j++) d[j] = -d[j];
        /* backtracking on the projected path */
        double alpha = 1.0, zn[ORC_MAX_PARAMS], Jn = INFINITY, gn[ORC_MAX_PARAMS];
        int ok = 0;
        for (int ls = 0; ls <= 20; ls++) {
            double dec = 0.0;
            for (int j = 0; j < D; j++) {
                double t = z[j] + alpha * d[j];
                zn[j] = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
                dec += g[j] * (zn[j] - z[j]);
            }
            Jn = misfit_z(mo, p_fixed, n_free, idx, lo, hi, logs, U, zn, NULL);
            if (Jn <= J + 1e-4 * dec && dec < 0.0) {
                ok = 1;
                break;
            }
            alpha *= 0.5;
        }
        if (!ok) break;
        misfit_z(mo, p_fixed, n_free, idx, lo, hi, logs, U, zn, gn);
        double s[ORC_MAX_PARAMS], y[ORC_MAX_PARAMS], sy = 0.0, ss = 0.0, yy = 0.0;
        for (int j = 0; j < D; j++) {
            s[j] = zn[j] - z[j];
            y[j] = gn[j] - g[j];
            sy += s[j] * y[j];
            ss += s[j] * s[j];
            yy += y[j] * y[j];
        }
        if (sy > 1e-12 * sqrt(ss) * sqrt(yy)) {
            for (int j = 0; j < D; j++) {
                S[head][j] = s[j];
                Y[head][j] = y[j];
            }
            rho[head] = 1.0 / sy;
            head = (head + 1) % HM;
            if (hn < HM) hn++;
        }
        for (int j = 0; j < D; j++) {
            z[j] = zn[j];
            g[j] = gn[j];
        }
        J = Jn;
    }
    return J;
}

/* ------------------------------------------------------------------------------------------ */
/* Euler-Bernoulli cantilever modes (paper Sec. 3.2, Eq. 6-7)                                 */
/* ------------------------------------------------------------------------------------------ */

/* Mode shape of Eq. 6 at x/L = xi for root x = beta L:
 *   Phi = [2 sin(bx) - 2G cos(bx) + (G - 1) e^{bx} + (G + 1) e^{-bx}] / 2,
 *   G   = (2 e^{-bL} sin bL - e^{-2bL} + 1) / (2 e^{-bL} cos bL + e^{-2bL} + 1).
 * The denominator's e^{-2bL} term is taken with a plus sign: that is the value for which
 * Phi''(L) = Phi'''(L) = 0 (free end); with the minus sign the free-end conditions fail. */
static double eb_G(double bL) {
    double e = exp(-bL);
    return (2.0 * e * sin(bL) - e * e + 1.0) / (2.0 * e * cos(bL) + e * e + 1.0);
}

double orc_eb_shape(double bL, double xi) {
    double G = eb_G(bL), bx = bL * xi;
    return (2.0 * sin(bx) - 2.0 * G * cos(bx) + (G - 1.0) * exp(bx) + (G + 1.0) * exp(-bx)) / 2.0;
}

/* i-th (1-based) root of cos(x) cosh(x) + 1 = 0 by Newton's method from (2i - 1) pi / 2. */
double orc_eb_root(int32_t i) {
    double x = (2.0 * i - 1.0) * M_PI / 2.0;
    if (i == 1) x = 1.875;
    for (int it = 0; it < 100; it++) {
        double f = cos(x) * cosh(x) + 1.0, fp = -sin(x) * cosh(x) + cos(x) * sinh(x);
        double dx = f / fp;
        x -= dx;
        if (fabs(dx) < 1e-15 * x) break;
    }
    return x;
}

/* Tip-normalised modal data for the first n modes from npts-point composite Simpson integration
 * of the mode shapes (npts odd): ratio_i = (b_i / b_1)^2 (w_i = b_i^2 sqrt(EI / (mu L^4))),
 * mass_i = int_0^L Phi_i^2 dx / (L Phi_i(L)^2) (modal mass over mu L) and the base-drive gain
 * gamma_i = int Phi_i dx / (Phi_i(L) int Phi_i^2 dx) * Phi_i(L)^2 = (int Phi_i/Phi_i(L) dx / L)
 * / mass_i, so that q_i'' + ... = F / (mu L mass_i) - gamma_i y_b''. */
void orc_eb_modes(int32_t n, int32_t npts, double *bL, double *ratio, double *mass, double *gain) {
    for (int32_t i = 0; i < n; i++) {
        bL[i] = orc_eb_root(i + 1);
        double tipv = orc_eb_shape(bL[i], 1.0), s1 = 0.0, s2 = 0.0, hx = 1.0 / (npts - 1);
        for (int32_t k = 0; k < npts; k++) {
            double wgt = (k == 0 || k == npts - 1) ? 1.0 : (k % 2 ? 4.0 : 2.0);
            double ph = orc_eb_shape(bL[i], k * hx) / tipv;
            s1 += wgt * ph;
            s2 += wgt * ph * ph;
        }
        s1 *= hx / 3.0;
        s2 *= hx / 3.0;
        ratio[i] = (bL[i] / bL[0]) * (bL[i] / bL[0]);
        mass[i] = s2;
        gain[i] = s1 / s2;
    }
}
