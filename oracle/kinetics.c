/* Stiff-chemistry reference integrator (test infrastructure, FP64).
 *
 * Only the test-suite and the CPU-baseline leg of the benchmark load this
 * library; it shares no code with the HIP path.  It stands in for the
 * conventional ODE solver the paper validates ODENet against (Sec. 5.1,
 * accuracy test) and produces training labels for the chemistry net.
 *
 * Model: ideal gas at constant pressure, adiabatic, per-species constant c_p.
 *   rho = P Wbar / (R T),  1/Wbar = sum_i Y_i / W_i,  c_i = rho Y_i / W_i
 *   q_r = k_r(T) prod_i c_i^nu'_ir,  k_r = A_r T^b_r exp(-Ea_r / (R T))
 *   dY_i/dt = (W_i / rho) sum_r (nu''_ir - nu'_ir) q_r
 *   dT/dt   = -sum_i h_i(T) dY_i/dt / cpbar,  h_i = hf_i + cp_i (T - T_ref),
 *             cpbar = sum_i Y_i cp_i
 * Units are SI (mol, m^3, J, kg, K, s).
 *
 * Time stepping: ROS2, the two-stage L-stable Rosenbrock method of Verwer,
 * Spee, Blom and Hundsdorfer (SIAM J. Sci. Comput. 20, 1999) with
 * gamma = 1 + 1/sqrt(2):
 *   (I - gamma h J) k1 = f(y_n)
 *   (I - gamma h J) k2 = f(y_n + h k1) - 2 k1
 *   y_(n+1) = y_n + 3/2 h k1 + 1/2 h k2
 * The embedded first-order solution y_n + h k1 gives the local error
 * estimate h (k1 + k2)/2; steps adapt to a weighted RMS norm of it.
 * The Jacobian is analytic; the linear solves use LU with partial pivoting.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KIN_MAXS 64
#define KIN_MAXN (KIN_MAXS + 1)
#define R_GAS 8.314462618

typedef struct {
    int S, R;
    const double *W, *hf, *cp;  /* [S] */
    double t_ref;
    const int32_t *nu_f, *nu_r; /* [R][S] reactant / product coefficients */
    const double *A, *b, *Ea;   /* [R] SI units */
} kin_mech;

/* Reactant list of reaction r: species indices with multiplicity (at most
 * KIN_MAXORD entries).  Returns the count. */
#define KIN_MAXORD 3
static int reactants(const kin_mech *m, int r, int *idx) {
    int n = 0;
    const int32_t *nf = m->nu_f + (size_t)r * m->S;
    for (int i = 0; i < m->S; ++i)
        for (int p = 0; p < nf[i] && n < KIN_MAXORD; ++p) idx[n++] = i;
    return n;
}

/* Rate constant and rate of progress of reaction r; with dq != NULL also
 * dq/dc_(idx[k]) for each listed reactant, and d q / d T at fixed c. */
static double rate(const kin_mech *m, int r, double T, const double *c, const int *idx, int n,
                   double *dq, double *dqT) {
    double k = m->A[r] * pow(T, m->b[r]) * exp(-m->Ea[r] / (R_GAS * T));
    double prod = 1.0;
    for (int a = 0; a < n; ++a) prod *= c[idx[a]];
    double q = k * prod;
    if (dqT) *dqT = q * (m->b[r] / T + m->Ea[r] / (R_GAS * T * T));
    if (dq)
        for (int a = 0; a < n; ++a) {
            /* product rule: derivative of the a-th factor, others kept */
            double rest = 1.0;
            for (int e = 0; e < n; ++e)
                if (e != a) rest *= c[idx[e]];
            dq[a] = k * rest;
        }
    return q;
}

static double mix_rho(const kin_mech *m, double P, const double *y, double *inv_wbar) {
    double s = 0.0;
    for (int i = 0; i < m->S; ++i) s += y[i] / m->W[i];
    if (inv_wbar) *inv_wbar = s;
    return P / (R_GAS * y[m->S] * s);
}

/* f = dy/dt for y = (Y_1..Y_S, T). */
int kin_rhs(const kin_mech *m, double P, const double *y, double *f) {
    const int S = m->S;
    double c[KIN_MAXS], w[KIN_MAXS];
    int idx[KIN_MAXORD];
    if (S > KIN_MAXS) return -1;
    double T = y[S];
    double rho = mix_rho(m, P, y, NULL);
    for (int i = 0; i < S; ++i) { c[i] = rho * y[i] / m->W[i]; w[i] = 0.0; }
    for (int r = 0; r < m->R; ++r) {
        int n = reactants(m, r, idx);
        double q = rate(m, r, T, c, idx, n, NULL, NULL);
        for (int i = 0; i < S; ++i) {
            int nu = m->nu_r[(size_t)r * S + i] - m->nu_f[(size_t)r * S + i];
            if (nu) w[i] += nu * q;
        }
    }
    double num = 0.0, cpbar = 0.0;
    for (int i = 0; i < S; ++i) {
        f[i] = m->W[i] * w[i] / rho;
        num += (m->hf[i] + m->cp[i] * (T - m->t_ref)) * f[i];
        cpbar += y[i] * m->cp[i];
    }
    f[S] = -num / cpbar;
    return 0;
}

/* Analytic Jacobian J[a][b] = d f_a / d y_b, row-major (S+1)^2. */
int kin_jac(const kin_mech *m, double P, const double *y, double *J) {
    const int S = m->S, N = S + 1, R = m->R;
    double c[KIN_MAXS], omega[KIN_MAXS], f[KIN_MAXN], drho[KIN_MAXN], g[KIN_MAXN];
    double dq[KIN_MAXORD], dqT;
    int idx[KIN_MAXORD];
    if (S > KIN_MAXS) return -1;
    double T = y[S], inv_wbar;
    double rho = mix_rho(m, P, y, &inv_wbar);
    for (int i = 0; i < S; ++i) { c[i] = rho * y[i] / m->W[i]; omega[i] = 0.0; }
    /* d rho / d Y_j = -rho (1/W_j) / (1/Wbar);  d rho / d T = -rho / T */
    for (int j = 0; j < S; ++j) drho[j] = -rho / (m->W[j] * inv_wbar);
    drho[S] = -rho / T;
    for (size_t e = 0; e < (size_t)N * N; ++e) J[e] = 0.0;
    /* d c_k / d y_b = (rho / W_k) [b == k] + (Y_k / W_k) drho_b */
    for (int r = 0; r < R; ++r) {
        int n = reactants(m, r, idx);
        double q = rate(m, r, T, c, idx, n, dq, &dqT);
        /* g_b = d q_r / d y_b */
        for (int b = 0; b < N; ++b) g[b] = (b == S) ? dqT : 0.0;
        for (int a = 0; a < n; ++a) {
            int k = idx[a];
            for (int b = 0; b < N; ++b) g[b] += dq[a] * (y[k] / m->W[k]) * drho[b];
            g[k] += dq[a] * rho / m->W[k];
        }
        for (int i = 0; i < S; ++i) {
            int nu = m->nu_r[(size_t)r * S + i] - m->nu_f[(size_t)r * S + i];
            if (!nu) continue;
            omega[i] += nu * q;
            for (int b = 0; b < N; ++b) J[(size_t)i * N + b] += nu * g[b];
        }
    }
    /* species rows: f_i = W_i omega_i / rho */
    for (int i = 0; i < S; ++i) {
        f[i] = m->W[i] * omega[i] / rho;
        for (int b = 0; b < N; ++b)
            J[(size_t)i * N + b] = m->W[i] * J[(size_t)i * N + b] / rho
                                   - m->W[i] * omega[i] * drho[b] / (rho * rho);
    }
    /* temperature row: f_T = -sum_i h_i f_i / cpbar */
    double cpbar = 0.0, hsum = 0.0;
    for (int i = 0; i < S; ++i) {
        cpbar += y[i] * m->cp[i];
        hsum += (m->hf[i] + m->cp[i] * (T - m->t_ref)) * f[i];
    }
    for (int b = 0; b < N; ++b) {
        double s = 0.0;
        for (int i = 0; i < S; ++i)
            s += (m->hf[i] + m->cp[i] * (T - m->t_ref)) * J[(size_t)i * N + b];
        if (b == S)
            for (int i = 0; i < S; ++i) s += m->cp[i] * f[i];
        double dcp = (b < S) ? m->cp[b] : 0.0;
        J[(size_t)S * N + b] = -s / cpbar + hsum * dcp / (cpbar * cpbar);
    }
    return 0;
}

/* In-place LU with partial pivoting of an N x N row-major matrix. */
static int lu_factor(double *a, int N, int *piv) {
    for (int k = 0; k < N; ++k) {
        int p = k;
        double best = fabs(a[(size_t)k * N + k]);
        for (int i = k + 1; i < N; ++i) {
            double v = fabs(a[(size_t)i * N + k]);
            if (v > best) { best = v; p = i; }
        }
        if (best == 0.0 || !isfinite(best)) return -1;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < N; ++j) {
                double t = a[(size_t)k * N + j];
                a[(size_t)k * N + j] = a[(size_t)p * N + j];
                a[(size_t)p * N + j] = t;
            }
        for (int i = k + 1; i < N; ++i) {
            double l = a[(size_t)i * N + k] / a[(size_t)k * N + k];
            a[(size_t)i * N + k] = l;
            for (int j = k + 1; j < N; ++j) a[(size_t)i * N + j] -= l * a[(size_t)k * N + j];
        }
    }
    return 0;
}

/* Solve with the factors of lu_factor.  Whole rows were swapped there, so
 * every interchange is applied to x before the forward substitution. */
static void lu_solve(const double *a, int N, const int *piv, double *x) {
    for (int k = 0; k < N; ++k)
        if (piv[k] != k) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
    for (int k = 0; k < N; ++k)
        for (int i = k + 1; i < N; ++i) x[i] -= a[(size_t)i * N + k] * x[k];
    for (int k = N - 1; k >= 0; --k) {
        for (int j = k + 1; j < N; ++j) x[k] -= a[(size_t)k * N + j] * x[j];
        x[k] /= a[(size_t)k * N + k];
    }
}

/* Integrate one state over dt.  y has S+1 entries (Y..., T) and is updated in
 * place.  Tolerances: species use atol, temperature atol_T; both rtol.
 * Returns the number of accepted steps, or a negative code on failure. */
int kin_ros2(const kin_mech *m, double P, double *y, double dt, double rtol,
             double atol, double atol_T, int max_steps) {
    const int S = m->S, N = S + 1;
    const double gam = 1.0 + 1.0 / sqrt(2.0);
    double J[KIN_MAXN * KIN_MAXN], M[KIN_MAXN * KIN_MAXN];
    double f0[KIN_MAXN], f1[KIN_MAXN], k1[KIN_MAXN], k2[KIN_MAXN], yt[KIN_MAXN], yn[KIN_MAXN];
    int piv[KIN_MAXN];
    if (S > KIN_MAXS) return -1;
    double t = 0.0, h = dt * 1e-6;
    int accepted = 0, tries = 0;
    while (t < dt) {
        if (++tries > max_steps) return -2;
        if (t + h > dt) h = dt - t;
        if (kin_jac(m, P, y, J) || kin_rhs(m, P, y, f0)) return -3;
        for (int i = 0; i < N * N; ++i) M[i] = -gam * h * J[i];
        for (int i = 0; i < N; ++i) M[(size_t)i * N + i] += 1.0;
        if (lu_factor(M, N, piv)) { h *= 0.25; continue; }
        memcpy(k1, f0, sizeof(double) * N);
        lu_solve(M, N, piv, k1);
        for (int i = 0; i < N; ++i) yt[i] = y[i] + h * k1[i];
        if (kin_rhs(m, P, yt, f1)) return -3;
        for (int i = 0; i < N; ++i) k2[i] = f1[i] - 2.0 * k1[i];
        lu_solve(M, N, piv, k2);
        double err = 0.0;
        int finite = 1;
        for (int i = 0; i < N; ++i) {
            yn[i] = y[i] + 1.5 * h * k1[i] + 0.5 * h * k2[i];
            double e = 0.5 * h * (k1[i] + k2[i]);
            double sc = (i < S ? atol : atol_T) + rtol * fmax(fabs(y[i]), fabs(yn[i]));
            err += (e / sc) * (e / sc);
            if (!isfinite(yn[i])) finite = 0;
        }
        err = sqrt(err / N);
        if (!finite || !isfinite(err)) { h *= 0.25; continue; }
        if (err <= 1.0) {
            t += h;
            memcpy(y, yn, sizeof(double) * N);
            ++accepted;
        }
        double fac = (err > 0.0) ? 0.9 / sqrt(err) : 5.0;
        fac = fmin(5.0, fmax(0.2, fac));
        h *= fac;
        if (h < 1e-300) return -4;
    }
    return accepted;
}

/* Integrate n independent states stored as T[n], P[n], Y[S][ld].
 * nsteps[i] receives kin_ros2's return value for state i.
 * Returns the number of states that failed. */
int kin_integrate(const kin_mech *m, int64_t n, int64_t ld, const double *T, const double *P,
                  const double *Y, double dt, double rtol, double atol, double atol_T,
                  int max_steps, double *T_out, double *Y_out, int32_t *nsteps, int nthreads) {
    const int S = m->S;
    int failed = 0;
    if (S > KIN_MAXS) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : failed)
#endif
    for (int64_t c = 0; c < n; ++c) {
        double y[KIN_MAXN];
        for (int i = 0; i < S; ++i) y[i] = Y[(size_t)i * ld + c];
        y[S] = T[c];
        int rc = kin_ros2(m, P[c], y, dt, rtol, atol, atol_T, max_steps);
        if (nsteps) nsteps[c] = rc;
        if (rc < 0) {
            ++failed;
            for (int i = 0; i < S; ++i) Y_out[(size_t)i * ld + c] = Y[(size_t)i * ld + c];
            T_out[c] = T[c];
        } else {
            for (int i = 0; i < S; ++i) Y_out[(size_t)i * ld + c] = y[i];
            T_out[c] = y[S];
        }
    }
    return failed;
}
