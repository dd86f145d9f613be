/*
 * pd_oracle.c -- plain FP64 direct-summation reference for the FCBM-EC
 * peridynamic operators.  TEST INFRASTRUCTURE ONLY: nothing in the product
 * library links, includes or calls this file; only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark use it.
 *
 * What it computes is the one-point (mid-point) quadrature of the
 * peridynamic integrals on a uniform grid, summed bond by bond over the
 * horizon stencil ("meshfree PD with direct quadrature", paper Sec. 1 and
 * Sec. 4.1.1, Eq. 55).  The fast method evaluates exactly these sums through
 * FFT convolutions, so the direct sum is the plain definition it must match.
 * No FFT, no blocking, no fusion: every function is a loop over nodes and,
 * inside, a loop over the bonds of that node.
 *
 * Conventions (readings of the paper where it is silent or ambiguous):
 *  - grid box nb[0] x nb[1] x nb[2] (x fastest, nb[2] = 1 in 2D); fields are
 *    stored component-major: f[c*N + (z*ny + y)*nx + x], N = nx*ny*nz;
 *  - node spacing dx[d]; cell volume dV = prod dx[d] (unit thickness in 2D);
 *  - bond offsets o != 0 with |o*dx|^2 <= delta^2 (1 + 1e-10)  (Eq. 16: the
 *    influence function vanishes beyond the horizon; the small relative
 *    slack makes grid points lying exactly on the horizon count as inside
 *    regardless of rounding);
 *  - influence function omega(r) = 1/r (the paper's choice, Sec. 5.1 and
 *    5.2) when influence == 0, omega = 1 when influence == 1;
 *  - periodic != 0: neighbour indices wrap around the box (periodic domain
 *    of Sec. 4.1); periodic == 0: neighbours outside the box do not exist.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the parallel loops below use (1 without OpenMP). */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

typedef struct {
    int dim;          /* 2 or 3 */
    int nb[3];        /* box size in nodes, nb[2] = 1 for dim == 2 */
    int periodic;     /* wrap neighbour indices around the box */
    double dx[3];     /* node spacing per axis */
    double delta;     /* horizon radius */
    int influence;    /* 0: omega = 1/r, 1: omega = 1 */
} orc_geom;

static const double ORC_PI = 3.14159265358979323846;

static double orc_dv(const orc_geom* g) {
    double v = g->dx[0] * g->dx[1];
    if (g->dim == 3) v *= g->dx[2];
    return v;
}

static long orc_nodes(const orc_geom* g) {
    return (long)g->nb[0] * g->nb[1] * g->nb[2];
}

static double orc_omega(const orc_geom* g, double r) {
    return g->influence == 0 ? 1.0 / r : 1.0;
}

/* Horizon stencil: every integer offset o != 0 whose bond vector o*dx lies
 * inside the horizon ball (Eq. 16 / Eq. 48 support).  Returns the count;
 * writes up to cap offsets as (ox, oy, oz) triples. */
int orc_stencil(const orc_geom* g, int* offs, int cap) {
    int M[3] = {0, 0, 0};
    for (int d = 0; d < g->dim; ++d) M[d] = (int)floor(g->delta / g->dx[d] + 1e-9) + 1;
    int n = 0;
    double lim = g->delta * g->delta * (1.0 + 1e-10);
    for (int oz = -M[2]; oz <= M[2]; ++oz)
        for (int oy = -M[1]; oy <= M[1]; ++oy)
            for (int ox = -M[0]; ox <= M[0]; ++ox) {
                if (ox == 0 && oy == 0 && oz == 0) continue;
                double xi0 = ox * g->dx[0], xi1 = oy * g->dx[1], xi2 = oz * g->dx[2];
                double r2 = xi0 * xi0 + xi1 * xi1 + (g->dim == 3 ? xi2 * xi2 : 0.0);
                if (r2 > lim) continue;
                if (n < cap) { offs[3 * n] = ox; offs[3 * n + 1] = oy; offs[3 * n + 2] = oz; }
                ++n;
            }
    return n;
}

/* The whole stencil in a buffer of its own size (free with free()). */
static int* orc_stencil_alloc(const orc_geom* g, int* ns) {
    int n = orc_stencil(g, NULL, 0);
    int* S = (int*)malloc(sizeof(int) * 3 * (size_t)(n > 0 ? n : 1));
    *ns = orc_stencil(g, S, n);
    return S;
}

/* Neighbour linear index of node (x, y, z) shifted by o, or -1 if the
 * neighbour falls outside a non-periodic box. */
static long orc_nbr(const orc_geom* g, int x, int y, int z, const int* o) {
    int p[3] = {x + o[0], y + o[1], z + o[2]};
    for (int d = 0; d < 3; ++d) {
        if (p[d] < 0 || p[d] >= g->nb[d]) {
            if (!g->periodic) return -1;
            p[d] = ((p[d] % g->nb[d]) + g->nb[d]) % g->nb[d];
        }
    }
    return ((long)p[2] * g->nb[1] + p[1]) * g->nb[0] + p[0];
}

/* Micromodulus constant alpha of the linearized bond-based solid
 * C(xi) = alpha * omega(|xi|) * xi (x) xi / |xi|^2  (Eq. 17), calibrated so
 * that the continuum limit matches classical isotropic elasticity with the
 * Poisson ratio bond-based models are restricted to: plane stress nu = 1/3
 * in 2D (alpha = 9E/(pi delta^3) for omega = 1/r, Sec. 5.2) and nu = 1/4 in
 * 3D.  Derivation: the effective Lame constant lambda equals
 *   (alpha/2) * A_d * int_0^delta omega(r) r^(d+1) dr,
 * with the angular moment A_2 = pi/4, A_3 = 4 pi/15; the target lambda is
 * 3E/8 in 2D plane stress and 2E/5 in 3D. */
double orc_bb_alpha(int dim, int influence, double E, double delta) {
    double I = (influence == 0) ? pow(delta, dim + 1) / (dim + 1) : pow(delta, dim + 2) / (dim + 2);
    double A = (dim == 2) ? ORC_PI / 4.0 : 4.0 * ORC_PI / 15.0;
    double lam = (dim == 2) ? 3.0 * E / 8.0 : 2.0 * E / 5.0;
    return 2.0 * lam / (A * I);
}

/* Linearized bond-based force density with bond weights phi(x) phi(x')
 * (Eq. 18 with the embedded-constraint mask of Eq. 75, the integrity
 * product of Eq. 46/100, or a heterogeneous micromodulus c0*s*s'):
 *   L_i(x) = phi(x) sum_o phi(x+o) alpha omega xi_i xi_j / r^2
 *            (u_j(x+o) - u_j(x)) dV                                        */
void orc_bb_force(const orc_geom* g, double alpha, const double* phi, const double* u, double* L) {
    int ns = 0;
    int* S = orc_stencil_alloc(g, &ns);
    long N = orc_nodes(g);
    int D = g->dim;
    double dV = orc_dv(g);
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
        int x = (int)(id % g->nb[0]);
        int y = (int)((id / g->nb[0]) % g->nb[1]);
        int z = (int)(id / ((long)g->nb[0] * g->nb[1]));
        double acc[3] = {0, 0, 0};
        if (phi[id] != 0.0) {
            for (int s = 0; s < ns; ++s) {
                long j = orc_nbr(g, x, y, z, &S[3 * s]);
                if (j < 0 || phi[j] == 0.0) continue;
                double xi[3] = {S[3 * s] * g->dx[0], S[3 * s + 1] * g->dx[1], S[3 * s + 2] * g->dx[2]};
                double r2 = 0;
                for (int d = 0; d < D; ++d) r2 += xi[d] * xi[d];
                double r = sqrt(r2);
                double eta_dot_xi = 0;
                for (int d = 0; d < D; ++d) eta_dot_xi += xi[d] * (u[d * N + j] - u[d * N + id]);
                double c = alpha * orc_omega(g, r) / r2 * phi[j] * dV;
                for (int i = 0; i < D; ++i) acc[i] += c * xi[i] * eta_dot_xi;
            }
        }
        for (int i = 0; i < D; ++i) L[i * N + id] = phi[id] * acc[i];
    }
    free(S);
}

/* Nonlinear, rotation-invariant bond-based solid (Sec. 3.2, Eq. 19-20), with
 * bond weights phi(x) phi(x') as for the linear model:
 *   L_i(x) = phi(x) sum_o phi(x+o) f_i dV,
 *   f = alpha omega(|xi|) |xi| (s + 3/2 s^2 + 1/2 s^3) (xi + eta)/|xi + eta|,
 *   s = (|xi + eta| - |xi|) / |xi|   (the bond strain),
 * xi = o*dx, eta = u(x+o) - u(x).  A bond whose deformed length is zero
 * carries no force (the limit of f, since s + 3/2 s^2 + 1/2 s^3 = 0 at
 * s = -1).  No linearisation: evaluated bond by bond as written. */
void orc_nbb_force(const orc_geom* g, double alpha, const double* phi, const double* u, double* L) {
    int ns = 0;
    int* S = orc_stencil_alloc(g, &ns);
    long N = orc_nodes(g);
    int D = g->dim;
    double dV = orc_dv(g);
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
        int x = (int)(id % g->nb[0]);
        int y = (int)((id / g->nb[0]) % g->nb[1]);
        int z = (int)(id / ((long)g->nb[0] * g->nb[1]));
        double acc[3] = {0, 0, 0};
        if (phi[id] != 0.0) {
            for (int s = 0; s < ns; ++s) {
                long j = orc_nbr(g, x, y, z, &S[3 * s]);
                if (j < 0 || phi[j] == 0.0) continue;
                double xi[3] = {S[3 * s] * g->dx[0], S[3 * s + 1] * g->dx[1], S[3 * s + 2] * g->dx[2]};
                double r2 = 0, y2 = 0, yv[3] = {0, 0, 0};
                for (int d = 0; d < D; ++d) {
                    yv[d] = xi[d] + (u[d * N + j] - u[d * N + id]);
                    r2 += xi[d] * xi[d];
                    y2 += yv[d] * yv[d];
                }
                double r = sqrt(r2), ry = sqrt(y2);
                if (ry == 0.0) continue;
                double st = (ry - r) / r;
                double mag = alpha * orc_omega(g, r) * r * (st + 1.5 * st * st + 0.5 * st * st * st) * phi[j] * dV;
                for (int i = 0; i < D; ++i) acc[i] += mag * yv[i] / ry;
            }
        }
        for (int i = 0; i < D; ++i) L[i * N + id] = phi[id] * acc[i];
    }
    free(S);
}

/* Strain energy density of the linearized bond-based solid with bond
 * weights (Eq. 42 with the bond weights inserted as the paper prescribes
 * for bond-breaking models, Eq. 47/102), in its direct bond form:
 *   W(x) = 1/2 phi(x) sum_o phi(x+o) alpha omega (xi . eta)^2 / r^2 dV      */
void orc_bb_energy(const orc_geom* g, double alpha, const double* phi, const double* u, double* W) {
    int ns = 0;
    int* S = orc_stencil_alloc(g, &ns);
    long N = orc_nodes(g);
    int D = g->dim;
    double dV = orc_dv(g);
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
        int x = (int)(id % g->nb[0]);
        int y = (int)((id / g->nb[0]) % g->nb[1]);
        int z = (int)(id / ((long)g->nb[0] * g->nb[1]));
        double acc = 0;
        if (phi[id] != 0.0) {
            for (int s = 0; s < ns; ++s) {
                long j = orc_nbr(g, x, y, z, &S[3 * s]);
                if (j < 0 || phi[j] == 0.0) continue;
                double xi[3] = {S[3 * s] * g->dx[0], S[3 * s + 1] * g->dx[1], S[3 * s + 2] * g->dx[2]};
                double r2 = 0, e = 0;
                for (int d = 0; d < D; ++d) {
                    r2 += xi[d] * xi[d];
                    e += xi[d] * (u[d * N + j] - u[d * N + id]);
                }
                acc += alpha * orc_omega(g, sqrt(r2)) * e * e / r2 * phi[j] * dV;
            }
        }
        W[id] = 0.5 * phi[id] * acc;
    }
    free(S);
}

/* Discrete weighted volume of the full horizon, m0 = sum_o omega r^2 dV
 * (Eq. 35 evaluated with the same one-point quadrature). */
double orc_m0(const orc_geom* g) {
    int ns = 0;
    int* S = orc_stencil_alloc(g, &ns);
    double dV = orc_dv(g), m0 = 0;
    for (int s = 0; s < ns; ++s) {
        double r2 = 0;
        for (int d = 0; d < g->dim; ++d) {
            double xi = S[3 * s + d] * g->dx[d];
            r2 += xi * xi;
        }
        m0 += orc_omega(g, sqrt(r2)) * r2 * dV;
    }
    free(S);
    return m0;
}

/* Linearized state-based (LPS) solid with the embedded-constraint mask chi
 * (Eq. 33-36 with the bond weights chi chi' of Eq. 75 and Eq. 92-94):
 *   m(x)     = chi sum_o chi' omega r^2 dV
 *   theta(x) = (3 chi / m(x)) sum_o chi' omega xi . (u' - u) dV  (0 if m = 0)
 *   L_i(x)   = chi sum_o chi' [ k_a omega xi_i (theta + theta')
 *                               + (30 mu / m0) omega xi_i xi_j / r^2 (u'_j - u_j) ] dV
 * with kappa = E / (3(1 - 2 nu)), mu = E / (2(1 + nu)), k_a = (3 kappa - 5 mu)/m0
 * and m0 the full-horizon weighted volume.  The force constants use m0, the
 * dilatation uses the local m(x) (Eq. 37 kernels are translation invariant;
 * Eq. 97 gives the local m).  theta_out may be NULL. */
void orc_lps_force(const orc_geom* g, double E, double nu, const double* chi, const double* u,
                   double* theta_out, double* L) {
    int ns = 0;
    int* S = orc_stencil_alloc(g, &ns);
    long N = orc_nodes(g);
    double dV = orc_dv(g);
    double m0 = orc_m0(g);
    double kappa = E / (3.0 * (1.0 - 2.0 * nu));
    double mu = E / (2.0 * (1.0 + nu));
    double ka = (3.0 * kappa - 5.0 * mu) / m0;
    double cC = 30.0 * mu / m0;
    double* th = (double*)malloc(sizeof(double) * N);
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
        int x = (int)(id % g->nb[0]);
        int y = (int)((id / g->nb[0]) % g->nb[1]);
        int z = (int)(id / ((long)g->nb[0] * g->nb[1]));
        double m = 0, s_ext = 0;
        if (chi[id] != 0.0) {
            for (int s = 0; s < ns; ++s) {
                long j = orc_nbr(g, x, y, z, &S[3 * s]);
                if (j < 0 || chi[j] == 0.0) continue;
                double xi[3] = {S[3 * s] * g->dx[0], S[3 * s + 1] * g->dx[1], S[3 * s + 2] * g->dx[2]};
                double r2 = 0, e = 0;
                for (int d = 0; d < 3; ++d) {
                    r2 += xi[d] * xi[d];
                    e += xi[d] * (u[d * N + j] - u[d * N + id]);
                }
                double w = orc_omega(g, sqrt(r2)) * chi[j] * dV;
                m += w * r2;
                s_ext += w * e;
            }
            m *= chi[id];
        }
        th[id] = (chi[id] != 0.0 && m != 0.0) ? 3.0 * chi[id] / m * s_ext : 0.0;
    }
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
        int x = (int)(id % g->nb[0]);
        int y = (int)((id / g->nb[0]) % g->nb[1]);
        int z = (int)(id / ((long)g->nb[0] * g->nb[1]));
        double acc[3] = {0, 0, 0};
        if (chi[id] != 0.0) {
            for (int s = 0; s < ns; ++s) {
                long j = orc_nbr(g, x, y, z, &S[3 * s]);
                if (j < 0 || chi[j] == 0.0) continue;
                double xi[3] = {S[3 * s] * g->dx[0], S[3 * s + 1] * g->dx[1], S[3 * s + 2] * g->dx[2]};
                double r2 = 0, e = 0;
                for (int d = 0; d < 3; ++d) {
                    r2 += xi[d] * xi[d];
                    e += xi[d] * (u[d * N + j] - u[d * N + id]);
                }
                double om = orc_omega(g, sqrt(r2)) * chi[j] * dV;
                for (int i = 0; i < 3; ++i)
                    acc[i] += ka * om * xi[i] * (th[id] + th[j]) + cC * om * xi[i] * e / r2;
            }
        }
        for (int i = 0; i < 3; ++i) L[i * N + id] = chi[id] * acc[i];
    }
    if (theta_out) memcpy(theta_out, th, sizeof(double) * N);
    free(th);
    free(S);
}

/* Damage index (Eq. 12 written as Eq. 49 with the integrity index, Eq. 44),
 * with the embedded-constraint mask: the count of intact bond partners
 * including the node itself,
 *   cnt(x)  = sum_{o in S u {0}} chi_B lambda (x+o),
 *   beta(x) = sum_{o in S u {0}} chi_B(x+o),
 *   d(x)    = 1 - chi_B lambda(x) cnt(x) / beta(x)   on chi_B = 1, else 0.
 * beta is the node's own family size within the body (Eq. 12). */
void orc_damage_index(const orc_geom* g, const uint8_t* chiB, const uint8_t* lam, double* d, int32_t* cnt_out) {
    int ns = 0;
    int* S = orc_stencil_alloc(g, &ns);
    long N = orc_nodes(g);
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
        int x = (int)(id % g->nb[0]);
        int y = (int)((id / g->nb[0]) % g->nb[1]);
        int z = (int)(id / ((long)g->nb[0] * g->nb[1]));
        int phi = (chiB[id] && lam[id]) ? 1 : 0;
        long cnt = phi, beta = chiB[id] ? 1 : 0;
        for (int s = 0; s < ns; ++s) {
            long j = orc_nbr(g, x, y, z, &S[3 * s]);
            if (j < 0) continue;
            cnt += (chiB[j] && lam[j]) ? 1 : 0;
            beta += chiB[j] ? 1 : 0;
        }
        d[id] = chiB[id] ? 1.0 - (double)(phi * cnt) / (double)beta : 0.0;
        if (cnt_out) cnt_out[id] = (int32_t)cnt;
    }
    free(S);
}

/* ------------------------------------------------------------------ */
/* Model description shared by the time integrator and the static solver */
typedef struct {
    int model;        /* 0: linearized bond-based, 1: linearized LPS (3D) */
    double E, nu;     /* Young modulus, Poisson ratio (LPS only) */
    double alpha;     /* bond-based micromodulus constant */
    double rho;       /* mass density */
    double Wc;        /* critical strain energy density (<= 0: no damage) */
} orc_model;

/* Force density with bond weights phi for either model.  For the LPS model
 * phi must be the 0/1 body mask. */
static void orc_force_any(const orc_geom* g, const orc_model* mdl, const double* phi, const double* u, double* L) {
    if (mdl->model == 0) orc_bb_force(g, mdl->alpha, phi, u, L);
    else orc_lps_force(g, mdl->E, mdl->nu, phi, u, NULL, L);
}

/* Bond weight phi = chi_B * lambda * s (lambda, s optional). */
static void orc_weights(long N, const uint8_t* chiB, const uint8_t* lam, const double* s, double* phi) {
    for (long i = 0; i < N; ++i) {
        double p = chiB[i] ? 1.0 : 0.0;
        if (lam && !lam[i]) p = 0.0;
        if (s) p *= s[i];
        phi[i] = p;
    }
}

/* Embedded-constraint velocity-Verlet dynamics (Eq. 67 with Eq. 83-84),
 * with the pointwise energy failure rule (Eq. 40, 43, 63) applied
 * irreversibly and one step behind the force (the integrity used for the
 * force at t + dt is lambda^{n+1} = lambda^n AND [W^n <= W_c], W^n being the
 * energy of (u^n, lambda^n)).  One step:
 *   u      <- chi_O [u + dt v + dt^2/(2 rho) F] + (1 - chi_O) w
 *   lambda <- lambda AND [W <= W_c]                    (if damage is on)
 *   F'     <- L(u; chi_B lambda s) + b,  W' <- W(u; chi_B lambda s)
 *   v      <- chi_O [v + dt/(2 rho) (F + F')]
 * chiO holds one 0/1 mask per displacement component (Eq. 74).  If init != 0
 * the force F and energy W of the initial state are computed first.
 * energy (optional, nsteps x 4): kinetic, internal potential
 * -1/2 dV <u, L>, external -dV <u, b>, and the discrete shadow energy
 * KE + PE + EXT - dt^2/(8 rho) dV |chi_O F|^2 that velocity Verlet
 * conserves exactly for a linear force. */
void orc_verlet(const orc_geom* g, const orc_model* mdl, const uint8_t* chiB, const uint8_t* chiO,
                uint8_t* lam, const double* s, double* u, double* v, double* F, double* W,
                const double* b, const double* w, double dt, int nsteps, int init, double* energy) {
    long N = orc_nodes(g);
    int D = g->dim;
    double dV = orc_dv(g);
    double* phi = (double*)malloc(sizeof(double) * N);
    double* Lt = (double*)malloc(sizeof(double) * N * D);
    const uint8_t* lw = (mdl->model == 0) ? lam : NULL;
    int damage = (mdl->Wc > 0 && lw != NULL);
    if (init) {
        orc_weights(N, chiB, lw, s, phi);
        orc_force_any(g, mdl, phi, u, Lt);
        for (long i = 0; i < N * D; ++i) F[i] = Lt[i] + (b ? b[i] : 0.0);
        if (damage && W) orc_bb_energy(g, mdl->alpha, phi, u, W);
    }
    for (int step = 0; step < nsteps; ++step) {
        for (long i = 0; i < N * D; ++i) {
            double wi = w ? w[i] : 0.0;
            u[i] = chiO[i] ? (u[i] + dt * v[i] + dt * dt / (2.0 * mdl->rho) * F[i]) : wi;
        }
        if (damage)
            for (long i = 0; i < N; ++i) lam[i] = (lam[i] && W[i] <= mdl->Wc) ? 1 : 0;
        orc_weights(N, chiB, lw, s, phi);
        orc_force_any(g, mdl, phi, u, Lt);
        if (damage && W) orc_bb_energy(g, mdl->alpha, phi, u, W);
        for (long i = 0; i < N * D; ++i) {
            double Fn = Lt[i] + (b ? b[i] : 0.0);
            v[i] = chiO[i] ? (v[i] + dt / (2.0 * mdl->rho) * (F[i] + Fn)) : 0.0;
            F[i] = Fn;
        }
        if (energy) {
            double ke = 0, pe = 0, ext = 0, f2 = 0;
            for (long i = 0; i < N * D; ++i) {
                ke += 0.5 * mdl->rho * v[i] * v[i];
                pe += -0.5 * u[i] * Lt[i];
                ext += -(b ? b[i] : 0.0) * u[i];
                if (chiO[i]) f2 += F[i] * F[i];
            }
            energy[4 * step + 0] = ke * dV;
            energy[4 * step + 1] = pe * dV;
            energy[4 * step + 2] = ext * dV;
            energy[4 * step + 3] = (ke + pe + ext) * dV - dt * dt / (8.0 * mdl->rho) * f2 * dV;
        }
    }
    free(Lt);
    free(phi);
}

/* Embedded-constraint statics (Eq. 85-89) by conjugate gradients.  The
 * unknowns are the components with chi_O = 1; u = w on the rest.  With
 * u = chi_O y + (1 - chi_O) w the residual R = chi_O (L(u) + b) = 0 becomes
 *   A y = rhs,  A = -chi_O L chi_O (symmetric positive definite on the
 *   unknowns),  rhs = chi_O (b + L((1 - chi_O) w)).
 * Plain CG from the initial guess in u, stopped when
 * |R(u)|_2 <= rtol |rhs|_2 or after maxit iterations.  Returns the iteration
 * count; *relres receives the final relative residual. */
int orc_static_cg(const orc_geom* g, const orc_model* mdl, const uint8_t* chiB, const uint8_t* chiO,
                  const double* b, const double* w, double* u, double rtol, int maxit, double* relres) {
    long N = orc_nodes(g);
    int D = g->dim;
    long n = N * D;
    double* phi = (double*)malloc(sizeof(double) * N);
    double* t = (double*)malloc(sizeof(double) * n);
    double* Lt = (double*)malloc(sizeof(double) * n);
    double* r = (double*)malloc(sizeof(double) * n);
    double* p = (double*)malloc(sizeof(double) * n);
    double* Ap = (double*)malloc(sizeof(double) * n);
    orc_weights(N, chiB, NULL, NULL, phi);
    /* rhs = chi_O (b + L((1 - chi_O) w)) */
    for (long i = 0; i < n; ++i) t[i] = chiO[i] ? 0.0 : (w ? w[i] : 0.0);
    orc_force_any(g, mdl, phi, t, Lt);
    double rhs_norm2 = 0;
    double* rhs = (double*)malloc(sizeof(double) * n);
    for (long i = 0; i < n; ++i) {
        rhs[i] = chiO[i] ? (b[i] + Lt[i]) : 0.0;
        rhs_norm2 += rhs[i] * rhs[i];
    }
    /* y0 = chi_O u;  r = rhs - A y0 = rhs + chi_O L(chi_O y0) */
    for (long i = 0; i < n; ++i) t[i] = chiO[i] ? u[i] : 0.0;
    orc_force_any(g, mdl, phi, t, Lt);
    double rr = 0;
    for (long i = 0; i < n; ++i) {
        r[i] = chiO[i] ? rhs[i] + Lt[i] : 0.0;
        p[i] = r[i];
        rr += r[i] * r[i];
    }
    double bn = sqrt(rhs_norm2);
    int it = 0;
    if (bn == 0.0) bn = 1.0;
    while (it < maxit && sqrt(rr) > rtol * bn) {
        orc_force_any(g, mdl, phi, p, Lt);
        double pAp = 0;
        for (long i = 0; i < n; ++i) {
            Ap[i] = chiO[i] ? -Lt[i] : 0.0;
            pAp += p[i] * Ap[i];
        }
        double a = rr / pAp;
        double rr_new = 0;
        for (long i = 0; i < n; ++i) {
            t[i] += a * p[i];
            r[i] -= a * Ap[i];
            rr_new += r[i] * r[i];
        }
        double beta = rr_new / rr;
        rr = rr_new;
        for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        ++it;
    }
    for (long i = 0; i < n; ++i) u[i] = chiO[i] ? t[i] : (w ? w[i] : 0.0);
    /* true residual of the returned iterate */
    orc_force_any(g, mdl, phi, u, Lt);
    double res2 = 0;
    for (long i = 0; i < n; ++i) {
        double R = chiO[i] ? Lt[i] + b[i] : 0.0;
        res2 += R * R;
    }
    if (relres) *relres = sqrt(res2) / bn;
    free(rhs); free(phi); free(t); free(Lt); free(r); free(p); free(Ap);
    return it;
}

/* Adjoint of the weighted bond-based force (derived from Eq. 46/100; the
 * paper has no adjoint).  For a cotangent g on L:
 *   u_bar   = L_phi(g)            (the operator is symmetric for fixed phi)
 *   phi_bar(y) = d <g, L_phi(u)> / d phi(y)
 *       = sum_o [ g_i(y) phi(y+o) C_ij(o) (u_j(y+o) - u_j(y))
 *               + g_i(y+o) phi(y+o) C_ij(o) (u_j(y) - u_j(y+o)) ] dV
 * written as a gather over the bonds of y (the second term is the bond seen
 * from its other end, C being even in o).  ubar or phibar may be NULL. */
void orc_bb_force_adjoint(const orc_geom* g, double alpha, const double* phi, const double* u,
                          const double* gb, double* ubar, double* phibar) {
    long N = orc_nodes(g);
    int D = g->dim;
    if (ubar) orc_bb_force(g, alpha, phi, gb, ubar);
    if (!phibar) return;
    int ns = 0;
    int* S = orc_stencil_alloc(g, &ns);
    double dV = orc_dv(g);
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
        int x = (int)(id % g->nb[0]);
        int y = (int)((id / g->nb[0]) % g->nb[1]);
        int z = (int)(id / ((long)g->nb[0] * g->nb[1]));
        double acc = 0;
        for (int s = 0; s < ns; ++s) {
            long j = orc_nbr(g, x, y, z, &S[3 * s]);
            if (j < 0) continue;
            double xi[3] = {S[3 * s] * g->dx[0], S[3 * s + 1] * g->dx[1], S[3 * s + 2] * g->dx[2]};
            double r2 = 0;
            for (int d = 0; d < D; ++d) r2 += xi[d] * xi[d];
            double c = alpha * orc_omega(g, sqrt(r2)) / r2 * dV;
            double e = 0, gy = 0, gj = 0;
            for (int d = 0; d < D; ++d) {
                e += xi[d] * (u[d * N + j] - u[d * N + id]);
                gy += xi[d] * gb[d * N + id];
                gj += xi[d] * gb[d * N + j];
            }
            /* C_ij g_i eta_j = c (xi . g)(xi . eta) */
            acc += c * phi[j] * gy * e - c * phi[j] * gj * e;
        }
        phibar[id] = acc;
    }
    free(S);
}

/* Reverse-mode sweep of the embedded-constraint Verlet rollout with fixed
 * bond weights phi, constant body force b and w = 0 on the constrained
 * components.  Forward step (as in orc_verlet without damage):
 *   u' = chi_O (u + dt v + c2 (L u + b)),  v' = chi_O (v + c1 (L u + b + L u' + b)),
 *   c1 = dt/(2 rho), c2 = dt^2/(2 rho).
 * Given ubar, vbar at the final time (overwritten with the cotangents of the
 * initial u0, v0) and returning d/dphi in phibar and d/db in bbar (both
 * accumulated; bbar may be NULL), the trajectory is stored and swept
 * backwards:
 *   a = chi_O vbar';  ut = ubar' + c1 L a;
 *   ubar = c1 L a + chi_O ut + c2 L(chi_O ut);  vbar = a + dt chi_O ut;
 *   phibar += c1 dphi<a, L(u + u')> + c2 dphi<chi_O ut, L u>;
 *   bbar += c2 chi_O ut + 2 c1 a   (b enters u' once through F = L u + b,
 *                                   and v' twice, through F and F').    */
void orc_verlet_adjoint(const orc_geom* g, double alpha, double rho, const uint8_t* chiO,
                        const double* phi, const double* b, const double* u0, const double* v0,
                        double dt, int nsteps, double* ubar, double* vbar, double* phibar, double* bbar) {
    long N = orc_nodes(g);
    int D = g->dim;
    long n = N * D;
    double c1 = dt / (2.0 * rho), c2 = dt * dt / (2.0 * rho);
    double* U = (double*)malloc(sizeof(double) * n * (nsteps + 1));
    double* v = (double*)malloc(sizeof(double) * n);
    double* F = (double*)malloc(sizeof(double) * n);
    double* Lt = (double*)malloc(sizeof(double) * n);
    memcpy(U, u0, sizeof(double) * n);
    memcpy(v, v0, sizeof(double) * n);
    orc_bb_force(g, alpha, phi, U, Lt);
    for (long i = 0; i < n; ++i) F[i] = Lt[i] + b[i];
    for (int st = 0; st < nsteps; ++st) {
        double* uc = U + n * st;
        double* un = U + n * (st + 1);
        for (long i = 0; i < n; ++i) un[i] = chiO[i] ? uc[i] + dt * v[i] + c2 * F[i] : 0.0;
        orc_bb_force(g, alpha, phi, un, Lt);
        for (long i = 0; i < n; ++i) {
            double Fn = Lt[i] + b[i];
            v[i] = chiO[i] ? v[i] + c1 * (F[i] + Fn) : 0.0;
            F[i] = Fn;
        }
    }
    double* a = (double*)malloc(sizeof(double) * n);
    double* ut = (double*)malloc(sizeof(double) * n);
    double* La = (double*)malloc(sizeof(double) * n);
    double* us = (double*)malloc(sizeof(double) * n);
    double* pb = (double*)malloc(sizeof(double) * N);
    for (int st = nsteps - 1; st >= 0; --st) {
        double* uc = U + n * st;
        double* un = U + n * (st + 1);
        for (long i = 0; i < n; ++i) a[i] = chiO[i] ? vbar[i] : 0.0;
        orc_bb_force(g, alpha, phi, a, La);
        for (long i = 0; i < n; ++i) {
            ut[i] = chiO[i] ? ubar[i] + c1 * La[i] : 0.0;
            us[i] = uc[i] + un[i];
        }
        orc_bb_force_adjoint(g, alpha, phi, us, a, NULL, pb);
        for (long i = 0; i < N; ++i) phibar[i] += c1 * pb[i];
        orc_bb_force(g, alpha, phi, ut, Lt);
        orc_bb_force_adjoint(g, alpha, phi, uc, ut, NULL, pb);
        for (long i = 0; i < N; ++i) phibar[i] += c2 * pb[i];
        for (long i = 0; i < n; ++i) {
            ubar[i] = c1 * La[i] + ut[i] + c2 * Lt[i];
            vbar[i] = a[i] + dt * ut[i];
            if (bbar) bbar[i] += c2 * ut[i] + 2.0 * c1 * a[i];
        }
    }
    free(a); free(ut); free(La); free(us); free(pb);
    free(U); free(v); free(F); free(Lt);
}

/* ------------------------------------------------------------------ */
/* Comparator only: the critical bond-strain failure rule of Sec. 2 (Eq. 10-12).
 * It removes bonds one by one and so has no convolution structure; the fast
 * method replaces it with the pointwise energy rule (Sec. 3.4), and these
 * functions exist to compare the two, as the paper does in Sec. 5.2.
 *
 * mu holds one intact flag per (node, stencil bond), node-major:
 * mu[id * ns + s] is the bond from node id along stencil offset s, in the
 * order orc_stencil lists the offsets.  Bonds whose partner lies outside a
 * non-periodic box or outside the body are ignored by every function. */

/* Critical stretch s_c calibrated to the fracture energy G0 (the rule the
 * paper cites for bond-strain models, Sec. 3.4.3 follows its idea): the
 * energy of every bond crossing a unit area of a planar crack equals G0.
 * With the linearized bond energy per pair of unit volumes
 *   w = 1/2 alpha omega(r) (xi . eta)^2 / r^2 = 1/2 alpha omega(r) s^2 r^2
 * at stretch s, a bond xi with normal component xi_n > 0 crosses the plane
 * for xi_n of the depths below it, so
 *   G0 = 1/2 alpha s_c^2 K,  K = int_{|xi| <= delta, xi_n > 0} omega(r) r^2 xi_n dxi,
 *   K = delta^4 / 2 (2D) or pi delta^5 / 5 (3D) for omega = 1/r,
 *   K = 2 delta^5 / 5 (2D) or pi delta^6 / 6 (3D) for omega = 1. */
double orc_bond_sc(int dim, int influence, double alpha, double G0, double delta) {
    double K;
    if (influence == 0) K = (dim == 2) ? pow(delta, 4) / 2.0 : ORC_PI * pow(delta, 5) / 5.0;
    else K = (dim == 2) ? 2.0 * pow(delta, 5) / 5.0 : ORC_PI * pow(delta, 6) / 6.0;
    return sqrt(2.0 * G0 / (alpha * K));
}

/* Linearized bond-based force with per-bond intact flags (Eq. 10 with the
 * integrand of Eq. 18):
 *   L_i(x) = chi_B(x) sum_o mu(x, o) chi_B(x+o) alpha omega xi_i xi_j / r^2
 *            (u_j(x+o) - u_j(x)) dV                                        */
void orc_bond_force(const orc_geom* g, double alpha, const uint8_t* chiB, const uint8_t* mu, const double* u,
                    double* L) {
    int ns = 0;
    int* S = orc_stencil_alloc(g, &ns);
    long N = orc_nodes(g);
    int D = g->dim;
    double dV = orc_dv(g);
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
        int x = (int)(id % g->nb[0]);
        int y = (int)((id / g->nb[0]) % g->nb[1]);
        int z = (int)(id / ((long)g->nb[0] * g->nb[1]));
        double acc[3] = {0, 0, 0};
        if (chiB[id]) {
            for (int s = 0; s < ns; ++s) {
                long j = orc_nbr(g, x, y, z, &S[3 * s]);
                if (j < 0 || !chiB[j] || !mu[id * ns + s]) continue;
                double xi[3] = {S[3 * s] * g->dx[0], S[3 * s + 1] * g->dx[1], S[3 * s + 2] * g->dx[2]};
                double r2 = 0, ed = 0;
                for (int d = 0; d < D; ++d) r2 += xi[d] * xi[d];
                for (int d = 0; d < D; ++d) ed += xi[d] * (u[d * N + j] - u[d * N + id]);
                double c = alpha * orc_omega(g, sqrt(r2)) / r2 * dV;
                for (int i = 0; i < D; ++i) acc[i] += c * xi[i] * ed;
            }
        }
        for (int i = 0; i < D; ++i) L[i * N + id] = acc[i];
    }
    free(S);
}

/* Break, for good, every body bond whose stretch exceeds s_c.  The stretch
 * of the linearized model is s = xi . eta / |xi|^2 (the first-order part of
 * (|xi + eta| - |xi|) / |xi|); it is the same seen from either end, so both
 * directions of a bond break together.  Returns the number of flags
 * cleared. */
long orc_bond_break(const orc_geom* g, double s_c, const uint8_t* chiB, uint8_t* mu, const double* u) {
    int ns = 0;
    int* S = orc_stencil_alloc(g, &ns);
    long N = orc_nodes(g);
    int D = g->dim;
    long broken = 0;
#pragma omp parallel for schedule(static) reduction(+ : broken)
    for (long id = 0; id < N; ++id) {
        int x = (int)(id % g->nb[0]);
        int y = (int)((id / g->nb[0]) % g->nb[1]);
        int z = (int)(id / ((long)g->nb[0] * g->nb[1]));
        if (!chiB[id]) continue;
        for (int s = 0; s < ns; ++s) {
            long j = orc_nbr(g, x, y, z, &S[3 * s]);
            if (j < 0 || !chiB[j] || !mu[id * ns + s]) continue;
            double xi[3] = {S[3 * s] * g->dx[0], S[3 * s + 1] * g->dx[1], S[3 * s + 2] * g->dx[2]};
            double r2 = 0, ed = 0;
            for (int d = 0; d < D; ++d) r2 += xi[d] * xi[d];
            for (int d = 0; d < D; ++d) ed += xi[d] * (u[d * N + j] - u[d * N + id]);
            if (ed / r2 > s_c) {
                mu[id * ns + s] = 0;
                ++broken;
            }
        }
    }
    free(S);
    return broken;
}

/* Damage index of Eq. 12 with the one-point quadrature (equal weights dV,
 * so the ratio of integrals is a ratio of bond counts):
 *   d(x) = 1 - sum_o mu(x, o) chi_B(x+o) / sum_o chi_B(x+o)   on chi_B = 1,
 * 0 off the body and for a node without body partners. */
void orc_bond_damage(const orc_geom* g, const uint8_t* chiB, const uint8_t* mu, double* d) {
    int ns = 0;
    int* S = orc_stencil_alloc(g, &ns);
    long N = orc_nodes(g);
#pragma omp parallel for schedule(static)
    for (long id = 0; id < N; ++id) {
        int x = (int)(id % g->nb[0]);
        int y = (int)((id / g->nb[0]) % g->nb[1]);
        int z = (int)(id / ((long)g->nb[0] * g->nb[1]));
        long tot = 0, intact = 0;
        if (chiB[id]) {
            for (int s = 0; s < ns; ++s) {
                long j = orc_nbr(g, x, y, z, &S[3 * s]);
                if (j < 0 || !chiB[j]) continue;
                ++tot;
                intact += mu[id * ns + s] ? 1 : 0;
            }
        }
        d[id] = tot ? 1.0 - (double)intact / (double)tot : 0.0;
    }
    free(S);
}

/* Velocity Verlet of the bond-based solid under the critical bond-strain
 * rule.  Bonds are checked on the new positions u^{n+1} and the force at
 * t + dt uses the bonds still intact after that check (bond-strain codes
 * break bonds as soon as they are overstretched; the energy rule of
 * orc_verlet instead lags one step, Eq. 63).  One step:
 *   u  <- chi_O [u + dt v + dt^2/(2 rho) F] + (1 - chi_O) w
 *   mu <- mu AND [s(u) <= s_c]
 *   F' <- L_mu(u) + b
 *   v  <- chi_O [v + dt/(2 rho) (F + F')]
 * If init != 0 the force of the initial state is computed first.  Returns
 * the number of bond flags cleared. */
long orc_bond_verlet(const orc_geom* g, double alpha, double rho, double s_c, const uint8_t* chiB,
                     const uint8_t* chiO, uint8_t* mu, double* u, double* v, double* F, const double* b,
                     const double* w, double dt, int nsteps, int init) {
    long N = orc_nodes(g);
    int D = g->dim;
    double* Lt = (double*)malloc(sizeof(double) * N * D);
    long broken = 0;
    if (init) {
        orc_bond_force(g, alpha, chiB, mu, u, Lt);
        for (long i = 0; i < N * D; ++i) F[i] = Lt[i] + (b ? b[i] : 0.0);
    }
    for (int step = 0; step < nsteps; ++step) {
        for (long i = 0; i < N * D; ++i) {
            double wi = w ? w[i] : 0.0;
            u[i] = chiO[i] ? (u[i] + dt * v[i] + dt * dt / (2.0 * rho) * F[i]) : wi;
        }
        broken += orc_bond_break(g, s_c, chiB, mu, u);
        orc_bond_force(g, alpha, chiB, mu, u, Lt);
        for (long i = 0; i < N * D; ++i) {
            double Fn = Lt[i] + (b ? b[i] : 0.0);
            v[i] = chiO[i] ? (v[i] + dt / (2.0 * rho) * (F[i] + Fn)) : 0.0;
            F[i] = Fn;
        }
    }
    free(Lt);
    return broken;
}
