/*
 * Plain FP64 CPU oracle of the advection-diffusion lattice Boltzmann model coupled to the
 * Maxwell-Stefan equations through a per-node relaxation time (Huang, Bao, Jiang, Zhang,
 * "A combined approach of LBM and Maxwell-Stefan equation for modeling multi-component
 * diffusion in SOFC", arXiv 1809.01600).
 *
 * TEST INFRASTRUCTURE.  This file exists only to check the HIP library; it is slow on purpose
 * and shares no code, header, table or helper with it.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.
 *
 * State: the pre-collision populations f[s][a][node] of the two evolved species s = 0 (H2) and
 * s = 1 (H2O); the inert third species (Ar) is the balance X_3 = 1 - X_1 - X_2.  node index =
 * (z * ny + y) * nx + x, x = diffusion direction (Dirichlet inlet at x = 0, reactive-flux outlet
 * at x = nx - 1), periodic in y and z.  Entries of solid nodes are ignored and written as 0.
 *
 * One step, in the paper's order (Eq. 28: collide, then stream):
 *   1. moments X_s = sum_a f_a (Eq. 29 makes f a mole-fraction distribution); X_3 by closure
 *      (Sec. 3.2, last paragraph).
 *   2. mole-fraction gradients in lattice units (Eq. 35 in x at the inlet column, Eq. 37 at the
 *      outlet column, central differences elsewhere, one-sided next to solid).
 *   3. Maxwell-Stefan matrix [B] (Eq. 32), generalized Fick fluxes J = -[B]^-1 grad X with
 *      Gamma = I (Eq. 30, 33, 34); N = J since the total molar flux is zero (Eq. 21 with u_M = 0).
 *   4. effective diffusivity of each evolved species from Eq. 24 with the flux vectors replaced
 *      by signed norms N_i -> -sgn(nu_i) |N_i|.
 *   5. relaxation time tau_i = D_i / c_s^2 + 1/2 with c_s^2 = 1/3 (Eq. 25).
 *   6. BGK collision toward f_eq = w_a X_s (Eq. 28 with Eq. 29), plus the source term of Eq. 27,
 *      F_a = w_a S_s, on the fluid nodes of the columns x >= src_x0 (zero unless a source is set).
 *   7. streaming; half-way bounce-back on solid links (Sec. 3.3, last paragraph).
 *   8. inlet: anti-bounce-back f_a = (w_a + w_abar) X_in - f_abar (Eq. 36);
 *      outlet: exact-flux rule f_a = f*_abar - (w_abar / W_n) Q_s imposing the electrode flux
 *      N_s = -nu_s I / (n F) (Eq. 39) as the net lattice outflow Q_s per open outlet node.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int lattice;          /* 0: D2Q9, 1: D3Q19, 2: D2Q5, 3: D3Q7 */
    int nx, ny, nz;       /* nz = 1 for D2Q9 */
    double Dl[3][3];      /* lattice binary diffusivities D*_ij = D_ij dt / dx^2 (symmetric) */
    double X_in[2];       /* inlet mole fractions of the evolved species */
    double Q[2];          /* lattice outflow per open outlet node per step, evolved species */
    double nu[3];         /* stoichiometric coefficients (Eq. 39) */
    int inlet_wall;       /* 1: the inlet face is a bounce-back wall (closed-box tests) */
    int ms_mode;          /* 0: flux-norm ratio from the local fluxes, 1: stoichiometric ratio */
    double eps;           /* regularizer of the flux-norm ratio (lattice units) */
    double tau_min, tau_max;
    double S[2];          /* source per fluid node and step of the columns x >= src_x0 (Eq. 27) */
    int src_x0;
    int trt;              /* 1: two-relaxation-time collision instead of BGK */
    double lambda_trt;    /* TRT: (tau_even - 1/2)(tau - 1/2), tau from Eq. 25 */
    double tau_flow;      /* advective coupling only: relaxation time of the velocity model */
} orc_params;

typedef struct {
    double inflow[2];     /* amount entering through the inlet face during the step */
    double outflow[2];    /* amount leaving through the outlet face during the step */
    long clamp_hits;      /* relaxation times that hit tau_min or tau_max */
} orc_stats;

#define ORC_QMAX 19

typedef struct {
    int q;
    int e[ORC_QMAX][3];
    double w[ORC_QMAX];
    int opp[ORC_QMAX];
    double Wn;            /* sum of the weights of the velocities with e_x = +1 */
} orc_lattice;

/* D2Q9 from Eq. 2 and Eq. 9; D3Q19 by enumerating the vectors of {-1,0,1}^3 with |e|^2 <= 2
 * (rest, then the six axis vectors, then the twelve edge vectors) with weights 1/3, 1/18, 1/36. */
static void build_lattice(int lattice, orc_lattice* L)
{
    memset(L, 0, sizeof(*L));
    if (lattice == 2) {
        /* D2Q5 (the paper names it beside D2Q9 in Sec. 2.3): rest and the four axis links, with
         * weights 1/3 and 1/6, which give sum_a w_a e_a e_a = I / 3 like D2Q9 */
        static const int ex[5] = {0, 1, 0, -1, 0}, ey[5] = {0, 0, 1, 0, -1};
        L->q = 5;
        for (int a = 0; a < 5; ++a) {
            L->e[a][0] = ex[a];
            L->e[a][1] = ey[a];
            L->e[a][2] = 0;
            L->w[a] = (a == 0) ? 1.0 / 3.0 : 1.0 / 6.0;
        }
    } else if (lattice == 3) {
        /* D3Q7: rest and the six axis links.  Sec. 3.1 fixes c_s^2 = 1/3 (so tau = 3 D* + 1/2,
         * Eq. 25); sum_a w_a e_a e_a = 2 w_axis I then needs w_axis = 1/6, and unit mass leaves
         * the rest link a weight of 0 */
        static const int ex[7] = {0, 1, -1, 0, 0, 0, 0}, ey[7] = {0, 0, 0, 1, -1, 0, 0},
                         ez[7] = {0, 0, 0, 0, 0, 1, -1};
        L->q = 7;
        for (int a = 0; a < 7; ++a) {
            L->e[a][0] = ex[a];
            L->e[a][1] = ey[a];
            L->e[a][2] = ez[a];
            L->w[a] = (a == 0) ? 0.0 : 1.0 / 6.0;
        }
    } else if (lattice == 0) {
        L->q = 9;
        for (int a = 0; a < 9; ++a) {
            double ex = 0.0, ey = 0.0;
            if (a >= 1 && a <= 4) {
                ex = cos((a - 1) * M_PI / 2.0);
                ey = sin((a - 1) * M_PI / 2.0);
            } else if (a >= 5) {
                ex = sqrt(2.0) * cos((a - 5) * M_PI / 2.0 + M_PI / 4.0);
                ey = sqrt(2.0) * sin((a - 5) * M_PI / 2.0 + M_PI / 4.0);
            }
            L->e[a][0] = (int)lround(ex);
            L->e[a][1] = (int)lround(ey);
            L->e[a][2] = 0;
            L->w[a] = (a == 0) ? 4.0 / 9.0 : (a <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
        }
    } else {
        int n = 0;
        for (int len2 = 0; len2 <= 2; ++len2)
            for (int ez = -1; ez <= 1; ++ez)
                for (int ey = -1; ey <= 1; ++ey)
                    for (int ex = -1; ex <= 1; ++ex) {
                        if (ex * ex + ey * ey + ez * ez != len2) continue;
                        L->e[n][0] = ex;
                        L->e[n][1] = ey;
                        L->e[n][2] = ez;
                        L->w[n] = (len2 == 0) ? 1.0 / 3.0 : (len2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
                        ++n;
                    }
        L->q = n; /* 19 */
    }
    for (int a = 0; a < L->q; ++a) {
        for (int b = 0; b < L->q; ++b)
            if (L->e[b][0] == -L->e[a][0] && L->e[b][1] == -L->e[a][1] && L->e[b][2] == -L->e[a][2])
                L->opp[a] = b;
        if (L->e[a][0] == 1) L->Wn += L->w[a];
    }
}

int orc_num_velocities(int lattice)
{
    orc_lattice L;
    build_lattice(lattice, &L);
    return L.q;
}

void orc_velocities(int lattice, int* e, double* w)
{
    orc_lattice L;
    build_lattice(lattice, &L);
    for (int a = 0; a < L.q; ++a) {
        e[3 * a + 0] = L.e[a][0];
        e[3 * a + 1] = L.e[a][1];
        e[3 * a + 2] = L.e[a][2];
        w[a] = L.w[a];
    }
}

static int wrap(int i, int n) { return ((i % n) + n) % n; }

static long node_index(const orc_params* p, int x, int y, int z)
{
    return ((long)z * p->ny + y) * p->nx + x;
}

/* sign convention of Eq. 24: N_i = -(nu_i / |nu_i|) |N_i|; zero for an inert species */
static double flux_sign(double nu)
{
    if (nu > 0.0) return -1.0;
    if (nu < 0.0) return 1.0;
    return 0.0;
}

/* Moments of all nodes: X[k][node], k = 0, 1 evolved species, k = 2 the balance species. */
void orc_moments(const orc_params* p, const uint8_t* solid, const double* f, double* X)
{
    orc_lattice L;
    build_lattice(p->lattice, &L);
    long N = (long)p->nx * p->ny * p->nz;
    for (long n = 0; n < N; ++n) {
        if (solid[n]) {
            X[n] = X[N + n] = X[2 * N + n] = 0.0;
            continue;
        }
        double xs[2];
        for (int s = 0; s < 2; ++s) {
            double sum = 0.0;
            for (int a = 0; a < L.q; ++a) sum += f[((long)s * L.q + a) * N + n];
            xs[s] = sum;
        }
        X[n] = xs[0];
        X[N + n] = xs[1];
        X[2 * N + n] = 1.0 - xs[0] - xs[1];
    }
}

/* Is (x, y, z) an existing fluid node?  y and z wrap; x does not. */
static int is_fluid(const orc_params* p, const uint8_t* solid, int x, int y, int z)
{
    if (x < 0 || x >= p->nx) return 0;
    return !solid[node_index(p, x, wrap(y, p->ny), wrap(z, p->nz))];
}

/* Eq. 32: the (n-1)x(n-1) matrix [B] for n = 3 species, from the full composition X[0..2]. */
static void ms_matrix(const orc_params* p, const double X[3], double B[2][2])
{
    const int n = 2; /* index of the last (balance) species */
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            if (i == j) {
                double b = X[i] / p->Dl[i][n];
                for (int k = 0; k < 3; ++k)
                    if (k != i) b += X[k] / p->Dl[i][k];
                B[i][i] = b;
            } else {
                B[i][j] = -X[i] * (1.0 / p->Dl[i][j] - 1.0 / p->Dl[i][n]);
            }
        }
}

/*
 * Steps 1-6 for every fluid node: f (pre-collision) -> fstar (post-collision).
 * Optionally returns the relaxation times tau[s][node] and the fluxes J[s][d][node].
 */
static int collide_all(const orc_params* p, const orc_lattice* L, const uint8_t* solid,
                       const double* f, double* fstar, double* tau_out, double* J_out,
                       long* clamp_hits)
{
    const long N = (long)p->nx * p->ny * p->nz;
    const int q = L->q;
    const int dims = (p->lattice == 1 || p->lattice == 3) ? 3 : 2;
    double* X = (double*)malloc(sizeof(double) * 3 * N);
    if (!X) return -8;
    orc_moments(p, solid, f, X);
    long hits = 0;

    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const long n = node_index(p, x, y, z);
                if (solid[n]) {
                    for (int s = 0; s < 2; ++s)
                        for (int a = 0; a < q; ++a) fstar[((long)s * q + a) * N + n] = 0.0;
                    continue;
                }
                double Xn[3] = {X[n], X[N + n], X[2 * N + n]};
                double B[2][2];
                ms_matrix(p, Xn, B);

                /* step 2: gradients g[s][d] in lattice units */
                double g[2][3] = {{0, 0, 0}, {0, 0, 0}};
                for (int d = 0; d < dims; ++d) {
                    if (d == 0 && x == p->nx - 1) {
                        /* Eq. 37: grad X = -C_t^-1 [D]^-1 J = -[B] J with the imposed flux */
                        for (int s = 0; s < 2; ++s)
                            g[s][0] = -(B[s][0] * p->Q[0] + B[s][1] * p->Q[1]);
                        continue;
                    }
                    int up[3] = {x, y, z}, dn[3] = {x, y, z};
                    up[d] += 1;
                    dn[d] -= 1;
                    int fu = is_fluid(p, solid, up[0], up[1], up[2]);
                    int fd = is_fluid(p, solid, dn[0], dn[1], dn[2]);
                    for (int s = 0; s < 2; ++s) {
                        double xc = X[(long)s * N + n];
                        double xu = fu ? X[(long)s * N + node_index(p, up[0], wrap(up[1], p->ny), wrap(up[2], p->nz))] : 0.0;
                        double xd = fd ? X[(long)s * N + node_index(p, dn[0], wrap(dn[1], p->ny), wrap(dn[2], p->nz))] : 0.0;
                        if (fu && fd)
                            g[s][d] = 0.5 * (xu - xd);
                        else if (fu)
                            g[s][d] = xu - xc;   /* forward (Eq. 35 at the inlet column) */
                        else if (fd)
                            g[s][d] = xc - xd;
                        else
                            g[s][d] = 0.0;
                    }
                }

                /* step 3: J = -[B]^-1 g per axis (Cramer's rule) */
                double det = B[0][0] * B[1][1] - B[0][1] * B[1][0];
                double J[2][3] = {{0, 0, 0}, {0, 0, 0}};
                for (int d = 0; d < dims; ++d) {
                    J[0][d] = -(B[1][1] * g[0][d] - B[0][1] * g[1][d]) / det;
                    J[1][d] = -(B[0][0] * g[1][d] - B[1][0] * g[0][d]) / det;
                }
                double norm[2];
                for (int s = 0; s < 2; ++s) {
                    double ss = 0.0;
                    for (int d = 0; d < dims; ++d) ss += J[s][d] * J[s][d];
                    norm[s] = sqrt(ss);
                }

                /* steps 4-5: Eq. 24 with signed flux norms, Eq. 25 */
                double tau[2];
                for (int i = 0; i < 2; ++i) {
                    double inv_D = 0.0;
                    double si = flux_sign(p->nu[i]);
                    for (int j = 0; j < 3; ++j) {
                        if (j == i) continue;
                        double sj = flux_sign(p->nu[j]);
                        double ratio = 0.0; /* N_j / N_i */
                        if (sj != 0.0) {
                            double rho;
                            if (p->ms_mode == 1)
                                rho = fabs(p->nu[j]) / fabs(p->nu[i]);
                            else
                                rho = (norm[j] + p->eps * fabs(p->nu[j])) /
                                      (norm[i] + p->eps * fabs(p->nu[i]));
                            ratio = (sj / si) * rho;
                        }
                        inv_D += (Xn[j] - Xn[i] * ratio) / p->Dl[i][j];
                    }
                    double D = 1.0 / inv_D;
                    double t = 3.0 * D + 0.5;
                    if (!(t >= p->tau_min)) { t = p->tau_min; ++hits; }
                    else if (t > p->tau_max) { t = p->tau_max; ++hits; }
                    tau[i] = t;
                }
                if (tau_out) {
                    tau_out[n] = tau[0];
                    tau_out[N + n] = tau[1];
                }
                if (J_out)
                    for (int s = 0; s < 2; ++s)
                        for (int d = 0; d < 3; ++d) J_out[((long)s * 3 + d) * N + n] = J[s][d];

                /* step 6: BGK collision toward w_a X_s, and the source term w_a S_s (Eq. 27).
                 * TRT variant: the odd part of each link pair, (f_a - f_abar) / 2, relaxes with
                 * tau (it carries the flux, so tau keeps setting D through Eq. 25); the even part,
                 * (f_a + f_abar) / 2 - w_a X, relaxes with tau_even = 1/2 + Lambda / (tau - 1/2). */
                for (int s = 0; s < 2; ++s) {
                    const double tau_even = 0.5 + p->lambda_trt / (tau[s] - 0.5);
                    for (int a = 0; a < q; ++a) {
                        long k = ((long)s * q + a) * N + n;
                        if (p->trt) {
                            long kb = ((long)s * q + L->opp[a]) * N + n;
                            const double fe = 0.5 * (f[k] + f[kb]), fo = 0.5 * (f[k] - f[kb]);
                            fstar[k] = f[k] - (fe - L->w[a] * Xn[s]) / tau_even - fo / tau[s];
                        } else {
                            fstar[k] = f[k] - (f[k] - L->w[a] * Xn[s]) / tau[s];
                        }
                        if (x >= p->src_x0) fstar[k] += L->w[a] * p->S[s];
                    }
                }
            }
    free(X);
    if (clamp_hits) *clamp_hits = hits;
    return 0;
}

/* Steps 1-6 only (post-collision populations of the current state). */
int orc_collide(const orc_params* p, const uint8_t* solid, const double* f, double* fstar,
                double* tau_out, double* J_out, orc_stats* st)
{
    orc_lattice L;
    build_lattice(p->lattice, &L);
    long hits = 0;
    int rc = collide_all(p, &L, solid, f, fstar, tau_out, J_out, &hits);
    if (st) {
        memset(st, 0, sizeof(*st));
        st->clamp_hits = hits;
    }
    return rc;
}

/* Steps 7-8: stream fstar into fnext with bounce-back and the two x boundaries. */
static void stream_all(const orc_params* p, const orc_lattice* L, const uint8_t* solid,
                       const double* fstar, double* fnext, orc_stats* st)
{
    const long N = (long)p->nx * p->ny * p->nz;
    const int q = L->q;
    double inflow[2] = {0, 0}, outflow[2] = {0, 0};

    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const long n = node_index(p, x, y, z);
                if (solid[n]) {
                    for (int s = 0; s < 2; ++s)
                        for (int a = 0; a < q; ++a) fnext[((long)s * q + a) * N + n] = 0.0;
                    continue;
                }
                int kind[ORC_QMAX]; /* 0 streamed or bounced, 1 inlet link, 2 outlet link */
                for (int a = 0; a < q; ++a) {
                    int sx = x - L->e[a][0];
                    int sy = wrap(y - L->e[a][1], p->ny);
                    int sz = wrap(z - L->e[a][2], p->nz);
                    kind[a] = 0;
                    if (sx < 0) { kind[a] = 1; continue; }
                    if (sx >= p->nx) { kind[a] = 2; continue; }
                    long src = node_index(p, sx, sy, sz);
                    for (int s = 0; s < 2; ++s) {
                        if (solid[src])
                            fnext[((long)s * q + a) * N + n] = fstar[((long)s * q + L->opp[a]) * N + n];
                        else
                            fnext[((long)s * q + a) * N + n] = fstar[((long)s * q + a) * N + src];
                    }
                }
                for (int a = 0; a < q; ++a) {
                    int b = L->opp[a];
                    for (int s = 0; s < 2; ++s) {
                        double* dst = &fnext[((long)s * q + a) * N + n];
                        double out_pop = fstar[((long)s * q + b) * N + n]; /* leaves through the face */
                        if (kind[a] == 1) {
                            if (p->inlet_wall)
                                *dst = out_pop;
                            else
                                *dst = (L->w[a] + L->w[b]) * p->X_in[s] - fnext[((long)s * q + b) * N + n];
                            inflow[s] += *dst - out_pop;
                        } else if (kind[a] == 2) {
                            *dst = out_pop - (L->w[b] / L->Wn) * p->Q[s];
                            outflow[s] += out_pop - *dst;
                        }
                    }
                }
            }
    if (st) {
        for (int s = 0; s < 2; ++s) {
            st->inflow[s] = inflow[s];
            st->outflow[s] = outflow[s];
        }
    }
}

/* One full step f -> fnext.  Returns 0, or -8 when memory runs out. */
int orc_step(const orc_params* p, const uint8_t* solid, const double* f, double* fnext,
             orc_stats* st)
{
    orc_lattice L;
    build_lattice(p->lattice, &L);
    const long N = (long)p->nx * p->ny * p->nz;
    double* fstar = (double*)malloc(sizeof(double) * 2 * L.q * N);
    if (!fstar) return -8;
    long hits = 0;
    int rc = collide_all(p, &L, solid, f, fstar, NULL, NULL, &hits);
    if (rc == 0) {
        orc_stats tmp;
        memset(&tmp, 0, sizeof(tmp));
        stream_all(p, &L, solid, fstar, fnext, &tmp);
        tmp.clamp_hits = hits;
        if (st) *st = tmp;
    }
    free(fstar);
    return rc;
}

/* nsteps steps in place on f (work must hold as many doubles as f).  Stats of the last step. */
int orc_run(const orc_params* p, const uint8_t* solid, double* f, double* work, long nsteps,
            orc_stats* st)
{
    orc_lattice L;
    build_lattice(p->lattice, &L);
    const long total = 2L * L.q * p->nx * p->ny * p->nz;
    long hits = 0;
    for (long t = 0; t < nsteps; ++t) {
        orc_stats s1;
        int rc = orc_step(p, solid, f, work, &s1);
        if (rc) return rc;
        memcpy(f, work, sizeof(double) * total);
        hits += s1.clamp_hits;
        if (st) *st = s1;
    }
    if (st) st->clamp_hits = hits;
    return 0;
}

/* Equilibrium initial state f_a = w_a X0_s for fluid nodes (X0 holds [3][N] or [2][N]). */
void orc_equilibrium(const orc_params* p, const uint8_t* solid, const double* X0, double* f)
{
    orc_lattice L;
    build_lattice(p->lattice, &L);
    const long N = (long)p->nx * p->ny * p->nz;
    for (int s = 0; s < 2; ++s)
        for (int a = 0; a < L.q; ++a)
            for (long n = 0; n < N; ++n)
                f[((long)s * L.q + a) * N + n] = solid[n] ? 0.0 : L.w[a] * X0[(long)s * N + n];
}

/*
 * Pore-space clean-up: fluid nodes that no chain of lattice links (periodic in y and z, not in
 * x) connects to a fluid node of the inlet column become solid.  Returns the number of fluid
 * nodes left in the outlet column (0 means the outlet cannot be reached).
 */
long orc_label(int lattice, int nx, int ny, int nz, const uint8_t* solid_in, uint8_t* solid_out)
{
    orc_lattice L;
    build_lattice(lattice, &L);
    const long N = (long)nx * ny * nz;
    uint8_t* seen = (uint8_t*)calloc(N, 1);
    long* queue = (long*)malloc(sizeof(long) * N);
    if (!seen || !queue) {
        free(seen);
        free(queue);
        return -8;
    }
    long head = 0, tail = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
            long n = ((long)z * ny + y) * nx;
            if (!solid_in[n]) {
                seen[n] = 1;
                queue[tail++] = n;
            }
        }
    while (head < tail) {
        long n = queue[head++];
        int x = (int)(n % nx);
        int y = (int)((n / nx) % ny);
        int z = (int)(n / ((long)nx * ny));
        for (int a = 1; a < L.q; ++a) {
            int xx = x + L.e[a][0];
            if (xx < 0 || xx >= nx) continue;
            int yy = wrap(y + L.e[a][1], ny);
            int zz = wrap(z + L.e[a][2], nz);
            long m = ((long)zz * ny + yy) * nx + xx;
            if (!solid_in[m] && !seen[m]) {
                seen[m] = 1;
                queue[tail++] = m;
            }
        }
    }
    long outlet = 0;
    for (long n = 0; n < N; ++n) {
        solid_out[n] = seen[n] ? 0 : 1;
        if (seen[n] && (n % nx) == nx - 1) ++outlet;
    }
    free(seen);
    free(queue);
    return outlet;
}

/*
 * ---------------------------------------------------------------------------------------------
 * Advective coupling (Sec. 3.1, Eq. 20-21 and 26): when the electrode reaction changes the number
 * of moles (nu_1 + nu_2 != 0), the total flux N_t = C_t u_M no longer vanishes and the species
 * equilibrium carries the molar-averaged velocity, f_eq = w_a X_s (1 + e_a . u_M / c_s^2) (Eq. 26
 * divided by the constant C_t).  u_M comes from a second lattice Boltzmann model, an
 * incompressible one whose density is the total concentration (Sec. 3.1, last paragraphs); here
 * its Stokes limit, g_eq = w_a (rho + e_a . u / c_s^2) with rho = C_t / C_t,ref = 1 + O(Ma^2),
 * u = sum_a e_a g_a, BGK with relaxation time tau_flow.  Its boundaries mirror the species ones:
 * no-slip half-way bounce-back on solid, the inlet (channel) at rho = 1 by the anti-bounce-back
 * rule, and at each open outlet node the net outflow Q_t = Q_1 + Q_2 (the electrode's total
 * molar flux in lattice units) by the same exact-flux rule.  This linear model carries an
 * undamped period-2 mode: populations at their equilibrium (so no collision acts on them) whose
 * node velocity alternates between neighbouring nodes and between consecutive steps while every
 * link flux stays uniform.  The species therefore see the mean of the node velocity over the last
 * two steps, u_M = (u^t + u^{t-1}) / 2, which removes that mode exactly and equals u at a steady
 * state.
 *
 * With advection the species populations carry N_s = X_s N_t + J_s, so the relaxation time must
 * reproduce the diffusive flux J_s = N_s - X_s N_t (Eq. 20) alone: Eq. 24 is read with J in place
 * of N (Eq. 19 holds with either), and the inert species now has J_3 = -J_1 - J_2 != 0.  The
 * flux ratio J_j / J_i of two vectors is read as the projection (J_j . J_i) / |J_i|^2, which is
 * the signed-norm rule of Eq. 24 for collinear fluxes; the regularization pulls it towards the
 * one-dimensional steady ratio (Nh_j - X_j Nh_t) / (Nh_i - X_i Nh_t), Nh_s = -nu_s, which is also
 * the stoichiometric variant.  At the outlet column Eq. 37's gradient uses the diffusive boundary
 * flux J_s = Q_s - X_s Q_t.  With nu_1 + nu_2 = 0 every step reduces to the equimolar method.
 * ---------------------------------------------------------------------------------------------
 */

/* the one-dimensional steady ratio J_j / J_i of diffusive fluxes for stoichiometric N */
static double stoich_ratio_adv(const orc_params* p, const double X[3], int i, int j)
{
    const double nt = -(p->nu[0] + p->nu[1] + p->nu[2]);
    return (-p->nu[j] - X[j] * nt) / (-p->nu[i] - X[i] * nt);
}

static int collide_adv(const orc_params* p, const orc_lattice* L, const uint8_t* solid,
                       const double* f, const double* g, const double* uprev, double* fstar,
                       double* gstar, double* ucur, double* tau_out, double* u_out,
                       long* clamp_hits)
{
    const long N = (long)p->nx * p->ny * p->nz;
    const int q = L->q;
    const int dims = (p->lattice == 1 || p->lattice == 3) ? 3 : 2;
    const double Qt = p->Q[0] + p->Q[1];
    double* X = (double*)malloc(sizeof(double) * 3 * N);
    if (!X) return -8;
    orc_moments(p, solid, f, X);
    long hits = 0;
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const long n = node_index(p, x, y, z);
                if (solid[n]) {
                    for (int a = 0; a < q; ++a) {
                        fstar[(long)a * N + n] = fstar[((long)q + a) * N + n] = 0.0;
                        gstar[(long)a * N + n] = 0.0;
                    }
                    for (int d = 0; d < 3; ++d) {
                        if (ucur) ucur[(long)d * N + n] = 0.0;
                        if (u_out) u_out[(long)d * N + n] = 0.0;
                    }
                    continue;
                }
                /* velocity model moments */
                double rho = 0.0, u[3] = {0.0, 0.0, 0.0};
                for (int a = 0; a < q; ++a) {
                    const double ga = g[(long)a * N + n];
                    rho += ga;
                    for (int d = 0; d < 3; ++d) u[d] += L->e[a][d] * ga;
                }
                /* the species see the two-step mean (removes the period-2 mode) */
                double um[3];
                for (int d = 0; d < 3; ++d) {
                    if (ucur) ucur[(long)d * N + n] = u[d];
                    um[d] = 0.5 * (u[d] + uprev[(long)d * N + n]);
                    if (u_out) u_out[(long)d * N + n] = um[d];
                }
                double Xn[3] = {X[n], X[N + n], X[2 * N + n]};
                double B[2][2];
                ms_matrix(p, Xn, B);
                /* gradients, as in the equimolar method except Eq. 37's diffusive boundary flux */
                double gr[2][3] = {{0, 0, 0}, {0, 0, 0}};
                for (int d = 0; d < dims; ++d) {
                    if (d == 0 && x == p->nx - 1) {
                        const double J0 = p->Q[0] - Xn[0] * Qt, J1 = p->Q[1] - Xn[1] * Qt;
                        for (int s = 0; s < 2; ++s) gr[s][0] = -(B[s][0] * J0 + B[s][1] * J1);
                        continue;
                    }
                    int up[3] = {x, y, z}, dn[3] = {x, y, z};
                    up[d] += 1;
                    dn[d] -= 1;
                    int fu = is_fluid(p, solid, up[0], up[1], up[2]);
                    int fd = is_fluid(p, solid, dn[0], dn[1], dn[2]);
                    for (int s = 0; s < 2; ++s) {
                        double xc = X[(long)s * N + n];
                        double xu = fu ? X[(long)s * N + node_index(p, up[0], wrap(up[1], p->ny), wrap(up[2], p->nz))] : 0.0;
                        double xd = fd ? X[(long)s * N + node_index(p, dn[0], wrap(dn[1], p->ny), wrap(dn[2], p->nz))] : 0.0;
                        if (fu && fd) gr[s][d] = 0.5 * (xu - xd);
                        else if (fu) gr[s][d] = xu - xc;
                        else if (fd) gr[s][d] = xc - xd;
                        else gr[s][d] = 0.0;
                    }
                }
                /* diffusive fluxes: generalized Fick (Eq. 34), J_3 by the zero sum of Eq. 20 */
                double det = B[0][0] * B[1][1] - B[0][1] * B[1][0];
                double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
                for (int d = 0; d < dims; ++d) {
                    J[0][d] = -(B[1][1] * gr[0][d] - B[0][1] * gr[1][d]) / det;
                    J[1][d] = -(B[0][0] * gr[1][d] - B[1][0] * gr[0][d]) / det;
                    J[2][d] = -J[0][d] - J[1][d];
                }
                double tau[2];
                for (int i = 0; i < 2; ++i) {
                    double inv_D = 0.0;
                    for (int j = 0; j < 3; ++j) {
                        if (j == i) continue;
                        double rho_ji = stoich_ratio_adv(p, Xn, i, j);
                        if (p->ms_mode != 1) {
                            double dot = 0.0, nn = 0.0;
                            for (int d = 0; d < dims; ++d) {
                                dot += J[j][d] * J[i][d];
                                nn += J[i][d] * J[i][d];
                            }
                            const double e2 = p->eps * p->eps;
                            rho_ji = (dot + e2 * rho_ji) / (nn + e2);
                        }
                        inv_D += (Xn[j] - Xn[i] * rho_ji) / p->Dl[i][j];
                    }
                    double t = 3.0 / inv_D + 0.5;
                    if (!(t >= p->tau_min)) { t = p->tau_min; ++hits; }
                    else if (t > p->tau_max) { t = p->tau_max; ++hits; }
                    tau[i] = t;
                }
                if (tau_out) {
                    tau_out[n] = tau[0];
                    tau_out[N + n] = tau[1];
                }
                /* BGK toward Eq. 26, and the velocity model toward its Stokes equilibrium */
                for (int a = 0; a < q; ++a) {
                    const double eu = L->e[a][0] * u[0] + L->e[a][1] * u[1] + L->e[a][2] * u[2];
                    const double em = L->e[a][0] * um[0] + L->e[a][1] * um[1] + L->e[a][2] * um[2];
                    for (int s = 0; s < 2; ++s) {
                        const long k = ((long)s * q + a) * N + n;
                        const double feq = L->w[a] * Xn[s] * (1.0 + 3.0 * em);
                        fstar[k] = f[k] - (f[k] - feq) / tau[s];
                    }
                    const long k = (long)a * N + n;
                    const double geq = L->w[a] * (rho + 3.0 * eu);
                    gstar[k] = g[k] - (g[k] - geq) / p->tau_flow;
                }
            }
    free(X);
    if (clamp_hits) *clamp_hits = hits;
    return 0;
}

/* Streaming of the velocity model: the species rules with rho_in = 1 at the inlet and the total
 * outflow Q_t per open outlet node. */
static void stream_flow(const orc_params* p, const orc_lattice* L, const uint8_t* solid,
                        const double* gstar, double* gnext)
{
    const long N = (long)p->nx * p->ny * p->nz;
    const int q = L->q;
    const double Qt = p->Q[0] + p->Q[1];
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const long n = node_index(p, x, y, z);
                if (solid[n]) {
                    for (int a = 0; a < q; ++a) gnext[(long)a * N + n] = 0.0;
                    continue;
                }
                int kind[ORC_QMAX];
                for (int a = 0; a < q; ++a) {
                    int sx = x - L->e[a][0];
                    int sy = wrap(y - L->e[a][1], p->ny);
                    int sz = wrap(z - L->e[a][2], p->nz);
                    kind[a] = 0;
                    if (sx < 0) { kind[a] = 1; continue; }
                    if (sx >= p->nx) { kind[a] = 2; continue; }
                    long src = node_index(p, sx, sy, sz);
                    gnext[(long)a * N + n] = solid[src] ? gstar[(long)L->opp[a] * N + n]
                                                        : gstar[(long)a * N + src];
                }
                for (int a = 0; a < q; ++a) {
                    int b = L->opp[a];
                    if (kind[a] == 1)
                        gnext[(long)a * N + n] = (L->w[a] + L->w[b]) * 1.0 - gnext[(long)b * N + n];
                    else if (kind[a] == 2)
                        gnext[(long)a * N + n] = gstar[(long)b * N + n] - (L->w[b] / L->Wn) * Qt;
                }
            }
}

/* One step of the coupled pair: (f, g, u^{t-1}) -> (fnext, gnext, u^t). */
int orc_step_adv(const orc_params* p, const uint8_t* solid, const double* f, const double* g,
                 const double* uprev, double* fnext, double* gnext, double* ucur, orc_stats* st)
{
    orc_lattice L;
    build_lattice(p->lattice, &L);
    const long N = (long)p->nx * p->ny * p->nz;
    double* fstar = (double*)malloc(sizeof(double) * 2 * L.q * N);
    double* gstar = (double*)malloc(sizeof(double) * L.q * N);
    if (!fstar || !gstar) {
        free(fstar);
        free(gstar);
        return -8;
    }
    long hits = 0;
    int rc = collide_adv(p, &L, solid, f, g, uprev, fstar, gstar, ucur, NULL, NULL, &hits);
    if (rc == 0) {
        orc_stats tmp;
        memset(&tmp, 0, sizeof(tmp));
        stream_all(p, &L, solid, fstar, fnext, &tmp);
        stream_flow(p, &L, solid, gstar, gnext);
        tmp.clamp_hits = hits;
        if (st) *st = tmp;
    }
    free(fstar);
    free(gstar);
    return rc;
}

/* nsteps coupled steps in place on (f, g, uprev) (fwork, gwork: scratch of the sizes of f, g). */
int orc_run_adv(const orc_params* p, const uint8_t* solid, double* f, double* g, double* uprev,
                double* fwork, double* gwork, long nsteps, orc_stats* st)
{
    orc_lattice L;
    build_lattice(p->lattice, &L);
    const long N = (long)p->nx * p->ny * p->nz;
    double* ucur = (double*)malloc(sizeof(double) * 3 * N);
    if (!ucur) return -8;
    long hits = 0;
    for (long t = 0; t < nsteps; ++t) {
        orc_stats s1;
        int rc = orc_step_adv(p, solid, f, g, uprev, fwork, gwork, ucur, &s1);
        if (rc) {
            free(ucur);
            return rc;
        }
        memcpy(f, fwork, sizeof(double) * 2 * L.q * N);
        memcpy(g, gwork, sizeof(double) * L.q * N);
        memcpy(uprev, ucur, sizeof(double) * 3 * N);
        hits += s1.clamp_hits;
        if (st) *st = s1;
    }
    free(ucur);
    if (st) st->clamp_hits = hits;
    return 0;
}

/* Post-collision state and diagnostics of the coupled pair: fstar, gstar, tau [2][N], and the
 * velocity the species see, u_M [3][N]. */
int orc_collide_adv(const orc_params* p, const uint8_t* solid, const double* f, const double* g,
                    const double* uprev, double* fstar, double* gstar, double* tau_out,
                    double* u_out, orc_stats* st)
{
    orc_lattice L;
    build_lattice(p->lattice, &L);
    long hits = 0;
    int rc = collide_adv(p, &L, solid, f, g, uprev, fstar, gstar, NULL, tau_out, u_out, &hits);
    if (st) {
        memset(st, 0, sizeof(*st));
        st->clamp_hits = hits;
    }
    return rc;
}

/* Velocity model at rest, g_a = w_a (rho = 1, u = 0), on fluid nodes. */
void orc_flow_rest(const orc_params* p, const uint8_t* solid, double* g)
{
    orc_lattice L;
    build_lattice(p->lattice, &L);
    const long N = (long)p->nx * p->ny * p->nz;
    for (int a = 0; a < L.q; ++a)
        for (long n = 0; n < N; ++n) g[(long)a * N + n] = solid[n] ? 0.0 : L.w[a];
}

