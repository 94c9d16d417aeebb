/*
 * FP64 CPU oracle for the Wilson / domain-wall hopping operator -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, obviously-correct reference the HIP kernels are checked against.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product library never calls into it and shares no code with it.
 *
 * Everything is evaluated from its definition: full 4x4 Dirac matrices, full 3x3 link matrices,
 * no spin projection, no link compression, no Ls batching. OpenMP parallelises over sites only.
 *
 * The paper (Grid, Section 4) names the Wilson fermion action, five-dimensional chiral fermions,
 * periodic boundary conditions and the conjugate gradient; it prints none of their formulas.
 * The readings used here are the standard ones:
 *
 *   Geometry   site i = x0 + L0 (x1 + L1 (x2 + L2 x3)), periodic in all four directions,
 *              mu = 0..3 is x, y, z, t (Section 2.3's Cshift semantics: x + mu-hat wraps).
 *   Gammas     Euclidean chiral basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = 1, 2, 3),
 *              gamma_4 = [[0, 1], [1, 0]]; direction mu uses gamma_{mu+1}; gamma_5 = g1 g2 g3 g4.
 *   Hopping    (H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x + mu)
 *                                 + (1 + gamma_mu) U_mu(x - mu)^dagger psi(x - mu);
 *              H^dagger is the same sum with the signs of gamma_mu flipped.
 *   Wilson     D = (4 + m) - H / 2,   D^dagger = (4 + m) - H^dagger / 2.
 *   DWF        (M psi)_s = (5 - M5) psi_s - H psi_s / 2 - P_- psi~_{s+1} - P_+ psi~_{s-1},
 *              P_+- = (1 +- gamma_5) / 2, walls psi~_{Ls} = -mf psi_0, psi~_{-1} = -mf psi_{Ls-1};
 *              M^dagger swaps P_+ and P_- and uses H^dagger.
 *   CG         Hestenes-Stiefel on A = Op^dagger Op, stopping on the true residual.
 *   Link grad  for L = Re <chi, c H psi>:
 *              dL/dU_mu(x) = c sum_spin { [(1 - gamma_mu) chi(x)] psi(x + mu)^dagger
 *                                        + psi(x) [(1 + gamma_mu) chi(x + mu)]^dagger }
 *              (complex gradient dL/dRe + i dL/dIm), summed over the fifth coordinate for 5D.
 *   Force      F = TA(G U^dagger), TA(M) = (M - M^dagger)/2 - tr(M - M^dagger)/6.
 *
 * Layouts (C order, complex = two interleaved doubles):
 *   U   [site][mu][a][b]          psi [site][s][spin][colour]  (s absent or Ls = 1 in 4D)
 *   G   [site][mu][a][b]
 */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef double complex cplx;

/* Dirac matrices gamma_{mu+1} (index 0..3) and gamma_5, built from the Pauli matrices. */
static cplx GAM[5][4][4];

static void build_gammas(void)
{
    cplx sigma[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(GAM, 0, sizeof(GAM));
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                GAM[k][a][2 + b] = -I * sigma[k][a][b];
                GAM[k][2 + a][b] = I * sigma[k][a][b];
            }
    for (int a = 0; a < 2; ++a) {
        GAM[3][a][2 + a] = 1;
        GAM[3][2 + a][a] = 1;
    }
    /* gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 by plain matrix products. */
    cplx t1[4][4], t2[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += GAM[0][i][k] * GAM[1][k][j];
            t1[i][j] = s;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += t1[i][k] * GAM[2][k][j];
            t2[i][j] = s;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += t2[i][k] * GAM[3][k][j];
            GAM[4][i][j] = s;
        }
}

/* Copy out a Dirac matrix: which = 0..3 gamma_{mu+1}, 4 gamma_5 (for the pin tests). */
void oracle_gamma(int which, double *out32)
{
    build_gammas();
    memcpy(out32, GAM[which], sizeof(GAM[which]));
}

int oracle_threads(void) { return omp_get_max_threads(); }

static long volume(const int *dims) { return (long)dims[0] * dims[1] * dims[2] * dims[3]; }

/* Periodic neighbour x + dir * mu-hat of site i. */
static long neighbour(const int *dims, long i, int mu, int dir)
{
    int x[4];
    long r = i;
    for (int d = 0; d < 4; ++d) {
        x[d] = (int)(r % dims[d]);
        r /= dims[d];
    }
    x[mu] = (x[mu] + dir + dims[mu]) % dims[mu];
    return x[0] + (long)dims[0] * (x[1] + (long)dims[1] * (x[2] + (long)dims[2] * x[3]));
}

/* out[s][a] += sum_t P[s][t] v[t][a] with P = 1 + sign * gamma. */
static void add_proj(cplx out[4][3], int mu, double sign, cplx v[4][3])
{
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx acc = 0;
            for (int t = 0; t < 4; ++t) {
                cplx p = (s == t ? 1.0 : 0.0) + sign * GAM[mu][s][t];
                acc += p * v[t][a];
            }
            out[s][a] += acc;
        }
}

/* (H psi)(x, s5) (dag = 0) or (H^dagger psi)(x, s5) (dag = 1) at one site, into acc. */
static void hop_site(const cplx *U, const cplx *psi, const int *dims, int Ls, int dag, long x, int s5,
                     cplx acc[4][3])
{
    const double sg = dag ? -1.0 : 1.0;
    memset(acc, 0, sizeof(cplx) * 12);
    for (int mu = 0; mu < 4; ++mu) {
        const long xp = neighbour(dims, x, mu, +1);
        const long xm = neighbour(dims, x, mu, -1);
        const cplx *uf = U + (x * 4 + mu) * 9;    /* U_mu(x)      */
        const cplx *ub = U + (xm * 4 + mu) * 9;   /* U_mu(x - mu) */
        const cplx *pf = psi + (xp * Ls + s5) * 12;
        const cplx *pb = psi + (xm * Ls + s5) * 12;
        cplx v[4][3], w[4][3];
        for (int t = 0; t < 4; ++t)
            for (int a = 0; a < 3; ++a) {
                cplx f = 0, b = 0;
                for (int c = 0; c < 3; ++c) {
                    f += uf[a * 3 + c] * pf[t * 3 + c];
                    b += conj(ub[c * 3 + a]) * pb[t * 3 + c];
                }
                v[t][a] = f;
                w[t][a] = b;
            }
        add_proj(acc, mu, -sg, v);   /* (1 - gamma) forward  (H), (1 + gamma) for H^dag */
        add_proj(acc, mu, +sg, w);   /* (1 + gamma) backward (H), (1 - gamma) for H^dag */
    }
}

/* Domain-wall (M psi)(x, s5) or (M^dagger psi)(x, s5) at one site, into o. */
static void dwf_site(const cplx *U, const cplx *psi, const int *dims, int Ls, double M5, double mf, int dag,
                     long x, int s5, cplx o[4][3])
{
    /* Chiral projectors from gamma_5; P_- is applied to s+1 and P_+ to s-1 (swapped for M^dag). */
    cplx Pp[4][4], Pm[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx d = (i == j) ? 1.0 : 0.0;
            Pp[i][j] = 0.5 * (d + GAM[4][i][j]);
            Pm[i][j] = 0.5 * (d - GAM[4][i][j]);
        }
    cplx (*Pup)[4] = dag ? Pp : Pm;
    cplx (*Pdn)[4] = dag ? Pm : Pp;
    cplx h[4][3];
    hop_site(U, psi, dims, Ls, dag, x, s5, h);
    const cplx *p = psi + (x * Ls + s5) * 12;
    const int sp = (s5 + 1) % Ls, sm = (s5 - 1 + Ls) % Ls;
    const double fp = (s5 == Ls - 1) ? -mf : 1.0;   /* psi~_{s+1} wall factor */
    const double fm = (s5 == 0) ? -mf : 1.0;        /* psi~_{s-1} wall factor */
    const cplx *pu = psi + (x * Ls + sp) * 12;
    const cplx *pd = psi + (x * Ls + sm) * 12;
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx acc = (5.0 - M5) * p[s * 3 + a] - 0.5 * h[s][a];
            for (int t = 0; t < 4; ++t) {
                acc -= Pup[s][t] * fp * pu[t * 3 + a];
                acc -= Pdn[s][t] * fm * pd[t * 3 + a];
            }
            o[s][a] = acc;
        }
}

/*
 * out = H psi (dag = 0) or H^dagger psi (dag = 1) on every fifth-dimension slice; Ls = 1 for 4D.
 * The same link field is used on every slice.
 */
void oracle_hop(const cplx *U, const cplx *psi, cplx *out, const int *dims, int Ls, int dag)
{
    build_gammas();
    const long V = volume(dims);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x)
        for (int s5 = 0; s5 < Ls; ++s5)
            hop_site(U, psi, dims, Ls, dag, x, s5, (cplx(*)[3])(out + (x * Ls + s5) * 12));
}

/* out = D psi or D^dagger psi, D = (4 + m) - H / 2 (4D, Ls = 1). */
void oracle_wilson(const cplx *U, const cplx *psi, cplx *out, const int *dims, double mass, int dag)
{
    const long n = volume(dims) * 12;
    oracle_hop(U, psi, out, dims, 1, dag);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) out[k] = (4.0 + mass) * psi[k] - 0.5 * out[k];
}

/* out = M psi or M^dagger psi for the Shamir domain-wall operator. */
void oracle_dwf(const cplx *U, const cplx *psi, cplx *out, const int *dims, int Ls, double M5,
                double mf, int dag)
{
    build_gammas();
    const long V = volume(dims);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x)
        for (int s5 = 0; s5 < Ls; ++s5)
            dwf_site(U, psi, dims, Ls, M5, mf, dag, x, s5, (cplx(*)[3])(out + (x * Ls + s5) * 12));
}

/*
 * Sampled evaluation for lattices too large to check whole: out[k] (12 complex) is the operator
 * at site idx[k] (a 5D index x * Ls + s). kind 0: H, 1: D = (4 + mass) - H/2 (Ls = 1), 2: M.
 */
void oracle_sites(const cplx *U, const cplx *psi, cplx *out, const int *dims, int Ls, int kind, double mass,
                  double M5, double mf, int dag, const long *idx, long n)
{
    build_gammas();
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) {
        const long x = idx[k] / Ls;
        const int s5 = (int)(idx[k] % Ls);
        cplx (*o)[3] = (cplx(*)[3])(out + k * 12);
        if (kind == 2) {
            dwf_site(U, psi, dims, Ls, M5, mf, dag, x, s5, o);
        } else {
            hop_site(U, psi, dims, Ls, dag, x, s5, o);
            if (kind == 1) {
                const cplx *p = psi + idx[k] * 12;
                for (int j = 0; j < 12; ++j) o[j / 3][j % 3] = (4.0 + mass) * p[j] - 0.5 * o[j / 3][j % 3];
            }
        }
    }
}

/* Operator selection for the normal-equation helpers and the CG. */
typedef struct {
    int kind;        /* 0: Wilson D (Ls must be 1), 1: domain-wall M */
    int Ls;
    double mass;     /* Wilson mass m */
    double M5, mf;   /* domain-wall height and quark mass */
} oracle_op;

static void apply_op(const oracle_op *op, const cplx *U, const cplx *in, cplx *out, const int *dims,
                     int dag)
{
    if (op->kind == 0)
        oracle_wilson(U, in, out, dims, op->mass, dag);
    else
        oracle_dwf(U, in, out, dims, op->Ls, op->M5, op->mf, dag);
}

/* out = Op^dagger Op in; tmp has the size of in. */
void oracle_normal(const cplx *U, const cplx *in, cplx *out, cplx *tmp, const int *dims,
                   const oracle_op *op)
{
    apply_op(op, U, in, tmp, dims, 0);
    apply_op(op, U, tmp, out, dims, 1);
}

/* Deterministic FP64 reductions: fixed chunking, partial sums added in order. */
#define NCHUNK 256
static double norm2(const cplx *a, long n)
{
    double part[NCHUNK];
#pragma omp parallel for schedule(static)
    for (int c = 0; c < NCHUNK; ++c) {
        long lo = n * c / NCHUNK, hi = n * (c + 1) / NCHUNK;
        double s = 0;
        for (long k = lo; k < hi; ++k) s += creal(a[k]) * creal(a[k]) + cimag(a[k]) * cimag(a[k]);
        part[c] = s;
    }
    double s = 0;
    for (int c = 0; c < NCHUNK; ++c) s += part[c];
    return s;
}

static double redot(const cplx *a, const cplx *b, long n)
{
    double part[NCHUNK];
#pragma omp parallel for schedule(static)
    for (int c = 0; c < NCHUNK; ++c) {
        long lo = n * c / NCHUNK, hi = n * (c + 1) / NCHUNK;
        double s = 0;
        for (long k = lo; k < hi; ++k) s += creal(conj(a[k]) * b[k]);
        part[c] = s;
    }
    double s = 0;
    for (int c = 0; c < NCHUNK; ++c) s += part[c];
    return s;
}

/*
 * Conjugate gradient (Hestenes-Stiefel) on A = Op^dagger Op, A x = b.
 * x holds the initial guess on entry and the solution on exit. The iterated residual decides
 * when to look; the stop is on the true relative residual |b - A x| / |b| <= tol, recomputed.
 * stats[0] = iterations, stats[1] = true relative residual. Returns 0 on convergence, 1 if
 * maxiter was reached, 2 on breakdown (<p, A p> <= 0 or non-finite).
 */
int oracle_cg(const cplx *U, const cplx *b, cplx *x, const int *dims, const oracle_op *op,
              double tol, int maxiter, double *stats)
{
    const long n = volume(dims) * (op->kind == 0 ? 1 : op->Ls) * 12;
    cplx *r = malloc(n * sizeof(cplx)), *p = malloc(n * sizeof(cplx));
    cplx *q = malloc(n * sizeof(cplx)), *t = malloc(n * sizeof(cplx));
    const double bnorm = sqrt(norm2(b, n));
    int status = 1, it = 0;
    double relres = 0;

    oracle_normal(U, x, q, t, dims, op);
    for (long k = 0; k < n; ++k) { r[k] = b[k] - q[k]; p[k] = r[k]; }
    double rho = norm2(r, n);
    if (bnorm == 0.0 || sqrt(rho) <= tol * bnorm) { status = 0; relres = bnorm > 0 ? sqrt(rho) / bnorm : 0; }

    /* progress on stderr every ORACLE_CG_PROGRESS iterations (long solves); no effect on the result */
    const char *pe = getenv("ORACLE_CG_PROGRESS");
    const int every = pe ? atoi(pe) : 0;
    for (it = 1; status == 1 && it <= maxiter; ++it) {
        if (every > 0 && it % every == 0) {
            fprintf(stderr, "oracle cg: iteration %d, |r|/|b| = %.3e\n", it, sqrt(rho) / bnorm);
            fflush(stderr);
        }
        oracle_normal(U, p, q, t, dims, op);
        const double pq = redot(p, q, n);
        if (!(pq > 0.0) || !isfinite(pq)) { status = 2; break; }
        const double alpha = rho / pq;
        for (long k = 0; k < n; ++k) { x[k] += alpha * p[k]; r[k] -= alpha * q[k]; }
        const double rho_new = norm2(r, n);
        if (!isfinite(rho_new)) { status = 2; break; }
        if (sqrt(rho_new) <= tol * bnorm) {
            oracle_normal(U, x, q, t, dims, op);
            for (long k = 0; k < n; ++k) t[k] = b[k] - q[k];
            relres = sqrt(norm2(t, n)) / bnorm;
            if (relres <= tol) { status = 0; break; }
        }
        const double beta = rho_new / rho;
        for (long k = 0; k < n; ++k) p[k] = r[k] + beta * p[k];
        rho = rho_new;
    }
    if (status != 0) {
        oracle_normal(U, x, q, t, dims, op);
        for (long k = 0; k < n; ++k) t[k] = b[k] - q[k];
        relres = sqrt(norm2(t, n)) / bnorm;
    }
    stats[0] = (double)(it > maxiter ? maxiter : it);
    stats[1] = relres;
    free(r); free(p); free(q); free(t);
    return status;
}

/*
 * Link gradient of L = Re <chi, c H psi> (dag = 0) or Re <chi, c H^dagger psi> (dag = 1):
 *   G_mu(x) = c sum_{s5, spin} { [(1 - sg gamma_mu) chi(x)] psi(x + mu)^dagger
 *                               + psi(x) [(1 + sg gamma_mu) chi(x + mu)]^dagger },  sg = +-1.
 * The gradient does not depend on U (L is linear in each link).
 */
void oracle_link_grad(const cplx *chi, const cplx *psi, cplx *G, const int *dims, int Ls, double c,
                      int dag)
{
    build_gammas();
    const long V = volume(dims);
    const double sg = dag ? -1.0 : 1.0;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        for (int mu = 0; mu < 4; ++mu) {
            const long xp = neighbour(dims, x, mu, +1);
            cplx g[3][3];
            memset(g, 0, sizeof(g));
            for (int s5 = 0; s5 < Ls; ++s5) {
                const cplx *chx = chi + (x * Ls + s5) * 12, *chp = chi + (xp * Ls + s5) * 12;
                const cplx *psx = psi + (x * Ls + s5) * 12, *psp = psi + (xp * Ls + s5) * 12;
                for (int s = 0; s < 4; ++s) {
                    cplx f[3], h[3];
                    for (int a = 0; a < 3; ++a) {
                        cplx fs = 0, hs = 0;
                        for (int t = 0; t < 4; ++t) {
                            const cplx d = (s == t) ? 1.0 : 0.0;
                            fs += (d - sg * GAM[mu][s][t]) * chx[t * 3 + a];
                            hs += (d + sg * GAM[mu][s][t]) * chp[t * 3 + a];
                        }
                        f[a] = fs;
                        h[a] = hs;
                    }
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b)
                            g[a][b] += f[a] * conj(psp[s * 3 + b]) + psx[s * 3 + a] * conj(h[b]);
                }
            }
            cplx *o = G + (x * 4 + mu) * 9;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) o[a * 3 + b] = c * g[a][b];
        }
    }
}

/* F = TA(G U^dagger) per link, TA(M) = (M - M^dagger)/2 - tr(M - M^dagger)/6 * 1. */
void oracle_force(const cplx *G, const cplx *U, cplx *F, long nlinks)
{
#pragma omp parallel for schedule(static)
    for (long l = 0; l < nlinks; ++l) {
        const cplx *g = G + l * 9, *u = U + l * 9;
        cplx m[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                cplx s = 0;
                for (int c = 0; c < 3; ++c) s += g[a * 3 + c] * conj(u[b * 3 + c]);
                m[a][b] = s;
            }
        cplx tr = 0;
        for (int a = 0; a < 3; ++a) tr += m[a][a] - conj(m[a][a]);
        cplx *f = F + l * 9;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                f[a * 3 + b] = 0.5 * (m[a][b] - conj(m[b][a])) - (a == b ? tr / 6.0 : 0.0);
    }
}
