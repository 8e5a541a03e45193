/*
 * Plain FP64 CPU oracle for the eddy-current theta-methods of
 * Ventre, Chiariello, Isernia, Mottola, Tamburrino,
 * "Modal Decomposition in Numerical Computation of Eddy Current Transients"
 * (arXiv 2407.11993).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * definition the GPU library is checked against.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it; the product
 * path never does.  It shares no code, header or helper with the GPU library.
 *
 * Storage: every dense matrix here is ROW-MAJOR, A[i*n + j].
 * Precision: IEEE double throughout (the paper fixes none; FP64 is the
 * paper's own setting, ScaLAPACK double routines, Sec. 4.6).
 *
 * What is computed (citations are to the paper's sections and equations):
 *   - the Galerkin circuit system  R I + L dI/dt + E^T phi = V0 + VD,
 *     E I = iD                                  (Sec. 3.1, eqs. discrete_version_1a/b)
 *   - the null-space split  I = K Ii + E^T (E E^T)^{-1} iD
 *                                               (Sec. 3.1, eq. current_electrodes)
 *   - the projected system with Ri = K^T R K, Li = K^T L K,
 *     R_D = K^T R E^T (E E^T)^{-1}, L_D = K^T L E^T (E E^T)^{-1}
 *                                               (Sec. 3.1, eqs. discrete_version_2,
 *                                                circuit_equations_v2)
 *   - the classical theta-method with a Cholesky factor of Li + theta dt Ri
 *                                               (Sec. 3.3.1, eq. time_integration)
 *   - the modal theta-method on the generalized eigenpairs of (Li, Ri)
 *                                               (Sec. 3.2 and Sec. 3.3.2)
 *   - the time constants tau of Li v = tau Ri v, from the standard form on
 *     Ri's side                                 (Sec. 3.2, eq. generalized_
 *                                                eigenvalues_discrete)
 *   - the Sylvester inertia of Ri - sigma Li (the number of eigenvalues
 *     below a shift, for checks at sizes Jacobi cannot reach)
 *   - exact integration of the decoupled modal equations for inputs linear
 *     between samples (the analytical route Sec. 3.3 leaves to later work;
 *     reading r11)
 *   - the modal forcing and probe weights, and both modal steppers on a chosen
 *     subset of the decoupled equations (the selective solution of Sec. 3.2;
 *     reading r13)
 *
 * Readings of the paper taken where it is silent or inconsistent:
 *   (r1) the modal right-hand side is the Cholesky right-hand side expressed in
 *        the modal basis (increment form of the forcing for both methods);
 *   (r2) Ln, Rn use the reduced Li, Ri; eigenvectors are Li-normalised, so
 *        Ln = 1 and Rn = lambda_n = 1/tau_n;
 *   (r3) the factored matrix is the reduced Z = Li + theta dt Ri;
 *   (r4) the source mutual inductances enter projected by K^T; M^D = 0;
 *   (r5) K is the orthonormal Householder complement of im(E^T);
 *   (r10) the probe signal after step k is P (I^{k+1} - I^k) / dt;
 *   (r11) "exact" integration takes every source waveform linear between its
 *        samples (first-order hold), so on a step the modal forcing is
 *        g(s) = e0 + e1 s and each mode is integrated in closed form;
 *   (r13) a mode left out of the selective solution keeps y_n = 0 (its
 *        equation is not solved); which modes to keep is decided outside this
 *        file, by the coupling score of the Python wrapper's select_modes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, ld) ((int64_t)(i) * (int64_t)(ld) + (int64_t)(j))

/* ------------------------------------------------------------------------ */
/* Step a0: inductance kernel of the synthetic plates.                       */
/* L_ij = h / sqrt(|x_i - x_j|^2 + h^2): a smooth SPD stand-in for the       */
/* Coulomb-gauge operator of Sec. 2.2 (eq. operat), whose Galerkin matrix    */
/* is the dense SPD L of Sec. 3.1.                                           */
/* ------------------------------------------------------------------------ */
void orc_assemble_L(int64_t n, const double *xyz, double h, double *L)
{
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double dx = xyz[3 * i + 0] - xyz[3 * j + 0];
            double dy = xyz[3 * i + 1] - xyz[3 * j + 1];
            double dz = xyz[3 * i + 2] - xyz[3 * j + 2];
            L[IDX(i, j, n)] = h / sqrt(dx * dx + dy * dy + dz * dz + h * h);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Dense Cholesky A = G G^T (lower), in place; the upper triangle is zeroed. */
/* Returns -1 on success, else the index of the first non-positive pivot.    */
/* (Sec. 3.3.1: the factorisation Z = C C^T; also Li = G G^T for the modal   */
/*  standard form.)                                                          */
/* ------------------------------------------------------------------------ */
int64_t orc_cholesky(int64_t n, double *A)
{
    for (int64_t j = 0; j < n; ++j) {
        double s = A[IDX(j, j, n)];
        for (int64_t k = 0; k < j; ++k)
            s -= A[IDX(j, k, n)] * A[IDX(j, k, n)];
        if (!(s > 0.0))
            return j;
        double gjj = sqrt(s);
        A[IDX(j, j, n)] = gjj;
        for (int64_t i = j + 1; i < n; ++i) {
            double t = A[IDX(i, j, n)];
            for (int64_t k = 0; k < j; ++k)
                t -= A[IDX(i, k, n)] * A[IDX(j, k, n)];
            A[IDX(i, j, n)] = t / gjj;
        }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j)
            A[IDX(i, j, n)] = 0.0;
    return -1;
}

/* Forward substitution G y = b (G lower), b overwritten by y. */
void orc_forward(int64_t n, const double *G, double *b)
{
    for (int64_t i = 0; i < n; ++i) {
        double t = b[i];
        for (int64_t k = 0; k < i; ++k)
            t -= G[IDX(i, k, n)] * b[k];
        b[i] = t / G[IDX(i, i, n)];
    }
}

/* Backward substitution G^T x = y (G lower), y overwritten by x. */
void orc_backward_T(int64_t n, const double *G, double *y)
{
    for (int64_t i = n - 1; i >= 0; --i) {
        double t = y[i];
        for (int64_t k = i + 1; k < n; ++k)
            t -= G[IDX(k, i, n)] * y[k];
        y[i] = t / G[IDX(i, i, n)];
    }
}

/* ------------------------------------------------------------------------ */
/* Cyclic-by-row Jacobi for a symmetric matrix (Golub & Van Loan, "Matrix   */
/* Computations", sec. 8.5): A = Q diag(lam) Q^T.  A is destroyed.  A       */
/* rotation is skipped when |a_pq| <= eps sqrt(|a_pp a_qq|) (the relative   */
/* threshold of Demmel & Veselic); the sweep loop stops after a sweep that  */
/* rotates nothing.  lam is returned ascending with Q's columns permuted to  */
/* match (the paper's tau_n = 1/lam_n in decreasing order, Sec. 2.3).        */
/* Q is row-major n x n, Q[i*n + j] = component i of eigenvector j.          */
/* Returns the number of sweeps, or -1 if max_sweeps were not enough.        */
/* ------------------------------------------------------------------------ */
int orc_jacobi(int64_t n, double *A, double *Q, double *lam, int max_sweeps)
{
    const double eps = 2.220446049250313e-16;
    /* Qt holds the eigenvectors as rows while rotating (contiguous updates) */
    double *Qt = (double *)malloc(sizeof(double) * (size_t)(n * n + 1));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            Qt[IDX(i, j, n)] = (i == j) ? 1.0 : 0.0;
    int sweep = 0, done = (n < 2);
    while (!done && sweep < max_sweeps) {
        int64_t rotated = 0;
        for (int64_t p = 0; p < n - 1; ++p) {
            for (int64_t q = p + 1; q < n; ++q) {
                double apq = A[IDX(p, q, n)];
                double app = A[IDX(p, p, n)];
                double aqq = A[IDX(q, q, n)];
                if (apq == 0.0 || fabs(apq) <= eps * sqrt(fabs(app * aqq)))
                    continue;
                /* symmetric 2x2 Schur decomposition: J = [c s; -s c] in the
                 * (p,q) plane makes (J^T A J)_pq vanish */
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0.0 ? 1.0 : -1.0) /
                           (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = t * c;
                /* A <- J^T A J.  Rows p and q equal columns p and q (A is
                 * symmetric): update them along the rows, mirror into the
                 * columns. */
                double *rp = A + p * n, *rq = A + q * n;
                for (int64_t k = 0; k < n; ++k) {
                    if (k == p || k == q)
                        continue;
                    double akp = rp[k], akq = rq[k];
                    double np_ = c * akp - s * akq;
                    double nq_ = s * akp + c * akq;
                    rp[k] = np_;
                    rq[k] = nq_;
                    A[IDX(k, p, n)] = np_;
                    A[IDX(k, q, n)] = nq_;
                }
                rp[p] = app - t * apq;
                rq[q] = aqq + t * apq;
                rp[q] = 0.0;
                rq[p] = 0.0;
                /* Q <- Q J, i.e. rows p, q of Qt */
                double *up = Qt + p * n, *uq = Qt + q * n;
                for (int64_t k = 0; k < n; ++k) {
                    double a = up[k], b = uq[k];
                    up[k] = c * a - s * b;
                    uq[k] = s * a + c * b;
                }
                ++rotated;
            }
        }
        ++sweep;
        if (rotated == 0)
            done = 1;
    }
    for (int64_t i = 0; i < n; ++i)
        lam[i] = A[IDX(i, i, n)];
    /* selection sort of the eigenpairs, ascending */
    for (int64_t i = 0; i < n; ++i) {
        int64_t m = i;
        for (int64_t j = i + 1; j < n; ++j)
            if (lam[j] < lam[m])
                m = j;
        if (m != i) {
            double t = lam[i];
            lam[i] = lam[m];
            lam[m] = t;
            for (int64_t k = 0; k < n; ++k) {
                double u = Qt[IDX(i, k, n)];
                Qt[IDX(i, k, n)] = Qt[IDX(m, k, n)];
                Qt[IDX(m, k, n)] = u;
            }
        }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            Q[IDX(i, j, n)] = Qt[IDX(j, i, n)];
    free(Qt);
    return done ? sweep : -1;
}

/* ------------------------------------------------------------------------ */
/* Orthonormal basis K (n x (n-m)) of ker E for E (m x n) of full row rank:  */
/* Householder QR of E^T = H_1 ... H_m [T; 0]; the last n-m columns of       */
/* H = H_1 ... H_m are orthonormal and orthogonal to im E^T = X_D, so they   */
/* span X_0 = ker E (Sec. 3.1, eq. direct_sum_discrete).  Returns 0, or 1 if */
/* E is rank deficient.                                                      */
/* ------------------------------------------------------------------------ */
int orc_null_basis(int64_t m, int64_t n, const double *E, double *K)
{
    double *A = (double *)malloc(sizeof(double) * (size_t)(n * (m > 0 ? m : 1)));
    double *V = (double *)malloc(sizeof(double) * (size_t)(n * (m > 0 ? m : 1)));
    double *H = (double *)malloc(sizeof(double) * (size_t)(n * n));
    double *beta = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    int bad = 0;
    /* A = E^T, n x m row-major */
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < m; ++j)
            A[IDX(i, j, m)] = E[IDX(j, i, n)];
    memset(V, 0, sizeof(double) * (size_t)(n * (m > 0 ? m : 1)));
    for (int64_t j = 0; j < m; ++j) {
        double nrm = 0.0, full = 0.0;
        for (int64_t i = 0; i < n; ++i)
            full += E[IDX(j, i, n)] * E[IDX(j, i, n)];
        for (int64_t i = j; i < n; ++i)
            nrm += A[IDX(i, j, m)] * A[IDX(i, j, m)];
        nrm = sqrt(nrm);
        /* rank test: what is left of column j after the previous reflectors */
        if (!(nrm > 1e-12 * sqrt(full))) {
            bad = 1;
            break;
        }
        double alpha = A[IDX(j, j, m)] >= 0.0 ? -nrm : nrm;
        /* v = a - alpha e_j, H_j = I - beta v v^T, beta = 2 / v^T v */
        double vv = 0.0;
        for (int64_t i = j; i < n; ++i) {
            double vi = A[IDX(i, j, m)] - (i == j ? alpha : 0.0);
            V[IDX(i, j, m)] = vi;
            vv += vi * vi;
        }
        beta[j] = 2.0 / vv;
        for (int64_t c = j; c < m; ++c) {
            double d = 0.0;
            for (int64_t i = j; i < n; ++i)
                d += V[IDX(i, j, m)] * A[IDX(i, c, m)];
            for (int64_t i = j; i < n; ++i)
                A[IDX(i, c, m)] -= beta[j] * d * V[IDX(i, j, m)];
        }
    }
    if (!bad) {
        /* H = H_1 H_2 ... H_m I : apply in reverse order to the identity */
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j)
                H[IDX(i, j, n)] = (i == j) ? 1.0 : 0.0;
        for (int64_t j = m - 1; j >= 0; --j) {
            for (int64_t c = 0; c < n; ++c) {
                double d = 0.0;
                for (int64_t i = j; i < n; ++i)
                    d += V[IDX(i, j, m)] * H[IDX(i, c, n)];
                for (int64_t i = j; i < n; ++i)
                    H[IDX(i, c, n)] -= beta[j] * d * V[IDX(i, j, m)];
            }
        }
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = m; j < n; ++j)
                K[IDX(i, j - m, n - m)] = H[IDX(i, j, n)];
    }
    free(A);
    free(V);
    free(H);
    free(beta);
    return bad;
}

/* C = A^T B for A (r x p), B (r x q), all row-major; C is p x q. */
static void matTmul(int64_t r, int64_t p, int64_t q, const double *A,
                    const double *B, double *C)
{
    memset(C, 0, sizeof(double) * (size_t)(p * q));
    for (int64_t k = 0; k < r; ++k)
        for (int64_t i = 0; i < p; ++i) {
            double a = A[IDX(k, i, p)];
            if (a == 0.0)
                continue;
            for (int64_t j = 0; j < q; ++j)
                C[IDX(i, j, q)] += a * B[IDX(k, j, q)];
        }
}

/* C = A B for A (p x r), B (r x q), row-major. */
static void matmul(int64_t p, int64_t r, int64_t q, const double *A,
                   const double *B, double *C)
{
    memset(C, 0, sizeof(double) * (size_t)(p * q));
    for (int64_t i = 0; i < p; ++i)
        for (int64_t k = 0; k < r; ++k) {
            double a = A[IDX(i, k, r)];
            if (a == 0.0)
                continue;
            for (int64_t j = 0; j < q; ++j)
                C[IDX(i, j, q)] += a * B[IDX(k, j, q)];
        }
}

/* ------------------------------------------------------------------------ */
/* The problem statement (Sec. 3.1, eqs. discrete_version_1a/b and           */
/* induced_voltages_0): R I + L I' + E^T phi = -M0 i0',  E I = iD,           */
/* observed through probe rows P.                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;       /* unknowns N */
    int64_t m;       /* electrode rows Ne-1 (0: no electrodes) */
    int64_t n_src;   /* solenoidal sources (columns of M0) */
    int64_t n_probe; /* probe rows */
    const double *L; /* n x n, SPD */
    const double *R; /* n x n, SPD */
    const double *E; /* m x n */
    const double *M; /* n x n_src */
    const double *P; /* n_probe x n */
} orc_problem;

/* The reduced quantities of Sec. 3.1 (eqs. discrete_version_2 and
 * circuit_equations_v2). */
typedef struct {
    int64_t n0;
    double *K;  /* n x n0 */
    double *Li; /* n0 x n0 */
    double *Ri; /* n0 x n0 */
    double *AD; /* n x m   : E^T (E E^T)^{-1} */
    double *RD; /* n0 x m  : K^T R AD */
    double *LD; /* n0 x m  : K^T L AD  (+ K^T M^D, taken as 0) */
    double *Mi; /* n0 x n_src : K^T M0 */
    double *PK; /* n_probe x n0 : P K */
    double *PD; /* n_probe x m  : P AD */
} orc_reduced;

static void free_reduced(orc_reduced *r)
{
    free(r->K);
    free(r->Li);
    free(r->Ri);
    free(r->AD);
    free(r->RD);
    free(r->LD);
    free(r->Mi);
    free(r->PK);
    free(r->PD);
}

static int reduce(const orc_problem *pb, orc_reduced *r)
{
    const int64_t n = pb->n, m = pb->m, n0 = n - m;
    const int64_t mm = m > 0 ? m : 1;
    memset(r, 0, sizeof(*r));
    r->n0 = n0;
    r->K = (double *)malloc(sizeof(double) * (size_t)(n * n0));
    r->Li = (double *)malloc(sizeof(double) * (size_t)(n0 * n0));
    r->Ri = (double *)malloc(sizeof(double) * (size_t)(n0 * n0));
    r->AD = (double *)calloc((size_t)(n * mm), sizeof(double));
    r->RD = (double *)calloc((size_t)(n0 * mm), sizeof(double));
    r->LD = (double *)calloc((size_t)(n0 * mm), sizeof(double));
    r->Mi = (double *)calloc((size_t)(n0 * (pb->n_src > 0 ? pb->n_src : 1)), sizeof(double));
    r->PK = (double *)calloc((size_t)((pb->n_probe > 0 ? pb->n_probe : 1) * n0), sizeof(double));
    r->PD = (double *)calloc((size_t)((pb->n_probe > 0 ? pb->n_probe : 1) * mm), sizeof(double));
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(n * (n > mm ? n : mm)));
    if (m == 0) {
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j)
                r->K[IDX(i, j, n)] = (i == j) ? 1.0 : 0.0;
        memcpy(r->Li, pb->L, sizeof(double) * (size_t)(n * n));
        memcpy(r->Ri, pb->R, sizeof(double) * (size_t)(n * n));
        if (pb->n_src > 0)
            memcpy(r->Mi, pb->M, sizeof(double) * (size_t)(n * pb->n_src));
        if (pb->n_probe > 0)
            memcpy(r->PK, pb->P, sizeof(double) * (size_t)(pb->n_probe * n));
        free(tmp);
        return 0;
    }
    if (orc_null_basis(m, n, pb->E, r->K)) {
        free(tmp);
        return 1;
    }
    /* Li = K^T L K, Ri = K^T R K (eq. discrete_version_2) */
    double *LK = (double *)malloc(sizeof(double) * (size_t)(n * n0));
    matmul(n, n, n0, pb->L, r->K, LK);
    matTmul(n, n0, n0, r->K, LK, r->Li);
    matmul(n, n, n0, pb->R, r->K, LK);
    matTmul(n, n0, n0, r->K, LK, r->Ri);
    free(LK);
    /* AD = E^T (E E^T)^{-1}  (eq. current_electrodes) */
    double *EEt = (double *)malloc(sizeof(double) * (size_t)(m * m));
    for (int64_t a = 0; a < m; ++a)
        for (int64_t b = 0; b < m; ++b) {
            double s = 0.0;
            for (int64_t k = 0; k < n; ++k)
                s += pb->E[IDX(a, k, n)] * pb->E[IDX(b, k, n)];
            EEt[IDX(a, b, m)] = s;
        }
    if (orc_cholesky(m, EEt) >= 0) {
        free(EEt);
        free(tmp);
        return 1;
    }
    /* row i of AD solves (E E^T) x = E[:, i] */
    for (int64_t i = 0; i < n; ++i) {
        double *x = r->AD + i * m;
        for (int64_t a = 0; a < m; ++a)
            x[a] = pb->E[IDX(a, i, n)];
        orc_forward(m, EEt, x);
        orc_backward_T(m, EEt, x);
    }
    free(EEt);
    /* R_D = K^T R AD, L_D = K^T L AD (eq. circuit_equations_v2, M^D = 0) */
    matmul(n, n, m, pb->R, r->AD, tmp);
    matTmul(n, n0, m, r->K, tmp, r->RD);
    matmul(n, n, m, pb->L, r->AD, tmp);
    matTmul(n, n0, m, r->K, tmp, r->LD);
    if (pb->n_src > 0)
        matTmul(n, n0, pb->n_src, r->K, pb->M, r->Mi);
    if (pb->n_probe > 0) {
        matmul(pb->n_probe, n, n0, pb->P, r->K, r->PK);
        matmul(pb->n_probe, n, m, pb->P, r->AD, r->PD);
    }
    free(tmp);
    return 0;
}

/* Forcing of one theta step (Sec. 3.3.1, eq. time_integration, reading r1):
 *   f = -dt R_D (iD^k + theta d iD) - L_D d iD - K^T M0 d i0,
 * with d x = x^{k+1} - x^k.  Written into f (n0). */
static void forcing(const orc_problem *pb, const orc_reduced *r, double theta,
                    double dt, int64_t k, const double *i_src,
                    const double *i_D, double *f)
{
    const int64_t n0 = r->n0, m = pb->m, ns = pb->n_src;
    for (int64_t i = 0; i < n0; ++i) {
        double s = 0.0;
        for (int64_t a = 0; a < m; ++a) {
            double iDk = i_D[IDX(k, a, m)];
            double diD = i_D[IDX(k + 1, a, m)] - iDk;
            s += -dt * r->RD[IDX(i, a, m)] * (iDk + theta * diD) -
                 r->LD[IDX(i, a, m)] * diD;
        }
        for (int64_t c = 0; c < ns; ++c) {
            double di0 = i_src[IDX(k + 1, c, ns)] - i_src[IDX(k, c, ns)];
            s += -r->Mi[IDX(i, c, ns)] * di0;
        }
        f[i] = s;
    }
}

/* Probe signal after step k (reading r10):
 *   s^{k+1} = P (K dIi + AD d iD) / dt. */
static void probe(const orc_problem *pb, const orc_reduced *r, double dt,
                  int64_t k, const double *dIi, const double *i_D, double *out)
{
    const int64_t n0 = r->n0, m = pb->m;
    for (int64_t p = 0; p < pb->n_probe; ++p) {
        double s = 0.0;
        for (int64_t i = 0; i < n0; ++i)
            s += r->PK[IDX(p, i, n0)] * dIi[i];
        for (int64_t a = 0; a < m; ++a)
            s += r->PD[IDX(p, a, m)] *
                 (i_D[IDX(k + 1, a, m)] - i_D[IDX(k, a, m)]);
        out[p] = s / dt;
    }
}

/* Full current I = K Ii + AD iD (eq. current_electrodes). */
static void full_current(const orc_problem *pb, const orc_reduced *r,
                         const double *Ii, const double *iD_k, double *I)
{
    const int64_t n = pb->n, n0 = r->n0, m = pb->m;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n0; ++j)
            s += r->K[IDX(i, j, n0)] * Ii[j];
        for (int64_t a = 0; a < m; ++a)
            s += r->AD[IDX(i, a, m)] * iD_k[a];
        I[i] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* The classical theta-method (Sec. 3.3.1, eq. time_integration): factor     */
/* Z = Li + theta dt Ri = C C^T once, then per step                          */
/*   Z dI = -dt Ri Ii^k + f^k,  Ii^{k+1} = Ii^k + dI,                        */
/* solved by forward then backward substitution.  Ii^0 = 0.                  */
/* signal: T x n_probe; I_hist: (T+1) x n full currents, or NULL.            */
/* Returns 0, 1 (bad electrodes), 2 (Z not SPD).                             */
/* ------------------------------------------------------------------------ */
int orc_theta_direct(const orc_problem *pb, double theta, double dt, int64_t T,
                     const double *i_src, const double *i_D, double *signal,
                     double *I_hist)
{
    orc_reduced r;
    if (reduce(pb, &r)) {
        free_reduced(&r);
        return 1;
    }
    const int64_t n0 = r.n0;
    double *Z = (double *)malloc(sizeof(double) * (size_t)(n0 * n0));
    for (int64_t i = 0; i < n0 * n0; ++i)
        Z[i] = r.Li[i] + theta * dt * r.Ri[i];
    if (orc_cholesky(n0, Z) >= 0) {
        free(Z);
        free_reduced(&r);
        return 2;
    }
    double *Ii = (double *)calloc((size_t)n0, sizeof(double));
    double *b = (double *)malloc(sizeof(double) * (size_t)n0);
    if (I_hist)
        full_current(pb, &r, Ii, i_D, I_hist);
    for (int64_t k = 0; k < T; ++k) {
        forcing(pb, &r, theta, dt, k, i_src, i_D, b);
        for (int64_t i = 0; i < n0; ++i) {
            double s = 0.0;
            for (int64_t j = 0; j < n0; ++j)
                s += r.Ri[IDX(i, j, n0)] * Ii[j];
            b[i] -= dt * s;
        }
        orc_forward(n0, Z, b);
        orc_backward_T(n0, Z, b);
        for (int64_t i = 0; i < n0; ++i)
            Ii[i] += b[i];
        if (signal)
            probe(pb, &r, dt, k, b, i_D, signal + k * pb->n_probe);
        if (I_hist)
            full_current(pb, &r, Ii, i_D + (k + 1) * pb->m,
                         I_hist + (k + 1) * pb->n);
    }
    free(Ii);
    free(b);
    free(Z);
    free_reduced(&r);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Standard form of the pencil (Sec. 3.2, eq. generalized_eigenvalues_      */
/* discrete, written with lambda = 1/tau):  Ri v = lambda Li v.  With        */
/* Li = G G^T, C = G^{-1} Ri G^{-T} has the same eigenvalues, and            */
/* v = G^{-T} q for each eigenvector q of C.  G is the lower Cholesky        */
/* factor (row-major n x n); C (n x n) is returned symmetrised.              */
/* ------------------------------------------------------------------------ */
void orc_standard_form(int64_t n, const double *G, const double *Ri, double *C)
{
    double *X = (double *)malloc(sizeof(double) * (size_t)(n * n));
    double *col = (double *)malloc(sizeof(double) * (size_t)n);
    /* X = G^{-1} Ri, column by column */
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < n; ++i)
            col[i] = Ri[IDX(i, j, n)];
        orc_forward(n, G, col);
        for (int64_t i = 0; i < n; ++i)
            X[IDX(i, j, n)] = col[i];
    }
    /* C = G^{-1} X^T  (X^T = Ri G^{-T}) */
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < n; ++i)
            col[i] = X[IDX(j, i, n)];
        orc_forward(n, G, col);
        for (int64_t i = 0; i < n; ++i)
            C[IDX(i, j, n)] = col[i];
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double s = 0.5 * (C[IDX(i, j, n)] + C[IDX(j, i, n)]);
            C[IDX(i, j, n)] = s;
            C[IDX(j, i, n)] = s;
        }
    free(X);
    free(col);
}

/* ------------------------------------------------------------------------ */
/* Modal decomposition of the reduced pencil (Sec. 3.2): eigenvalues        */
/* lam (ascending, lam_n = R_n / L_n = 1/tau_n) and the Li-normalised        */
/* eigenvectors V = G^{-T} Q (n0 x n0, column j = mode j), or NULL.          */
/* Returns 0, 1 (bad electrodes), 2 (Li not SPD), 3 (Jacobi did not         */
/* converge).                                                                */
/* ------------------------------------------------------------------------ */
static int modal_parts(const orc_problem *pb, orc_reduced *r, double *lam,
                       double *V, int *sweeps)
{
    if (reduce(pb, r))
        return 1;
    const int64_t n0 = r->n0;
    double *G = (double *)malloc(sizeof(double) * (size_t)(n0 * n0));
    memcpy(G, r->Li, sizeof(double) * (size_t)(n0 * n0));
    if (orc_cholesky(n0, G) >= 0) {
        free(G);
        return 2;
    }
    double *C = (double *)malloc(sizeof(double) * (size_t)(n0 * n0));
    double *Q = (double *)malloc(sizeof(double) * (size_t)(n0 * n0));
    orc_standard_form(n0, G, r->Ri, C);
    int sw = orc_jacobi(n0, C, Q, lam, 100);
    if (sweeps)
        *sweeps = sw;
    if (sw < 0) {
        free(G);
        free(C);
        free(Q);
        return 3;
    }
    /* V = G^{-T} Q, column by column */
    double *col = (double *)malloc(sizeof(double) * (size_t)n0);
    for (int64_t j = 0; j < n0; ++j) {
        for (int64_t i = 0; i < n0; ++i)
            col[i] = Q[IDX(i, j, n0)];
        orc_backward_T(n0, G, col);
        for (int64_t i = 0; i < n0; ++i)
            V[IDX(i, j, n0)] = col[i];
    }
    free(col);
    free(G);
    free(C);
    free(Q);
    return 0;
}

int orc_modal_eigen(const orc_problem *pb, double *lam, double *V, int *sweeps)
{
    orc_reduced r;
    double *Vtmp = V;
    int64_t n0 = pb->n - pb->m;
    if (!Vtmp)
        Vtmp = (double *)malloc(sizeof(double) * (size_t)(n0 * n0));
    int rc = modal_parts(pb, &r, lam, Vtmp, sweeps);
    if (!V)
        free(Vtmp);
    free_reduced(&r);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* The time constants of the pencil as the paper writes its eigenproblem    */
/* (Sec. 3.2, eq. generalized_eigenvalues_discrete):  Li v = tau Ri v.  With  */
/* Ri = H H^T, C' = H^{-1} Li H^{-T} has the eigenvalues tau (the standard   */
/* form taken from the other side of the pencil than orc_modal_eigen).       */
/* tau is returned ascending (n0 values).  Returns 0, 1 (bad electrodes),    */
/* 2 (Ri not SPD), 3 (Jacobi did not converge).                              */
/* ------------------------------------------------------------------------ */
int orc_time_constants(const orc_problem *pb, double *tau)
{
    orc_reduced r;
    if (reduce(pb, &r)) {
        free_reduced(&r);
        return 1;
    }
    const int64_t n0 = r.n0;
    double *H = (double *)malloc(sizeof(double) * (size_t)(n0 * n0));
    memcpy(H, r.Ri, sizeof(double) * (size_t)(n0 * n0));
    int rc = 0;
    if (orc_cholesky(n0, H) >= 0) {
        rc = 2;
    } else {
        double *C = (double *)malloc(sizeof(double) * (size_t)(n0 * n0));
        double *Q = (double *)malloc(sizeof(double) * (size_t)(n0 * n0));
        orc_standard_form(n0, H, r.Li, C);
        if (orc_jacobi(n0, C, Q, tau, 100) < 0)
            rc = 3;
        free(C);
        free(Q);
    }
    free(H);
    free_reduced(&r);
    return rc;
}

/* Modal coupling weights (Sec. 3.2, eq. modal_decomposition_discrete): with */
/* the Li-normalised eigenvectors V, the forcing of mode n by column j of    */
/* [RD | LD | Mi] is W(n, j) = (V^T [RD | LD | Mi])(n, j), and its weight in  */
/* probe p is Pw(n, p) = (P K V)(p, n).  A mode with a zero row in W is never */
/* excited from I(0) = 0; one with a zero row in Pw is never seen by a probe. */
/* W is n0 x (2m + n_src), Pw n0 x n_probe, both row-major; lam may be NULL. */
int orc_mode_weights(const orc_problem *pb, double *lam_out, double *W, double *Pw)
{
    orc_reduced r;
    const int64_t n0 = pb->n - pb->m, m = pb->m, ns = pb->n_src;
    const int64_t nf = 2 * m + ns, np = pb->n_probe;
    double *lam = (double *)malloc(sizeof(double) * (size_t)n0);
    double *V = (double *)malloc(sizeof(double) * (size_t)(n0 * n0));
    int rc = modal_parts(pb, &r, lam, V, NULL);
    if (rc) {
        free(lam);
        free(V);
        free_reduced(&r);
        return rc;
    }
    for (int64_t nn = 0; nn < n0; ++nn) {
        for (int64_t j = 0; j < nf; ++j) {
            double s = 0.0;
            for (int64_t i = 0; i < n0; ++i) {
                double f;
                if (j < m)
                    f = r.RD[IDX(i, j, m)];
                else if (j < 2 * m)
                    f = r.LD[IDX(i, j - m, m)];
                else
                    f = r.Mi[IDX(i, j - 2 * m, ns)];
                s += V[IDX(i, nn, n0)] * f;
            }
            W[IDX(nn, j, nf)] = s;
        }
        for (int64_t p = 0; p < np; ++p) {
            double s = 0.0;
            for (int64_t i = 0; i < n0; ++i)
                s += r.PK[IDX(p, i, n0)] * V[IDX(i, nn, n0)];
            Pw[IDX(nn, p, np)] = s;
        }
    }
    if (lam_out)
        memcpy(lam_out, lam, sizeof(double) * (size_t)n0);
    free(lam);
    free(V);
    free_reduced(&r);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The modal theta-method (Sec. 3.3.2).  In the basis of Li-normalised       */
/* generalized eigenvectors V the system decouples into                      */
/*   I_n' + lam_n I_n = (V^T g)_n    (eq. modal_decomposition_discrete)      */
/* and each mode is stepped by the theta-method:                             */
/*   (1 + theta dt lam_n) dy_n = -dt lam_n y_n + (V^T f^k)_n,                */
/* where f^k is the same forcing as in the Cholesky method (reading r1).     */
/* Ii = V y, so the probe signal is P (K V dy + AD d iD) / dt.               */
/* lam_out (n0) and I_hist ((T+1) x n) may be NULL.  keep (n0 flags, or      */
/* NULL = every mode) solves only the flagged decoupled equations (the       */
/* selective solution that Sec. 3.2 allows); the others stay at y_n = 0.     */
/* ------------------------------------------------------------------------ */
int orc_theta_modal(const orc_problem *pb, double theta, double dt, int64_t T,
                    const double *i_src, const double *i_D, double *signal,
                    double *lam_out, double *I_hist, const unsigned char *keep)
{
    orc_reduced r;
    const int64_t n0 = pb->n - pb->m;
    double *lam = (double *)malloc(sizeof(double) * (size_t)n0);
    double *V = (double *)malloc(sizeof(double) * (size_t)(n0 * n0));
    int rc = modal_parts(pb, &r, lam, V, NULL);
    if (rc) {
        free(lam);
        free(V);
        free_reduced(&r);
        return rc;
    }
    double *y = (double *)calloc((size_t)n0, sizeof(double));
    double *dy = (double *)malloc(sizeof(double) * (size_t)n0);
    double *f = (double *)malloc(sizeof(double) * (size_t)n0);
    double *dIi = (double *)malloc(sizeof(double) * (size_t)n0);
    double *Ii = (double *)malloc(sizeof(double) * (size_t)n0);
    if (I_hist) {
        memset(Ii, 0, sizeof(double) * (size_t)n0);
        full_current(pb, &r, Ii, i_D, I_hist);
    }
    for (int64_t k = 0; k < T; ++k) {
        forcing(pb, &r, theta, dt, k, i_src, i_D, f);
        for (int64_t nn = 0; nn < n0; ++nn) {
            double e = 0.0; /* modal forcing (V^T f)_n */
            for (int64_t i = 0; i < n0; ++i)
                e += V[IDX(i, nn, n0)] * f[i];
            dy[nn] = (keep && !keep[nn])
                         ? 0.0
                         : (-dt * lam[nn] * y[nn] + e) / (1.0 + theta * dt * lam[nn]);
        }
        for (int64_t nn = 0; nn < n0; ++nn)
            y[nn] += dy[nn];
        for (int64_t i = 0; i < n0; ++i) {
            double s = 0.0;
            for (int64_t nn = 0; nn < n0; ++nn)
                s += V[IDX(i, nn, n0)] * dy[nn];
            dIi[i] = s;
        }
        if (signal)
            probe(pb, &r, dt, k, dIi, i_D, signal + k * pb->n_probe);
        if (I_hist) {
            for (int64_t i = 0; i < n0; ++i) {
                double s = 0.0;
                for (int64_t nn = 0; nn < n0; ++nn)
                    s += V[IDX(i, nn, n0)] * y[nn];
                Ii[i] = s;
            }
            full_current(pb, &r, Ii, i_D + (k + 1) * pb->m,
                         I_hist + (k + 1) * pb->n);
        }
    }
    if (lam_out)
        memcpy(lam_out, lam, sizeof(double) * (size_t)n0);
    free(y);
    free(dy);
    free(f);
    free(dIi);
    free(Ii);
    free(lam);
    free(V);
    free_reduced(&r);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Exact integration of one mode over a step of length dt (reading r11):     */
/*   y' + lam y = e0 + e1 s,  s in [0, dt]                                    */
/* gives y(dt) = exp(-lam dt) y(0) + e0 phi1 + e1 phi2 with                   */
/*   phi1 = int_0^dt exp(-lam (dt - s)) ds   = dt  sum_k (-x)^k / (k+1)!      */
/*   phi2 = int_0^dt exp(-lam (dt - s)) s ds = dt^2 sum_k (-x)^k / (k+2)!     */
/* (x = lam dt).  The series are summed for x < 1/2; above, the closed forms */
/* phi1 = (1 - exp(-x)) / lam, phi2 = (dt - phi1) / lam have no cancellation. */
/* ------------------------------------------------------------------------ */
void orc_exact_phi(double lam, double dt, double *phi1, double *phi2)
{
    const double x = lam * dt;
    if (x < 0.5) {
        double t1 = 1.0, t2 = 0.5, s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < 40; ++k) {
            s1 += t1;
            s2 += t2;
            t1 *= -x / (double)(k + 2);
            t2 *= -x / (double)(k + 3);
        }
        *phi1 = dt * s1;
        *phi2 = dt * dt * s2;
    } else {
        *phi1 = -expm1(-x) / lam;
        *phi2 = (dt - *phi1) / lam;
    }
}

/* Modal stepping with exact per-mode integration (reading r11).  With the   */
/* waveforms linear on step k (d x = x^{k+1} - x^k), the reduced forcing of   */
/* eq. circuit_equations_v2 is                                               */
/*   f(s) = f0 + f1 s,  f0 = -R_D iD^k - L_D d iD / dt - K^T M0 d i0 / dt,    */
/*                      f1 = -R_D d iD / dt,                                 */
/* its modal components e0 = V^T f0, e1 = V^T f1, and every mode advances as */
/* in orc_exact_phi.  Probe signal, history and keep as in orc_theta_modal. */
/* ------------------------------------------------------------------------ */
int orc_exact_modal(const orc_problem *pb, double dt, int64_t T,
                    const double *i_src, const double *i_D, double *signal,
                    double *I_hist, const unsigned char *keep)
{
    orc_reduced r;
    const int64_t n0 = pb->n - pb->m, m = pb->m, ns = pb->n_src;
    double *lam = (double *)malloc(sizeof(double) * (size_t)n0);
    double *V = (double *)malloc(sizeof(double) * (size_t)(n0 * n0));
    int rc = modal_parts(pb, &r, lam, V, NULL);
    if (rc) {
        free(lam);
        free(V);
        free_reduced(&r);
        return rc;
    }
    double *decay = (double *)malloc(sizeof(double) * (size_t)n0);
    double *p1 = (double *)malloc(sizeof(double) * (size_t)n0);
    double *p2 = (double *)malloc(sizeof(double) * (size_t)n0);
    for (int64_t nn = 0; nn < n0; ++nn) {
        decay[nn] = exp(-lam[nn] * dt);
        orc_exact_phi(lam[nn], dt, &p1[nn], &p2[nn]);
    }
    double *y = (double *)calloc((size_t)n0, sizeof(double));
    double *dy = (double *)malloc(sizeof(double) * (size_t)n0);
    double *f0 = (double *)malloc(sizeof(double) * (size_t)n0);
    double *f1 = (double *)malloc(sizeof(double) * (size_t)n0);
    double *dIi = (double *)malloc(sizeof(double) * (size_t)n0);
    double *Ii = (double *)malloc(sizeof(double) * (size_t)n0);
    if (I_hist) {
        memset(Ii, 0, sizeof(double) * (size_t)n0);
        full_current(pb, &r, Ii, i_D, I_hist);
    }
    for (int64_t k = 0; k < T; ++k) {
        for (int64_t i = 0; i < n0; ++i) {
            double a = 0.0, b = 0.0;
            for (int64_t e = 0; e < m; ++e) {
                const double iDk = i_D[IDX(k, e, m)];
                const double diD = i_D[IDX(k + 1, e, m)] - iDk;
                a += -r.RD[IDX(i, e, m)] * iDk - r.LD[IDX(i, e, m)] * diD / dt;
                b += -r.RD[IDX(i, e, m)] * diD / dt;
            }
            for (int64_t c = 0; c < ns; ++c) {
                const double di0 = i_src[IDX(k + 1, c, ns)] - i_src[IDX(k, c, ns)];
                a += -r.Mi[IDX(i, c, ns)] * di0 / dt;
            }
            f0[i] = a;
            f1[i] = b;
        }
        for (int64_t nn = 0; nn < n0; ++nn) {
            double e0 = 0.0, e1 = 0.0;
            for (int64_t i = 0; i < n0; ++i) {
                e0 += V[IDX(i, nn, n0)] * f0[i];
                e1 += V[IDX(i, nn, n0)] * f1[i];
            }
            const double ynew = decay[nn] * y[nn] + e0 * p1[nn] + e1 * p2[nn];
            dy[nn] = (keep && !keep[nn]) ? 0.0 : ynew - y[nn];
        }
        for (int64_t nn = 0; nn < n0; ++nn)
            y[nn] += dy[nn];
        for (int64_t i = 0; i < n0; ++i) {
            double s = 0.0;
            for (int64_t nn = 0; nn < n0; ++nn)
                s += V[IDX(i, nn, n0)] * dy[nn];
            dIi[i] = s;
        }
        if (signal)
            probe(pb, &r, dt, k, dIi, i_D, signal + k * pb->n_probe);
        if (I_hist) {
            for (int64_t i = 0; i < n0; ++i) {
                double s = 0.0;
                for (int64_t nn = 0; nn < n0; ++nn)
                    s += V[IDX(i, nn, n0)] * y[nn];
                Ii[i] = s;
            }
            full_current(pb, &r, Ii, i_D + (k + 1) * pb->m,
                         I_hist + (k + 1) * pb->n);
        }
    }
    free(decay);
    free(p1);
    free(p2);
    free(y);
    free(dy);
    free(f0);
    free(f1);
    free(dIi);
    free(Ii);
    free(lam);
    free(V);
    free_reduced(&r);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the probe-signal misfit over runs that share one waveform     */
/* (gradient of the theta-method of Sec. 3.3.1, eq. time_integration).      */
/* Run c drives source column c of M (n x C) with the waveform i (T+1       */
/* samples) and observes probe row c of P (C x n); no electrodes.  With     */
/* Z = L + theta dt R and the residual of step k                            */
/*     F_k = Z dI_k + dt R I_k - M_c u_k,   u_k = -(i_{k+1} - i_k),          */
/* the misfit J = sum_c sum_k (P_c dI_k / dt - obs_c[k])^2 has the adjoint   */
/*     Z lambda_k = g_k P_c^T - dt R mu_k,   mu_k = sum_{j > k} lambda_j,    */
/*     g_k = 2 (P_c dI_k / dt - obs_c[k]) / dt,                             */
/* and the gradients                                                        */
/*     dJ/dR(a,b) = - sum_{c,k} lambda_k(a) (theta dt dI_k(b) + dt I_k(b)),  */
/*     dJ/du_k    =   sum_c lambda_k^T M_c,                                  */
/*     dJ/di_j    =   dJ/du_j - dJ/du_{j-1}.                                 */
/* Every entry of R is treated as independent (dJdR is n x n, row-major).   */
/* Every state is kept (no checkpoints).  Returns 0, or 2 if Z is not SPD.   */
/* ------------------------------------------------------------------------ */
int orc_adjoint_direct(int64_t n, const double *L, const double *R, int64_t C,
                       const double *M, const double *P, double theta,
                       double dt, int64_t T, const double *i_src,
                       const double *obs, double *J, double *dJdR,
                       double *dJdi)
{
    double *Z = (double *)malloc(sizeof(double) * (size_t)(n * n));
    for (int64_t a = 0; a < n * n; ++a)
        Z[a] = L[a] + theta * dt * R[a];
    if (orc_cholesky(n, Z) >= 0) {
        free(Z);
        return 2;
    }
    double *I = (double *)malloc(sizeof(double) * (size_t)((T + 1) * n));
    double *dI = (double *)malloc(sizeof(double) * (size_t)((T > 0 ? T : 1) * n));
    double *g = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1));
    double *lam = (double *)malloc(sizeof(double) * (size_t)n);
    double *mu = (double *)malloc(sizeof(double) * (size_t)n);
    double *b = (double *)malloc(sizeof(double) * (size_t)n);
    double *dJdu = (double *)calloc((size_t)(T > 0 ? T : 1), sizeof(double));
    *J = 0.0;
    for (int64_t a = 0; a < n * n; ++a)
        dJdR[a] = 0.0;
    for (int64_t c = 0; c < C; ++c) {
        /* forward: every I_k and dI_k of run c */
        for (int64_t a = 0; a < n; ++a)
            I[a] = 0.0;
        for (int64_t k = 0; k < T; ++k) {
            const double u = -(i_src[k + 1] - i_src[k]);
            const double *Ik = I + k * n;
            for (int64_t a = 0; a < n; ++a) {
                double s = 0.0;
                for (int64_t q = 0; q < n; ++q)
                    s += R[IDX(a, q, n)] * Ik[q];
                b[a] = -dt * s + M[IDX(a, c, C)] * u;
            }
            orc_forward(n, Z, b);
            orc_backward_T(n, Z, b);
            double s = 0.0;
            for (int64_t a = 0; a < n; ++a) {
                dI[k * n + a] = b[a];
                I[(k + 1) * n + a] = Ik[a] + b[a];
                s += P[IDX(c, a, n)] * b[a];
            }
            const double res = s / dt - obs[c * T + k];
            *J += res * res;
            g[k] = 2.0 * res / dt;
        }
        /* backward */
        for (int64_t a = 0; a < n; ++a)
            mu[a] = 0.0;
        for (int64_t k = T - 1; k >= 0; --k) {
            for (int64_t a = 0; a < n; ++a) {
                double s = 0.0;
                for (int64_t q = 0; q < n; ++q)
                    s += R[IDX(a, q, n)] * mu[q];
                lam[a] = g[k] * P[IDX(c, a, n)] - dt * s;
            }
            orc_forward(n, Z, lam);
            orc_backward_T(n, Z, lam);
            double du = 0.0;
            for (int64_t a = 0; a < n; ++a)
                du += lam[a] * M[IDX(a, c, C)];
            dJdu[k] += du;
            for (int64_t a = 0; a < n; ++a) {
                const double la = lam[a];
                if (la == 0.0)
                    continue;
                for (int64_t q = 0; q < n; ++q)
                    dJdR[IDX(a, q, n)] -=
                        la * (theta * dt * dI[k * n + q] + dt * I[k * n + q]);
            }
            for (int64_t a = 0; a < n; ++a)
                mu[a] += lam[a];
        }
    }
    for (int64_t j = 0; j <= T; ++j)
        dJdi[j] = (j < T ? dJdu[j] : 0.0) - (j > 0 ? dJdu[j - 1] : 0.0);
    free(Z);
    free(I);
    free(dI);
    free(g);
    free(lam);
    free(mu);
    free(b);
    free(dJdu);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sylvester inertia of a symmetric matrix by the symmetric-indefinite       */
/* factorisation P A P^T = L D L^T with Bunch-Kaufman pivoting (Bunch &      */
/* Kaufman, "Some stable methods for calculating inertia and solving         */
/* symmetric linear systems", Math. Comp. 31, 1977; Golub & Van Loan 4.4).   */
/* D is block diagonal with 1x1 and 2x2 blocks; A and D are congruent, so    */
/* by Sylvester's law of inertia they have the same numbers of negative,     */
/* zero and positive eigenvalues.  Only the lower triangle of the trailing   */
/* matrix is read and updated (A[i*n + j], i >= j); A is destroyed.  L is    */
/* not kept: only D's blocks are needed.                                     */
/* counts[0] = #negative, counts[1] = #zero, counts[2] = #positive.          */
/* ------------------------------------------------------------------------ */
static double lo_get(const double *A, int64_t n, int64_t i, int64_t j)
{
    return i >= j ? A[IDX(i, j, n)] : A[IDX(j, i, n)];
}

/* Symmetric interchange of rows and columns p < q of the trailing matrix    */
/* A[k:, k:] in lower-triangle storage.                                      */
static void lo_swap(double *A, int64_t n, int64_t k, int64_t p, int64_t q)
{
    double t;
    if (p == q)
        return;
    for (int64_t j = k; j < p; ++j) {          /* row entries left of p */
        t = A[IDX(p, j, n)];
        A[IDX(p, j, n)] = A[IDX(q, j, n)];
        A[IDX(q, j, n)] = t;
    }
    t = A[IDX(p, p, n)];                        /* the two diagonal entries */
    A[IDX(p, p, n)] = A[IDX(q, q, n)];
    A[IDX(q, q, n)] = t;
    for (int64_t i = p + 1; i < q; ++i) {       /* column p below p, row q left of q */
        t = A[IDX(i, p, n)];
        A[IDX(i, p, n)] = A[IDX(q, i, n)];
        A[IDX(q, i, n)] = t;
    }
    for (int64_t i = q + 1; i < n; ++i) {       /* columns p and q below q */
        t = A[IDX(i, p, n)];
        A[IDX(i, p, n)] = A[IDX(i, q, n)];
        A[IDX(i, q, n)] = t;
    }
}

void orc_ldlt_inertia(int64_t n, double *A, int64_t *counts)
{
    const double alpha = (1.0 + sqrt(17.0)) / 8.0;
    double *u = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    counts[0] = counts[1] = counts[2] = 0;
    int64_t k = 0;
    while (k < n) {
        /* largest off-diagonal entry of column k of the trailing matrix */
        double lam = 0.0;
        int64_t r = k;
        for (int64_t i = k + 1; i < n; ++i)
            if (fabs(A[IDX(i, k, n)]) > lam) {
                lam = fabs(A[IDX(i, k, n)]);
                r = i;
            }
        const double akk = fabs(A[IDX(k, k, n)]);
        if (akk == 0.0 && lam == 0.0) {         /* zero row and column */
            counts[1] += 1;
            k += 1;
            continue;
        }
        int two = 0;
        if (akk < alpha * lam) {
            /* largest off-diagonal entry of row/column r of the trailing matrix */
            double sig = 0.0;
            for (int64_t j = k; j < n; ++j)
                if (j != r && fabs(lo_get(A, n, r, j)) > sig)
                    sig = fabs(lo_get(A, n, r, j));
            if (akk * sig >= alpha * lam * lam) {
                /* 1x1 pivot a_kk */
            } else if (fabs(A[IDX(r, r, n)]) >= alpha * sig) {
                lo_swap(A, n, k, k, r);         /* 1x1 pivot a_rr */
            } else {
                lo_swap(A, n, k, k + 1, r);     /* 2x2 pivot on rows k, r */
                two = 1;
            }
        }
        if (!two) {
            const double d = A[IDX(k, k, n)];
            counts[d > 0.0 ? 2 : (d < 0.0 ? 0 : 1)] += 1;
            for (int64_t i = k + 1; i < n; ++i)
                u[i] = A[IDX(i, k, n)];
            /* A22 -= u u^T / d on the lower triangle */
            for (int64_t i = k + 1; i < n; ++i) {
                const double li = u[i] / d;
                double *row = A + IDX(i, 0, n);
                for (int64_t j = k + 1; j <= i; ++j)
                    row[j] -= li * u[j];
            }
            k += 1;
        } else {
            const double a = A[IDX(k, k, n)], b = A[IDX(k + 1, k, n)];
            const double c = A[IDX(k + 1, k + 1, n)];
            const double det = a * c - b * b;
            if (det < 0.0) {
                counts[0] += 1;
                counts[2] += 1;
            } else if (det > 0.0) {
                counts[a + c > 0.0 ? 2 : 0] += 2;
            } else {
                counts[1] += 1;
                counts[a + c > 0.0 ? 2 : (a + c < 0.0 ? 0 : 1)] += 1;
            }
            for (int64_t i = k + 2; i < n; ++i) {
                u[i] = A[IDX(i, k, n)];
                w[i] = A[IDX(i, k + 1, n)];
            }
            /* A22 -= [u w] D^{-1} [u w]^T on the lower triangle */
            for (int64_t i = k + 2; i < n; ++i) {
                const double l1 = (c * u[i] - b * w[i]) / det;
                const double l2 = (a * w[i] - b * u[i]) / det;
                double *row = A + IDX(i, 0, n);
                for (int64_t j = k + 2; j <= i; ++j)
                    row[j] -= l1 * u[j] + l2 * w[j];
            }
            k += 2;
        }
    }
    free(u);
    free(w);
}

/* Inertia of Ri - sigma Li (Sec. 3.2, eq. generalized_eigenvalues_discrete, */
/* lambda = 1/tau).  Ri - sigma Li = G (C - sigma I) G^T with Li = G G^T, a   */
/* congruence, so counts[0] = #{lambda_n < sigma}, counts[1] = #{lambda_n =  */
/* sigma} (exact zeros only) and counts[2] = #{lambda_n > sigma}.  Without   */
/* electrodes the pencil is (R, L) itself and no reduction is formed.        */
/* Returns 0, or 1 if the electrode matrix is rank deficient.                */
int orc_inertia(const orc_problem *pb, double sigma, int64_t *counts)
{
    const int64_t n0 = pb->n - pb->m;
    double *A = (double *)malloc(sizeof(double) * (size_t)(n0 * n0));
    if (pb->m == 0) {
        for (int64_t a = 0; a < n0 * n0; ++a)
            A[a] = pb->R[a] - sigma * pb->L[a];
    } else {
        orc_reduced r;
        if (reduce(pb, &r)) {
            free_reduced(&r);
            free(A);
            return 1;
        }
        for (int64_t a = 0; a < n0 * n0; ++a)
            A[a] = r.Ri[a] - sigma * r.Li[a];
        free_reduced(&r);
    }
    orc_ldlt_inertia(n0, A, counts);
    free(A);
    return 0;
}
