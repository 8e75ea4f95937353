/*
 * lrpr_oracle.c -- plain, slow FP64 CPU oracle for Parareal with low-rank
 * coarse solvers (Gander, Ohlberger, Rave, arXiv 2508.08873).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * table or helper with the HIP library; the library never links it.
 *
 * Everything is double precision, written as the textbook loops in the
 * paper's order.  OpenMP is used only across independent right-hand-side
 * columns; every column's arithmetic is a plain sequential loop.
 *
 * Storage conventions (all owned by the caller):
 *   band   : n x (2b+1) row-major, band[i*(2b+1) + (j - i + b)] = M[i][j]
 *            for |i - j| <= b.  After ora_band_lu it holds L (strictly
 *            lower part, unit diagonal implied) and U (upper part incl.
 *            diagonal) in the same positions.
 *   X, Y.. : column-major, element (i, c) at X[i + c*ld].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define BAND(a, bw, i, j) (a)[(size_t)(i) * (size_t)(2 * (bw) + 1) + (size_t)((j) - (i) + (bw))]

static int imax(int a, int b) { return a > b ? a : b; }
static int imin(int a, int b) { return a < b ? a : b; }

/* ------------------------------------------------------------------------
 * Operator assembly (finite differences; homogeneous Dirichlet).
 *
 * The paper discretises with linear finite elements and backward Euler
 * (Sec. 4, first paragraph).  Here the spatial operator is the
 * finite-difference analogue of  -nu*Laplace(u) + beta.grad(u) + c*u  on the
 * unit interval / unit square with first-order upwinding, and the fine step
 * is implicit Euler, so one step solves  (I + dt*A) x_new = x_old + dt*f.
 *
 * 1D (dim=1): n = nx, h = 1/(nx+1), half-bandwidth b = 1.
 * 2D (dim=2): n = nx*nx, h = 1/(nx+1), index r = i + nx*j (x fastest),
 *             half-bandwidth b = nx.
 * Off-diagonal entries: -nu/h^2 - beta_plus/h  towards the upwind neighbour
 * (the west/south neighbour when the velocity component is positive),
 * -nu/h^2 - beta_minus/h towards the other one; the diagonal carries
 * 2*dim*nu/h^2 + sum_d |beta_d|/h + c.  Neighbours outside the domain are
 * dropped (zero boundary values).
 * Writes M = I + dt*A into band (n x (2b+1)); returns b.
 * ---------------------------------------------------------------------- */
int ora_assemble(int dim, int nx, double nu, double beta1, double beta2,
                 double c, double dt, double *band)
{
    const double h = 1.0 / (double)(nx + 1);
    const double dif = nu / (h * h);
    const double b1p = beta1 > 0 ? beta1 : 0.0, b1m = beta1 < 0 ? -beta1 : 0.0;
    const double b2p = beta2 > 0 ? beta2 : 0.0, b2m = beta2 < 0 ? -beta2 : 0.0;
    int n, bw;
    if (dim == 1) { n = nx; bw = 1; }
    else          { n = nx * nx; bw = nx; }
    memset(band, 0, sizeof(double) * (size_t)n * (size_t)(2 * bw + 1));
    if (dim == 1) {
        for (int i = 0; i < nx; i++) {
            double diag = 2.0 * dif + fabs(beta1) / h + c;
            BAND(band, bw, i, i) = 1.0 + dt * diag;
            if (i > 0)      BAND(band, bw, i, i - 1) = dt * (-dif - b1p / h);
            if (i < nx - 1) BAND(band, bw, i, i + 1) = dt * (-dif - b1m / h);
        }
    } else {
        for (int j = 0; j < nx; j++) {
            for (int i = 0; i < nx; i++) {
                int r = i + nx * j;
                double diag = 4.0 * dif + (fabs(beta1) + fabs(beta2)) / h + c;
                BAND(band, bw, r, r) = 1.0 + dt * diag;
                if (i > 0)      BAND(band, bw, r, r - 1)  = dt * (-dif - b1p / h);
                if (i < nx - 1) BAND(band, bw, r, r + 1)  = dt * (-dif - b1m / h);
                if (j > 0)      BAND(band, bw, r, r - nx) = dt * (-dif - b2p / h);
                if (j < nx - 1) BAND(band, bw, r, r + nx) = dt * (-dif - b2m / h);
            }
        }
    }
    return bw;
}

/* ------------------------------------------------------------------------
 * The same operator with homogeneous Neumann boundaries (the paper's variant
 * of its first experiment, Sec. 4): nx grid points per axis including both
 * boundary points, h = 1/(nx-1), x_i = i h.  The boundary condition is
 * imposed with a mirrored ghost point (u_{-1} = u_1, u_{nx} = u_{nx-2}), so
 * the coefficient of the missing neighbour moves onto the mirrored one.
 * Every row of A sums to c: constants are an eigenvector (the undamped
 * constant mode when c = 0).  Returns the half-bandwidth.
 * ------------------------------------------------------------------------ */
static void neumann_axis(int i, int nx, double dif, double beta, double h,
                         double *diag, double *lo, double *hi)
{
    const double bp = beta > 0 ? beta : 0.0, bm = beta < 0 ? -beta : 0.0;
    double left = -dif - bp / h, right = -dif - bm / h;
    *diag = 2.0 * dif + fabs(beta) / h;
    if (i == 0)      { right += left; left = 0.0; }
    if (i == nx - 1) { left += right; right = 0.0; }
    *lo = left;
    *hi = right;
}

int ora_assemble_neumann(int dim, int nx, double nu, double beta1, double beta2,
                         double c, double dt, double *band)
{
    const double h = 1.0 / (double)(nx - 1);
    const double dif = nu / (h * h);
    int n, bw;
    if (dim == 1) { n = nx; bw = 1; }
    else          { n = nx * nx; bw = nx; }
    memset(band, 0, sizeof(double) * (size_t)n * (size_t)(2 * bw + 1));
    if (dim == 1) {
        for (int i = 0; i < nx; i++) {
            double d, lo, hi;
            neumann_axis(i, nx, dif, beta1, h, &d, &lo, &hi);
            BAND(band, bw, i, i) = 1.0 + dt * (d + c);
            if (i > 0)      BAND(band, bw, i, i - 1) = dt * lo;
            if (i < nx - 1) BAND(band, bw, i, i + 1) = dt * hi;
        }
    } else {
        for (int j = 0; j < nx; j++) {
            for (int i = 0; i < nx; i++) {
                const int r = i + nx * j;
                double dx, lx, hx, dy, ly, hy;
                neumann_axis(i, nx, dif, beta1, h, &dx, &lx, &hx);
                neumann_axis(j, nx, dif, beta2, h, &dy, &ly, &hy);
                BAND(band, bw, r, r) = 1.0 + dt * (dx + dy + c);
                if (i > 0)      BAND(band, bw, r, r - 1)  = dt * lx;
                if (i < nx - 1) BAND(band, bw, r, r + 1)  = dt * hx;
                if (j > 0)      BAND(band, bw, r, r - nx) = dt * ly;
                if (j < nx - 1) BAND(band, bw, r, r + nx) = dt * hy;
            }
        }
    }
    return bw;
}

/* ------------------------------------------------------------------------
 * Banded LU without pivoting (Doolittle, right-looking, ascending loops).
 * The paper's fine solver factors the backward-Euler matrix with a direct
 * solver and reuses the factors for all right-hand sides of a step
 * (Sec. 4.4).  For each pivot q: L[i][q] = a[i][q]/a[q][q] and
 * a[i][j] -= L[i][q]*a[q][j] for rows and columns inside the band.
 * Returns 0, or q+1 if pivot q is zero or not finite.
 * ---------------------------------------------------------------------- */
int ora_band_lu(int n, int bw, double *band)
{
    for (int q = 0; q < n; q++) {
        double piv = BAND(band, bw, q, q);
        if (piv == 0.0 || !isfinite(piv)) return q + 1;
        int iend = imin(q + bw, n - 1);
        /* rows of one pivot step are independent: every entry still receives
         * its updates in pivot order (threads only for wide bands) */
#pragma omp parallel for schedule(static) if (bw >= 128)
        for (int i = q + 1; i <= iend; i++) {
            double lij = BAND(band, bw, i, q) / piv;
            BAND(band, bw, i, q) = lij;
            for (int j = q + 1; j <= imin(q + bw, n - 1); j++)
                BAND(band, bw, i, j) -= lij * BAND(band, bw, q, j);
        }
    }
    return 0;
}

/* Copy column-major X (n x w, ld) into row-major work W (n x w). */
static void to_rows(int n, int w, const double *X, long ld, double *W)
{
    for (int c = 0; c < w; c++)
        for (int i = 0; i < n; i++) W[(size_t)i * w + c] = X[i + (size_t)c * ld];
}
static void from_rows(int n, int w, const double *W, double *X, long ld)
{
    for (int c = 0; c < w; c++)
        for (int i = 0; i < n; i++) X[i + (size_t)c * ld] = W[(size_t)i * w + c];
}

/* One solve M x = r with M = LU, for the w columns of row-major W in place.
 * Forward substitution y_i = r_i - sum_{q=i-b}^{i-1} L[i][q] y_q (ascending),
 * back substitution x_i = (y_i - sum_{q=i+1}^{i+b} U[i][q] x_q) / U[i][i]
 * (descending i, ascending q). */
static void lu_solve_rows(int n, int bw, const double *lu, int w, double *W)
{
    for (int i = 0; i < n; i++) {
        double *yi = W + (size_t)i * w;
        for (int q = imax(0, i - bw); q < i; q++) {
            const double l = BAND(lu, bw, i, q);
            const double *yq = W + (size_t)q * w;
            for (int c = 0; c < w; c++) yi[c] -= l * yq[c];
        }
    }
    for (int i = n - 1; i >= 0; i--) {
        double *xi = W + (size_t)i * w;
        for (int q = i + 1; q <= imin(n - 1, i + bw); q++) {
            const double u = BAND(lu, bw, i, q);
            const double *xq = W + (size_t)q * w;
            for (int c = 0; c < w; c++) xi[c] -= u * xq[c];
        }
        const double d = BAND(lu, bw, i, i);
        for (int c = 0; c < w; c++) xi[c] /= d;
    }
}

/* One solve M^T z = x with M = LU, i.e. U^T (L^T z) = x:
 * forward with U^T: t_i = (x_i - sum_{q<i} U[q][i] t_q) / U[i][i] (ascending),
 * back with L^T:    z_i = t_i - sum_{q>i} L[q][i] z_q (descending). */
static void lu_solve_t_rows(int n, int bw, const double *lu, int w, double *W)
{
    for (int i = 0; i < n; i++) {
        double *ti = W + (size_t)i * w;
        for (int q = imax(0, i - bw); q < i; q++) {
            const double u = BAND(lu, bw, q, i);
            const double *tq = W + (size_t)q * w;
            for (int c = 0; c < w; c++) ti[c] -= u * tq[c];
        }
        const double d = BAND(lu, bw, i, i);
        for (int c = 0; c < w; c++) ti[c] /= d;
    }
    for (int i = n - 1; i >= 0; i--) {
        double *zi = W + (size_t)i * w;
        for (int q = i + 1; q <= imin(n - 1, i + bw); q++) {
            const double l = BAND(lu, bw, q, i);
            const double *zq = W + (size_t)q * w;
            for (int c = 0; c < w; c++) zi[c] -= l * zq[c];
        }
    }
}

#define COLS_PER_TASK 8

/* ------------------------------------------------------------------------
 * Fine propagator: m implicit-Euler steps for each of the w columns of X.
 * Step j (0-based) solves (I + dt*A) x_{j+1} = x_j + dt * f(t_{j+1}), with
 * the source of column c equal to fscale[c*m + j] * f[:, fcol[c]] (fcol[c] < 0
 * or f == NULL: no source).  This is F_n (Sec. 2, the affine fine solver);
 * with no source it is the linear part F_n' = T_n = M^{-m}.
 * ---------------------------------------------------------------------- */
void ora_fine_steps(int n, int bw, const double *lu, double dt, int m,
                    double *X, long ldx, int w,
                    const double *f, long ldf, const int *fcol, const double *fscale)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int c0 = 0; c0 < w; c0 += COLS_PER_TASK) {
        int wc = imin(COLS_PER_TASK, w - c0);
        double *W = (double *)malloc(sizeof(double) * (size_t)n * wc);
        to_rows(n, wc, X + (size_t)c0 * ldx, ldx, W);
        for (int j = 0; j < m; j++) {
            if (f) {
                for (int c = 0; c < wc; c++) {
                    int fc = fcol ? fcol[c0 + c] : 0;
                    if (fc < 0) continue;
                    double s = dt * (fscale ? fscale[(size_t)(c0 + c) * m + j] : 1.0);
                    const double *fv = f + (size_t)fc * ldf;
                    for (int i = 0; i < n; i++) W[(size_t)i * wc + c] += s * fv[i];
                }
            }
            lu_solve_rows(n, bw, lu, wc, W);
        }
        from_rows(n, wc, W, X + (size_t)c0 * ldx, ldx);
        free(W);
    }
}

/* Adjoint of the source-free fine propagator: X <- (M^T)^{-m} X = T_n^T X.
 * (Sec. 2.1 step 3; the Euclidean inner product makes the adjoint the
 * transpose.) */
void ora_adjoint_steps(int n, int bw, const double *lu, int m,
                       double *X, long ldx, int w)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int c0 = 0; c0 < w; c0 += COLS_PER_TASK) {
        int wc = imin(COLS_PER_TASK, w - c0);
        double *W = (double *)malloc(sizeof(double) * (size_t)n * wc);
        to_rows(n, wc, X + (size_t)c0 * ldx, ldx, W);
        for (int j = 0; j < m; j++) lu_solve_t_rows(n, bw, lu, wc, W);
        from_rows(n, wc, W, X + (size_t)c0 * ldx, ldx);
        free(W);
    }
}

/* ------------------------------------------------------------------------
 * Thin Householder QR of Y (n x l, column-major, n >= l): Y = Q R with Q
 * n x l orthonormal columns and R l x l upper triangular, normalised so
 * that R[j][j] >= 0.  This provides the orthonormal bases of steps 2 and 4
 * of the randomized SVD (Sec. 2.1).
 * Q: n x l (ld n), R: l x l (ld l).  Returns 0.
 * ---------------------------------------------------------------------- */
int ora_householder_qr(int n, int l, const double *Y, long ldy, double *Q, double *R)
{
    double *A = (double *)malloc(sizeof(double) * (size_t)n * l);
    double *V = (double *)calloc((size_t)n * l, sizeof(double)); /* reflectors */
    double *beta = (double *)calloc((size_t)l, sizeof(double));
    for (int c = 0; c < l; c++) memcpy(A + (size_t)c * n, Y + (size_t)c * ldy, sizeof(double) * n);
    for (int j = 0; j < l; j++) {
        double *a = A + (size_t)j * n;
        double nrm2 = 0.0;
        for (int i = j; i < n; i++) nrm2 += a[i] * a[i];
        double nrm = sqrt(nrm2);
        double *v = V + (size_t)j * n;
        if (nrm == 0.0) { beta[j] = 0.0; continue; }
        double alpha = a[j] >= 0 ? -nrm : nrm;      /* H a = alpha e_j */
        for (int i = j; i < n; i++) v[i] = a[i];
        v[j] -= alpha;
        double vv = 0.0;
        for (int i = j; i < n; i++) vv += v[i] * v[i];
        beta[j] = vv > 0 ? 2.0 / vv : 0.0;
        /* apply H = I - beta v v^T to columns j..l-1 */
        for (int c = j; c < l; c++) {
            double *ac = A + (size_t)c * n;
            double s = 0.0;
            for (int i = j; i < n; i++) s += v[i] * ac[i];
            s *= beta[j];
            for (int i = j; i < n; i++) ac[i] -= s * v[i];
        }
    }
    /* R = upper triangle of A */
    for (int c = 0; c < l; c++)
        for (int r = 0; r < l; r++) R[r + (size_t)c * l] = (r <= c) ? A[r + (size_t)c * n] : 0.0;
    /* Q = H_0 H_1 ... H_{l-1} [I_l; 0], applied right to left */
    for (int c = 0; c < l; c++) {
        double *qc = Q + (size_t)c * n;
        memset(qc, 0, sizeof(double) * n);
        qc[c] = 1.0;
    }
    for (int j = l - 1; j >= 0; j--) {
        const double *v = V + (size_t)j * n;
        if (beta[j] == 0.0) continue;
        for (int c = 0; c < l; c++) {
            double *qc = Q + (size_t)c * n;
            double s = 0.0;
            for (int i = j; i < n; i++) s += v[i] * qc[i];
            s *= beta[j];
            for (int i = j; i < n; i++) qc[i] -= s * v[i];
        }
    }
    /* sign normalisation: R[j][j] >= 0 */
    for (int j = 0; j < l; j++) {
        if (R[j + (size_t)j * l] < 0) {
            for (int c = j; c < l; c++) R[j + (size_t)c * l] = -R[j + (size_t)c * l];
            double *qj = Q + (size_t)j * n;
            for (int i = 0; i < n; i++) qj[i] = -qj[i];
        }
    }
    free(A); free(V); free(beta);
    return 0;
}

/* ------------------------------------------------------------------------
 * One-sided (Hestenes) Jacobi SVD of a square l x l matrix Mm (column-major):
 * Mm = U diag(S) V^T, S sorted descending.  Plane rotations orthogonalise
 * pairs of columns until every pair satisfies
 * |a_p.a_q| <= l*eps*||a_p||*||a_q||; then S_j = ||a_j||, U_j = a_j/S_j.
 * This is the small SVD of step 5 of the randomized SVD (Sec. 2.1).
 * Returns the number of sweeps, or -1 if not converged after 100 sweeps.
 * ---------------------------------------------------------------------- */
int ora_jacobi_svd(int l, const double *Mm, double *U, double *S, double *V)
{
    double *A = (double *)malloc(sizeof(double) * (size_t)l * l);
    double *Vw = (double *)malloc(sizeof(double) * (size_t)l * l);
    memcpy(A, Mm, sizeof(double) * (size_t)l * l);
    for (int c = 0; c < l; c++)
        for (int r = 0; r < l; r++) Vw[r + (size_t)c * l] = (r == c) ? 1.0 : 0.0;
    const double tol = (double)l * 2.220446049250313e-16;
    int sweeps = 0, converged = 0;
    while (!converged && sweeps < 100) {
        converged = 1;
        sweeps++;
        for (int p = 0; p < l - 1; p++) {
            for (int q = p + 1; q < l; q++) {
                double *ap = A + (size_t)p * l, *aq = A + (size_t)q * l;
                double alpha = 0, beta = 0, gamma = 0;
                for (int i = 0; i < l; i++) {
                    alpha += ap[i] * ap[i];
                    beta += aq[i] * aq[i];
                    gamma += ap[i] * aq[i];
                }
                if (fabs(gamma) <= tol * sqrt(alpha * beta) || gamma == 0.0) continue;
                converged = 0;
                double zeta = (beta - alpha) / (2.0 * gamma);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                for (int i = 0; i < l; i++) {
                    double x = ap[i], y = aq[i];
                    ap[i] = cs * x - sn * y;
                    aq[i] = sn * x + cs * y;
                }
                double *vp = Vw + (size_t)p * l, *vq = Vw + (size_t)q * l;
                for (int i = 0; i < l; i++) {
                    double x = vp[i], y = vq[i];
                    vp[i] = cs * x - sn * y;
                    vq[i] = sn * x + cs * y;
                }
            }
        }
    }
    /* column norms, then selection sort by descending norm */
    double *nrm = (double *)malloc(sizeof(double) * l);
    int *ord = (int *)malloc(sizeof(int) * l);
    for (int c = 0; c < l; c++) {
        double s = 0;
        for (int i = 0; i < l; i++) s += A[i + (size_t)c * l] * A[i + (size_t)c * l];
        nrm[c] = sqrt(s);
        ord[c] = c;
    }
    for (int a = 0; a < l; a++) {
        int best = a;
        for (int b = a + 1; b < l; b++) if (nrm[ord[b]] > nrm[ord[best]]) best = b;
        int tmp = ord[a]; ord[a] = ord[best]; ord[best] = tmp;
    }
    for (int a = 0; a < l; a++) {
        int c = ord[a];
        S[a] = nrm[c];
        for (int i = 0; i < l; i++) {
            U[i + (size_t)a * l] = nrm[c] > 0 ? A[i + (size_t)c * l] / nrm[c] : 0.0;
            V[i + (size_t)a * l] = Vw[i + (size_t)c * l];
        }
    }
    free(A); free(Vw); free(nrm); free(ord);
    return converged ? sweeps : -1;
}

/* C = A * B with A: m x k (lda), B: k x nc (ldb), C: m x nc (ldc), col-major */
static void matmul(int m, int k, int nc, const double *A, long lda,
                   const double *B, long ldb, double *C, long ldc)
{
    #pragma omp parallel for schedule(static)
    for (int c = 0; c < nc; c++) {
        double *cc = C + (size_t)c * ldc;
        for (int i = 0; i < m; i++) cc[i] = 0.0;
        for (int q = 0; q < k; q++) {
            double bq = B[q + (size_t)c * ldb];
            const double *aq = A + (size_t)q * lda;
            for (int i = 0; i < m; i++) cc[i] += aq[i] * bq;
        }
    }
}

/* ------------------------------------------------------------------------
 * Randomized SVD of the transfer operator T = M^{-m} of one slice
 * (Sec. 2.1, steps 1-6), with l = k + p test vectors Omega (n x l):
 *   Y = T Omega;  Y = Q R (Householder);  Z = T^T Q;  Z = Qz Rz;
 *   small matrix Mm = Rz^T, whose (i,j) entry is (T^T w_i, v_j);
 *   Mm = Uh diag(S) Vh^T (Jacobi);  Uk = Q Uh[:, :k],  Vk = Qz Vh[:, :k].
 * The left singular vectors are combinations of the range basis Q and the
 * right ones of the co-range basis Qz, since T ~ Q Q^T T = Q Mm Qz^T.
 * Signs: each pair (Uk[:,r], Vk[:,r]) is flipped jointly so that the entry
 * of Uk[:,r] with the largest magnitude (lowest index on ties) is positive.
 * Outputs: Uk, Vk: n x k (ld n); S: all l singular values of Mm.
 * Returns Jacobi sweep count (or -1).
 *
 * Power iterations (Sec. 2.1, for slowly decaying singular values): with
 * q >= 1 the range space is W = span (T T^T)^q T Omega.  It is reached by q
 * rounds of "orthonormalise, apply T^T, orthonormalise, apply T" after step
 * 1, so that the small directions are not lost to rounding; steps 2-6 then
 * run on the final Y.
 * ---------------------------------------------------------------------- */
int ora_rsvd_q(int n, int bw, const double *lu, int m, int k, int p, int q,
               const double *Omega, long ldo, double *Uk, double *S, double *Vk);

int ora_rsvd(int n, int bw, const double *lu, int m, int k, int p,
             const double *Omega, long ldo, double *Uk, double *S, double *Vk)
{
    return ora_rsvd_q(n, bw, lu, m, k, p, 0, Omega, ldo, Uk, S, Vk);
}

int ora_rsvd_q(int n, int bw, const double *lu, int m, int k, int p, int q,
               const double *Omega, long ldo, double *Uk, double *S, double *Vk)
{
    const int l = k + p;
    double *Y = (double *)malloc(sizeof(double) * (size_t)n * l);
    double *Q = (double *)malloc(sizeof(double) * (size_t)n * l);
    double *Qz = (double *)malloc(sizeof(double) * (size_t)n * l);
    double *R = (double *)malloc(sizeof(double) * (size_t)l * l);
    double *Mm = (double *)malloc(sizeof(double) * (size_t)l * l);
    double *Uh = (double *)malloc(sizeof(double) * (size_t)l * l);
    double *Vh = (double *)malloc(sizeof(double) * (size_t)l * l);
    for (int c = 0; c < l; c++) memcpy(Y + (size_t)c * n, Omega + (size_t)c * ldo, sizeof(double) * n);
    ora_fine_steps(n, bw, lu, 0.0, m, Y, n, l, NULL, 0, NULL, NULL);     /* step 1 */
    for (int it = 0; it < q; it++) {                                      /* power iterations */
        ora_householder_qr(n, l, Y, n, Q, R);
        memcpy(Y, Q, sizeof(double) * (size_t)n * l);
        ora_adjoint_steps(n, bw, lu, m, Y, n, l);                         /* T^T Q */
        ora_householder_qr(n, l, Y, n, Qz, R);
        memcpy(Y, Qz, sizeof(double) * (size_t)n * l);
        ora_fine_steps(n, bw, lu, 0.0, m, Y, n, l, NULL, 0, NULL, NULL);  /* T Qz */
    }
    ora_householder_qr(n, l, Y, n, Q, R);                                /* step 2 */
    memcpy(Y, Q, sizeof(double) * (size_t)n * l);
    ora_adjoint_steps(n, bw, lu, m, Y, n, l);                             /* step 3 */
    ora_householder_qr(n, l, Y, n, Qz, R);                               /* step 4 */
    for (int i = 0; i < l; i++)
        for (int j = 0; j < l; j++) Mm[i + (size_t)j * l] = R[j + (size_t)i * l];
    int sw = ora_jacobi_svd(l, Mm, Uh, S, Vh);                            /* step 5 */
    matmul(n, l, k, Q, n, Uh, l, Uk, n);                                  /* step 6 */
    matmul(n, l, k, Qz, n, Vh, l, Vk, n);
    for (int r = 0; r < k; r++) {
        double *u = Uk + (size_t)r * n, *v = Vk + (size_t)r * n;
        int im = 0;
        for (int i = 1; i < n; i++) if (fabs(u[i]) > fabs(u[im])) im = i;
        if (u[im] < 0) {
            for (int i = 0; i < n; i++) { u[i] = -u[i]; v[i] = -v[i]; }
        }
    }
    free(Y); free(Q); free(Qz); free(R); free(Mm); free(Uh); free(Vh);
    return sw;
}

/* ------------------------------------------------------------------------
 * Randomized SVD with the adjoint evaluated on independent test vectors
 * (Sec. 2.2: more parallelism at some loss of accuracy, the two-sided
 * sketch).  Reading: Psi (n x l) is a second Gaussian matrix drawn
 * independently of Omega, so Z = T^T Psi does not wait for the range basis;
 * with Q the orthonormal basis of Y = T Omega, the approximation is
 *   T ~ Q X,  X = (Psi^T Q)^{-1} Psi^T T = (Psi^T Q)^{-1} Z^T,
 * i.e. the operator that agrees with Q Q^T T on the test space Psi.  Its
 * truncated SVD: X^T = Qx Rx (Householder), Q X = Q Rx^T Qx^T, and
 * Rx^T = Uh diag(S) Vh^T (Jacobi);  Uk = Q Uh[:, :k],  Vk = Qx Vh[:, :k].
 * X^T = Z (Psi^T Q)^{-T} is formed by Gaussian elimination with partial
 * pivoting on (Psi^T Q)^T.  Signs as in ora_rsvd.  Returns the Jacobi sweep
 * count, -1 if Jacobi did not converge, -2 if Psi^T Q is singular.
 * ---------------------------------------------------------------------- */
int ora_rsvd_two_sided(int n, int bw, const double *lu, int m, int k, int p,
                       const double *Omega, const double *Psi, long ld,
                       double *Uk, double *S, double *Vk)
{
    const int l = k + p;
    double *Y = (double *)malloc(sizeof(double) * (size_t)n * l);
    double *Z = (double *)malloc(sizeof(double) * (size_t)n * l);
    double *Q = (double *)malloc(sizeof(double) * (size_t)n * l);
    double *Qx = (double *)malloc(sizeof(double) * (size_t)n * l);
    double *C = (double *)malloc(sizeof(double) * (size_t)l * l);
    double *R = (double *)malloc(sizeof(double) * (size_t)l * l);
    double *Mm = (double *)malloc(sizeof(double) * (size_t)l * l);
    double *Uh = (double *)malloc(sizeof(double) * (size_t)l * l);
    double *Vh = (double *)malloc(sizeof(double) * (size_t)l * l);
    int *piv = (int *)malloc(sizeof(int) * (size_t)l);
    int ret = 0;
    for (int c = 0; c < l; c++) {
        memcpy(Y + (size_t)c * n, Omega + (size_t)c * ld, sizeof(double) * n);
        memcpy(Z + (size_t)c * n, Psi + (size_t)c * ld, sizeof(double) * n);
    }
    ora_fine_steps(n, bw, lu, 0.0, m, Y, n, l, NULL, 0, NULL, NULL);     /* Y = T Omega */
    ora_adjoint_steps(n, bw, lu, m, Z, n, l);                             /* Z = T^T Psi */
    ora_householder_qr(n, l, Y, n, Q, R);                                /* Y = Q R */
    /* Ct = (Psi^T Q)^T = Q^T Psi, column-major l x l: Ct[i + j l] = q_i . psi_j */
    for (int i = 0; i < l; i++)
        for (int j = 0; j < l; j++) {
            double acc = 0.0;
            for (int r = 0; r < n; r++) acc += Q[r + (size_t)i * n] * Psi[r + (size_t)j * ld];
            C[i + (size_t)j * l] = acc;
        }
    /* LU with partial pivoting of Ct: Ct = P^T L U (in place) */
    for (int c = 0; c < l && ret == 0; c++) {
        int pr = c;
        for (int r = c + 1; r < l; r++) if (fabs(C[r + (size_t)c * l]) > fabs(C[pr + (size_t)c * l])) pr = r;
        piv[c] = pr;
        if (C[pr + (size_t)c * l] == 0.0) { ret = -2; break; }
        if (pr != c)
            for (int j = 0; j < l; j++) {
                const double t = C[c + (size_t)j * l];
                C[c + (size_t)j * l] = C[pr + (size_t)j * l];
                C[pr + (size_t)j * l] = t;
            }
        for (int r = c + 1; r < l; r++) {
            C[r + (size_t)c * l] /= C[c + (size_t)c * l];
            for (int j = c + 1; j < l; j++) C[r + (size_t)j * l] -= C[r + (size_t)c * l] * C[c + (size_t)j * l];
        }
    }
    if (ret == 0) {
        /* X^T = Z Ct^{-1}: row z of Z gives x with Ct^T... solve x Ct = z, i.e. Ct^T x^T = z^T.
         * With Ct = P^T L U: Ct^T = U^T L^T P, so solve U^T w = z^T, L^T v = w, x^T = P^T v. */
        double *w = (double *)malloc(sizeof(double) * (size_t)l);
        for (int r = 0; r < n; r++) {
            for (int i = 0; i < l; i++) {                 /* U^T w = z (forward, U^T lower) */
                double v = Z[r + (size_t)i * n];
                for (int j = 0; j < i; j++) v -= C[j + (size_t)i * l] * w[j];
                w[i] = v / C[i + (size_t)i * l];
            }
            for (int i = l - 1; i >= 0; i--) {            /* L^T v = w (backward, unit diagonal) */
                double v = w[i];
                for (int j = i + 1; j < l; j++) v -= C[j + (size_t)i * l] * w[j];
                w[i] = v;
            }
            for (int i = l - 1; i >= 0; i--) {            /* undo the row swaps: x = P^T v */
                const double t = w[i];
                w[i] = w[piv[i]];
                w[piv[i]] = t;
            }
            for (int i = 0; i < l; i++) Z[r + (size_t)i * n] = w[i];
        }
        free(w);
        ora_householder_qr(n, l, Z, n, Qx, R);                           /* X^T = Qx Rx */
        for (int i = 0; i < l; i++)
            for (int j = 0; j < l; j++) Mm[i + (size_t)j * l] = R[j + (size_t)i * l];
        ret = ora_jacobi_svd(l, Mm, Uh, S, Vh);                           /* Rx^T = Uh S Vh^T */
        matmul(n, l, k, Q, n, Uh, l, Uk, n);
        matmul(n, l, k, Qx, n, Vh, l, Vk, n);
        for (int r = 0; r < k; r++) {
            double *u = Uk + (size_t)r * n, *v = Vk + (size_t)r * n;
            int im = 0;
            for (int i = 1; i < n; i++) if (fabs(u[i]) > fabs(u[im])) im = i;
            if (u[im] < 0) {
                for (int i = 0; i < n; i++) { u[i] = -u[i]; v[i] = -v[i]; }
            }
        }
    }
    free(Y); free(Z); free(Q); free(Qx); free(C); free(R); free(Mm); free(Uh); free(Vh); free(piv);
    return ret;
}

/* ------------------------------------------------------------------------
 * Linear part of the low-rank coarse solver, Sec. 2 (definition of G_n):
 * out = Uk (S .* (Vk^T v)) for w vectors v (columns of Vin); k inner
 * products followed by a combination of k vectors (Sec. 2.2, last
 * paragraph).  Uk, Vk: n x k (ld n); Vin, Out: n x w (ld n).
 * ---------------------------------------------------------------------- */
void ora_lowrank_apply(int n, int k, const double *Uk, const double *S,
                       const double *Vk, int w, const double *Vin, double *Out)
{
    double *coef = (double *)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
    for (int c = 0; c < w; c++) {
        const double *v = Vin + (size_t)c * n;
        double *o = Out + (size_t)c * n;
        for (int r = 0; r < k; r++) {
            double s = 0.0;
            const double *vr = Vk + (size_t)r * n;
            for (int i = 0; i < n; i++) s += vr[i] * v[i];
            coef[r] = S[r] * s;
        }
        for (int i = 0; i < n; i++) o[i] = 0.0;
        for (int r = 0; r < k; r++) {
            const double *ur = Uk + (size_t)r * n;
            for (int i = 0; i < n; i++) o[i] += ur[i] * coef[r];
        }
    }
    free(coef);
}
