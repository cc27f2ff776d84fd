/*
 * Geometric multigrid on (I - alpha L_h) u = b for the oracle
 * (TEST INFRASTRUCTURE ONLY).  Included twice by mg.c: once with
 * REAL=double / SFX=or (FP64) and once with REAL=float / SFX=orf (the FP32
 * inner solver of the mixed-precision form).
 *
 * The V-cycle follows the paper's multigrid description (Sec. 4.1.1 and
 * Sec. 4.2.1): linear interpolation, full-weighting restriction, pre- and
 * post-smoothing.  Readings where the paper is silent: the coarse operator
 * is re-discretised (I - alpha L_2h, same alpha); coarsening continues
 * while the grid has n >= 3 odd points per dimension and n in {1,2} is
 * solved exactly.
 */
#define CAT2_(a, b) a##b
#define CAT_(a, b) CAT2_(a, b)
#define FN(name) CAT_(SFX, name)

/* u at 0-based (i,j,k) with zero outside the interior. */
static inline REAL FN(_at)(const REAL *u, int n, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i >= n || j >= n || k >= n) return (REAL)0;
    return u[(size_t)i + (size_t)n * ((size_t)j + (size_t)n * (size_t)k)];
}

/* Sum over dimensions of the 3-point second difference (not yet divided
 * by h^2) at 0-based point (i,j,k). */
static inline REAL FN(_d2)(int dim, int n, const REAL *u, int i, int j, int k)
{
    REAL c = FN(_at)(u, n, i, j, k);
    REAL s = FN(_at)(u, n, i - 1, j, k) - 2 * c + FN(_at)(u, n, i + 1, j, k);
    if (dim >= 2) s += FN(_at)(u, n, i, j - 1, k) - 2 * c + FN(_at)(u, n, i, j + 1, k);
    if (dim >= 3) s += FN(_at)(u, n, i, j, k - 1) - 2 * c + FN(_at)(u, n, i, j, k + 1);
    return s;
}

static inline size_t FN(_len)(int dim, int n)
{
    size_t l = 1;
    for (int d = 0; d < dim; ++d) l *= (size_t)n;
    return l;
}

#define NY_(dim, n) ((dim) >= 2 ? (n) : 1)
#define NZ_(dim, n) ((dim) >= 3 ? (n) : 1)

void FN(_resid)(int dim, int n, double alpha, const REAL *b, const REAL *u, REAL *r)
{
    const REAL ah = (REAL)(alpha * (double)(n + 1) * (double)(n + 1));
    const int ny = NY_(dim, n), nz = NZ_(dim, n);
#pragma omp parallel for schedule(static) if (nz > 8)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < n; ++i) {
                size_t x = (size_t)i + (size_t)n * ((size_t)j + (size_t)n * (size_t)k);
                REAL hu = u[x] - ah * FN(_d2)(dim, n, u, i, j, k);
                r[x] = b[x] - hu;
            }
}

/* Weighted Jacobi: u <- u + omega (b - H u) / diag(H).
 * Red-black: the same update applied first to red points, then to black
 * points, each colour seeing the latest values of the other. */
void FN(_smooth)(int dim, int n, double alpha, int smoother, double omega,
                 const REAL *b, REAL *u)
{
    const REAL ah = (REAL)(alpha * (double)(n + 1) * (double)(n + 1));
    const REAL diag = (REAL)(1.0 + 2.0 * dim * alpha * (double)(n + 1) * (double)(n + 1));
    const REAL w = (REAL)omega;
    const int ny = NY_(dim, n), nz = NZ_(dim, n);
    const size_t len = FN(_len)(dim, n);
    if (smoother == OR_JACOBI) {
        REAL *r = (REAL *)malloc(len * sizeof(REAL));
        FN(_resid)(dim, n, alpha, b, u, r);
#pragma omp parallel for schedule(static) if (len > 4096)
        for (size_t x = 0; x < len; ++x) u[x] = u[x] + w * r[x] / diag;
        free(r);
        return;
    }
    for (int colour = 0; colour < 2; ++colour) {     /* 0 red, 1 black */
#pragma omp parallel for schedule(static) if (nz > 8)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < n; ++i) {
                    /* 1-based index sum; red when even */
                    int sum1 = (i + 1) + (dim >= 2 ? j + 1 : 0) + (dim >= 3 ? k + 1 : 0);
                    if ((sum1 & 1) != colour) continue;
                    size_t x = (size_t)i + (size_t)n * ((size_t)j + (size_t)n * (size_t)k);
                    REAL hu = u[x] - ah * FN(_d2)(dim, n, u, i, j, k);
                    u[x] = u[x] + w * (b[x] - hu) / diag;
                }
    }
}

/* Full weighting: coarse point J (1-based) sits on fine point 2J; weights
 * (1/4, 1/2, 1/4) in each dimension. */
void FN(_restrict_fw)(int dim, int n, const REAL *r, REAL *bc)
{
    const int nc = (n + 1) / 2 - 1;
    const int ncy = NY_(dim, nc), ncz = NZ_(dim, nc);
    const REAL w1[3] = {(REAL)0.25, (REAL)0.5, (REAL)0.25};
#pragma omp parallel for schedule(static) if (ncz > 8)
    for (int K = 0; K < ncz; ++K)
        for (int J = 0; J < ncy; ++J)
            for (int I = 0; I < nc; ++I) {
                /* 0-based fine centre: 1-based 2(I+1) -> 0-based 2I+1 */
                int fi = 2 * I + 1, fj = (dim >= 2) ? 2 * J + 1 : 0, fk = (dim >= 3) ? 2 * K + 1 : 0;
                REAL acc = 0;
                for (int oz = (dim >= 3 ? -1 : 0); oz <= (dim >= 3 ? 1 : 0); ++oz)
                    for (int oy = (dim >= 2 ? -1 : 0); oy <= (dim >= 2 ? 1 : 0); ++oy)
                        for (int ox = -1; ox <= 1; ++ox) {
                            REAL w = w1[ox + 1];
                            if (dim >= 2) w *= w1[oy + 1];
                            if (dim >= 3) w *= w1[oz + 1];
                            acc += w * FN(_at)(r, n, fi + ox, fj + oy, fk + oz);
                        }
                bc[(size_t)I + (size_t)nc * ((size_t)J + (size_t)nc * (size_t)K)] = acc;
            }
}

/* d-linear interpolation with zero boundary: fine 1-based index i takes
 * coarse value i/2 when even, the mean of (i-1)/2 and (i+1)/2 when odd. */
void FN(_prolong_add)(int dim, int nc, const REAL *ec, REAL *u)
{
    const int n = 2 * (nc + 1) - 1;
    const int ny = NY_(dim, n), nz = NZ_(dim, n);
#pragma omp parallel for schedule(static) if (nz > 8)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < n; ++i) {
                int idx1[3] = {i + 1, j + 1, k + 1};
                int lo[3], hi[3];
                REAL wl[3], wh[3];
                for (int d = 0; d < 3; ++d) {
                    if (d >= dim) { lo[d] = hi[d] = 1; wl[d] = 1; wh[d] = 0; continue; }
                    if ((idx1[d] & 1) == 0) { lo[d] = hi[d] = idx1[d] / 2; wl[d] = 1; wh[d] = 0; }
                    else { lo[d] = (idx1[d] - 1) / 2; hi[d] = (idx1[d] + 1) / 2; wl[d] = (REAL)0.5; wh[d] = (REAL)0.5; }
                }
                REAL acc = 0;
                for (int cz = 0; cz < 2; ++cz)
                    for (int cy = 0; cy < 2; ++cy)
                        for (int cx = 0; cx < 2; ++cx) {
                            REAL w = (cx ? wh[0] : wl[0]) * (cy ? wh[1] : wl[1]) * (cz ? wh[2] : wl[2]);
                            if (w == 0) continue;
                            int I = cx ? hi[0] : lo[0], J = cy ? hi[1] : lo[1], K = cz ? hi[2] : lo[2];
                            /* 1-based coarse indices 0 and nc+1 are boundary zeros */
                            REAL v = FN(_at)(ec, nc, I - 1, dim >= 2 ? J - 1 : 0, dim >= 3 ? K - 1 : 0);
                            acc += w * v;
                        }
                size_t x = (size_t)i + (size_t)n * ((size_t)j + (size_t)n * (size_t)k);
                u[x] += acc;
            }
}

/* Exact solve on n in {1,2}: assemble the dense (I - alpha L_h) column by
 * column and eliminate with partial pivoting (in double). */
void FN(_coarsest)(int dim, int n, double alpha, const REAL *b, REAL *u)
{
    const int len = (int)FN(_len)(dim, n);
    double A[64 * 64], rhs[64];
    const double ah = alpha * (double)(n + 1) * (double)(n + 1);
    for (int c = 0; c < len; ++c) {
        double e[64] = {0};
        e[c] = 1.0;
        for (int r = 0; r < len; ++r) {
            int i = r % n, j = (dim >= 2) ? (r / n) % n : 0, k = (dim >= 3) ? r / (n * n) : 0;
            double s = 0, cc = e[r];
            /* second difference of the unit vector e at point r */
#define EAT(ii, jj, kk) (((ii) < 0 || (jj) < 0 || (kk) < 0 || (ii) >= n || (jj) >= n || (kk) >= n) ? 0.0 : e[(ii) + n * ((jj) + n * (kk))])
            s = EAT(i - 1, j, k) - 2 * cc + EAT(i + 1, j, k);
            if (dim >= 2) s += EAT(i, j - 1, k) - 2 * cc + EAT(i, j + 1, k);
            if (dim >= 3) s += EAT(i, j, k - 1) - 2 * cc + EAT(i, j, k + 1);
#undef EAT
            A[r * len + c] = cc - ah * s;
        }
    }
    for (int r = 0; r < len; ++r) rhs[r] = (double)b[r];
    for (int c = 0; c < len; ++c) {
        int piv = c;
        for (int r = c + 1; r < len; ++r)
            if (fabs(A[r * len + c]) > fabs(A[piv * len + c])) piv = r;
        if (piv != c) {
            for (int q = 0; q < len; ++q) { double t = A[c * len + q]; A[c * len + q] = A[piv * len + q]; A[piv * len + q] = t; }
            double t = rhs[c]; rhs[c] = rhs[piv]; rhs[piv] = t;
        }
        for (int r = c + 1; r < len; ++r) {
            double f = A[r * len + c] / A[c * len + c];
            for (int q = c; q < len; ++q) A[r * len + q] -= f * A[c * len + q];
            rhs[r] -= f * rhs[c];
        }
    }
    for (int r = len - 1; r >= 0; --r) {
        double s = rhs[r];
        for (int q = r + 1; q < len; ++q) s -= A[r * len + q] * rhs[q];
        rhs[r] = s / A[r * len + r];
    }
    for (int r = 0; r < len; ++r) u[r] = (REAL)rhs[r];
}

void FN(_vcycle)(int dim, int n, double alpha, int smoother, double omega,
                 int nu1, int nu2, const REAL *b, REAL *u)
{
    if (n <= 2) {
        FN(_coarsest)(dim, n, alpha, b, u);
        return;
    }
    const size_t len = FN(_len)(dim, n);
    const int nc = (n + 1) / 2 - 1;
    const size_t lenc = FN(_len)(dim, nc);
    for (int s = 0; s < nu1; ++s) FN(_smooth)(dim, n, alpha, smoother, omega, b, u);
    REAL *r = (REAL *)malloc(len * sizeof(REAL));
    REAL *bc = (REAL *)malloc(lenc * sizeof(REAL));
    REAL *ec = (REAL *)calloc(lenc, sizeof(REAL));
    FN(_resid)(dim, n, alpha, b, u, r);
    FN(_restrict_fw)(dim, n, r, bc);
    FN(_vcycle)(dim, nc, alpha, smoother, omega, nu1, nu2, bc, ec);
    FN(_prolong_add)(dim, nc, ec, u);
    free(r);
    free(bc);
    free(ec);
    for (int s = 0; s < nu2; ++s) FN(_smooth)(dim, n, alpha, smoother, omega, b, u);
}

#undef NY_
#undef NZ_
#undef FN
#undef CAT_
#undef CAT2_
