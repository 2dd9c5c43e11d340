/*
 * oracle.c -- plain, slow, FP64 CPU reference for the time-stepping method of
 * "Heterogeneous computing in a strongly-connected CPU-GPU environment: fast
 * multiple time-evolution equation-based modeling accelerated using
 * data-driven approach" (Ichimura et al., arXiv:2409.20380).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the HIP library: every number here is
 * derived from the definitions written out below.
 *
 * What it computes (paper Sec. 3.1 and 3.2):
 *   - second-order (10-node) tetrahedral elements for linear elasticity;
 *     element stiffness and consistent mass integrated exactly with the
 *     closed form for barycentric monomials over a tetrahedron;
 *   - the assembled 3x3-block CRS matrices M, K and
 *     A = (4/dt^2 + 2 a_R/dt) M + (1 + 2 b_R/dt) K   (Eq. GE:DIS, Rayleigh C),
 *     with identity rows/columns for fixed degrees of freedom;
 *   - Algorithm 1 (3x3 block-Jacobi preconditioned CG) with the recursive
 *     stop test ||r||/||f|| < eps, followed by a true-residual check;
 *   - the Adams-Bashforth 4-step guess (Sec. 3.2);
 *   - the regional data-driven predictor of Sec. 3.2: modified Gram-Schmidt
 *     of past Adams-Bashforth errors X gives U (P = XU orthonormal),
 *     c = P^T x, y = Y U c;
 *   - the Newmark-beta (beta = 1/4, gamma = 1/2) update of Eq. timestep.
 *
 * Readings where the paper's printed formulas are garbled (each justified in
 * the design notes): the system matrix uses 4/dt^2 and 2/dt (average
 * acceleration); the acceleration update subtracts (4/dt) v; the unknown is
 * the increment du = u^it - u^(it-1) with right-hand side
 * f + C v + M (a + (4/dt) v) - K u; the predictor maps the AB error of one
 * step to that of the next (inputs = older column, outputs = newer column).
 *
 * Vectors are node-major, xyz interleaved: dof = 3*node + component.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Polynomials in the four barycentric coordinates L0..L3                    */
/* ------------------------------------------------------------------------ */
#define PMAX 16
typedef struct {
    int n;
    double c[PMAX];
    int e[PMAX][4];
} poly;

static double fact(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

/* Integral over a tetrahedron of volume V of L0^a L1^b L2^c L3^d:
 * 6 V a! b! c! d! / (a+b+c+d+3)!  (the classical barycentric closed form). */
static double monomial_integral(const int e[4], double V) {
    int s = e[0] + e[1] + e[2] + e[3];
    return 6.0 * V * fact(e[0]) * fact(e[1]) * fact(e[2]) * fact(e[3]) / fact(s + 3);
}

static double poly_integrate(const poly* p, double V) {
    double s = 0.0;
    for (int t = 0; t < p->n; ++t) s += p->c[t] * monomial_integral(p->e[t], V);
    return s;
}

static poly poly_mul(const poly* a, const poly* b) {
    poly r;
    r.n = 0;
    for (int i = 0; i < a->n; ++i)
        for (int j = 0; j < b->n; ++j) {
            r.c[r.n] = a->c[i] * b->c[j];
            for (int k = 0; k < 4; ++k) r.e[r.n][k] = a->e[i][k] + b->e[j][k];
            r.n++;
        }
    return r;
}

/* d/dL_k, treating the four barycentric coordinates as independent variables
 * (valid for the chain rule grad N = sum_k dN/dL_k grad L_k). */
static poly poly_diff(const poly* a, int k) {
    poly r;
    r.n = 0;
    for (int i = 0; i < a->n; ++i) {
        if (a->e[i][k] == 0) continue;
        r.c[r.n] = a->c[i] * a->e[i][k];
        for (int m = 0; m < 4; ++m) r.e[r.n][m] = a->e[i][m];
        r.e[r.n][k] -= 1;
        r.n++;
    }
    return r;
}

static void add_term(poly* p, double c, int e0, int e1, int e2, int e3) {
    p->c[p->n] = c;
    p->e[p->n][0] = e0; p->e[p->n][1] = e1; p->e[p->n][2] = e2; p->e[p->n][3] = e3;
    p->n++;
}

/* Edges of the 10-node tetrahedron, in local node order 4..9. */
static const int EDGE[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};

/* Quadratic Lagrange shape functions on the tetrahedron:
 * vertex i: L_i (2 L_i - 1); edge (i,j): 4 L_i L_j. */
static void p2_shape(poly N[10]) {
    for (int i = 0; i < 4; ++i) {
        int e2[4] = {0, 0, 0, 0}, e1[4] = {0, 0, 0, 0};
        e2[i] = 2; e1[i] = 1;
        N[i].n = 0;
        add_term(&N[i], 2.0, e2[0], e2[1], e2[2], e2[3]);
        add_term(&N[i], -1.0, e1[0], e1[1], e1[2], e1[3]);
    }
    for (int m = 0; m < 6; ++m) {
        int e[4] = {0, 0, 0, 0};
        e[EDGE[m][0]] = 1; e[EDGE[m][1]] = 1;
        N[4 + m].n = 0;
        add_term(&N[4 + m], 4.0, e[0], e[1], e[2], e[3]);
    }
}

/* Barycentric gradients and volume of a straight tetrahedron from its four
 * vertices. L(x) = J^{-1}(x - x0) for L1..L3 with J = [x1-x0, x2-x0, x3-x0];
 * L0 = 1 - L1 - L2 - L3.  Returns the signed volume det(J)/6. */
static double tet_geometry(const double xv[4][3], double gradL[4][3]) {
    double J[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) J[r][c] = xv[c + 1][r] - xv[0][r];
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double inv[3][3];
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    for (int a = 0; a < 3; ++a) {
        gradL[1][a] = inv[0][a];
        gradL[2][a] = inv[1][a];
        gradL[3][a] = inv[2][a];
        gradL[0][a] = -(inv[0][a] + inv[1][a] + inv[2][a]);
    }
    return det / 6.0;
}

/* Element stiffness and consistent mass (30x30, row-major, dof 3*i+c) of a
 * straight 10-node tetrahedron with Lame constants lam, mu and density rho.
 *   K[(i,a),(j,b)] = int lam dN_i/dx_a dN_j/dx_b
 *                        + mu (dN_i/dx_b dN_j/dx_a + delta_ab gradN_i.gradN_j)
 *   M[(i,a),(j,b)] = rho delta_ab int N_i N_j
 * Every integrand is a polynomial in L, integrated exactly.
 * Returns the element volume (negative if the vertex order is inverted). */
double orc_element_matrices(const double* xv_flat, double lam, double mu, double rho,
                            double* Ke, double* Me) {
    double xv[4][3], gL[4][3];
    memcpy(xv, xv_flat, sizeof(xv));
    double V = tet_geometry(xv, gL);
    double Va = fabs(V);
    poly N[10], D[10][4];
    p2_shape(N);
    for (int i = 0; i < 10; ++i)
        for (int k = 0; k < 4; ++k) D[i][k] = poly_diff(&N[i], k);

    /* G[i][j][a][b] = int dN_i/dx_a dN_j/dx_b
     *              = sum_{k,l} gradL_k[a] gradL_l[b] int dN_i/dL_k dN_j/dL_l */
    static const int nn = 10;
    double G[10][10][3][3];
    for (int i = 0; i < nn; ++i)
        for (int j = 0; j < nn; ++j) {
            double I[4][4];
            for (int k = 0; k < 4; ++k)
                for (int l = 0; l < 4; ++l) {
                    poly pr = poly_mul(&D[i][k], &D[j][l]);
                    I[k][l] = poly_integrate(&pr, Va);
                }
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double s = 0.0;
                    for (int k = 0; k < 4; ++k)
                        for (int l = 0; l < 4; ++l) s += gL[k][a] * gL[l][b] * I[k][l];
                    G[i][j][a][b] = s;
                }
        }
    for (int i = 0; i < nn; ++i)
        for (int j = 0; j < nn; ++j) {
            double dot = G[i][j][0][0] + G[i][j][1][1] + G[i][j][2][2];
            poly pr = poly_mul(&N[i], &N[j]);
            double mij = rho * poly_integrate(&pr, Va);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double k = lam * G[i][j][a][b] + mu * G[i][j][b][a] + (a == b ? mu * dot : 0.0);
                    Ke[(3 * i + a) * 30 + 3 * j + b] = k;
                    Me[(3 * i + a) * 30 + 3 * j + b] = (a == b) ? mij : 0.0;
                }
        }
    return V;
}

/* ------------------------------------------------------------------------ */
/* Assembled model: 3x3 block CRS (Sec. 3.2, "3x3 block CRS format")         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;          /* nodes */
    int64_t nnzb;       /* stored 3x3 blocks */
    int64_t* rowptr;    /* [n+1] */
    int32_t* col;       /* [nnzb] */
    double* Mv;         /* [nnzb][9] mass */
    double* Kv;         /* [nnzb][9] stiffness */
    double* Av;         /* [nnzb][9] A with identity rows/cols on fixed dofs */
    uint8_t* fixed;     /* [n*3] */
    double cM, cK;
    double* Binv;       /* [n][9] inverse diagonal blocks of A */
} orc_model;

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

static int64_t find_block(const orc_model* m, int64_t row, int32_t col) {
    int64_t lo = m->rowptr[row], hi = m->rowptr[row + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (m->col[mid] == col) return mid;
        if (m->col[mid] < col) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

void orc_destroy(orc_model* m) {
    if (!m) return;
    free(m->rowptr); free(m->col); free(m->Mv); free(m->Kv); free(m->Av);
    free(m->fixed); free(m->Binv); free(m);
}

/* 3x3 inverse by the cofactor formula (row-major). */
static void inv3(const double a[9], double r[9]) {
    double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6])
               + a[2] * (a[3] * a[7] - a[4] * a[6]);
    r[0] = (a[4] * a[8] - a[5] * a[7]) / det;
    r[1] = (a[2] * a[7] - a[1] * a[8]) / det;
    r[2] = (a[1] * a[5] - a[2] * a[4]) / det;
    r[3] = (a[5] * a[6] - a[3] * a[8]) / det;
    r[4] = (a[0] * a[8] - a[2] * a[6]) / det;
    r[5] = (a[2] * a[3] - a[0] * a[5]) / det;
    r[6] = (a[3] * a[7] - a[4] * a[6]) / det;
    r[7] = (a[1] * a[6] - a[0] * a[7]) / det;
    r[8] = (a[0] * a[4] - a[1] * a[3]) / det;
}

/* Build M, K and A = cM M + cK K (identity rows/cols on fixed dofs) and the
 * block-Jacobi inverse.  mat rows are (rho, vp, vs): mu = rho vs^2,
 * lam = rho (vp^2 - 2 vs^2).  Returns NULL on bad input (*err set). */
orc_model* orc_create(int64_t n_nodes, const double* coords, int64_t n_elems, const int32_t* conn,
                      const int32_t* elem_mat, int32_t n_mat, const double* mat, const uint8_t* fixed,
                      double cM, double cK, int* err) {
    *err = 0;
    orc_model* m = (orc_model*)calloc(1, sizeof(orc_model));
    m->n = n_nodes;
    m->cM = cM;
    m->cK = cK;
    /* node -> elements */
    int64_t* ecount = (int64_t*)calloc(n_nodes + 1, sizeof(int64_t));
    for (int64_t e = 0; e < n_elems; ++e)
        for (int i = 0; i < 10; ++i) {
            int32_t v = conn[e * 10 + i];
            if (v < 0 || v >= n_nodes) { *err = 1; free(ecount); free(m); return NULL; }
            ecount[v + 1]++;
        }
    for (int64_t i = 0; i < n_nodes; ++i) ecount[i + 1] += ecount[i];
    int64_t* epos = (int64_t*)malloc(sizeof(int64_t) * (n_nodes + 1));
    memcpy(epos, ecount, sizeof(int64_t) * (n_nodes + 1));
    int64_t* elist = (int64_t*)malloc(sizeof(int64_t) * ecount[n_nodes]);
    for (int64_t e = 0; e < n_elems; ++e)
        for (int i = 0; i < 10; ++i) elist[epos[conn[e * 10 + i]]++] = e;
    /* sparsity: node i couples with every node of every element containing i */
    m->rowptr = (int64_t*)calloc(n_nodes + 1, sizeof(int64_t));
    int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * 10 * 64);
    int32_t** rows = (int32_t**)malloc(sizeof(int32_t*) * n_nodes);
    int64_t* rlen = (int64_t*)malloc(sizeof(int64_t) * n_nodes);
    for (int64_t v = 0; v < n_nodes; ++v) {
        int64_t ne = ecount[v + 1] - ecount[v];
        int32_t* buf = (ne * 10 <= 640) ? tmp : (int32_t*)malloc(sizeof(int32_t) * 10 * ne);
        int64_t k = 0;
        for (int64_t t = ecount[v]; t < ecount[v + 1]; ++t)
            for (int i = 0; i < 10; ++i) buf[k++] = conn[elist[t] * 10 + i];
        qsort(buf, k, sizeof(int32_t), cmp_i32);
        int64_t u = 0;
        for (int64_t t = 0; t < k; ++t)
            if (u == 0 || buf[t] != buf[u - 1]) buf[u++] = buf[t];
        rows[v] = (int32_t*)malloc(sizeof(int32_t) * (u > 0 ? u : 1));
        memcpy(rows[v], buf, sizeof(int32_t) * u);
        rlen[v] = u;
        m->rowptr[v + 1] = m->rowptr[v] + u;
        if (buf != tmp) free(buf);
    }
    free(tmp);
    m->nnzb = m->rowptr[n_nodes];
    m->col = (int32_t*)malloc(sizeof(int32_t) * m->nnzb);
    for (int64_t v = 0; v < n_nodes; ++v) {
        memcpy(m->col + m->rowptr[v], rows[v], sizeof(int32_t) * rlen[v]);
        free(rows[v]);
    }
    free(rows); free(rlen); free(ecount); free(epos); free(elist);

    m->Mv = (double*)calloc(m->nnzb * 9, sizeof(double));
    m->Kv = (double*)calloc(m->nnzb * 9, sizeof(double));
    m->Av = (double*)calloc(m->nnzb * 9, sizeof(double));
    m->fixed = (uint8_t*)malloc(n_nodes * 3);
    memcpy(m->fixed, fixed, n_nodes * 3);

    double Ke[900], Me[900];
    for (int64_t e = 0; e < n_elems; ++e) {
        const int32_t* c = conn + e * 10;
        double xv[12];
        for (int i = 0; i < 4; ++i)
            for (int a = 0; a < 3; ++a) xv[3 * i + a] = coords[3 * (int64_t)c[i] + a];
        int32_t mi = elem_mat[e];
        if (mi < 0 || mi >= n_mat) { *err = 2; orc_destroy(m); return NULL; }
        double rho = mat[3 * mi], vp = mat[3 * mi + 1], vs = mat[3 * mi + 2];
        double mu = rho * vs * vs, lam = rho * (vp * vp - 2.0 * vs * vs);
        double V = orc_element_matrices(xv, lam, mu, rho, Ke, Me);
        if (!(V > 0.0)) { *err = 3; orc_destroy(m); return NULL; }
        for (int i = 0; i < 10; ++i)
            for (int j = 0; j < 10; ++j) {
                int64_t b = find_block(m, c[i], c[j]);
                for (int a = 0; a < 3; ++a)
                    for (int bb = 0; bb < 3; ++bb) {
                        m->Mv[9 * b + 3 * a + bb] += Me[(3 * i + a) * 30 + 3 * j + bb];
                        m->Kv[9 * b + 3 * a + bb] += Ke[(3 * i + a) * 30 + 3 * j + bb];
                    }
            }
    }
    /* A = cM M + cK K, then identity rows and columns for fixed dofs */
    for (int64_t v = 0; v < n_nodes; ++v)
        for (int64_t b = m->rowptr[v]; b < m->rowptr[v + 1]; ++b) {
            int32_t w = m->col[b];
            for (int a = 0; a < 3; ++a)
                for (int bb = 0; bb < 3; ++bb) {
                    double val = cM * m->Mv[9 * b + 3 * a + bb] + cK * m->Kv[9 * b + 3 * a + bb];
                    int fr = fixed[3 * v + a], fc = fixed[3 * (int64_t)w + bb];
                    if (fr || fc) val = (v == w && a == bb) ? 1.0 : 0.0;
                    m->Av[9 * b + 3 * a + bb] = val;
                }
        }
    /* 3x3 block Jacobi: B = diagonal blocks of A */
    m->Binv = (double*)malloc(sizeof(double) * 9 * n_nodes);
    for (int64_t v = 0; v < n_nodes; ++v) {
        int64_t b = find_block(m, v, (int32_t)v);
        inv3(m->Av + 9 * b, m->Binv + 9 * v);
    }
    return m;
}

int64_t orc_nnzb(const orc_model* m) { return m->nnzb; }

void orc_copy_binv(const orc_model* m, double* out) { memcpy(out, m->Binv, sizeof(double) * 9 * m->n); }

/* Copy the assembled matrix (0 = M, 1 = K, 2 = A) as BCSR arrays. */
void orc_copy_bcsr(const orc_model* m, int which, int64_t* rowptr, int32_t* col, double* val) {
    const double* src = which == 0 ? m->Mv : which == 1 ? m->Kv : m->Av;
    memcpy(rowptr, m->rowptr, sizeof(int64_t) * (m->n + 1));
    memcpy(col, m->col, sizeof(int32_t) * m->nnzb);
    memcpy(val, src, sizeof(double) * 9 * m->nnzb);
}

/* y = X p with X = M (0), K (1) or A (2): the 3x3 block CRS product. */
void orc_spmv(const orc_model* m, int which, const double* p, double* y) {
    const double* val = which == 0 ? m->Mv : which == 1 ? m->Kv : m->Av;
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < m->n; ++v) {
        double s0 = 0, s1 = 0, s2 = 0;
        for (int64_t b = m->rowptr[v]; b < m->rowptr[v + 1]; ++b) {
            const double* B = val + 9 * b;
            const double* x = p + 3 * (int64_t)m->col[b];
            s0 += B[0] * x[0] + B[1] * x[1] + B[2] * x[2];
            s1 += B[3] * x[0] + B[4] * x[1] + B[5] * x[2];
            s2 += B[6] * x[0] + B[7] * x[1] + B[8] * x[2];
        }
        y[3 * v] = s0; y[3 * v + 1] = s1; y[3 * v + 2] = s2;
    }
}

static double dot(int64_t n, const double* a, const double* b) {
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* z = B^{-1} r, blockwise. */
void orc_precond(const orc_model* m, const double* r, double* z) {
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < m->n; ++v) {
        const double* B = m->Binv + 9 * v;
        const double* x = r + 3 * v;
        for (int a = 0; a < 3; ++a) z[3 * v + a] = B[3 * a] * x[0] + B[3 * a + 1] * x[1] + B[3 * a + 2] * x[2];
    }
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1: conjugate gradient with 3x3 block Jacobi preconditioner      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t iters;       /* loop trips (products q = A p), r0 product excluded */
    int32_t restarts;    /* true-residual restarts */
    double res0;         /* ||f - A xbar|| / ||f|| */
    double res_rec;      /* recursive residual at exit */
    double res_true;     /* ||f - A x|| / ||f|| at exit */
    double fnorm;
    int32_t status;      /* 0 converged, 1 not converged */
    int32_t pad;
} orc_solve_stats;

int orc_pcg(const orc_model* m, const double* f, double* x, double tol, int max_iter, orc_solve_stats* st) {
    int64_t n3 = 3 * m->n;
    memset(st, 0, sizeof(*st));
    double fn = sqrt(dot(n3, f, f));
    st->fnorm = fn;
    if (fn == 0.0) {
        memset(x, 0, sizeof(double) * n3);
        return 0;
    }
    double* r = (double*)malloc(sizeof(double) * n3);
    double* z = (double*)malloc(sizeof(double) * n3);
    double* p = (double*)calloc(n3, sizeof(double));
    double* q = (double*)malloc(sizeof(double) * n3);
    /* r = f - A x */
    orc_spmv(m, 2, x, q);
    for (int64_t i = 0; i < n3; ++i) r[i] = f[i] - q[i];
    st->res0 = sqrt(dot(n3, r, r)) / fn;
    int status = 0;
    for (;;) {
        double beta = 0.0, rho_b = 0.0;
        int i = 1;
        while (sqrt(dot(n3, r, r)) / fn >= tol) {
            if (st->iters >= max_iter) { status = 1; break; }
            orc_precond(m, r, z);
            double rho_a = dot(n3, z, r);
            if (i > 1) beta = rho_a / rho_b;
            for (int64_t k = 0; k < n3; ++k) p[k] = z[k] + beta * p[k];
            orc_spmv(m, 2, p, q);
            double alpha = rho_a / dot(n3, p, q);
            rho_b = rho_a;
            for (int64_t k = 0; k < n3; ++k) {
                r[k] -= alpha * q[k];
                x[k] += alpha * p[k];
            }
            i++;
            st->iters++;
        }
        st->res_rec = sqrt(dot(n3, r, r)) / fn;
        orc_spmv(m, 2, x, q);
        for (int64_t k = 0; k < n3; ++k) r[k] = f[k] - q[k];
        st->res_true = sqrt(dot(n3, r, r)) / fn;
        if (st->res_true < tol || status) break;
        /* recursive residual drifted from the true one: restart from x */
        st->restarts++;
        if (st->restarts > 20) { status = 1; break; }
    }
    st->status = status;
    free(r); free(z); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Right-hand side of Eq. GE:DIS for the increment (reading: unknown = du)   */
/* ------------------------------------------------------------------------ */
/* b = f + C v + M (a + (4/dt) v) - K u,  C = aR M + bR K,
 * f = f_add - sum_k g_k M r_k  (r_k the unit rigid translation along axis k:
 * the effective inertial load of a uniform base acceleration g),
 * then b = 0 on fixed dofs.  f_add and g may be NULL. */
void orc_rhs(const orc_model* m, const double* f_add, const double* g, const double* u, const double* v,
             const double* a, double dt, double aR, double bR, double* b) {
    int64_t n3 = 3 * m->n;
    double* t1 = (double*)malloc(sizeof(double) * n3);
    double* t2 = (double*)malloc(sizeof(double) * n3);
    for (int64_t i = 0; i < n3; ++i) b[i] = f_add ? f_add[i] : 0.0;
    if (g) {
        for (int k = 0; k < 3; ++k) {
            for (int64_t i = 0; i < n3; ++i) t1[i] = (i % 3 == k) ? 1.0 : 0.0;
            orc_spmv(m, 0, t1, t2);
            for (int64_t i = 0; i < n3; ++i) b[i] -= g[k] * t2[i];
        }
    }
    /* C v = aR M v + bR K v */
    orc_spmv(m, 0, v, t2);
    for (int64_t i = 0; i < n3; ++i) b[i] += aR * t2[i];
    orc_spmv(m, 1, v, t2);
    for (int64_t i = 0; i < n3; ++i) b[i] += bR * t2[i];
    /* M (a + 4/dt v) */
    for (int64_t i = 0; i < n3; ++i) t1[i] = a[i] + (4.0 / dt) * v[i];
    orc_spmv(m, 0, t1, t2);
    for (int64_t i = 0; i < n3; ++i) b[i] += t2[i];
    /* - K u */
    orc_spmv(m, 1, u, t2);
    for (int64_t i = 0; i < n3; ++i) b[i] -= t2[i];
    for (int64_t i = 0; i < n3; ++i)
        if (m->fixed[i]) b[i] = 0.0;
    free(t1); free(t2);
}

/* ------------------------------------------------------------------------ */
/* Predictors                                                                */
/* ------------------------------------------------------------------------ */
/* Adams-Bashforth 4-step increment (Sec. 3.2):
 * du_AB = dt/24 (55 v^{it-1} - 59 v^{it-2} + 37 v^{it-3} - 9 v^{it-4}).
 * vh[k] points at v^{it-1-k}. */
void orc_ab4(int64_t n3, double dt, const double* v1, const double* v2, const double* v3, const double* v4,
             double* out) {
    for (int64_t i = 0; i < n3; ++i)
        out[i] = dt / 24.0 * (55.0 * v1[i] - 59.0 * v2[i] + 37.0 * v3[i] - 9.0 * v4[i]);
}

/* Data-driven map of Sec. 3.2 on one region (rows = the region's dofs).
 * X = {x_1..x_s} inputs, Y = {y_1..y_s} outputs, x the query.
 * Modified Gram-Schmidt gives upper-triangular U with P = X U orthonormal;
 * c = P^T x; y = Y U c.  A column whose norm after orthogonalisation falls
 * below drop * (its original norm) is dropped (its column of U is zero).
 * X, Y: column pointers into full-length vectors, rows listed in idx[nr].
 * Returns the number of columns kept. */
static int mgs_predict_region(int s, const double* const* X, const double* const* Y, const double* x,
                              const int64_t* idx, int64_t nr, double drop, double* out, double* work) {
    double* P = work;                 /* [s][nr] */
    double* U = work + (int64_t)s * nr; /* [s][s], column j stored at U[j*s + i] */
    int* keep = (int*)(U + s * s);
    int kept = 0;
    memset(U, 0, sizeof(double) * s * s);
    for (int j = 0; j < s; ++j) {
        double* pj = P + (int64_t)j * nr;
        double n0 = 0.0;
        for (int64_t t = 0; t < nr; ++t) {
            pj[t] = X[j][idx[t]];
            n0 += pj[t] * pj[t];
        }
        n0 = sqrt(n0);
        U[j * s + j] = 1.0;
        for (int i = 0; i < j; ++i) {
            if (!keep[i]) continue;
            const double* pi = P + (int64_t)i * nr;
            double rij = 0.0;
            for (int64_t t = 0; t < nr; ++t) rij += pi[t] * pj[t];
            for (int64_t t = 0; t < nr; ++t) pj[t] -= rij * pi[t];
            for (int k = 0; k <= i; ++k) U[j * s + k] -= rij * U[i * s + k];
        }
        double nj = 0.0;
        for (int64_t t = 0; t < nr; ++t) nj += pj[t] * pj[t];
        nj = sqrt(nj);
        if (n0 == 0.0 || nj < drop * n0) {
            keep[j] = 0;
            for (int k = 0; k < s; ++k) U[j * s + k] = 0.0;
            for (int64_t t = 0; t < nr; ++t) pj[t] = 0.0;
            continue;
        }
        keep[j] = 1;
        kept++;
        for (int64_t t = 0; t < nr; ++t) pj[t] /= nj;
        for (int k = 0; k <= j; ++k) U[j * s + k] /= nj;
    }
    /* c = P^T x ; w = U c ; out = Y w */
    double* c = (double*)malloc(sizeof(double) * s * 2);
    double* w = c + s;
    for (int j = 0; j < s; ++j) {
        const double* pj = P + (int64_t)j * nr;
        double t0 = 0.0;
        for (int64_t t = 0; t < nr; ++t) t0 += pj[t] * x[idx[t]];
        c[j] = t0;
    }
    for (int k = 0; k < s; ++k) {
        double t0 = 0.0;
        for (int j = 0; j < s; ++j) t0 += U[j * s + k] * c[j];
        w[k] = t0;
    }
    for (int64_t t = 0; t < nr; ++t) {
        double t0 = 0.0;
        for (int k = 0; k < s; ++k) t0 += Y[k][idx[t]] * w[k];
        out[idx[t]] = t0;
    }
    free(c);
    return kept;
}

/* Regional predictor over the whole vector: for each region (nodes with the
 * same id in region_of_node), apply mgs_predict_region to its dofs.
 * X[j], Y[j] (j = 0..s-1, oldest first) and x are full-length vectors.
 * out receives the prediction (dofs of every region). */
void orc_predict_regional(int64_t n_nodes, const int32_t* region_of_node, int32_t n_regions, int s,
                          const double* const* X, const double* const* Y, const double* x, double drop,
                          double* out) {
    int64_t* cnt = (int64_t*)calloc(n_regions + 1, sizeof(int64_t));
    for (int64_t v = 0; v < n_nodes; ++v) cnt[region_of_node[v] + 1] += 3;
    for (int32_t r = 0; r < n_regions; ++r) cnt[r + 1] += cnt[r];
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * 3 * n_nodes);
    int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (n_regions + 1));
    memcpy(pos, cnt, sizeof(int64_t) * (n_regions + 1));
    for (int64_t v = 0; v < n_nodes; ++v)
        for (int c = 0; c < 3; ++c) idx[pos[region_of_node[v]]++] = 3 * v + c;
#pragma omp parallel for schedule(dynamic)
    for (int32_t r = 0; r < n_regions; ++r) {
        int64_t nr = cnt[r + 1] - cnt[r];
        if (nr == 0) continue;
        double* work = (double*)malloc(sizeof(double) * ((int64_t)s * nr + s * s) + sizeof(int) * (s + 1));
        mgs_predict_region(s, X, Y, x, idx + cnt[r], nr, drop, out, work);
        free(work);
    }
    free(cnt); free(idx); free(pos);
}

/* ------------------------------------------------------------------------ */
/* One time step: predict -> Algorithm 1 -> Newmark update                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    double dt, aR, bR, tol, drop;
    int32_t max_iter, s, kind; /* kind: 0 zero guess, 1 AB4, 2 AB4 + regional snapshots */
    int32_t want_ab_residual;
    int32_t s_min;             /* kind 2: the map needs at least this many column pairs (<= 0: 1) */
    int32_t guard;             /* kind 2: keep the AB4 guess when its initial residual is smaller,
                                  and restart the snapshot window (see orc_step) */
    double skip_ratio;         /* guard: the AB4 guess is not evaluated while the map's residual is
                                  below skip_ratio x the last evaluated AB4 residual (<= 0: always) */
    double col_cost;           /* guard: cost of one window column in PCG trips; > 0 enables the
                                  window-length probes (see orc_step), <= 0 keeps the length s */
    int32_t probe_every;       /* steps with a full window between probes (<= 0: 8) */
    int32_t probe_step;        /* columns a probe adds or removes (<= 0: 8) */
} orc_params;

/* Window state carried from step to step (kind 2). */
typedef struct {
    int32_t win;         /* first step whose AB error may enter the window (>= 1) */
    int32_t s_cap;       /* current window length cap in column pairs (0: s) */
    int32_t since;       /* steps with a full window since the last probe */
    int32_t grow_next;   /* direction of the next probe: 1 longer, 0 shorter */
    double rho_ab;       /* last evaluated initial relative residual of the AB4 guess (<= 0: none) */
    double rate;         /* ln(res0 / res_end) / trips of the last solve (<= 0: none) */
} orc_window;

typedef struct {
    int32_t it;          /* index of the step just solved */
    int32_t s_eff;       /* column pairs of the map used (0: no map) */
    int32_t iters;
    int32_t status;
    int32_t pick;        /* guard: 1 map kept, 0 AB4 kept (window restarted); -1 no comparison */
    int32_t first;       /* the window used held e^first .. e^{it-1} (0: no map) */
    int32_t skipped;     /* guard: 1 if the AB4 guess was not evaluated (map far ahead) */
    int32_t probe;       /* window length probed against s_eff this step (0: none) */
    int32_t s_cap;       /* window length cap after this step */
    int32_t pad;
    double res_ab;       /* initial relative residual of the AB4 guess (guard or if requested) */
    double res_map;      /* initial relative residual of the map's guess (guard only) */
    double res_probe;    /* the same for the probed window length */
    double res0;         /* initial relative residual of the guess actually used */
    double res_rec, res_true, fnorm;
} orc_step_stats;

/* Relative residual ||b - A x|| / ||b|| (0 when b = 0). */
static double rel_residual(const orc_model* m, const double* b, const double* x, double* tmp) {
    int64_t n3 = 3 * m->n;
    orc_spmv(m, 2, x, tmp);
    double s = 0.0;
    for (int64_t i = 0; i < n3; ++i) s += (b[i] - tmp[i]) * (b[i] - tmp[i]);
    double fn = sqrt(dot(n3, b, b));
    return fn > 0 ? sqrt(s) / fn : sqrt(s);
}

/* Trips per unit of log initial residual, in units of 1 / rate (the average
 * per-trip decay of a solve): a lower initial residual saves more trips than
 * the average decay suggests, because the guess removes mostly the slowly
 * converging components.  Measured on the 64 x 64 x 32-cell mesh at steady
 * state: s = 8 -> 16 lowers ln(res0) by 0.31 and saves 3.9 trips, 1.9 times
 * 0.31 / rate (rate 0.15). */
/* Lower end of the window length: the paper draws s from [8, 32] (Sec. 4, Fig. 3). */
#define LEN_FLOOR 8
#define TRIP_GAIN 2.0

/* Guess of the map over the window e^first .. e^{n-1} (s_eff column pairs):
 * inputs X = e^first .. e^{n-2}, outputs Y = e^{first+1} .. e^{n-1} (one step
 * later), query e^{n-1}; dab + the regional map, zero on fixed dofs. */
static void map_guess(const orc_model* m, const orc_params* P, const int32_t* region_of_node, int32_t n_regions,
                      double* const* ring, int n, int first, const double* dab, double* xm) {
    int64_t n3 = 3 * m->n;
    int s_eff = n - 1 - first;
    const double** X = (const double**)malloc(sizeof(double*) * s_eff);
    const double** Y = (const double**)malloc(sizeof(double*) * s_eff);
    int S1 = P->s + 1;
    for (int j = 0; j < s_eff; ++j) {
        X[j] = ring[(first + j - 1) % S1]; /* e^{first+j}   */
        Y[j] = ring[(first + j) % S1];     /* e^{first+j+1} */
    }
    const double* q = ring[(n - 2) % S1]; /* query e^{n-1} */
    memset(xm, 0, sizeof(double) * n3);
    orc_predict_regional(m->n, region_of_node, n_regions, s_eff, X, Y, q, P->drop, xm);
    for (int64_t i = 0; i < n3; ++i) xm[i] = m->fixed[i] ? 0.0 : dab[i] + xm[i];
    free(X); free(Y);
}

/* State arrays (all length 3N, owned by the caller):
 *   u, v, a                    displacement, velocity, acceleration at step it
 *   vh[0..3]                   v^{it}, v^{it-1}, v^{it-2}, v^{it-3}  (v^{j<=0} = 0)
 *   ring[0..s]                 AB errors e^j = du^j - du_AB^j, e^j stored in
 *                              slot (j-1) mod (s+1)
 *   *ws                        window state (may be NULL: window from step 1,
 *                              length s, no probes, no skipped evaluations)
 * *it is the number of completed steps; this call advances it by one.
 * g: base acceleration at the new time (3 values, may be NULL); f_add: extra
 * nodal force at the new time (may be NULL).  du_out, guess_out optional.
 *
 * Guess of step n = it + 1 (kind 2; Sec. 3.2): the AB4 increment plus the
 * regional map fitted on the window of AB errors e^first .. e^{n-1}, with
 * first = max(win, n - 1 - s_cap): s_eff = n - 1 - first column pairs, the map
 * used when s_eff >= s_min (the predictor as defined uses whatever history
 * the window holds, s_min = 1; a larger s_min waits for more pairs).
 *
 * With the guard, the AB4 guess is evaluated too and kept when its residual
 * ||b - A x|| is strictly smaller; the window then restarts at this step (win =
 * n): the map's columns up to e^{n-1} are discarded, so a window that spans a
 * change of regime (the start from rest, a kink in the input) is not fitted
 * again.  The AB4 guess is not evaluated (the map kept) while the map's
 * relative residual is below skip_ratio times the last evaluated AB4 one.
 *
 * Window length (the paper adjusts s during the run to balance predictor and
 * solver time; on one device the two add up, so the length that minimises
 * their sum is sought): with col_cost > 0, after every probe_every steps whose
 * window was full (s_eff = s_cap), the step also evaluates the map over
 * s_cap - d or s_cap + d column pairs (d = probe_step; alternating, whichever is
 * possible: at least max(s_min, min(8, s)), the paper drawing s from [8, 32],
 * at most s, and enough columns since win).  The
 * difference in trips is estimated from the two initial residuals with the
 * per-trip convergence rate of the previous solve, TRIP_GAIN x ln(rho_probe /
 * rho_map) / rate, and the cap moves to the probed length when the trips it
 * saves exceed col_cost x d (shorter: extra trips below col_cost x d; longer:
 * trips saved above it).  The step itself uses the window of length s_cap. */
int orc_step(const orc_model* m, const orc_params* P, const int32_t* region_of_node, int32_t n_regions,
             double* u, double* v, double* a, double* const* vh, double* const* ring, int32_t* it,
             orc_window* ws, const double* g, const double* f_add, double* du_out, double* guess_out,
             orc_step_stats* st) {
    int64_t n3 = 3 * m->n;
    int n = *it + 1; /* new step index */
    memset(st, 0, sizeof(*st));
    st->it = n;
    st->pick = -1;
    double* b = (double*)malloc(sizeof(double) * n3);
    double* dab = (double*)malloc(sizeof(double) * n3);
    double* x = (double*)malloc(sizeof(double) * n3);
    orc_rhs(m, f_add, g, u, v, a, P->dt, P->aR, P->bR, b);
    /* Adams-Bashforth increment from the stored velocities */
    orc_ab4(n3, P->dt, vh[0], vh[1], vh[2], vh[3], dab);
    memcpy(x, dab, sizeof(double) * n3);
    if (P->kind == 0) memset(x, 0, sizeof(double) * n3);
    for (int64_t i = 0; i < n3; ++i)
        if (m->fixed[i]) x[i] = 0.0;
    orc_window wl0 = {1, 0, 0, 0, 0.0, 0.0};
    orc_window* W = ws ? ws : &wl0;
    if (W->win < 1) W->win = 1;
    const int s_min = P->s_min < 1 ? 1 : (P->s_min < P->s ? P->s_min : P->s);
    const int len_floor = P->s < LEN_FLOOR ? P->s : LEN_FLOOR;
    const int len_min = s_min > len_floor ? s_min : len_floor;   /* shortest window length */
    if (W->s_cap < len_min || W->s_cap > P->s) W->s_cap = P->s;
    const int s_cap = W->s_cap;
    int first = n - 1 - s_cap;
    if (first < W->win) first = W->win;
    int s_eff = n - 1 - first;
    double* tmp = (double*)malloc(sizeof(double) * n3);
    int new_cap = s_cap;
    if (P->kind == 2 && P->s >= 1 && s_eff >= s_min) {
        double* xm = (double*)malloc(sizeof(double) * n3);
        map_guess(m, P, region_of_node, n_regions, ring, n, first, dab, xm);
        st->s_eff = s_eff;
        st->first = first;
        if (P->guard) {
            st->res_map = rel_residual(m, b, xm, tmp);
            /* window-length probe */
            const int d = P->probe_step > 0 ? P->probe_step : 8;
            const int every = P->probe_every > 0 ? P->probe_every : 8;
            if (P->col_cost > 0 && s_eff == s_cap) {
                if (W->since + 1 >= every) {
                    const int can_grow = s_cap + d <= P->s && n - 1 - (s_cap + d) >= W->win;
                    const int can_shrink = s_cap - d >= len_min;
                    int alt = 0;
                    if (W->grow_next && can_grow) alt = s_cap + d;
                    else if (can_shrink) alt = s_cap - d;
                    else if (can_grow) alt = s_cap + d;
                    if (alt) {
                        double* xp = (double*)malloc(sizeof(double) * n3);
                        map_guess(m, P, region_of_node, n_regions, ring, n, n - 1 - alt, dab, xp);
                        st->res_probe = rel_residual(m, b, xp, tmp);
                        st->probe = alt;
                        free(xp);
                        if (W->rate > 0 && st->res_map > 0 && st->res_probe > 0) {
                            const double dtrips = TRIP_GAIN * log(st->res_probe / st->res_map) / W->rate;
                            const double cols = P->col_cost * d;
                            if (alt < s_cap ? dtrips < cols : -dtrips > cols) new_cap = alt;
                        }
                        W->grow_next = alt < s_cap;
                    }
                    W->since = 0;
                } else {
                    W->since += 1;
                }
            }
            /* guard: the AB4 guess against the map's */
            if (P->skip_ratio > 0 && W->rho_ab > 0 && st->res_map < P->skip_ratio * W->rho_ab) {
                st->skipped = 1;
                st->pick = 1;
                memcpy(x, xm, sizeof(double) * n3);
            } else {
                st->res_ab = rel_residual(m, b, x, tmp);
                W->rho_ab = st->res_ab;
                if (st->res_ab < st->res_map) {
                    st->pick = 0;
                    W->win = n;
                } else {
                    st->pick = 1;
                    memcpy(x, xm, sizeof(double) * n3);
                }
            }
        } else {
            memcpy(x, xm, sizeof(double) * n3);
        }
        free(xm);
    }
    W->s_cap = new_cap;
    st->s_cap = new_cap;
    if (guess_out) memcpy(guess_out, x, sizeof(double) * n3);
    if (P->want_ab_residual && st->pick < 0) {
        double* xab = (double*)malloc(sizeof(double) * n3);
        for (int64_t i = 0; i < n3; ++i) xab[i] = m->fixed[i] ? 0.0 : dab[i];
        st->res_ab = rel_residual(m, b, xab, tmp);
        free(xab);
    }
    free(tmp);
    orc_solve_stats ss;
    int status = orc_pcg(m, b, x, P->tol, P->max_iter, &ss);
    st->iters = ss.iters;
    st->res0 = ss.res0;
    st->res_rec = ss.res_rec;
    st->res_true = ss.res_true;
    st->fnorm = ss.fnorm;
    st->status = status;
    /* per-trip convergence rate of this solve (for the next window-length probe) */
    if (ss.iters > 0 && ss.res0 > 0 && ss.res_rec > 0) W->rate = log(ss.res0 / ss.res_rec) / ss.iters;
    /* Newmark-beta (beta = 1/4, gamma = 1/2) update, Eq. timestep */
    double dt = P->dt;
    for (int64_t i = 0; i < n3; ++i) {
        double du = x[i];
        double vo = v[i];
        u[i] += du;
        v[i] = -vo + 2.0 / dt * du;
        a[i] = -a[i] - 4.0 / dt * vo + 4.0 / (dt * dt) * du;
    }
    /* velocity history: vh[0] <- v^{n}; older entries shift down */
    double* last = vh[3];
    memcpy(last, vh[2], sizeof(double) * n3);
    memcpy(vh[2], vh[1], sizeof(double) * n3);
    memcpy(vh[1], vh[0], sizeof(double) * n3);
    memcpy(vh[0], v, sizeof(double) * n3);
    /* AB error of this step into the ring */
    if (P->s >= 1) {
        double* e = ring[(n - 1) % (P->s + 1)];
        for (int64_t i = 0; i < n3; ++i) e[i] = x[i] - dab[i];
    }
    if (du_out) memcpy(du_out, x, sizeof(double) * n3);
    *it = n;
    free(b); free(dab); free(x);
    return status;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of later parallel loops (timing; the dot products' reduction order, and so their
 * rounding, follows the thread count). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
