/*
 * Oracle: plain, slow, FP64 CPU implementation of the Wilson-clover solve
 * used by all-mode averaging (von Hippel, Rae, Shintani, Wittig,
 * arXiv:1605.00564).  TEST INFRASTRUCTURE ONLY: nothing in the product
 * library links, loads or calls this code; only the tests, the smoke check
 * and the CPU-baseline leg of the benchmark do.
 *
 * It shares no code with the HIP library.  Every loop runs over
 * lexicographically ordered sites, in complex double, in the order in which
 * the definitions are written.  OpenMP parallelises independent sites or
 * independent Schwarz blocks only (no reordering of any sum over terms of
 * one output element).
 *
 * Conventions (the paper names the O(a)-improved Wilson operator but writes
 * none of it down; these are the readings adopted):
 *   dims = {T, X, Y, Z}, mu = 0 is time, site i = z + Z*(y + Y*(x + X*t));
 *   psi[i][spin][colour], U[i][mu][a][b] with U_mu(x) linking x -> x+mu;
 *   Euclidean chiral gamma basis:  gamma_0 = [[0,-1],[-1,0]],
 *   gamma_k = [[0,-i sigma_k],[i sigma_k,0]], gamma_5 = diag(1,1,-1,-1);
 *   sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu];
 *   kappa-normalised operator  M = A - kappa H,
 *   (H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                     + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu),
 *   A(x) = 1 + i kappa c_sw sum_{mu<nu} sigma_{mu nu} (x) Fhat_{mu nu}(x),
 *   Fhat_{mu nu} = (Q_{mu nu} - Q_{mu nu}^+)/8 with Q the sum of the four
 *   plaquette leaves in the mu-nu plane that start and end at x;
 *   fermion boundary: factor bc_t (-1 antiperiodic) on hops across t=T-1|0,
 *   gauge links periodic, no boundary phase inside the clover leaves.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* Dirac algebra                                                        */
/* ------------------------------------------------------------------ */

static cplx G[5][4][4];      /* gamma_0..gamma_3, gamma_5 */
static cplx SIG[6][4][4];    /* sigma_{mu nu} for the 6 pairs mu<nu */
static const int PAIR_MU[6] = {0, 0, 0, 1, 1, 2};
static const int PAIR_NU[6] = {1, 2, 3, 2, 3, 3};
static int g_init = 0;

static void init_gamma(void)
{
    if (g_init) return;
    const cplx im = _Complex_I;
    cplx pauli[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -im}, {im, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(G, 0, sizeof(G));
    for (int a = 0; a < 2; ++a) {          /* gamma_0: off-diagonal -1 blocks */
        G[0][a][a + 2] = -1;
        G[0][a + 2][a] = -1;
    }
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                G[k + 1][a][b + 2] = -im * pauli[k][a][b];
                G[k + 1][a + 2][b] = im * pauli[k][a][b];
            }
    /* gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3 */
    cplx t1[4][4], t2[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += G[0][i][k] * G[1][k][j];
            t1[i][j] = s;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += t1[i][k] * G[2][k][j];
            t2[i][j] = s;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += t2[i][k] * G[3][k][j];
            G[4][i][j] = s;
        }
    /* sigma_{mu nu} = (i/2)(gamma_mu gamma_nu - gamma_nu gamma_mu) */
    for (int p = 0; p < 6; ++p) {
        int mu = PAIR_MU[p], nu = PAIR_NU[p];
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                cplx s = 0;
                for (int k = 0; k < 4; ++k)
                    s += G[mu][i][k] * G[nu][k][j] - G[nu][i][k] * G[mu][k][j];
                SIG[p][i][j] = 0.5 * im * s;
            }
    }
    g_init = 1;
}

/* Export the gamma matrices so that tests can check the algebra. */
void orc_gamma(double complex *g /* [5][4][4] */, double complex *sig /* [6][4][4] */)
{
    init_gamma();
    memcpy(g, G, sizeof(G));
    memcpy(sig, SIG, sizeof(SIG));
}

/* ------------------------------------------------------------------ */
/* Geometry                                                             */
/* ------------------------------------------------------------------ */

typedef struct {
    int L[4];
    long V;
    double kappa, csw;
    int bc_t;
} lat_t;

static lat_t make_lat(const int *dims, double kappa, double csw, int bc_t)
{
    lat_t l;
    for (int m = 0; m < 4; ++m) l.L[m] = dims[m];
    l.V = (long)dims[0] * dims[1] * dims[2] * dims[3];
    l.kappa = kappa;
    l.csw = csw;
    l.bc_t = bc_t;
    init_gamma();   /* before any parallel region reads the tables */
    return l;
}

static void site_coords(const lat_t *l, long i, int c[4])
{
    c[3] = (int)(i % l->L[3]);
    i /= l->L[3];
    c[2] = (int)(i % l->L[2]);
    i /= l->L[2];
    c[1] = (int)(i % l->L[1]);
    c[0] = (int)(i / l->L[1]);
}

static long site_index(const lat_t *l, const int c[4])
{
    return c[3] + (long)l->L[3] * (c[2] + (long)l->L[2] * (c[1] + (long)l->L[1] * c[0]));
}

/* neighbour of site i one step in direction mu, forward (dir=+1) or back */
static long neighbour(const lat_t *l, long i, int mu, int dir)
{
    int c[4];
    site_coords(l, i, c);
    c[mu] = (c[mu] + dir + l->L[mu]) % l->L[mu];
    return site_index(l, c);
}

/* fermion boundary factor of the hop from site i in direction (mu, dir) */
static double hop_sign(const lat_t *l, long i, int mu, int dir)
{
    if (mu != 0 || l->bc_t == 1) return 1.0;
    int c[4];
    site_coords(l, i, c);
    if (dir > 0 && c[0] == l->L[0] - 1) return (double)l->bc_t;
    if (dir < 0 && c[0] == 0) return (double)l->bc_t;
    return 1.0;
}

/* ------------------------------------------------------------------ */
/* SU(3) helpers                                                        */
/* ------------------------------------------------------------------ */

static const cplx *link(const cplx *U, long i, int mu) { return U + (i * 4 + mu) * 9; }

static void mat_mul(const cplx *a, const cplx *b, cplx *c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += a[i * 3 + k] * b[k * 3 + j];
            c[i * 3 + j] = s;
        }
}

static void mat_dag(const cplx *a, cplx *c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c[i * 3 + j] = conj(a[j * 3 + i]);
}

/* product of four 3x3 matrices */
static void mul4(const cplx *a, const cplx *b, const cplx *c, const cplx *d, cplx *out)
{
    cplx t1[9], t2[9];
    mat_mul(a, b, t1);
    mat_mul(t1, c, t2);
    mat_mul(t2, d, out);
}

/* ------------------------------------------------------------------ */
/* Clover field strength  Fhat_{mu nu}(x) = (Q - Q^+)/8                 */
/* ------------------------------------------------------------------ */

void orc_fhat(const int *dims, const double complex *U, double complex *F /* [V][6][3][3] */)
{
    lat_t l = make_lat(dims, 0, 0, 1);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < l.V; ++x) {
        for (int p = 0; p < 6; ++p) {
            int mu = PAIR_MU[p], nu = PAIR_NU[p];
            long xm = neighbour(&l, x, mu, -1);   /* x - mu */
            long xn = neighbour(&l, x, nu, -1);   /* x - nu */
            long xpm = neighbour(&l, x, mu, +1);  /* x + mu */
            long xpn = neighbour(&l, x, nu, +1);  /* x + nu */
            long xmn = neighbour(&l, xm, nu, -1); /* x - mu - nu */
            long xpm_mn = neighbour(&l, xpm, nu, -1); /* x + mu - nu */
            long xmm_pn = neighbour(&l, xm, nu, +1);  /* x - mu + nu */
            cplx d1[9], d2[9], d3[9], d4[9], leaf[9], Q[9];
            memset(Q, 0, sizeof(Q));
            /* leaf 1: +mu, +nu, -mu, -nu */
            mat_dag(link(U, xpn, mu), d1);
            mat_dag(link(U, x, nu), d2);
            mul4(link(U, x, mu), link(U, xpm, nu), d1, d2, leaf);
            for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
            /* leaf 2: +nu, -mu, -nu, +mu */
            mat_dag(link(U, xmm_pn, mu), d1);
            mat_dag(link(U, xm, nu), d2);
            mul4(link(U, x, nu), d1, d2, link(U, xm, mu), leaf);
            for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
            /* leaf 3: -mu, -nu, +mu, +nu */
            mat_dag(link(U, xm, mu), d1);
            mat_dag(link(U, xmn, nu), d2);
            mul4(d1, d2, link(U, xmn, mu), link(U, xn, nu), leaf);
            for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
            /* leaf 4: -nu, +mu, +nu, -mu */
            mat_dag(link(U, xn, nu), d3);
            mat_dag(link(U, x, mu), d4);
            mul4(d3, link(U, xn, mu), link(U, xpm_mn, nu), d4, leaf);
            for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
            cplx *f = F + (x * 6 + p) * 9;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) f[a * 3 + b] = (Q[a * 3 + b] - conj(Q[b * 3 + a])) / 8.0;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Site-local operators                                                 */
/* ------------------------------------------------------------------ */

/* out = A(x) in from the clover field strength (definition above) */
static void clover_from_fhat(const lat_t *l, const cplx *F, long x, const cplx *in, cplx *out)
{
    const cplx coef = _Complex_I * l->kappa * l->csw;
    for (int k = 0; k < 12; ++k) out[k] = in[k];
    for (int p = 0; p < 6; ++p) {
        const cplx *f = F + (x * 6 + p) * 9;
        for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) {
                cplx acc = 0;
                for (int s2 = 0; s2 < 4; ++s2) {
                    if (SIG[p][s][s2] == 0) continue;
                    for (int b = 0; b < 3; ++b) acc += SIG[p][s][s2] * f[a * 3 + b] * in[s2 * 3 + b];
                }
                out[s * 3 + a] += coef * acc;
            }
    }
}

/* out = A(x) in with the site's stored 12x12 clover matrix Am[x] */
static void clover_site(const cplx *Am, long x, const cplx *in, cplx *out)
{
    const cplx *m = Am + x * 144;
    for (int i = 0; i < 12; ++i) {
        cplx s = 0;
        for (int j = 0; j < 12; ++j) s += m[i * 12 + j] * in[j];
        out[i] = s;
    }
}

/* Full 12x12 matrix A(x), index sc = 3*spin + colour. */
static void clover_matrix(const lat_t *l, const cplx *F, long x, cplx *Am /* [12][12] */)
{
    cplx e[12], col[12];
    for (int j = 0; j < 12; ++j) {
        memset(e, 0, sizeof(e));
        e[j] = 1;
        clover_from_fhat(l, F, x, e, col);
        for (int i = 0; i < 12; ++i) Am[i * 12 + j] = col[i];
    }
}

/* In-place inverse of an n x n complex matrix, Gauss-Jordan with partial
 * pivoting.  Returns 0 on success, -1 when a pivot vanishes.           */
static int invert_matrix(cplx *a, int n)
{
    int *piv = (int *)malloc(sizeof(int) * n);
    cplx *inv = (cplx *)calloc((size_t)n * n, sizeof(cplx));
    for (int i = 0; i < n; ++i) inv[i * n + i] = 1;
    int rc = 0;
    for (int c = 0; c < n; ++c) {
        int best = c;
        double bv = cabs(a[c * n + c]);
        for (int r = c + 1; r < n; ++r)
            if (cabs(a[r * n + c]) > bv) {
                bv = cabs(a[r * n + c]);
                best = r;
            }
        if (bv == 0.0) {
            rc = -1;
            break;
        }
        if (best != c)
            for (int k = 0; k < n; ++k) {
                cplx t = a[c * n + k];
                a[c * n + k] = a[best * n + k];
                a[best * n + k] = t;
                t = inv[c * n + k];
                inv[c * n + k] = inv[best * n + k];
                inv[best * n + k] = t;
            }
        cplx d = 1.0 / a[c * n + c];
        for (int k = 0; k < n; ++k) {
            a[c * n + k] *= d;
            inv[c * n + k] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            cplx f = a[r * n + c];
            if (f == 0) continue;
            for (int k = 0; k < n; ++k) {
                a[r * n + k] -= f * a[c * n + k];
                inv[r * n + k] -= f * inv[c * n + k];
            }
        }
    }
    if (rc == 0) memcpy(a, inv, sizeof(cplx) * (size_t)n * n);
    free(inv);
    free(piv);
    return rc;
}

/* Ainv[V][12][12] = Am[x]^{-1} at every site.  Returns number of singular sites. */
int orc_clover_inverse(long V, const double complex *Am, double complex *Ainv)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (long x = 0; x < V; ++x) {
        cplx *m = Ainv + x * 144;
        memcpy(m, Am + x * 144, sizeof(cplx) * 144);
        if (invert_matrix(m, 12) != 0) bad++;
    }
    return bad;
}

/* Clover matrices A(x) as 12x12 at every site (for tests). */
void orc_clover_matrices(const int *dims, double kappa, double csw, const double complex *F,
                         double complex *Am)
{
    lat_t l = make_lat(dims, kappa, csw, 1);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < l.V; ++x) clover_matrix(&l, F, x, Am + x * 144);
}

/* One hop term: out += sign * (1 - dir*gamma_mu) W in, with W = U_mu(x) for
 * dir=+1 and U_mu(x-mu)^+ for dir=-1; in/out [4][3]. */
static void add_hop(int mu, int dir, double sign, const cplx *W, int dagger, const cplx *in, cplx *out)
{
    init_gamma();
    cplx ucol[4][3];
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx acc = 0;
            for (int b = 0; b < 3; ++b) acc += (dagger ? conj(W[b * 3 + a]) : W[a * 3 + b]) * in[s * 3 + b];
            ucol[s][a] = acc;
        }
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx acc = ucol[s][a];
            for (int s2 = 0; s2 < 4; ++s2) acc -= (double)dir * G[mu][s][s2] * ucol[s2][a];
            out[s * 3 + a] += sign * acc;
        }
}

/* (H psi)(x) restricted by an optional predicate on the neighbour. */
static void hop_site(const lat_t *l, const cplx *U, long x, const cplx *in, cplx *out,
                     const int *blk, int drop_outside)
{
    for (int k = 0; k < 12; ++k) out[k] = 0;
    for (int mu = 0; mu < 4; ++mu) {
        long xf = neighbour(l, x, mu, +1);
        long xb = neighbour(l, x, mu, -1);
        if (!drop_outside || blk[xf] == blk[x])
            add_hop(mu, +1, hop_sign(l, x, mu, +1), link(U, x, mu), 0, in + xf * 12, out);
        if (!drop_outside || blk[xb] == blk[x])
            add_hop(mu, -1, hop_sign(l, x, mu, -1), link(U, xb, mu), 1, in + xb * 12, out);
    }
}

/* ------------------------------------------------------------------ */
/* The Dirac operator  M = A - kappa H  (section 2.2, D psi = eta)      */
/* ------------------------------------------------------------------ */

void orc_dirac(const int *dims, double kappa, int bc_t, const double complex *U, const double complex *Am,
               const double complex *in, double complex *out)
{
    lat_t l = make_lat(dims, kappa, 0, bc_t);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < l.V; ++x) {
        cplx a[12], h[12];
        clover_site(Am, x, in + x * 12, a);
        hop_site(&l, U, x, in, h, NULL, 0);
        for (int k = 0; k < 12; ++k) out[x * 12 + k] = a[k] - l.kappa * h[k];
    }
}

/* Hopping term alone, out = H in (for tests). */
void orc_hop(const int *dims, int bc_t, const double complex *U, const double complex *in,
             double complex *out)
{
    lat_t l = make_lat(dims, 0, 0, bc_t);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < l.V; ++x) hop_site(&l, U, x, in, out + x * 12, NULL, 0);
}

/* ------------------------------------------------------------------ */
/* Schwarz blocks (section 2.2: checkerboard of blocks Omega, Omega*)   */
/* ------------------------------------------------------------------ */

typedef struct {
    int b[4];    /* block extents */
    int nb[4];   /* blocks per direction */
    long Nb;     /* number of blocks */
    long Vb;     /* sites per block */
} blocks_t;

/* Returns 0, or -2 when the block grid is not a valid checkerboard. */
static int make_blocks(const lat_t *l, const int *b, blocks_t *g)
{
    g->Nb = 1;
    g->Vb = 1;
    for (int m = 0; m < 4; ++m) {
        if (b[m] <= 0 || l->L[m] % b[m] != 0) return -2;
        g->b[m] = b[m];
        g->nb[m] = l->L[m] / b[m];
        if (g->nb[m] % 2 != 0) return -2;  /* checkerboard must close periodically */
        if (b[m] % 2 != 0) return -2;      /* block parity = global parity */
        g->Nb *= g->nb[m];
        g->Vb *= b[m];
    }
    return 0;
}

/* lexicographic block index of site x */
static long block_of(const lat_t *l, const blocks_t *g, long x)
{
    int c[4];
    site_coords(l, x, c);
    long B = 0;
    for (int m = 0; m < 4; ++m) B = B * g->nb[m] + c[m] / g->b[m];
    return B;
}

static int block_colour(const blocks_t *g, long B)
{
    int s = 0;
    for (int m = 3; m >= 0; --m) {
        s += (int)(B % g->nb[m]);
        B /= g->nb[m];
    }
    return s & 1;
}

/* global site of local (lexicographic within block) index j in block B */
static long block_site(const lat_t *l, const blocks_t *g, long B, long j)
{
    int Bc[4], c[4];
    for (int m = 3; m >= 0; --m) {
        Bc[m] = (int)(B % g->nb[m]);
        B /= g->nb[m];
    }
    for (int m = 3; m >= 0; --m) {
        c[m] = Bc[m] * g->b[m] + (int)(j % g->b[m]);
        j /= g->b[m];
    }
    return site_index(l, c);
}

static int parity_of(const lat_t *l, long x)
{
    int c[4];
    site_coords(l, x, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* Map every site to its block (blk[V]), colour list etc.  Exported for tests. */
int orc_block_map(const int *dims, const int *b, long *blk /* [V] */, int *colour /* [Nb] */)
{
    lat_t l = make_lat(dims, 0, 0, 1);
    blocks_t g;
    if (make_blocks(&l, b, &g)) return -2;
    for (long x = 0; x < l.V; ++x) blk[x] = block_of(&l, &g, x);
    for (long B = 0; B < g.Nb; ++B) colour[B] = block_colour(&g, B);
    return 0;
}

/* Block-restricted (Dirichlet) Dirac operator D_Omega for every block at
 * once: hops whose neighbour lies in another block are dropped. */
int orc_dirac_dirichlet(const int *dims, double kappa, int bc_t, const int *b, const double complex *U,
                        const double complex *Am, const double complex *in, double complex *out)
{
    lat_t l = make_lat(dims, kappa, 0, bc_t);
    blocks_t g;
    if (make_blocks(&l, b, &g)) return -2;
    int *blk = (int *)malloc(sizeof(int) * l.V);
    for (long x = 0; x < l.V; ++x) blk[x] = (int)block_of(&l, &g, x);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < l.V; ++x) {
        cplx a[12], h[12];
        clover_site(Am, x, in + x * 12, a);
        hop_site(&l, U, x, in, h, blk, 1);
        for (int k = 0; k < 12; ++k) out[x * 12 + k] = a[k] - l.kappa * h[k];
    }
    free(blk);
    return 0;
}

/* ------------------------------------------------------------------ */
/* SAP (section 2.2):  psi -> psi + D_Lambda^{-1}(eta - D psi) on all    */
/* blocks of one colour, then the other; n_cy cycles from psi = 0.      */
/* The block solve D_Lambda delta = rho uses the even-odd reduced block */
/* operator  Dhat = A_ee - kappa^2 H_eo A_oo^{-1} H_oe  and n_mr        */
/* minimal-residual steps on it, starting from zero.                    */
/* ------------------------------------------------------------------ */

/* block-local work space: fields indexed by local site j (lexicographic) */
typedef struct {
    long *site;   /* global site of local j */
    int *par;     /* parity of local j */
    int *nbr;     /* [j][8]: local index of neighbour (mu,dir), -1 if outside */
} blockgeo_t;

static void block_geometry(const lat_t *l, const blocks_t *g, long B, blockgeo_t *bg)
{
    for (long j = 0; j < g->Vb; ++j) {
        bg->site[j] = block_site(l, g, B, j);
        bg->par[j] = parity_of(l, bg->site[j]);
    }
    /* local coordinates of j */
    for (long j = 0; j < g->Vb; ++j) {
        int c[4];
        long r = j;
        for (int m = 3; m >= 0; --m) {
            c[m] = (int)(r % g->b[m]);
            r /= g->b[m];
        }
        for (int mu = 0; mu < 4; ++mu)
            for (int d = 0; d < 2; ++d) {
                int cc[4] = {c[0], c[1], c[2], c[3]};
                cc[mu] += d == 0 ? +1 : -1;
                long k = -1;
                if (cc[mu] >= 0 && cc[mu] < g->b[mu]) {
                    k = 0;
                    for (int m = 0; m < 4; ++m) k = k * g->b[m] + cc[m];
                }
                bg->nbr[j * 8 + mu * 2 + d] = (int)k;
            }
    }
}

/* out_j = (H^Lambda in)_j on local sites of parity p (others untouched) */
static void block_hop(const lat_t *l, const cplx *U, const blocks_t *g, const blockgeo_t *bg, int p,
                      const cplx *in, cplx *out)
{
    for (long j = 0; j < g->Vb; ++j) {
        if (bg->par[j] != p) continue;
        cplx *o = out + j * 12;
        for (int k = 0; k < 12; ++k) o[k] = 0;
        long x = bg->site[j];
        for (int mu = 0; mu < 4; ++mu) {
            int jf = bg->nbr[j * 8 + mu * 2 + 0];
            int jb = bg->nbr[j * 8 + mu * 2 + 1];
            if (jf >= 0) add_hop(mu, +1, hop_sign(l, x, mu, +1), link(U, x, mu), 0, in + jf * 12, o);
            if (jb >= 0) add_hop(mu, -1, hop_sign(l, x, mu, -1), link(U, bg->site[jb], mu), 1, in + jb * 12, o);
        }
    }
}

static void mat12_vec(const cplx *m, const cplx *in, cplx *out)
{
    for (int i = 0; i < 12; ++i) {
        cplx s = 0;
        for (int j = 0; j < 12; ++j) s += m[i * 12 + j] * in[j];
        out[i] = s;
    }
}

/* delta = approximate D_Lambda^{-1} rho on one block (local arrays). */
static void block_solve(const lat_t *l, const cplx *U, const cplx *Am, const cplx *Ainv,
                        const blocks_t *g, const blockgeo_t *bg, int nmr, const cplx *rho,
                        cplx *delta, cplx *w1, cplx *w2, cplx *w3, cplx *w4)
{
    const long Vb = g->Vb;
    const double k = l->kappa;
    /* s_o = A_oo^{-1} rho_o  (kept in delta on odd sites) */
    for (long j = 0; j < Vb; ++j)
        if (bg->par[j] == 1) mat12_vec(Ainv + bg->site[j] * 144, rho + j * 12, delta + j * 12);
    /* rhat_e = rho_e + kappa H_eo s_o  -> r (w1) on even sites; x_e (w2) = 0 */
    block_hop(l, U, g, bg, 0, delta, w1);
    for (long j = 0; j < Vb; ++j)
        if (bg->par[j] == 0)
            for (int c = 0; c < 12; ++c) {
                w1[j * 12 + c] = rho[j * 12 + c] + k * w1[j * 12 + c];
                w2[j * 12 + c] = 0;
            }
    for (int it = 0; it < nmr; ++it) {
        /* p = Dhat r:  t_o = A_oo^{-1} H_oe r ;  p_e = A_ee r_e - kappa^2 H_eo t_o */
        block_hop(l, U, g, bg, 1, w1, w3);
        for (long j = 0; j < Vb; ++j)
            if (bg->par[j] == 1) {
                cplx t[12];
                mat12_vec(Ainv + bg->site[j] * 144, w3 + j * 12, t);
                for (int c = 0; c < 12; ++c) w3[j * 12 + c] = t[c];
            }
        block_hop(l, U, g, bg, 0, w3, w4);
        cplx pr = 0;
        double pp = 0;
        for (long j = 0; j < Vb; ++j)
            if (bg->par[j] == 0) {
                cplx a[12];
                clover_site(Am, bg->site[j], w1 + j * 12, a);
                for (int c = 0; c < 12; ++c) {
                    cplx p = a[c] - k * k * w4[j * 12 + c];
                    w4[j * 12 + c] = p;
                    pr += conj(p) * w1[j * 12 + c];
                    pp += creal(conj(p) * p);
                }
            }
        cplx alpha = pp > 0 ? pr / pp : 0;
        for (long j = 0; j < Vb; ++j)
            if (bg->par[j] == 0)
                for (int c = 0; c < 12; ++c) {
                    w2[j * 12 + c] += alpha * w1[j * 12 + c];
                    w1[j * 12 + c] -= alpha * w4[j * 12 + c];
                }
    }
    /* delta_e = x_e ;  delta_o = s_o + kappa A_oo^{-1} H_oe x_e */
    block_hop(l, U, g, bg, 1, w2, w3);
    for (long j = 0; j < Vb; ++j) {
        if (bg->par[j] == 0) {
            for (int c = 0; c < 12; ++c) delta[j * 12 + c] = w2[j * 12 + c];
        } else {
            cplx t[12];
            mat12_vec(Ainv + bg->site[j] * 144, w3 + j * 12, t);
            for (int c = 0; c < 12; ++c) delta[j * 12 + c] += k * t[c];
        }
    }
}

/* psi = M_SAP eta  (n_cy cycles from psi = 0). Returns 0 or -2 (geometry). */
int orc_sap(const int *dims, double kappa, int bc_t, const int *b, int ncy, int nmr,
            const double complex *U, const double complex *Am, const double complex *Ainv,
            const double complex *eta, double complex *psi)
{
    lat_t l = make_lat(dims, kappa, 0, bc_t);
    blocks_t g;
    if (make_blocks(&l, b, &g)) return -2;
    long V = l.V;
    cplx *rho = (cplx *)malloc(sizeof(cplx) * V * 12);
    memset(psi, 0, sizeof(cplx) * V * 12);
    for (int cy = 0; cy < ncy; ++cy) {
        for (int col = 0; col < 2; ++col) {
            /* rho = eta - M psi with the current psi (neighbours included) */
            orc_dirac(dims, kappa, bc_t, U, Am, psi, rho);
            for (long i = 0; i < V * 12; ++i) rho[i] = eta[i] - rho[i];
#pragma omp parallel
            {
                blockgeo_t bg;
                bg.site = (long *)malloc(sizeof(long) * g.Vb);
                bg.par = (int *)malloc(sizeof(int) * g.Vb);
                bg.nbr = (int *)malloc(sizeof(int) * g.Vb * 8);
                cplx *wk = (cplx *)malloc(sizeof(cplx) * g.Vb * 12 * 6);
#pragma omp for schedule(dynamic)
                for (long B = 0; B < g.Nb; ++B) {
                    if (block_colour(&g, B) != col) continue;
                    block_geometry(&l, &g, B, &bg);
                    cplx *r = wk, *d = wk + g.Vb * 12;
                    for (long j = 0; j < g.Vb; ++j)
                        for (int c = 0; c < 12; ++c) r[j * 12 + c] = rho[bg.site[j] * 12 + c];
                    block_solve(&l, U, Am, Ainv, &g, &bg, nmr, r, d, wk + 2 * g.Vb * 12,
                                wk + 3 * g.Vb * 12, wk + 4 * g.Vb * 12, wk + 5 * g.Vb * 12);
                    for (long j = 0; j < g.Vb; ++j)
                        for (int c = 0; c < 12; ++c) psi[bg.site[j] * 12 + c] += d[j * 12 + c];
                }
                free(wk);
                free(bg.site);
                free(bg.par);
                free(bg.nbr);
            }
        }
    }
    free(rho);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Little Dirac operator  A_kl = (phi_k, D phi_l)  (eq. little)          */
/* for block-local deflation fields phi[Nb][Ns][Vb][12] (local lex).    */
/* Stored by coupling direction: Alit[B][d][k][l], d = 0 self,          */
/* d = 1 + 2*mu (+mu neighbour block), d = 2 + 2*mu (-mu neighbour).    */
/* When a direction has only two blocks, +mu and -mu name the same      */
/* block and the two entries add up to its coupling.                    */
/* ------------------------------------------------------------------ */

int orc_little_op(const int *dims, double kappa, int bc_t, const int *b, int Ns, const double complex *U,
                  const double complex *Am, const double complex *phi, double complex *Alit)
{
    lat_t l = make_lat(dims, kappa, 0, bc_t);
    blocks_t g;
    if (make_blocks(&l, b, &g)) return -2;
    const long Vb = g.Vb;
    /* local index of each global site and its block */
    long *loc = (long *)malloc(sizeof(long) * l.V);
    long *bof = (long *)malloc(sizeof(long) * l.V);
    for (long B = 0; B < g.Nb; ++B)
        for (long j = 0; j < Vb; ++j) {
            long x = block_site(&l, &g, B, j);
            loc[x] = j;
            bof[x] = B;
        }
    memset(Alit, 0, sizeof(cplx) * g.Nb * 9 * Ns * Ns);
#pragma omp parallel
    {
        cplx *Dphi = (cplx *)malloc(sizeof(cplx) * 9 * Ns * Vb * 12);
#pragma omp for schedule(dynamic)
        for (long B = 0; B < g.Nb; ++B) {
            /* Dphi[d][l][j] = contribution to (D phi_{B_d, l})(x_j), x_j in B */
            memset(Dphi, 0, sizeof(cplx) * 9 * Ns * Vb * 12);
            for (long j = 0; j < Vb; ++j) {
                long x = block_site(&l, &g, B, j);
                for (int ll = 0; ll < Ns; ++ll) {
                    const cplx *own = phi + ((B * Ns + ll) * Vb) * 12;
                    cplx a[12], h[12];
                    /* self: clover + hops inside the block */
                    clover_site(Am, x, own + j * 12, a);
                    for (int c = 0; c < 12; ++c) h[c] = 0;
                    for (int mu = 0; mu < 4; ++mu)
                        for (int d = 0; d < 2; ++d) {
                            int dir = d == 0 ? +1 : -1;
                            long y = neighbour(&l, x, mu, dir);
                            long By = bof[y];
                            const cplx *W = dir > 0 ? link(U, x, mu) : link(U, y, mu);
                            const cplx *src = phi + ((By * Ns + ll) * Vb + loc[y]) * 12;
                            if (By == B) {
                                add_hop(mu, dir, hop_sign(&l, x, mu, dir), W, dir < 0, src, h);
                            } else {
                                cplx hh[12] = {0};
                                add_hop(mu, dir, hop_sign(&l, x, mu, dir), W, dir < 0, src, hh);
                                cplx *o = Dphi + (((1 + 2 * mu + d) * Ns + ll) * Vb + j) * 12;
                                for (int c = 0; c < 12; ++c) o[c] += -l.kappa * hh[c];
                            }
                        }
                    cplx *o = Dphi + ((0 * Ns + ll) * Vb + j) * 12;
                    for (int c = 0; c < 12; ++c) o[c] = a[c] - l.kappa * h[c];
                }
            }
            for (int d = 0; d < 9; ++d)
                for (int kk = 0; kk < Ns; ++kk)
                    for (int ll = 0; ll < Ns; ++ll) {
                        const cplx *pk = phi + ((B * Ns + kk) * Vb) * 12;
                        const cplx *q = Dphi + ((d * Ns + ll) * Vb) * 12;
                        cplx s = 0;
                        for (long i = 0; i < Vb * 12; ++i) s += conj(pk[i]) * q[i];
                        Alit[((B * 9 + d) * Ns + kk) * Ns + ll] = s;
                    }
        }
        free(Dphi);
    }
    free(loc);
    free(bof);
    return 0;
}

/* Neighbour block of B in coupling direction d (as used by orc_little_op). */
int orc_block_neighbours(const int *dims, const int *b, long *nbr /* [Nb][9] */)
{
    lat_t l = make_lat(dims, 0, 0, 1);
    blocks_t g;
    if (make_blocks(&l, b, &g)) return -2;
    for (long B = 0; B < g.Nb; ++B) {
        int Bc[4];
        long r = B;
        for (int m = 3; m >= 0; --m) {
            Bc[m] = (int)(r % g.nb[m]);
            r /= g.nb[m];
        }
        nbr[B * 9] = B;
        for (int mu = 0; mu < 4; ++mu)
            for (int d = 0; d < 2; ++d) {
                int c[4] = {Bc[0], Bc[1], Bc[2], Bc[3]};
                c[mu] = (c[mu] + (d == 0 ? 1 : -1) + g.nb[mu]) % g.nb[mu];
                long k = 0;
                for (int m = 0; m < 4; ++m) k = k * g.nb[m] + c[m];
                nbr[B * 9 + 1 + 2 * mu + d] = k;
            }
    }
    return 0;
}

/* Block-local site list: glob[B][j] = global site of local j in block B. */
int orc_block_sites(const int *dims, const int *b, long *glob)
{
    lat_t l = make_lat(dims, 0, 0, 1);
    blocks_t g;
    if (make_blocks(&l, b, &g)) return -2;
    for (long B = 0; B < g.Nb; ++B)
        for (long j = 0; j < g.Vb; ++j) glob[B * g.Vb + j] = block_site(&l, &g, B, j);
    return 0;
}

/* Counter-based generator (SplitMix64, Steele-Lea-Flood 2014): the n-th
 * output for state key.  Used for the random fields the method draws. */
static unsigned long long sm64(unsigned long long key, unsigned long long n)
{
    unsigned long long z = key + (n + 1ULL) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Complex Gaussian fields: component j (over n complex numbers) takes
 * Box-Muller numbers 2j (real) and 2j+1 (imaginary) of stream key. */
void orc_gaussian_fill(unsigned long long key, long n, double complex *out)
{
#pragma omp parallel for schedule(static)
    for (long j = 0; j < n; ++j) {
        double g[2];
        unsigned long long pair = (unsigned long long)j;  /* Gaussians 2j, 2j+1 share pair j */
        double u1 = 1.0 - (double)(sm64(key, 2 * pair) >> 11) * 0x1.0p-53;
        double u2 = (double)(sm64(key, 2 * pair + 1) >> 11) * 0x1.0p-53;
        double r = sqrt(-2.0 * log(u1));
        g[0] = r * cos(2.0 * M_PI * u2);
        g[1] = r * sin(2.0 * M_PI * u2);
        out[j] = g[0] + _Complex_I * g[1];
    }
}
