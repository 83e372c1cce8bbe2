/*
 * rlbm_oracle.c -- plain FP64 CPU oracle for the relativistic lattice
 * Boltzmann method (RLBM) for massless particles in (2+1) dimensions of
 * Bazzanini, Gabbana, Simeoni, Succi and Tripiccione, "A Lattice Boltzmann
 * Method for Relativistic Rarefied Flows in (2+1) Dimensions",
 * arXiv:2011.06856.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header,
 * table or constant with the GPU library: it has its own quadrature (root
 * bracketing on the Laguerre recurrence), its own polynomial basis (Cholesky
 * orthonormalisation of the light-cone monomials in the exact continuum inner
 * product), its own equilibrium coefficients (the covariant moment tensor of
 * the Maxwell-Juttner distribution), its own Landau-frame solver (bisection on
 * the characteristic cubic) and unfused stream / collide passes.
 *
 * Conventions (lattice units): metric eta = diag(+,-,-), c = 1, dx = dy = 1,
 * weighting temperature T0 = 1.  Velocity index v = i*K + j for radial shell i
 * and angle j.  Populations are stored f[v][y][x].
 *
 * Each function names the passage of the paper it follows.  Where the paper
 * is silent or garbled the reading taken is stated at the point of use.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef long double ld;

#define PI_L 3.141592653589793238462643383279502884L

/* ------------------------------------------------------------------------- */
/* Quadrature (Sec. 2.3, the product rule and its rotated off-lattice form)  */
/* ------------------------------------------------------------------------- */

/* Laguerre polynomial L_n(x) by its three-term recurrence. */
static ld laguerre(int n, ld x)
{
    ld l0 = 1.0L, l1 = 1.0L - x;
    if (n == 0) return l0;
    for (int k = 1; k < n; ++k) {
        ld l2 = ((2.0L * k + 1.0L - x) * l1 - k * l0) / (k + 1.0L);
        l0 = l1;
        l1 = l2;
    }
    return l1;
}

/* Roots of L_n: scan for sign changes on a fine grid, then bisect each
 * bracket until the interval no longer shrinks in long double. */
static int laguerre_roots(int n, ld* roots)
{
    const ld hi = 4.0L * n + 12.0L;
    const ld h = 1.0e-3L;
    int found = 0;
    ld xa = 1.0e-12L, fa = laguerre(n, xa);
    for (ld xb = xa + h; xb <= hi && found < n; xb += h) {
        ld fb = laguerre(n, xb);
        if ((fa < 0) != (fb < 0)) {
            ld lo = xa, up = xb, flo = fa;
            for (int it = 0; it < 200; ++it) {
                ld mid = 0.5L * (lo + up);
                if (mid <= lo || mid >= up) break;
                ld fm = laguerre(n, mid);
                if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; }
                else up = mid;
            }
            roots[found++] = 0.5L * (lo + up);
        }
        xa = xb;
        fa = fb;
    }
    return found;
}

typedef struct {
    int Np, K, N, nvel, nb, rotate;
    double *p, *theta, *w, *cth, *sth;   /* [nvel] */
    int *ea, *eb, *ec;                   /* monomial exponents, [nb] */
    ld *Linv;                            /* [nb][nb], J_b = sum_c Linv[b][c] m_c */
    double *J;                           /* [nb][nvel] basis values at the nodes */
} orc_quad;

/* Integral over [0, 2pi) of cos^b sin^c: zero unless b and c are both even,
 * otherwise 2 pi (b-1)!! (c-1)!! / (b+c)!!. */
static ld ang_int(int b, int c)
{
    if ((b & 1) || (c & 1)) return 0.0L;
    ld num = 1.0L, den = 1.0L;
    for (int k = b - 1; k > 0; k -= 2) num *= k;
    for (int k = c - 1; k > 0; k -= 2) num *= k;
    for (int k = b + c; k > 0; k -= 2) den *= k;
    return 2.0L * PI_L * num / den;
}

static ld factl(int k)
{
    ld r = 1.0L;
    for (int i = 2; i <= k; ++i) r *= i;
    return r;
}

/* Monomial m_c = (p^0)^a (p^x)^b (p^y)^c evaluated on the light cone. */
static ld mono_eval(int a, int b, int c, ld p, ld ct, ld st)
{
    ld r = 1.0L;
    for (int k = 0; k < a; ++k) r *= p;
    for (int k = 0; k < b; ++k) r *= p * ct;
    for (int k = 0; k < c; ++k) r *= p * st;
    return r;
}

void orc_quad_free(orc_quad* q)
{
    if (!q) return;
    free(q->p); free(q->theta); free(q->w); free(q->cth); free(q->sth);
    free(q->ea); free(q->eb); free(q->ec); free(q->Linv); free(q->J);
    free(q);
}

/*
 * Build the quadrature and the basis.
 *   Np      radial shells: the roots p_i of the Laguerre polynomial L_Np, with
 *           weights p_i / ((Np+1)^2 L_{Np+1}(p_i)^2) (Gauss-Laguerre, Sec. 2.3).
 *   K       angles per shell, theta_ij = (j + i/Np) 2 pi / K when rotate != 0
 *           (Eq. off-lattice-quad; the paper writes the offset i/(N+1) with
 *           N+1 shells, read here as i/Np so that shells spread evenly for any
 *           order), theta_ij = 2 pi j / K when rotate == 0.
 *   N       order of the truncated equilibrium expansion.
 * The basis J_b of Eq. mj-feq-expansion is not printed in the paper; here it
 * is the orthonormalisation (Cholesky of the Gram matrix, i.e. Gram-Schmidt in
 * degree order) of the (N+1)^2 independent light-cone monomials
 * (p^0)^a (p^x)^b (p^y)^c, a in {0,1}, a+b+c <= N, in the continuum inner
 * product <f,g> = int_0^inf int_0^2pi e^{-p} f g dtheta dp, whose weight is
 * the rest-frame equilibrium omega(p^0) with T0 = 1 (Sec. 2.2).
 */
orc_quad* orc_quad_new(int Np, int K, int N, int rotate)
{
    if (Np < 1 || Np > 16 || K < 1 || N < 0 || N > 8) return NULL;
    orc_quad* q = (orc_quad*)calloc(1, sizeof(orc_quad));
    q->Np = Np; q->K = K; q->N = N; q->rotate = rotate ? 1 : 0;
    q->nvel = Np * K;
    q->nb = (N + 1) * (N + 1);
    int nv = q->nvel, nb = q->nb;
    q->p = (double*)malloc(sizeof(double) * nv);
    q->theta = (double*)malloc(sizeof(double) * nv);
    q->w = (double*)malloc(sizeof(double) * nv);
    q->cth = (double*)malloc(sizeof(double) * nv);
    q->sth = (double*)malloc(sizeof(double) * nv);

    ld roots[16];
    if (laguerre_roots(Np, roots) != Np) { orc_quad_free(q); return NULL; }
    for (int i = 0; i < Np; ++i) {
        ld pi_ = roots[i];
        ld lnext = laguerre(Np + 1, pi_);
        ld wr = pi_ / ((ld)(Np + 1) * (Np + 1) * lnext * lnext);
        for (int j = 0; j < K; ++j) {
            int v = i * K + j;
            ld off = q->rotate ? (ld)i / (ld)Np : 0.0L;
            ld th = ((ld)j + off) * (2.0L * PI_L) / (ld)K;
            q->p[v] = (double)pi_;
            q->theta[v] = (double)th;
            q->w[v] = (double)(wr * (2.0L * PI_L) / (ld)K);
            q->cth[v] = (double)cosl(th);
            q->sth[v] = (double)sinl(th);
        }
    }

    /* light-cone monomials in degree order */
    q->ea = (int*)malloc(sizeof(int) * nb);
    q->eb = (int*)malloc(sizeof(int) * nb);
    q->ec = (int*)malloc(sizeof(int) * nb);
    int c = 0;
    for (int d = 0; d <= N; ++d)
        for (int a = 0; a <= 1 && a <= d; ++a)
            for (int b = d - a; b >= 0; --b) {
                q->ea[c] = a; q->eb[c] = b; q->ec[c] = d - a - b; ++c;
            }

    /* Gram matrix in the continuum inner product, then Cholesky G = L L^T
     * and J = L^{-1} m. */
    ld* G = (ld*)calloc((size_t)nb * nb, sizeof(ld));
    ld* L = (ld*)calloc((size_t)nb * nb, sizeof(ld));
    q->Linv = (ld*)calloc((size_t)nb * nb, sizeof(ld));
    for (int r = 0; r < nb; ++r)
        for (int s = 0; s < nb; ++s) {
            int deg = q->ea[r] + q->eb[r] + q->ec[r] + q->ea[s] + q->eb[s] + q->ec[s];
            G[r * nb + s] = factl(deg) * ang_int(q->eb[r] + q->eb[s], q->ec[r] + q->ec[s]);
        }
    for (int r = 0; r < nb; ++r) {
        for (int s = 0; s <= r; ++s) {
            ld acc = G[r * nb + s];
            for (int k = 0; k < s; ++k) acc -= L[r * nb + k] * L[s * nb + k];
            if (r == s) {
                if (acc <= 0) { free(G); free(L); orc_quad_free(q); return NULL; }
                L[r * nb + r] = sqrtl(acc);
            } else {
                L[r * nb + s] = acc / L[s * nb + s];
            }
        }
    }
    for (int col = 0; col < nb; ++col) {          /* forward substitution */
        for (int r = 0; r < nb; ++r) {
            ld acc = (r == col) ? 1.0L : 0.0L;
            for (int k = 0; k < r; ++k) acc -= L[r * nb + k] * q->Linv[k * nb + col];
            q->Linv[r * nb + col] = acc / L[r * nb + r];
        }
    }
    free(G); free(L);

    q->J = (double*)malloc(sizeof(double) * (size_t)nb * nv);
    for (int v = 0; v < nv; ++v) {
        ld ct = (ld)q->cth[v], st = (ld)q->sth[v], pp = (ld)q->p[v];
        ld m[81];
        for (int s = 0; s < nb; ++s) m[s] = mono_eval(q->ea[s], q->eb[s], q->ec[s], pp, ct, st);
        for (int b = 0; b < nb; ++b) {
            ld acc = 0.0L;
            for (int s = 0; s <= b; ++s) acc += q->Linv[b * nb + s] * m[s];
            q->J[(size_t)b * nv + v] = (double)acc;
        }
    }
    return q;
}

int orc_quad_nvel(const orc_quad* q) { return q->nvel; }
int orc_quad_nbasis(const orc_quad* q) { return q->nb; }

void orc_quad_get(const orc_quad* q, double* p, double* theta, double* w, double* cth, double* sth)
{
    for (int v = 0; v < q->nvel; ++v) {
        if (p) p[v] = q->p[v];
        if (theta) theta[v] = q->theta[v];
        if (w) w[v] = q->w[v];
        if (cth) cth[v] = q->cth[v];
        if (sth) sth[v] = q->sth[v];
    }
}

/* Basis values at the nodes, J[b][v], and the exponents of monomial b. */
void orc_quad_basis(const orc_quad* q, double* J, int* expo /* [nb][3] or NULL */)
{
    memcpy(J, q->J, sizeof(double) * (size_t)q->nb * q->nvel);
    if (expo)
        for (int b = 0; b < q->nb; ++b) {
            expo[3 * b] = q->ea[b]; expo[3 * b + 1] = q->eb[b]; expo[3 * b + 2] = q->ec[b];
        }
}

/* ------------------------------------------------------------------------- */
/* Equilibrium moments and coefficients (Sec. 2.1 Eq. feq_dist, Sec. 2.2)    */
/* ------------------------------------------------------------------------- */

static ld dfact(int m)
{
    ld r = 1.0L;
    for (int k = m; k > 1; k -= 2) r *= k;
    return r;
}

/* Sum over partial pairings of the index positions not yet used: a paired
 * couple contributes eta^{mu nu}, an unpaired index contributes U^mu, and a
 * pairing with l couples is weighted (-1)^l (2k-2l-1)!!. */
static ld pair_sum(const int* idx, int k, unsigned used, int l, ld prod, const ld* U)
{
    int first = -1;
    for (int i = 0; i < k; ++i)
        if (!(used & (1u << i))) { first = i; break; }
    if (first < 0) {
        ld sgn = (l & 1) ? -1.0L : 1.0L;
        return sgn * dfact(2 * k - 2 * l - 1) * prod;
    }
    unsigned u1 = used | (1u << first);
    ld acc = pair_sum(idx, k, u1, l, prod * U[idx[first]], U);
    for (int j = first + 1; j < k; ++j) {
        if (used & (1u << j)) continue;
        ld eta = (idx[first] != idx[j]) ? 0.0L : (idx[first] == 0 ? 1.0L : -1.0L);
        if (eta == 0.0L) continue;
        acc += pair_sum(idx, k, u1 | (1u << j), l + 1, prod * eta, U);
    }
    return acc;
}

/*
 * Rank-k moment of the Maxwell-Juttner equilibrium of a massless gas in 2+1D,
 *   int f_eq p^{mu_1} ... p^{mu_k} d^2p / p^0,
 * with f_eq = n / (2 pi T^2) exp(-U.p / T) (Eq. feq_dist with epsilon = 0,
 * normalised so that N^mu = n U^mu).  From the generating integral
 * int exp(-beta.p) d^2p/p^0 = 2 pi (beta.beta)^{-1/2} one finds
 *   n T^{k-1} sum_l (-1)^l (2k-2l-1)!! [U^{k-2l} eta^l]_sym,
 * the bracket summing over all ways of placing the l metric factors.
 * idx[i] in {0,1,2}; U = (U^0, U^x, U^y).
 */
static ld mj_moment(const int* idx, int k, ld n, ld T, const ld* U)
{
    return n * powl(T, (ld)(k - 1)) * pair_sum(idx, k, 0u, 0, 1.0L, U);
}

double orc_mj_moment(int k, const int* idx, double n, double T, double ux, double uy)
{
    ld U[3] = {sqrtl(1.0L + (ld)ux * ux + (ld)uy * uy), ux, uy};
    return (double)mj_moment(idx, k, n, T, U);
}

/* Expansion coefficients a_b = int f_eq J_b d^2p/p^0 (Eq.
 * mj-projection-coefficients), each J_b being a combination of monomials. */
static void eq_coeffs(const orc_quad* q, ld n, ld T, const ld* U, const ld* phi, ld* a)
{
    int nb = q->nb;
    ld mu[81];
    for (int s = 0; s < nb; ++s) {
        int idx[16], k = 0;
        for (int t = 0; t < q->ea[s]; ++t) idx[k++] = 0;
        for (int t = 0; t < q->eb[s]; ++t) idx[k++] = 1;
        for (int t = 0; t < q->ec[s]; ++t) idx[k++] = 2;
        /* Fermi-Dirac / Bose-Einstein: the rank-k moment is the
         * Maxwell-Juttner one scaled by phi[k] (see qs_G below) */
        mu[s] = mj_moment(idx, k, n, T, U) * (phi ? phi[k] : 1.0L);
    }
    for (int b = 0; b < nb; ++b) {
        ld acc = 0.0L;
        for (int s = 0; s <= b; ++s) acc += q->Linv[b * nb + s] * mu[s];
        a[b] = acc;
    }
}

/* Discrete truncated equilibrium f_eq_v = w_v sum_b a_b J_b(p_v)
 * (Eq. mj-feq-expansion-truncated).  The truncation is not clamped. */
static void feq_site(const orc_quad* q, ld n, ld T, const ld* U, const ld* phi, double* feq)
{
    ld a[81];
    eq_coeffs(q, n, T, U, phi, a);
    for (int v = 0; v < q->nvel; ++v) {
        ld acc = 0.0L;
        for (int b = 0; b < q->nb; ++b) acc += a[b] * (ld)q->J[(size_t)b * q->nvel + v];
        feq[v] = (double)((ld)q->w[v] * acc);
    }
}

void orc_feq(const orc_quad* q, double n, double T, double ux, double uy, double* feq)
{
    ld U[3] = {sqrtl(1.0L + (ld)ux * ux + (ld)uy * uy), ux, uy};
    feq_site(q, n, T, U, NULL, feq);
}

void orc_eq_coeffs(const orc_quad* q, double n, double T, double ux, double uy, double* a)
{
    ld U[3] = {sqrtl(1.0L + (ld)ux * ux + (ld)uy * uy), ux, uy};
    ld al[81];
    eq_coeffs(q, n, T, U, NULL, al);
    for (int b = 0; b < q->nb; ++b) a[b] = (double)al[b];
}

/* ------------------------------------------------------------------------- */
/* Fermi-Dirac and Bose-Einstein equilibria (Eq. feq_dist, epsilon = +-1)    */
/* ------------------------------------------------------------------------- */

/*
 * f_eq = A / (z^-1 exp(U.p / T) + epsilon), z = exp(mu / T), with the fixed
 * normalisation A = 1/(2 pi) (the paper writes f_eq only up to a factor;
 * with it epsilon -> 0 gives the Maxwell-Juttner form used above, with
 * z = n / T^2).  Since f_eq depends on p only through U.p / T, its rank-k
 * moment is A T^(k+1) k! G_k(z) times the same angular tensor as the
 * Maxwell-Juttner one, with the radial integral
 *   G_k(z) = (1/k!) int_0^inf x^k / (z^-1 e^x + epsilon) dx
 *          = z (MJ), -Li_{k+1}(-z) (FD), Li_{k+1}(z) (BE, z <= 1).
 * Hence n = T^2 G_1(z), and the rank-k moment equals the Maxwell-Juttner one
 * at the same (n, T, U) times phi_k = G_k(z) / G_1(z); eps = 2 n T phi_2,
 * P = eps / 2 as before.  Statistics: 0 MJ, 1 FD, 2 BE.
 */
enum { STAT_MJ = 0, STAT_FD = 1, STAT_BE = 2 };

/* zeta(n) for integer n != 1: n >= 2 by a direct sum with the
 * Euler-Maclaurin tail; zeta(0) = -1/2; zeta(-m) = 0 for even m > 0 and
 * zeta(1 - 2k) = (-1)^k 2 (2k-1)! zeta(2k) / (2 pi)^(2k). */
static ld zeta_eval(int n)
{
    if (n >= 2) {
        const int M = 1000;
        ld s = 0.0L;
        for (int j = M - 1; j >= 1; --j) s += powl((ld)j, (ld)-n);
        ld Mn = powl((ld)M, (ld)-n);
        s += powl((ld)M, (ld)(1 - n)) / (n - 1) + 0.5L * Mn + n * Mn / (12.0L * M)
           - (ld)n * (n + 1) * (n + 2) * Mn / (720.0L * M * M * M);
        return s;
    }
    if (n == 0) return -0.5L;
    int m = -n;
    if (m % 2 == 0) return 0.0L;
    int k = (m + 1) / 2;
    ld f = 1.0L;
    for (int i = 2; i <= 2 * k - 1; ++i) f *= i;
    return ((k & 1) ? -1.0L : 1.0L) * 2.0L * f * zeta_eval(2 * k) / powl(2.0L * PI_L, (ld)(2 * k));
}

/* zeta(n) for -ZMIN <= n <= ZMAX, tabulated once when the library loads. */
#define ZMIN 80
#define ZMAX 24
static ld zeta_tab[ZMIN + ZMAX + 1];
__attribute__((constructor)) static void zeta_init(void)
{
    for (int n = -ZMIN; n <= ZMAX; ++n) zeta_tab[n + ZMIN] = n == 1 ? 0.0L : zeta_eval(n);
}
static ld zeta_int(int n) { return zeta_tab[n + ZMIN]; }

static ld ipow(ld x, int e)
{
    ld r = 1.0L;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

/* sum_{j>=1} (-1)^(j+1) x^j / j^s = -Li_s(-x) for 0 <= x <= 1, by the
 * alternating-series acceleration of Cohen, Rodriguez Villegas and Zagier
 * (their algorithm 1; the terms form a moment sequence). */
static ld alt_polylog(int s, ld x)
{
    const int N = 40;
    ld d = powl(3.0L + sqrtl(8.0L), (ld)N);
    d = 0.5L * (d + 1.0L / d);
    ld b = -1.0L, c = -d, sum = 0.0L, xp = 1.0L;
    for (int k = 0; k < N; ++k) {
        c = b - c;
        xp *= x;
        sum += c * xp / ipow((ld)(k + 1), s);
        b = (ld)(k + N) * (ld)(k - N) * b / ((k + 0.5L) * (k + 1.0L));
    }
    return sum / d;
}

/* -Li_s(-x), x >= 0, s >= 1: the accelerated series for x <= 1, else the
 * inversion formula
 *   -Li_s(-x) = mu^s/s! + 2 sum_{j=1}^{s/2} eta(2j) mu^(s-2j)/(s-2j)! + (-1)^s Li_s(-1/x),
 * mu = ln x, eta(2j) = (1 - 2^(1-2j)) zeta(2j). */
static ld fd_polylog(int s, ld x)
{
    if (x <= 1.0L) return alt_polylog(s, x);
    ld mu = logl(x), r = 0.0L, f = 1.0L;
    for (int i = 2; i <= s; ++i) f *= i;
    r = powl(mu, (ld)s) / f;
    for (int j = 1; 2 * j <= s; ++j) {
        ld g = 1.0L;
        for (int i = 2; i <= s - 2 * j; ++i) g *= i;
        r += 2.0L * (1.0L - powl(2.0L, (ld)(1 - 2 * j))) * zeta_int(2 * j) * powl(mu, (ld)(s - 2 * j)) / g;
    }
    return r - ((s & 1) ? -1.0L : 1.0L) * alt_polylog(s, 1.0L / x);
}

/* Li_s(x), 0 <= x <= 1, s >= 1: -ln(1 - x) for s = 1; the power series for
 * x <= 1/2; else the expansion in mu = ln x (|mu| < 2 pi)
 *   Li_s(e^mu) = sum_{j != s-1} zeta(s-j) mu^j/j! + mu^(s-1)/(s-1)! (H_{s-1} - ln(-mu)). */
static ld be_polylog(int s, ld x)
{
    if (s == 1) return -log1pl(-x);
    if (x <= 0.5L) {
        ld sum = 0.0L, xp = 1.0L;
        for (int j = 1; j < 200; ++j) {
            xp *= x;
            ld t = xp / ipow((ld)j, s);
            sum += t;
            if (t < 1e-24L * sum) break;
        }
        return sum;
    }
    if (x >= 1.0L) return zeta_int(s);
    ld mu = logl(x), sum = 0.0L, term = 1.0L;   /* term = mu^j / j! */
    for (int j = 0; j < 60 && s - j >= -ZMIN; ++j) {
        if (j == s - 1) {
            ld H = 0.0L;
            for (int i = 1; i <= s - 1; ++i) H += 1.0L / i;
            sum += term * (H - logl(-mu));
        } else {
            sum += zeta_int(s - j) * term;
        }
        term *= mu / (j + 1);
    }
    return sum;
}

/* G_k(z) of the statistics stat. */
static ld qs_G(int k, ld z, int stat)
{
    if (stat == STAT_FD) return fd_polylog(k + 1, z);
    if (stat == STAT_BE) return be_polylog(k + 1, z);
    return z;
}

double orc_qs_G(int k, double z, int stat) { return (double)qs_G(k, z, stat); }

/* z of the initial state (n, T): G_1(z) = n / T^2, by bisection in ln z
 * (G_1 increases with z).  Returns 0, or 1 without a solution (BE above
 * G_1(1) = zeta(2)). */
static int qs_z_of_nT(ld n, ld T, int stat, ld* z)
{
    ld target = n / (T * T);
    if (stat == STAT_MJ) { *z = target; return 0; }
    ld lo = -80.0L, hi = stat == STAT_BE ? 0.0L : 80.0L;
    if (!(qs_G(1, expl(hi), stat) >= target)) return 1;
    for (int it = 0; it < 120; ++it) {
        ld mid = 0.5L * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (qs_G(1, expl(mid), stat) < target) lo = mid; else hi = mid;
    }
    *z = expl(0.5L * (lo + hi));
    return 0;
}

/* eps^2 / n^3 of the equilibrium of fugacity e^y: 4 G_2^2 / G_1^3. */
static ld qs_h(ld y, int stat)
{
    ld z = expl(y), g1 = qs_G(1, z, stat), g2 = qs_G(2, z, stat);
    return 4.0L * g2 * g2 / (g1 * g1 * g1);
}

/* Temperature, fugacity and moment factors of a Landau frame (n, eps):
 * z solves 4 G_2(z)^2 / G_1(z)^3 = eps^2 / n^3 (decreasing in z; bisection
 * in ln z), T = sqrt(n / G_1(z)), phi_k = G_k / G_1 for k <= kmax.
 * Returns 0, or 1 without a solution (FD below the degenerate limit 8/9, BE
 * below the value at z = 1). */
static int qs_frame(ld n, ld eps, int stat, int kmax, ld* T, ld* z, ld* phi)
{
    if (stat == STAT_MJ) {
        *T = eps / (2.0L * n);
        *z = n / (*T * *T);
        for (int k = 0; k <= kmax; ++k) phi[k] = 1.0L;
        return 0;
    }
    ld r = eps * eps / (n * n * n);
    ld lo = -80.0L, hi = stat == STAT_BE ? 0.0L : 80.0L;
    if (!(qs_h(hi, stat) <= r)) return 1;
    for (int it = 0; it < 120; ++it) {
        ld mid = 0.5L * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (qs_h(mid, stat) > r) lo = mid; else hi = mid;
    }
    *z = expl(0.5L * (lo + hi));
    ld G1 = qs_G(1, *z, stat);
    *T = sqrtl(n / G1);
    for (int k = 0; k <= kmax; ++k) phi[k] = qs_G(k, *z, stat) / G1;
    return 0;
}

/* The discrete truncated equilibrium of (n, T, U) under statistics stat
 * (rlbm_oracle's Maxwell-Juttner route with the factors phi_k); returns 1
 * if (n, T) has no equilibrium of that statistics. */
int orc_feq_qs(const orc_quad* q, double n, double T, double ux, double uy, int stat, double* feq)
{
    ld U[3] = {sqrtl(1.0L + (ld)ux * ux + (ld)uy * uy), ux, uy};
    ld z, phi[17];
    if (qs_z_of_nT(n, T, stat, &z)) return 1;
    ld G1 = qs_G(1, z, stat);
    for (int k = 0; k <= q->N + 1 && k < 17; ++k) phi[k] = stat == STAT_MJ ? 1.0L : qs_G(k, z, stat) / G1;
    feq_site(q, n, T, U, phi, feq);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Moments and the Landau frame (Eq. discrete_sum_moments, the eigenvalue    */
/* problem eps U^a = T^{ab} U_b, and the ideal equation of state eps = 2nT)  */
/* ------------------------------------------------------------------------- */

/* mom = (N^0, N^x, N^y, T^00, T^0x, T^0y, T^xx, T^xy, T^yy), summed in v order. */
static void moments_site(const orc_quad* q, const double* f, long stride, double* mom)
{
    double m[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int v = 0; v < q->nvel; ++v) {
        double fv = f[(long)v * stride];
        double p0 = q->p[v], px = q->p[v] * q->cth[v], py = q->p[v] * q->sth[v];
        m[0] += p0 * fv;      m[1] += px * fv;      m[2] += py * fv;
        m[3] += p0 * p0 * fv; m[4] += p0 * px * fv; m[5] += p0 * py * fv;
        m[6] += px * px * fv; m[7] += px * py * fv; m[8] += py * py * fv;
    }
    memcpy(mom, m, sizeof(m));
}

void orc_moments(const orc_quad* q, const double* f, double* mom) { moments_site(q, f, 1, mom); }

/* det(T^{mu nu} - lambda eta^{mu nu}) */
static ld char_poly(const ld* t, ld lam)
{
    ld a00 = t[3] - lam, a01 = t[4], a02 = t[5];
    ld a11 = t[6] + lam, a12 = t[7], a22 = t[8] + lam;
    return a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02) + a02 * (a01 * a12 - a11 * a02);
}

/*
 * Landau frame: eps is the largest root of det(T - lambda eta) = 0, found by
 * bisection on [0, G] with G the Gershgorin bound of T^mu_nu; u_mu spans the
 * null space of T - eps eta (largest cross product of two rows); U^mu = eta
 * u, normalised to U.U = 1 with U^0 > 0; n = U_mu N^mu; T = eps / (2n).
 * Returns 0, or 1 when the state is not physical (no positive root above the
 * others, no timelike eigenvector, n <= 0 or eps <= 0).
 * out = (n, eps, U^x, U^y, T, U^0).
 */
static int landau_site(const double* mom, ld* out)
{
    ld t[9];
    for (int i = 0; i < 9; ++i) t[i] = (ld)mom[i];
    ld g0 = fabsl(t[3]) + fabsl(t[4]) + fabsl(t[5]);
    ld g1 = fabsl(t[6]) + fabsl(t[4]) + fabsl(t[7]);
    ld g2 = fabsl(t[8]) + fabsl(t[5]) + fabsl(t[7]);
    ld hi = g0 > g1 ? g0 : g1;
    hi = hi > g2 ? hi : g2;
    ld lo = 0.0L;
    if (!(hi > 0) || !(char_poly(t, lo) > 0)) return 1;
    for (int it = 0; it < 400; ++it) {
        ld mid = 0.5L * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (char_poly(t, mid) > 0) lo = mid; else hi = mid;
    }
    ld eps = 0.5L * (lo + hi);
    ld M[3][3] = {{t[3] - eps, t[4], t[5]}, {t[4], t[6] + eps, t[7]}, {t[5], t[7], t[8] + eps}};
    ld best[3] = {0, 0, 0}, bn = -1.0L;
    for (int r = 0; r < 3; ++r)
        for (int s = r + 1; s < 3; ++s) {
            ld c[3] = {M[r][1] * M[s][2] - M[r][2] * M[s][1],
                       M[r][2] * M[s][0] - M[r][0] * M[s][2],
                       M[r][0] * M[s][1] - M[r][1] * M[s][0]};
            ld nn = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
            if (nn > bn) { bn = nn; best[0] = c[0]; best[1] = c[1]; best[2] = c[2]; }
        }
    ld U0 = best[0], Ux = -best[1], Uy = -best[2];
    ld norm2 = U0 * U0 - Ux * Ux - Uy * Uy;
    if (!(norm2 > 0)) return 1;
    ld s = 1.0L / sqrtl(norm2);
    if (U0 < 0) s = -s;
    U0 *= s; Ux *= s; Uy *= s;
    ld n = U0 * t[0] - Ux * t[1] - Uy * t[2];
    if (!(n > 0) || !(eps > 0)) return 1;
    out[0] = n; out[1] = eps; out[2] = Ux; out[3] = Uy; out[4] = eps / (2.0L * n); out[5] = U0;
    return 0;
}

/* Landau frame and statistics of nine moments: out8 = (n, eps, U^x, U^y, T,
 * U^0, z, phi_2); returns 1 for a state without such an equilibrium. */
int orc_qs_landau(const double* mom, int stat, double* out8)
{
    ld o[6], T = 0, z = 0, phi[3] = {0, 0, 0};
    int bad = landau_site(mom, o) || qs_frame(o[0], o[1], stat, 2, &T, &z, phi);
    out8[0] = (double)o[0]; out8[1] = (double)o[1]; out8[2] = (double)o[2]; out8[3] = (double)o[3];
    out8[4] = (double)T; out8[5] = (double)o[5]; out8[6] = (double)z; out8[7] = (double)phi[2];
    if (bad)
        for (int i = 0; i < 8; ++i) out8[i] = NAN;
    return bad;
}

int orc_landau(const double* mom, double* out6)
{
    ld o[6];
    int bad = landau_site(mom, o);
    for (int i = 0; i < 6; ++i) out6[i] = bad ? NAN : (double)o[i];
    return bad;
}

/* ------------------------------------------------------------------------- */
/* Lattice evolution (Eq. discrete-rbe split into Eq. streaming with the     */
/* bilinear interpolation of Eq. interpolation, then Eq. collision)          */
/* ------------------------------------------------------------------------- */

/* Boundary condition per axis.  The paper uses a box domain without stating
 * its boundaries and names boundary conditions as the next step (Sec. 4);
 * beyond periodic and zero-gradient (clamp) edges, two kinds are defined
 * here for an upwind point that falls outside the grid:
 *   WALL   halfway bounce-back: the point takes the population of the
 *          reversed velocity (theta + pi, same shell) at the target cell
 *          itself, so what a cell sends toward the wall returns to it
 *          reversed (mass and energy conserved per cell, momentum not);
 *   FIXED  a reservoir: the point takes the initial population (the
 *          truncated equilibrium of the initial fields) of the edge cell it
 *          is clamped to, for ever (inflow at a fixed state; outflow of
 *          whatever reaches the edge).
 * A point across a wall takes the wall's value even where the other axis is
 * FIXED. */
enum { BC_PERIODIC = 0, BC_CLAMP = 1, BC_WALL = 2, BC_FIXED = 3 };

typedef struct {
    const orc_quad* q;
    int nx, ny, bcx, bcy;       /* BC_* per axis */
    double tau, dt;
    double *f, *fs;             /* [nvel][ny][nx] */
    double *f0;                 /* initial populations (FIXED edges), or NULL */
    int stat;                   /* STAT_MJ, STAT_FD, STAT_BE */
    long nonphys;
} orc_sim;

static int wrap(int i, int n, int bc)
{
    if (i >= 0 && i < n) return i;
    if (bc == BC_PERIODIC) return ((i % n) + n) % n;
    return i < 0 ? 0 : n - 1;
}

/* The reversed velocity of v: angle theta + pi on the same shell. */
static int reversed(const orc_quad* q, int v)
{
    int i = v / q->K, j = v % q->K;
    return i * q->K + (j + q->K / 2) % q->K;
}

static int site_eq(const orc_quad* q, double n, double T, double ux, double uy, int stat, double* out, long stride)
{
    double tmp[4096];
    double* buf = q->nvel <= 4096 ? tmp : (double*)malloc(sizeof(double) * q->nvel);
    int bad = orc_feq_qs(q, n, T, ux, uy, stat, buf);
    for (int v = 0; v < q->nvel; ++v) out[(long)v * stride] = buf[v];
    if (buf != tmp) free(buf);
    return bad;
}

/* Initial populations: the truncated equilibrium of the given fields
 * (host arrays [ny][nx]; u = spatial part U^i of the four-velocity). */
orc_sim* orc_sim_new(const orc_quad* q, int nx, int ny, const double* n, const double* T,
                     const double* ux, const double* uy, double tau, double dt, int bcx, int bcy, int stat)
{
    if (!q || nx < 1 || ny < 1) return NULL;
    if (stat < STAT_MJ || stat > STAT_BE) return NULL;
    if (bcx < BC_PERIODIC || bcx > BC_FIXED || bcy < BC_PERIODIC || bcy > BC_FIXED) return NULL;
    if ((bcx == BC_WALL || bcy == BC_WALL) && (q->K % 2)) return NULL;   /* no reversed velocity */
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->q = q; s->nx = nx; s->ny = ny; s->bcx = bcx; s->bcy = bcy; s->tau = tau; s->dt = dt; s->stat = stat;
    long S = (long)nx * ny;
    s->f = (double*)malloc(sizeof(double) * S * q->nvel);
    s->fs = (double*)malloc(sizeof(double) * S * q->nvel);
    long bad = 0;
    #pragma omp parallel for schedule(static) reduction(+ : bad)
    for (long i = 0; i < S; ++i)
        bad += site_eq(q, n[i], T[i], ux ? ux[i] : 0.0, uy ? uy[i] : 0.0, stat, s->f + i, S);
    if (bad) {   /* (n, T) without an equilibrium of this statistics */
        free(s->f); free(s->fs); free(s);
        return NULL;
    }
    if (bcx == BC_FIXED || bcy == BC_FIXED) {
        s->f0 = (double*)malloc(sizeof(double) * S * q->nvel);
        memcpy(s->f0, s->f, sizeof(double) * S * q->nvel);
    }
    return s;
}

void orc_sim_free(orc_sim* s)
{
    if (!s) return;
    free(s->f); free(s->fs); free(s->f0); free(s);
}

/* Streaming with bilinear interpolation from the upwind cell quad.  In
 * lattice units (dx = dy = 1) the weights are a_x = dt |cos theta| for the
 * node displaced by -sgn(cos theta) in x, (1 - a_x) for the own column, and
 * likewise in y; sgn(0) = +1.  The printed formula lacks its "+" signs and
 * mixes dimensional factors; this is the standard upwind bilinear reading. */
static void stream_pass(orc_sim* s)
{
    const orc_quad* q = s->q;
    int nx = s->nx, ny = s->ny;
    long S = (long)nx * ny;
    #pragma omp parallel for schedule(static) collapse(2)
    for (int v = 0; v < q->nvel; ++v)
        for (int y = 0; y < ny; ++y) {
            double c = q->cth[v], sn = q->sth[v];
            double ax = s->dt * fabs(c), ay = s->dt * fabs(sn);
            int sx = c >= 0 ? 1 : -1, sy = sn >= 0 ? 1 : -1;
            const double* fv = s->f + (long)v * S;
            double* ov = s->fs + (long)v * S;
            int y1 = wrap(y - sy, ny, s->bcy);
            /* upwind points outside the grid (WALL and FIXED edges only) */
            int yo = (y - sy < 0 || y - sy >= ny) && s->bcy >= BC_WALL;
            const double* rv = s->f + (long)(s->bcx == BC_WALL || s->bcy == BC_WALL ? reversed(q, v) : v) * S;
            const double* iv = s->f0 ? s->f0 + (long)v * S : fv;
            for (int x = 0; x < nx; ++x) {
                int x1 = wrap(x - sx, nx, s->bcx);
                int xo = (x - sx < 0 || x - sx >= nx) && s->bcx >= BC_WALL;
                double f00 = fv[(long)y * nx + x], f10 = fv[(long)y * nx + x1];
                double f01 = fv[(long)y1 * nx + x], f11 = fv[(long)y1 * nx + x1];
                if (xo || yo) {
                    int xw = xo && s->bcx == BC_WALL, yw = yo && s->bcy == BC_WALL;
                    double back = rv[(long)y * nx + x];   /* reversed population of the target */
                    /* FIXED: the initial population at the clamped point
                     * (x1, y1 are clamped on a FIXED axis) */
                    if (xo) f10 = xw ? back : iv[(long)y * nx + x1];
                    if (yo) f01 = yw ? back : iv[(long)y1 * nx + x];
                    f11 = (xw || yw) ? back : iv[(long)y1 * nx + x1];
                }
                ov[(long)y * nx + x] = (1 - ax) * (1 - ay) * f00 + ax * (1 - ay) * f10
                                     + (1 - ax) * ay * f01 + ax * ay * f11;
            }
        }
}

/* Relaxation toward the local equilibrium built from the post-streaming
 * moments of the same site:
 *   f_new = f* + dt (p.U)/(p^0 tau) (f_eq - f*),  p.U / p^0 = U^0 - U.n_v.
 * The collision equation of the paper prints (f* - f_eq), which contradicts
 * Eq. discrete-rbe and would drive the state away from equilibrium; the sign
 * of Eq. discrete-rbe is used.  tau = +inf means no collision. */
static void collide_pass(orc_sim* s)
{
    const orc_quad* q = s->q;
    long S = (long)s->nx * s->ny;
    double rate = isinf(s->tau) ? 0.0 : s->dt / s->tau;
    long bad = 0;
    #pragma omp parallel reduction(+ : bad)
    {
        double* feq = (double*)malloc(sizeof(double) * q->nvel);
        #pragma omp for schedule(static)
        for (long i = 0; i < S; ++i) {
            double mom[9];
            moments_site(q, s->fs + i, S, mom);
            ld o[6];
            if (landau_site(mom, o)) {
                ++bad;
                for (int v = 0; v < q->nvel; ++v) s->f[(long)v * S + i] = s->fs[(long)v * S + i];
                continue;
            }
            ld U[3] = {o[5], o[2], o[3]};
            ld Tq, zq, phi[17];
            if (qs_frame(o[0], o[1], s->stat, q->N < 16 ? q->N : 16, &Tq, &zq, phi)) {
                ++bad;   /* no equilibrium of this statistics: streamed without collision */
                for (int v = 0; v < q->nvel; ++v) s->f[(long)v * S + i] = s->fs[(long)v * S + i];
                continue;
            }
            feq_site(q, o[0], Tq, U, phi, feq);
            for (int v = 0; v < q->nvel; ++v) {
                double om = rate * (double)(o[5] - o[2] * (ld)q->cth[v] - o[3] * (ld)q->sth[v]);
                double fsv = s->fs[(long)v * S + i];
                s->f[(long)v * S + i] = fsv + om * (feq[v] - fsv);
            }
        }
        free(feq);
    }
    s->nonphys += bad;
}

void orc_sim_step(orc_sim* s, int nsteps)
{
    for (int t = 0; t < nsteps; ++t) {
        stream_pass(s);
        collide_pass(s);
    }
}

/* Stream only (tau = inf) without touching the collision: used by tests of
 * the interpolation operator alone. */
void orc_sim_stream(orc_sim* s, int nsteps)
{
    long tot = (long)s->nx * s->ny * s->q->nvel;
    for (int t = 0; t < nsteps; ++t) {
        stream_pass(s);
        memcpy(s->f, s->fs, sizeof(double) * tot);
    }
}

/* Macroscopic fields n, eps, U^x, U^y of the stored populations. */
long orc_sim_fields(const orc_sim* s, double* n, double* eps, double* ux, double* uy)
{
    long S = (long)s->nx * s->ny;
    long bad = 0;
    #pragma omp parallel for schedule(static) reduction(+ : bad)
    for (long i = 0; i < S; ++i) {
        double mom[9];
        moments_site(s->q, s->f + i, S, mom);
        ld o[6];
        if (landau_site(mom, o)) {
            ++bad;
            o[0] = o[1] = o[2] = o[3] = NAN;
        }
        if (n) n[i] = (double)o[0];
        if (eps) eps[i] = (double)o[1];
        if (ux) ux[i] = (double)o[2];
        if (uy) uy[i] = (double)o[3];
    }
    return bad;
}

/* All nine moments per site, mom[9][ny][nx]. */
void orc_sim_moments(const orc_sim* s, double* mom)
{
    long S = (long)s->nx * s->ny;
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < S; ++i) {
        double m[9];
        moments_site(s->q, s->f + i, S, m);
        for (int k = 0; k < 9; ++k) mom[k * S + i] = m[k];
    }
}

/* Global charges sum_x (N^0, T^00, T^0x, T^0y). */
void orc_sim_charges(const orc_sim* s, double* ch)
{
    long S = (long)s->nx * s->ny;
    ld acc[4] = {0, 0, 0, 0};
    for (long i = 0; i < S; ++i) {
        double m[9];
        moments_site(s->q, s->f + i, S, m);
        acc[0] += m[0]; acc[1] += m[3]; acc[2] += m[4]; acc[3] += m[5];
    }
    for (int k = 0; k < 4; ++k) ch[k] = (double)acc[k];
}

void orc_sim_get_f(const orc_sim* s, double* f)
{
    memcpy(f, s->f, sizeof(double) * (size_t)s->nx * s->ny * s->q->nvel);
}

void orc_sim_set_f(orc_sim* s, const double* f)
{
    memcpy(s->f, f, sizeof(double) * (size_t)s->nx * s->ny * s->q->nvel);
}

long orc_sim_nonphys(const orc_sim* s) { return s->nonphys; }

int orc_num_threads(void) { return omp_get_max_threads(); }

/* Threads of the parallel loops that follow (the benchmark's single-core leg). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
