/*
 * tbkpm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, serial FP64 CPU implementation of what the density-of-states
 * hot path computes: neighbour pairs, the orthogonal tight-binding Hamiltonian
 * of Eq. (1), the kernel-polynomial (Chebyshev) moments over random-phase
 * vectors, Jackson damping and the DOS of Eq. (4); plus, for the learned-hopping
 * variant, the Chebyshev radial descriptor of Eq. (2), a per-bond MLP forward and
 * analytic backward with BF16 operand rounding, and one AdamW step; and the
 * counter-based random-phase generator the GPU can use instead of stored phases;
 * and the velocity-autocorrelation conductivity of Eq. (3) (velocity operator,
 * Chebyshev time evolution, correlation moments, running time integral); and
 * the s, p (and s, p, d) Slater-Koster orbital Hamiltonian of the multi-orbital
 * models; and the transport post-processing (integrated DOS, frame averages,
 * semiclassical conductivity and mobility).
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this file.  It shares no code, header or constant generator with the HIP
 * library; it is never called by the product path.
 *
 * Where the paper only names an ingredient (Sec. 2.4 names Chebyshev expansion,
 * KPM, sparse matrix-vector products and random phases), the steps follow the
 * published kernel polynomial method: Weisse, Wellein, Alvermann & Fehske,
 * Rev. Mod. Phys. 78, 275 (2006) -- Chebyshev recurrence (their Sec. II.A),
 * stochastic trace (Sec. II.D), Jackson kernel (Sec. II.C.3) and the DOS
 * reconstruction (Sec. III.A).
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (see oracle/build.py).
 * Every routine is serial and allocation-light; errors are reported by a
 * negative return value, never by aborting.
 */
#define _DEFAULT_SOURCE 1   /* jn() (Bessel functions of the first kind) from libm */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Geometry: minimum-image displacement (periodic axes) and neighbour pairs.  */
/* ------------------------------------------------------------------------- */

/* Nearest periodic image of a displacement along one axis of length L. */
static double orc_min_image(double d, double L, int periodic)
{
    if (!periodic) return d;
    return d - L * nearbyint(d / L);
}

/* Displacement x_j - x_i under the minimum-image convention; returns |d|. */
static double orc_displacement(const double *pos, int64_t i, int64_t j,
                               const double box[3], const int32_t periodic[3],
                               double d[3])
{
    for (int k = 0; k < 3; ++k)
        d[k] = orc_min_image(pos[3 * j + k] - pos[3 * i + k], box[k], periodic[k]);
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

/* Cell index of a coordinate along one axis with n cells over [lo, lo + L). */
static int64_t orc_cell_of(double x, double lo, double L, int64_t n, int periodic)
{
    double u = (x - lo) / L;
    if (periodic) u -= floor(u);
    int64_t c = (int64_t)floor(u * (double)n);
    if (c < 0) c = 0;
    if (c >= n) c = n - 1;
    return c;
}

/*
 * All unordered pairs {i, j}, i < j, whose minimum-image distance is strictly
 * below r_cut (the neighbour set N(i) of Eq. (1)).  Brute force over all pairs
 * for n <= 5000, a plain cell list above.  Pairs are written in an arbitrary
 * order; callers needing an order sort them.
 *
 * Returns the number of pairs found; if it exceeds `cap`, only the first `cap`
 * are stored (call again with a larger buffer).  Returns -1 on a bad argument
 * (periodic box shorter than 2 r_cut, non-finite coordinate, r_cut <= 0).
 */
int64_t orc_neighbor_pairs(int64_t n, const double *pos, const double box[3],
                           const int32_t periodic[3], double r_cut, int64_t cap,
                           int32_t *pi, int32_t *pj, double *dist)
{
    if (n < 0 || !(r_cut > 0.0)) return -1;
    for (int k = 0; k < 3; ++k)
        if (periodic[k] && !(box[k] >= 2.0 * r_cut)) return -1;
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!isfinite(pos[i])) return -1;

    int64_t count = 0;
    double d[3];
    if (n <= 5000) {
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j) {
                double r = orc_displacement(pos, i, j, box, periodic, d);
                if (r < r_cut) {
                    if (count < cap) { pi[count] = (int32_t)i; pj[count] = (int32_t)j; dist[count] = r; }
                    ++count;
                }
            }
        return count;
    }

    /* Cell list: cells at least r_cut wide; an axis with fewer than three cells
     * is scanned whole so that no cell is visited twice. */
    double lo[3], len[3];
    int64_t nc[3];
    for (int k = 0; k < 3; ++k) {
        if (periodic[k]) { lo[k] = 0.0; len[k] = box[k]; }
        else {
            double mn = pos[k], mx = pos[k];
            for (int64_t i = 1; i < n; ++i) {
                if (pos[3 * i + k] < mn) mn = pos[3 * i + k];
                if (pos[3 * i + k] > mx) mx = pos[3 * i + k];
            }
            lo[k] = mn; len[k] = (mx - mn) + 1e-9;
        }
        nc[k] = (int64_t)floor(len[k] / r_cut);
        if (nc[k] < 1) nc[k] = 1;
    }
    int64_t ncell = nc[0] * nc[1] * nc[2];
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!head || !next || !cell) { free(head); free(next); free(cell); return -2; }
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    for (int64_t i = n - 1; i >= 0; --i) {
        int64_t c0 = orc_cell_of(pos[3 * i + 0], lo[0], len[0], nc[0], periodic[0]);
        int64_t c1 = orc_cell_of(pos[3 * i + 1], lo[1], len[1], nc[1], periodic[1]);
        int64_t c2 = orc_cell_of(pos[3 * i + 2], lo[2], len[2], nc[2], periodic[2]);
        cell[i] = (c2 * nc[1] + c1) * nc[0] + c0;
        next[i] = head[cell[i]];
        head[cell[i]] = i;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t ci[3];
        ci[0] = cell[i] % nc[0];
        ci[1] = (cell[i] / nc[0]) % nc[1];
        ci[2] = cell[i] / (nc[0] * nc[1]);
        /* Offsets per axis: {-1,0,1} when there are >= 3 cells, else every cell. */
        int64_t off[3][3], noff[3];
        for (int k = 0; k < 3; ++k) {
            if (nc[k] >= 3) { off[k][0] = -1; off[k][1] = 0; off[k][2] = 1; noff[k] = 3; }
            else { noff[k] = nc[k]; for (int64_t t = 0; t < nc[k]; ++t) off[k][t] = t - ci[k]; }
        }
        for (int64_t a = 0; a < noff[2]; ++a)
            for (int64_t b = 0; b < noff[1]; ++b)
                for (int64_t c = 0; c < noff[0]; ++c) {
                    int64_t cc[3] = {ci[0] + off[0][c], ci[1] + off[1][b], ci[2] + off[2][a]};
                    int skip = 0;
                    for (int k = 0; k < 3; ++k) {
                        if (cc[k] < 0 || cc[k] >= nc[k]) {
                            if (periodic[k]) cc[k] = (cc[k] + nc[k]) % nc[k];
                            else skip = 1;
                        }
                    }
                    if (skip) continue;
                    int64_t cid = (cc[2] * nc[1] + cc[1]) * nc[0] + cc[0];
                    for (int64_t j = head[cid]; j >= 0; j = next[j]) {
                        if (j <= i) continue;
                        double r = orc_displacement(pos, i, j, box, periodic, d);
                        if (r < r_cut) {
                            if (count < cap) { pi[count] = (int32_t)i; pj[count] = (int32_t)j; dist[count] = r; }
                            ++count;
                        }
                    }
                }
    }
    free(head); free(next); free(cell);
    return count;
}

/* ------------------------------------------------------------------------- */
/* Hamiltonian of Eq. (1) in CSR form.                                        */
/* ------------------------------------------------------------------------- */

/* Distance-scaled hopping between species s and u at distance r. */
static double orc_hopping(double r, int32_t s, int32_t u, int32_t n_species,
                          const double *t_pair, double r0, double beta)
{
    return t_pair[s * n_species + u] * exp(-beta * (r / r0 - 1.0));
}

static int orc_cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * CSR of the off-diagonal part of H (Eq. (1)): for every pair {i, j} found by
 * orc_neighbor_pairs, H_ij = H_ji = t_pair[s_i][s_j] * exp(-beta (r/r0 - 1)).
 * Columns of each row are sorted ascending.  When `t_scale` is non-NULL the
 * hopping of pair p is multiplied by t_scale[p] (used for the learned and the
 * target Hamiltonians, whose per-bond factors are computed by the callers).
 * The onsite part H_ii = onsite[s_i] goes to `diag` [n].
 *
 * row_ptr has n+1 entries; col/val have 2*npairs entries.
 * Returns 0, or -1 on a species index outside [0, n_species).
 */
int orc_assemble_csr(int64_t n, const int32_t *species, int32_t n_species,
                     const double *onsite, const double *t_pair, double r0, double beta,
                     int64_t npairs, const int32_t *pi, const int32_t *pj,
                     const double *dist, const double *t_scale,
                     int64_t *row_ptr, int32_t *col, double *val, double *diag)
{
    for (int64_t i = 0; i < n; ++i)
        if (species[i] < 0 || species[i] >= n_species) return -1;
    for (int64_t i = 0; i <= n; ++i) row_ptr[i] = 0;
    for (int64_t p = 0; p < npairs; ++p) { row_ptr[pi[p] + 1]++; row_ptr[pj[p] + 1]++; }
    for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!fill) return -2;
    for (int64_t i = 0; i < n; ++i) fill[i] = row_ptr[i];
    for (int64_t p = 0; p < npairs; ++p) { col[fill[pi[p]]++] = pj[p]; col[fill[pj[p]]++] = pi[p]; }
    free(fill);
    for (int64_t i = 0; i < n; ++i)
        qsort(col + row_ptr[i], (size_t)(row_ptr[i + 1] - row_ptr[i]), sizeof(int32_t), orc_cmp_i32);
    /* Values: look the pair up again so that each entry is computed from its own
     * distance (both triangles from the same number, hence exactly symmetric). */
    for (int64_t p = 0; p < npairs; ++p) {
        int32_t i = pi[p], j = pj[p];
        double t = orc_hopping(dist[p], species[i], species[j], n_species, t_pair, r0, beta);
        if (t_scale) t *= t_scale[p];
        for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) if (col[q] == j) val[q] = t;
        for (int64_t q = row_ptr[j]; q < row_ptr[j + 1]; ++q) if (col[q] == i) val[q] = t;
    }
    for (int64_t i = 0; i < n; ++i) diag[i] = onsite[species[i]];
    return 0;
}

/* Row Gershgorin bounds of H = diag + off-diagonal CSR: [min_i (H_ii - sum|H_ij|),
 * max_i (H_ii + sum|H_ij|)]. */
void orc_gershgorin(int64_t n, const int64_t *row_ptr, const double *val,
                    const double *diag, double bounds[2])
{
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) s += fabs(val[q]);
        if (diag[i] - s < lo) lo = diag[i] - s;
        if (diag[i] + s > hi) hi = diag[i] + s;
    }
    bounds[0] = lo;
    bounds[1] = hi;
}

/* ------------------------------------------------------------------------- */
/* Kernel polynomial method.                                                  */
/* ------------------------------------------------------------------------- */

/* y = Htilde x with Htilde = (H - b) / a. */
static void orc_apply_scaled(int64_t n, const int64_t *row_ptr, const int32_t *col,
                             const double *val, const double *diag, double a, double b,
                             const double complex *x, double complex *y)
{
    for (int64_t i = 0; i < n; ++i) {
        double complex s = (diag[i] - b) * x[i];
        for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) s += val[q] * x[col[q]];
        y[i] = s / a;
    }
}

/* Re and Im of <r|t> = sum_i conj(r_i) t_i. */
static double complex orc_dot(int64_t n, const double complex *r, const double complex *t)
{
    double complex s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += conj(r[i]) * t[i];
    return s;
}

/*
 * Chebyshev moments mu_n^(v) = <r_v| T_n(Htilde) |r_v>, n = 0..M-1, for each
 * of the R vectors r_v (stored interleaved: element (i, v) at r[i*R + v]).
 * T_0 = r, T_1 = Htilde r, T_{n+1} = 2 Htilde T_n - T_{n-1}.  The moment is
 * the direct overlap with the starting vector (no doubling identities).
 * Outputs mu_re and mu_im, each [R][M].  Returns 0, -1 on bad arguments.
 */
int orc_kpm_moments(int64_t n, const int64_t *row_ptr, const int32_t *col,
                    const double *val, const double *diag, double a, double b,
                    const double complex *r, int32_t R, int32_t M,
                    double *mu_re, double *mu_im)
{
    if (n <= 0 || R < 1 || M < 1 || !(a > 0.0)) return -1;
    double complex *rv = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    double complex *t0 = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    double complex *t1 = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    double complex *t2 = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    if (!rv || !t0 || !t1 || !t2) { free(rv); free(t0); free(t1); free(t2); return -2; }
    for (int32_t v = 0; v < R; ++v) {
        for (int64_t i = 0; i < n; ++i) rv[i] = r[i * R + v];
        double complex m;
        /* n = 0 */
        for (int64_t i = 0; i < n; ++i) t0[i] = rv[i];
        m = orc_dot(n, rv, t0);
        mu_re[(int64_t)v * M + 0] = creal(m); mu_im[(int64_t)v * M + 0] = cimag(m);
        if (M == 1) continue;
        /* n = 1 */
        orc_apply_scaled(n, row_ptr, col, val, diag, a, b, t0, t1);
        m = orc_dot(n, rv, t1);
        mu_re[(int64_t)v * M + 1] = creal(m); mu_im[(int64_t)v * M + 1] = cimag(m);
        /* n >= 2 */
        for (int32_t k = 2; k < M; ++k) {
            orc_apply_scaled(n, row_ptr, col, val, diag, a, b, t1, t2);
            for (int64_t i = 0; i < n; ++i) t2[i] = 2.0 * t2[i] - t0[i];
            m = orc_dot(n, rv, t2);
            mu_re[(int64_t)v * M + k] = creal(m); mu_im[(int64_t)v * M + k] = cimag(m);
            double complex *tmp = t0; t0 = t1; t1 = t2; t2 = tmp;
        }
    }
    free(rv); free(t0); free(t1); free(t2);
    return 0;
}

/*
 * The recurrence of orc_kpm_moments split over calls (a checkpoint of the
 * Chebyshev expansion): state [R][2][n] carries, per vector, the last two
 * vectors of the recurrence.  n_start = 0 starts from r (T_0 = r,
 * T_1 = Htilde r) and writes moments 0..M-1; n_start in [2, M) reads
 * T_{n_start-2}, T_{n_start-1} from state and writes moments n_start..M-1.
 * Either way state holds T_{M-2}, T_{M-1} on return, so a run split at any
 * k performs exactly the operations of the one-shot run.  Returns 0, -1 on
 * bad arguments, -2 when out of memory.
 */
int orc_kpm_moments_state(int64_t n, const int64_t *row_ptr, const int32_t *col,
                          const double *val, const double *diag, double a, double b,
                          const double complex *r, int32_t R, int32_t M, int32_t n_start,
                          double complex *state, double *mu_re, double *mu_im)
{
    if (n <= 0 || R < 1 || M < 2 || !(a > 0.0) || !state) return -1;
    if (!(n_start == 0 || (n_start >= 2 && n_start < M))) return -1;
    double complex *rv = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    double complex *t0 = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    double complex *t1 = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    double complex *t2 = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    if (!rv || !t0 || !t1 || !t2) { free(rv); free(t0); free(t1); free(t2); return -2; }
    for (int32_t v = 0; v < R; ++v) {
        double complex *sv = state + (int64_t)v * 2 * n;     /* older, then newer vector */
        for (int64_t i = 0; i < n; ++i) rv[i] = r[i * R + v];
        double complex m;
        int32_t k;
        if (n_start == 0) {
            for (int64_t i = 0; i < n; ++i) t0[i] = rv[i];
            m = orc_dot(n, rv, t0);
            mu_re[(int64_t)v * M + 0] = creal(m); mu_im[(int64_t)v * M + 0] = cimag(m);
            orc_apply_scaled(n, row_ptr, col, val, diag, a, b, t0, t1);
            m = orc_dot(n, rv, t1);
            mu_re[(int64_t)v * M + 1] = creal(m); mu_im[(int64_t)v * M + 1] = cimag(m);
            k = 2;
        } else {
            for (int64_t i = 0; i < n; ++i) { t0[i] = sv[i]; t1[i] = sv[n + i]; }
            k = n_start;
        }
        for (; k < M; ++k) {
            orc_apply_scaled(n, row_ptr, col, val, diag, a, b, t1, t2);
            for (int64_t i = 0; i < n; ++i) t2[i] = 2.0 * t2[i] - t0[i];
            m = orc_dot(n, rv, t2);
            mu_re[(int64_t)v * M + k] = creal(m); mu_im[(int64_t)v * M + k] = cimag(m);
            double complex *tmp = t0; t0 = t1; t1 = t2; t2 = tmp;
        }
        for (int64_t i = 0; i < n; ++i) { sv[i] = t0[i]; sv[n + i] = t1[i]; }
    }
    free(rv); free(t0); free(t1); free(t2);
    return 0;
}

/* Jackson damping factors g_n, n = 0..M-1, for an expansion of M moments. */
void orc_jackson(int32_t M, double *g)
{
    double q = ORC_PI / (M + 1.0);
    for (int32_t k = 0; k < M; ++k)
        g[k] = ((M - k + 1.0) * cos(q * k) + sin(q * k) * cos(q) / sin(q)) / (M + 1.0);
}

/*
 * DOS of Eq. (4) from moments mu (already averaged over random vectors):
 *   rho(E) = [g_0 mu_0 + 2 sum_{n>=1} g_n mu_n T_n(x)] / (a pi sqrt(1 - x^2)),
 *   x = (E - b)/a,  rho = 0 for |x| >= 1.
 * The result is in states per energy unit for the whole system (it integrates
 * to mu_0); the spin and volume factor 2/Omega of Eq. (4) is left to callers.
 * kernel = 0: Jackson damping; kernel = 1: no damping (g_n = 1).
 */
int orc_kpm_dos(const double *mu, int32_t M, double a, double b, int32_t kernel,
                const double *E, int32_t nE, double *rho)
{
    if (M < 1 || !(a > 0.0) || (kernel != 0 && kernel != 1)) return -1;
    double *g = (double *)malloc(sizeof(double) * (size_t)M);
    if (!g) return -2;
    if (kernel == 0) orc_jackson(M, g);
    else for (int32_t k = 0; k < M; ++k) g[k] = 1.0;
    for (int32_t e = 0; e < nE; ++e) {
        double x = (E[e] - b) / a;
        if (!(fabs(x) < 1.0)) { rho[e] = 0.0; continue; }
        double s = g[0] * mu[0];
        double tm = 1.0, tn = x;      /* T_0(x), T_1(x) */
        for (int32_t k = 1; k < M; ++k) {
            s += 2.0 * g[k] * mu[k] * tn;
            double tp = 2.0 * x * tn - tm;
            tm = tn; tn = tp;
        }
        rho[e] = s / (a * ORC_PI * sqrt(1.0 - x * x));
    }
    free(g);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Seeded random phases (counter-based): output k of SplitMix64.              */
/* ------------------------------------------------------------------------- */

/*
 * Output number k (k = 0, 1, ...) of SplitMix64 started at state `seed`
 * (Steele, Lea & Flood, OOPSLA 2014; Vigna's reference splitmix64.c): the state
 * advances by the odd constant 0x9e3779b97f4a7c15 before each output, and each
 * output is the state after k + 1 advances passed through the mixing function
 * z ^= z >> 30; z *= 0xbf58476d1ce4e5b9; z ^= z >> 27; z *= 0x94d049bb133111eb;
 * z ^= z >> 31 (arithmetic mod 2^64).
 */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1u) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

/*
 * Random-phase vectors r[i][v] = exp(i phi), phi = 2 pi u, u = (x >> 11) 2^-53
 * with x = output number i R + v of the generator above (i = atom, v = vector).
 * re/im are [n][R].
 */
void orc_random_phase(int64_t n, int32_t R, uint64_t seed, double *re, double *im)
{
    for (int64_t i = 0; i < n; ++i)
        for (int32_t v = 0; v < R; ++v) {
            uint64_t x = orc_splitmix64(seed, (uint64_t)i * (uint64_t)R + (uint64_t)v);
            double u = (double)(x >> 11) * (1.0 / 9007199254740992.0);
            double phi = 2.0 * ORC_PI * u;
            re[i * R + v] = cos(phi);
            im[i * R + v] = sin(phi);
        }
}

/* ------------------------------------------------------------------------- */
/* Learned hoppings: descriptor of Eq. (2), per-bond MLP, AdamW.              */
/* ------------------------------------------------------------------------- */

/* Smooth cutoff f_c(r) = (1 + cos(pi r / rc)) / 2 for r < rc, else 0. */
static double orc_fc(double r, double rc)
{
    return r < rc ? 0.5 * (1.0 + cos(ORC_PI * r / rc)) : 0.0;
}

/* Chebyshev radial functions f_k(r) = (T_k(2 (r/rc - 1)^2 - 1) + 1) / 2 * f_c(r),
 * k = 0..nk-1, with T_k evaluated by its three-term recurrence. */
void orc_radial(double r, double rc, int32_t nk, double *f)
{
    double u = r / rc - 1.0;
    double x = 2.0 * u * u - 1.0;
    double c = orc_fc(r, rc);
    double tm = 1.0, tn = x;
    for (int32_t k = 0; k < nk; ++k) {
        double tk;
        if (k == 0) tk = 1.0;
        else if (k == 1) tk = x;
        else { double tp = 2.0 * x * tn - tm; tm = tn; tn = tp; tk = tp; }
        f[k] = 0.5 * (tk + 1.0) * c;
    }
}

/* Bond descriptor of Eq. (2): C_n(r) = sum_k c_nk f_k(r) with the coefficients
 * c [nk][nk] of the bond's species pair, or C_n = f_n (c = NULL: identity). */
static void orc_bond_basis(double r, double rc, int32_t nk, const double *c, double *C)
{
    double f[64];
    orc_radial(r, rc, nk, f);
    for (int32_t a = 0; a < nk; ++a) {
        if (!c) { C[a] = f[a]; continue; }
        double s = 0.0;
        for (int32_t k = 0; k < nk; ++k) s += c[a * nk + k] * f[k];
        C[a] = s;
    }
}

/* Coefficients of the species pair of atoms i and j: cnk [ns][ns][nk][nk]
 * (NULL: identity for every pair). */
static const double *orc_pair_cnk(const double *cnk, const int32_t *species, int32_t ns, int32_t nk,
                                  int32_t i, int32_t j)
{
    if (!cnk) return NULL;
    return cnk + ((int64_t)species[i] * ns + species[j]) * nk * nk;
}

/* Node feature v_i = sum_{j in N(i)} C(r_ij) (Eq. (2)), from the pair list of a
 * descriptor cutoff: v [n][nk].  cnk [ns][ns][nk][nk] (symmetric in the species
 * pair) and species [n], or cnk = NULL for the identity c_nk. */
void orc_descriptor(int64_t n, int64_t npairs, const int32_t *pi, const int32_t *pj,
                    const double *dist, double rc, int32_t nk, const int32_t *species, int32_t ns,
                    const double *cnk, double *v)
{
    double C[64];
    for (int64_t i = 0; i < n * nk; ++i) v[i] = 0.0;
    for (int64_t p = 0; p < npairs; ++p) {
        orc_bond_basis(dist[p], rc, nk, orc_pair_cnk(cnk, species, ns, nk, pi[p], pj[p]), C);
        for (int32_t k = 0; k < nk; ++k) { v[(int64_t)pi[p] * nk + k] += C[k]; v[(int64_t)pj[p] * nk + k] += C[k]; }
    }
}

/* Round a double to the nearest bfloat16 value (ties to even), returned as a
 * double.  bfloat16 keeps 8 significand bits and the FP32 exponent range. */
double orc_bf16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    double m = frexp(x, &e);            /* x = m 2^e, 0.5 <= |m| < 1 */
    if (e < -125) {                     /* subnormal range of FP32 */
        double q = ldexp(1.0, -133);    /* spacing of bfloat16 subnormals */
        return nearbyint(x / q) * q;
    }
    double s = ldexp(m, 8);             /* 8 significand bits */
    return ldexp(nearbyint(s), e - 8);  /* default rounding: nearest, ties to even */
}

/*
 * Per-bond MLP  x (16) -> 32 -> tanh -> 32 -> tanh -> 1, applied to B rows of X
 * [B][16] (already normalised).  Parameters, packed in this order:
 *   W1 [32][16], b1 [32], W2 [32][32], b2 [32], W3 [32], b3 [1]   (1633 values).
 * bf16 != 0: every multiply's two operands are rounded to bfloat16 (RNE) first
 * (weights and activations of the three matrix products), accumulation is FP64.
 * Outputs y [B]; when h1/h2 are non-NULL the post-tanh activations [B][32] are
 * stored for the backward pass.
 */
#define ORC_NI 16
#define ORC_NH 32
static double orc_rnd(double x, int bf16) { return bf16 ? orc_bf16(x) : x; }

void orc_mlp_forward(int64_t B, const double *X, const double *prm, int32_t bf16,
                     double *y, double *h1, double *h2)
{
    const double *W1 = prm, *b1 = W1 + ORC_NH * ORC_NI, *W2 = b1 + ORC_NH;
    const double *b2 = W2 + ORC_NH * ORC_NH, *W3 = b2 + ORC_NH, *b3 = W3 + ORC_NH;
    double a1[ORC_NH], a2[ORC_NH];
    for (int64_t e = 0; e < B; ++e) {
        const double *x = X + e * ORC_NI;
        for (int h = 0; h < ORC_NH; ++h) {
            double s = 0.0;
            for (int k = 0; k < ORC_NI; ++k) s += orc_rnd(W1[h * ORC_NI + k], bf16) * orc_rnd(x[k], bf16);
            a1[h] = tanh(s + b1[h]);
        }
        for (int h = 0; h < ORC_NH; ++h) {
            double s = 0.0;
            for (int k = 0; k < ORC_NH; ++k) s += orc_rnd(W2[h * ORC_NH + k], bf16) * orc_rnd(a1[k], bf16);
            a2[h] = tanh(s + b2[h]);
        }
        double s = 0.0;
        for (int k = 0; k < ORC_NH; ++k) s += orc_rnd(W3[k], bf16) * orc_rnd(a2[k], bf16);
        y[e] = s + b3[0];
        if (h1) for (int h = 0; h < ORC_NH; ++h) h1[e * ORC_NH + h] = a1[h];
        if (h2) for (int h = 0; h < ORC_NH; ++h) h2[e * ORC_NH + h] = a2[h];
    }
}

/*
 * Loss L = (1/B) sum_e w_e (y_e - y*_e)^2 and its gradient with respect to the
 * packed parameters (same layout as orc_mlp_forward), by the chain rule through
 * the three layers.  The backward products use the same bf16 operand rounding
 * as the forward ones when bf16 != 0: in dL/dW3 and dL/dW2, dL/dW1 both factors;
 * in the propagated deltas (delta2 = (W3 dy) * (1 - h2^2), delta1 = (W2^T delta2)
 * * (1 - h1^2)) the weight and the incoming delta.  `w` may be NULL (all ones).
 * Returns the loss.
 */
double orc_mlp_loss_grad(int64_t B, const double *X, const double *target,
                         const double *w, const double *prm, int32_t bf16, double *grad)
{
    const double *W1 = prm, *W2 = W1 + ORC_NH * ORC_NI + ORC_NH;
    const double *W3 = W2 + ORC_NH * ORC_NH + ORC_NH;
    double *gW1 = grad, *gb1 = gW1 + ORC_NH * ORC_NI, *gW2 = gb1 + ORC_NH;
    double *gb2 = gW2 + ORC_NH * ORC_NH, *gW3 = gb2 + ORC_NH, *gb3 = gW3 + ORC_NH;
    for (int i = 0; i < 1633; ++i) grad[i] = 0.0;
    double h1[ORC_NH], h2[ORC_NH], d1[ORC_NH], d2[ORC_NH], y;
    double loss = 0.0;
    for (int64_t e = 0; e < B; ++e) {
        const double *x = X + e * ORC_NI;
        orc_mlp_forward(1, x, prm, bf16, &y, h1, h2);
        double we = w ? w[e] : 1.0;
        double diff = y - target[e];
        loss += we * diff * diff;
        double dy = 2.0 * we * diff / (double)B;
        /* output layer */
        gb3[0] += dy;
        for (int k = 0; k < ORC_NH; ++k) gW3[k] += orc_rnd(dy, bf16) * orc_rnd(h2[k], bf16);
        for (int k = 0; k < ORC_NH; ++k) d2[k] = orc_rnd(W3[k], bf16) * orc_rnd(dy, bf16) * (1.0 - h2[k] * h2[k]);
        /* second hidden layer */
        for (int h = 0; h < ORC_NH; ++h) {
            gb2[h] += d2[h];
            for (int k = 0; k < ORC_NH; ++k) gW2[h * ORC_NH + k] += orc_rnd(d2[h], bf16) * orc_rnd(h1[k], bf16);
        }
        for (int k = 0; k < ORC_NH; ++k) {
            double s = 0.0;
            for (int h = 0; h < ORC_NH; ++h) s += orc_rnd(W2[h * ORC_NH + k], bf16) * orc_rnd(d2[h], bf16);
            d1[k] = s * (1.0 - h1[k] * h1[k]);
        }
        /* first hidden layer */
        for (int h = 0; h < ORC_NH; ++h) {
            gb1[h] += d1[h];
            for (int k = 0; k < ORC_NI; ++k) gW1[h * ORC_NI + k] += orc_rnd(d1[h], bf16) * orc_rnd(x[k], bf16);
        }
    }
    return loss / (double)B;
}

/*
 * One AdamW step (Loshchilov & Hutter, decoupled weight decay) on n parameters:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr * ( (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps) + wd * p ),
 * with t the 1-based step count after this update.
 */
void orc_adamw_step(int64_t n, double *p, const double *g, double *m, double *v,
                    int64_t t, double lr, double beta1, double beta2, double eps, double wd)
{
    double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        p[i] -= lr * (mh / (sqrt(vh) + eps) + wd * p[i]);
    }
}

/*
 * Per-bond MLP input of the learned model: for pair p = {i, j},
 *   x_p = [C_0..C_{nk-1}(r_ij) || v_i + v_j]      (2 nk values, symmetric in i, j)
 * with C the bond descriptor of the pair's species (orc_bond_basis; f itself
 * when cnk = NULL)
 * followed by the fixed standardisation x <- (x - shift) / scale per feature.
 * X is [npairs][2 nk].
 */
void orc_bond_features(int64_t npairs, const int32_t *pi, const int32_t *pj,
                       const double *dist, const double *v, double rc, int32_t nk,
                       const int32_t *species, int32_t ns, const double *cnk,
                       const double *shift, const double *scale, double *X)
{
    double f[64];
    for (int64_t p = 0; p < npairs; ++p) {
        double *x = X + p * 2 * nk;
        orc_bond_basis(dist[p], rc, nk, orc_pair_cnk(cnk, species, ns, nk, pi[p], pj[p]), f);
        for (int32_t k = 0; k < nk; ++k) x[k] = f[k];
        for (int32_t k = 0; k < nk; ++k) x[nk + k] = v[(int64_t)pi[p] * nk + k] + v[(int64_t)pj[p] * nk + k];
        for (int32_t k = 0; k < 2 * nk; ++k) x[k] = (x[k] - shift[k]) / scale[k];
    }
}

/*
 * Synthetic "true" hopping factor of the learned-hopping workload: the plain
 * distance formula times a coordination correction
 *   s_p = 1 + kappa (z_i + z_j - 2 z0),   z_i = sum_{j: r_ij < rc} f_c(r_ij),
 * where z is the zeroth radial descriptor component v_{i,0}.
 */
void orc_target_scale(int64_t npairs, const int32_t *pi, const int32_t *pj,
                      const double *v, int32_t nk, double kappa, double z0, double *s)
{
    for (int64_t p = 0; p < npairs; ++p)
        s[p] = 1.0 + kappa * (v[(int64_t)pi[p] * nk] + v[(int64_t)pj[p] * nk] - 2.0 * z0);
}

/* ------------------------------------------------------------------------- */
/* Velocity autocorrelation, Eq. (3): velocity operator, time evolution, the  */
/* correlation moments and the running conductivity integral.                 */
/* ------------------------------------------------------------------------- */

#define ORC_HBAR 0.6582119569 /* reduced Planck constant, eV fs (CODATA 2018) */

/*
 * Velocity operator along `axis`, V = (i / hbar) [H, X]: in the site basis
 * V_ij = (i / hbar) H_ij (x_j - x_i), the displacement taken with the
 * minimum-image convention (the bond the hopping belongs to), and V_ii = 0.
 * Stored as the real coefficient vx[q] = H_ij (x_j - x_i) / hbar of each CSR
 * entry q = (i, j), so that (V psi)_i = i sum_q vx[q] psi_j (Angstrom / fs).
 * With n_orb orbitals per atom (orbital index = n_orb atom + a), x is the
 * position of the orbital's atom.
 */
void orc_velocity_values(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                         const double *pos, const double box[3], const int32_t periodic[3],
                         int32_t axis, int32_t n_orb, double *vx)
{
    /* n rows = n_orb orbitals per atom; an orbital sits at its atom's position */
    double d[3];
    for (int64_t i = 0; i < n; ++i)
        for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
            orc_displacement(pos, i / n_orb, col[q] / n_orb, box, periodic, d);
            vx[q] = val[q] * d[axis] / ORC_HBAR;
        }
}

/* y = V x, (V x)_i = i sum_q vx[q] x_col[q]. */
static void orc_apply_velocity(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *vx,
                               const double complex *x, double complex *y)
{
    for (int64_t i = 0; i < n; ++i) {
        double complex s = 0.0;
        for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) s += vx[q] * x[col[q]];
        y[i] = I * s;
    }
}

/*
 * psi <- exp(-i H dt / hbar) psi (dt in fs) by the Chebyshev expansion of the
 * propagator on the scaled spectrum H = a Htilde + b:
 *   exp(-i H dt/hbar) = exp(-i b dt/hbar) sum_k (2 - delta_k0) (-i)^k J_k(a dt/hbar) T_k(Htilde),
 * truncated after n_cheb terms; J_k is the C library's Bessel function jn.
 * Returns 0, -1 on a bad argument, -2 when out of memory.
 */
int orc_evolve(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
               const double *diag, double a, double b, double dt, int32_t n_cheb, double complex *psi)
{
    if (n <= 0 || !(a > 0.0) || n_cheb < 1) return -1;
    double complex *t0 = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    double complex *t1 = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    double complex *t2 = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    double complex *acc = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    if (!t0 || !t1 || !t2 || !acc) { free(t0); free(t1); free(t2); free(acc); return -2; }
    const double z = a * dt / ORC_HBAR;
    const double complex phase = cexp(-I * b * dt / ORC_HBAR);
    double complex ik = 1.0;                                    /* (-i)^k */
    for (int64_t i = 0; i < n; ++i) { t0[i] = psi[i]; acc[i] = jn(0, z) * t0[i]; }
    if (n_cheb > 1) {
        orc_apply_scaled(n, row_ptr, col, val, diag, a, b, t0, t1);
        ik = -I;
        double complex c = 2.0 * ik * jn(1, z);
        for (int64_t i = 0; i < n; ++i) acc[i] += c * t1[i];
    }
    for (int32_t k = 2; k < n_cheb; ++k) {
        orc_apply_scaled(n, row_ptr, col, val, diag, a, b, t1, t2);
        for (int64_t i = 0; i < n; ++i) t2[i] = 2.0 * t2[i] - t0[i];
        ik *= -I;
        double complex c = 2.0 * ik * jn(k, z);
        for (int64_t i = 0; i < n; ++i) acc[i] += c * t2[i];
        double complex *tmp = t0; t0 = t1; t1 = t2; t2 = tmp;
    }
    for (int64_t i = 0; i < n; ++i) psi[i] = phase * acc[i];
    free(t0); free(t1); free(t2); free(acc);
    return 0;
}

/*
 * Correlation moments of Eq. (3) with the random-phase trace (Sec. 2.4).  For
 * each start vector phi_v (r, interleaved [n][R]):
 *   phi_R(0) = phi, phi_L(0) = V phi, and for time step j = 0..n_t-1
 *     nu[j][v][m] = Re <phi_L(t_j)| T_m(Htilde) V |phi_R(t_j)>,  m = 0..M-1,
 *     then phi_R <- U phi_R and phi_L <- U phi_L, U = exp(-i H dt/hbar) (orc_evolve).
 * With phi_R(t) = U(t) phi and phi_L(t) = U(t) V phi the bracket is
 * <phi| V U(t)^+ T_m V U(t) |phi>, whose trace over phi is
 * Tr[T_m(Htilde) V(t) V] with V(t) = U(t)^+ V U(t); the real part is the
 * T_m-moment of Tr[delta(E - H) Re(V V(t))].
 * Returns 0, -1 on a bad argument, -2 when out of memory.
 */
int orc_vac_moments(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                    const double *diag, const double *vx, double a, double b,
                    const double complex *r, int32_t R, int32_t M, int32_t n_t, double dt,
                    int32_t n_cheb, double *nu)
{
    if (n <= 0 || R < 1 || M < 1 || n_t < 1 || !(a > 0.0) || n_cheb < 1) return -1;
    size_t bytes = sizeof(double complex) * (size_t)n;
    double complex *pr = malloc(bytes), *pl = malloc(bytes), *w = malloc(bytes);
    double complex *t0 = malloc(bytes), *t1 = malloc(bytes), *t2 = malloc(bytes);
    if (!pr || !pl || !w || !t0 || !t1 || !t2) {
        free(pr); free(pl); free(w); free(t0); free(t1); free(t2);
        return -2;
    }
    int rc = 0;
    for (int32_t v = 0; v < R && rc == 0; ++v) {
        for (int64_t i = 0; i < n; ++i) pr[i] = r[i * R + v];
        orc_apply_velocity(n, row_ptr, col, vx, pr, pl);
        for (int32_t j = 0; j < n_t && rc == 0; ++j) {
            double *out = nu + ((int64_t)j * R + v) * M;
            orc_apply_velocity(n, row_ptr, col, vx, pr, w);
            /* <phi_L| T_m w>, T_0 = w */
            for (int64_t i = 0; i < n; ++i) t0[i] = w[i];
            out[0] = creal(orc_dot(n, pl, t0));
            if (M > 1) {
                orc_apply_scaled(n, row_ptr, col, val, diag, a, b, t0, t1);
                out[1] = creal(orc_dot(n, pl, t1));
            }
            for (int32_t m = 2; m < M; ++m) {
                orc_apply_scaled(n, row_ptr, col, val, diag, a, b, t1, t2);
                for (int64_t i = 0; i < n; ++i) t2[i] = 2.0 * t2[i] - t0[i];
                out[m] = creal(orc_dot(n, pl, t2));
                double complex *tmp = t0; t0 = t1; t1 = t2; t2 = tmp;
            }
            if (j + 1 < n_t) {
                rc = orc_evolve(n, row_ptr, col, val, diag, a, b, dt, n_cheb, pr);
                if (rc == 0) rc = orc_evolve(n, row_ptr, col, val, diag, a, b, dt, n_cheb, pl);
            }
        }
    }
    free(pr); free(pl); free(w); free(t0); free(t1); free(t2);
    return rc;
}

/*
 * Running conductivity of Eq. (3) without its prefactor 2 e^2 / Omega:
 *   C_j(E) = the KPM reconstruction (orc_kpm_dos, same kernel) of the moments
 *            nu[j][m] (already averaged over vectors) at correlation time t_j = j dt,
 *   s[j][e] = integral_0^{t_j} C(E, tau) dtau by the trapezoidal rule over the
 *            samples (s[0] = 0).
 * Units: (Angstrom / fs)^2 per eV times fs.  Returns 0 or -1.
 */
int orc_vac_sigma(const double *nu, int32_t M, int32_t n_t, double dt, double a, double b,
                  int32_t kernel, const double *E, int32_t nE, double *s)
{
    if (n_t < 1 || nE < 0) return -1;
    double *cprev = malloc(sizeof(double) * (size_t)(nE > 0 ? nE : 1));
    double *cj = malloc(sizeof(double) * (size_t)(nE > 0 ? nE : 1));
    if (!cprev || !cj) { free(cprev); free(cj); return -2; }
    int rc = orc_kpm_dos(nu, M, a, b, kernel, E, nE, cprev);
    for (int32_t e = 0; e < nE; ++e) s[e] = 0.0;
    for (int32_t j = 1; j < n_t && rc == 0; ++j) {
        rc = orc_kpm_dos(nu + (int64_t)j * M, M, a, b, kernel, E, nE, cj);
        for (int32_t e = 0; e < nE; ++e) {
            s[(int64_t)j * nE + e] = s[(int64_t)(j - 1) * nE + e] + 0.5 * dt * (cprev[e] + cj[e]);
            cprev[e] = cj[e];
        }
    }
    free(cprev); free(cj);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Transport post-processing: integrated DOS, frame averages, mobility.       */
/* ------------------------------------------------------------------------- */

/*
 * Integrated DOS N(E) = integral of rho(E') dE' from the bottom of the spectrum
 * to E, for the kernel-damped expansion of orc_kpm_dos, in closed form: with
 * x = (E - b)/a = cos(theta),
 *   integral_{-1}^{x} T_0(y) / (pi sqrt(1 - y^2)) dy = 1 - theta / pi,
 *   integral_{-1}^{x} T_n(y) / (pi sqrt(1 - y^2)) dy = -sin(n theta) / (n pi),  n >= 1,
 * so N = g_0 mu_0 (1 - theta/pi) - (2/pi) sum_{n>=1} g_n mu_n sin(n theta) / n;
 * N = 0 for x <= -1 and g_0 mu_0 for x >= 1.  States of the whole system (no
 * spin factor), as orc_kpm_dos.  Returns 0, -1 on a bad argument.
 */
int orc_integrated_dos(const double *mu, int32_t M, double a, double b, int32_t kernel,
                       const double *E, int32_t nE, double *N)
{
    if (M < 1 || !(a > 0.0) || (kernel != 0 && kernel != 1) || nE < 0) return -1;
    double *g = (double *)malloc(sizeof(double) * (size_t)M);
    if (!g) return -2;
    if (kernel == 0) orc_jackson(M, g);
    else for (int32_t k = 0; k < M; ++k) g[k] = 1.0;
    for (int32_t e = 0; e < nE; ++e) {
        double x = (E[e] - b) / a;
        if (x <= -1.0) { N[e] = 0.0; continue; }
        if (x >= 1.0) { N[e] = g[0] * mu[0]; continue; }
        double theta = acos(x);
        double s = g[0] * mu[0] * (1.0 - theta / ORC_PI);
        for (int32_t k = 1; k < M; ++k)
            s -= 2.0 / ORC_PI * g[k] * mu[k] * sin(k * theta) / k;
        N[e] = s;
    }
    free(g);
    return 0;
}

/*
 * Frame averages and mobility (Sec. 2.4: results of several MD frames are
 * averaged; Sec. 3: mobility against carrier concentration).
 *   sigma [F][n_t][nE]  running conductivity of each frame (orc_vac_sigma units),
 *   N     [F][nE]       integrated DOS of each frame (orc_integrated_dos),
 *   n_ref               integrated DOS at charge neutrality (states),
 * out:
 *   sigma_sc[e] = max over j of (1/F) sum_f sigma[f][j][e]   (semiclassical
 *                 conductivity: the plateau of the frame-averaged running value),
 *   carriers[e] = (1/F) sum_f N[f][e] - n_ref                 (carriers, states),
 *   mobility[e] = 0.1 sigma_sc[e] / |carriers[e]|             (cm^2 / (V s)).
 * The factor: sigma = (2 e^2 / A) sigma_sc and n = 2 carriers / A (spin 2, area A
 * in Angstrom^2), so mu = sigma / (e n) = e sigma_sc / carriers, and
 * e Angstrom^2 / (eV fs) = Angstrom^2 / (V fs) = 1e-16 cm^2 / (1e-15 V s).
 * mobility = NaN where carriers = 0.  Returns 0, -1 on a bad argument.
 */
int orc_mobility(const double *sigma, int32_t F, int32_t n_t, int32_t nE, const double *N, double n_ref,
                 double *sigma_sc, double *carriers, double *mobility)
{
    if (F < 1 || n_t < 1 || nE < 0) return -1;
    for (int32_t e = 0; e < nE; ++e) {
        double best = -INFINITY;
        for (int32_t j = 0; j < n_t; ++j) {
            double m = 0.0;
            for (int32_t f = 0; f < F; ++f) m += sigma[((int64_t)f * n_t + j) * nE + e];
            m /= F;
            if (m > best) best = m;
        }
        double nb = 0.0;
        for (int32_t f = 0; f < F; ++f) nb += N[(int64_t)f * nE + e];
        nb = nb / F - n_ref;
        sigma_sc[e] = best;
        carriers[e] = nb;
        mobility[e] = nb != 0.0 ? 0.1 * best / fabs(nb) : NAN;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Multi-orbital Slater-Koster Hamiltonian (s, p or s, p, d per atom).        */
/* ------------------------------------------------------------------------- */

/*
 * Two-centre block E[a][b] = <a_i|H|b_j> / f of a bond with direction cosines
 * c = (l, m, n) from atom i to atom j, orbitals in the order
 *   s, px, py, pz, dxy, dyz, dzx, dx2-y2, d3z2-r2
 * (Slater & Koster, Phys. Rev. 94, 1498 (1954), Table I), from the ten
 * integrals v = {ss_sigma, sp_sigma, pp_sigma, pp_pi, sd_sigma, pd_sigma,
 * pd_pi, dd_sigma, dd_pi, dd_delta}.  The table gives the blocks with the
 * lower angular momentum first; the others follow from Hermiticity and parity,
 * E[b][a](c) = E[a][b](-c) = (-1)^(l_a + l_b) E[a][b](c).
 */
static const int lq[9] = {0, 1, 1, 1, 2, 2, 2, 2, 2};   /* angular momentum of each orbital */

static void orc_sk_table(const double c[3], const double v[10], double E[9][9])
{
    const double l = c[0], m = c[1], n = c[2], s3 = sqrt(3.0);
    const double l2 = l * l, m2 = m * m, n2 = n * n;
    const double ss = v[0], sp = v[1], pps = v[2], ppp = v[3], sd = v[4], pds = v[5], pdp = v[6];
    const double dds = v[7], ddp = v[8], ddd = v[9];
    double sdrow[5], pd[3][5], dd[5][5];
    for (int a = 0; a < 9; ++a)
        for (int b = 0; b < 9; ++b) E[a][b] = 0.0;
    /* s-s, s-p, p-p */
    E[0][0] = ss;
    for (int a = 0; a < 3; ++a) {
        E[0][1 + a] = c[a] * sp;
        for (int b = 0; b < 3; ++b)
            E[1 + a][1 + b] = c[a] * c[b] * pps + ((a == b ? 1.0 : 0.0) - c[a] * c[b]) * ppp;
    }
    /* s-d */
    sdrow[0] = s3 * l * m * sd;
    sdrow[1] = s3 * m * n * sd;
    sdrow[2] = s3 * n * l * sd;
    sdrow[3] = 0.5 * s3 * (l2 - m2) * sd;
    sdrow[4] = (n2 - 0.5 * (l2 + m2)) * sd;
    /* p-d */
    pd[0][0] = s3 * l2 * m * pds + m * (1.0 - 2.0 * l2) * pdp;
    pd[0][1] = s3 * l * m * n * pds - 2.0 * l * m * n * pdp;
    pd[0][2] = s3 * l2 * n * pds + n * (1.0 - 2.0 * l2) * pdp;
    pd[0][3] = 0.5 * s3 * l * (l2 - m2) * pds + l * (1.0 - l2 + m2) * pdp;
    pd[0][4] = l * (n2 - 0.5 * (l2 + m2)) * pds - s3 * l * n2 * pdp;
    pd[1][0] = s3 * m2 * l * pds + l * (1.0 - 2.0 * m2) * pdp;
    pd[1][1] = s3 * m2 * n * pds + n * (1.0 - 2.0 * m2) * pdp;
    pd[1][2] = s3 * l * m * n * pds - 2.0 * l * m * n * pdp;
    pd[1][3] = 0.5 * s3 * m * (l2 - m2) * pds - m * (1.0 + l2 - m2) * pdp;
    pd[1][4] = m * (n2 - 0.5 * (l2 + m2)) * pds - s3 * m * n2 * pdp;
    pd[2][0] = s3 * l * m * n * pds - 2.0 * l * m * n * pdp;
    pd[2][1] = s3 * n2 * m * pds + m * (1.0 - 2.0 * n2) * pdp;
    pd[2][2] = s3 * n2 * l * pds + l * (1.0 - 2.0 * n2) * pdp;
    pd[2][3] = 0.5 * s3 * n * (l2 - m2) * pds - n * (l2 - m2) * pdp;
    pd[2][4] = n * (n2 - 0.5 * (l2 + m2)) * pds + s3 * n * (l2 + m2) * pdp;
    /* d-d (symmetric in the two d orbitals) */
    dd[0][0] = 3.0 * l2 * m2 * dds + (l2 + m2 - 4.0 * l2 * m2) * ddp + (n2 + l2 * m2) * ddd;
    dd[1][1] = 3.0 * m2 * n2 * dds + (m2 + n2 - 4.0 * m2 * n2) * ddp + (l2 + m2 * n2) * ddd;
    dd[2][2] = 3.0 * n2 * l2 * dds + (n2 + l2 - 4.0 * n2 * l2) * ddp + (m2 + n2 * l2) * ddd;
    dd[0][1] = 3.0 * l * m2 * n * dds + l * n * (1.0 - 4.0 * m2) * ddp + l * n * (m2 - 1.0) * ddd;
    dd[0][2] = 3.0 * l2 * m * n * dds + m * n * (1.0 - 4.0 * l2) * ddp + m * n * (l2 - 1.0) * ddd;
    dd[1][2] = 3.0 * l * m * n2 * dds + l * m * (1.0 - 4.0 * n2) * ddp + l * m * (n2 - 1.0) * ddd;
    dd[0][3] = 1.5 * l * m * (l2 - m2) * dds + 2.0 * l * m * (m2 - l2) * ddp + 0.5 * l * m * (l2 - m2) * ddd;
    dd[1][3] = 1.5 * m * n * (l2 - m2) * dds - m * n * (1.0 + 2.0 * (l2 - m2)) * ddp
             + m * n * (1.0 + 0.5 * (l2 - m2)) * ddd;
    dd[2][3] = 1.5 * n * l * (l2 - m2) * dds + n * l * (1.0 - 2.0 * (l2 - m2)) * ddp
             - n * l * (1.0 - 0.5 * (l2 - m2)) * ddd;
    dd[0][4] = s3 * (l * m * (n2 - 0.5 * (l2 + m2)) * dds - 2.0 * l * m * n2 * ddp + 0.5 * l * m * (1.0 + n2) * ddd);
    dd[1][4] = s3 * (m * n * (n2 - 0.5 * (l2 + m2)) * dds + m * n * (l2 + m2 - n2) * ddp
                     - 0.5 * m * n * (l2 + m2) * ddd);
    dd[2][4] = s3 * (l * n * (n2 - 0.5 * (l2 + m2)) * dds + l * n * (l2 + m2 - n2) * ddp
                     - 0.5 * l * n * (l2 + m2) * ddd);
    dd[3][3] = 0.75 * (l2 - m2) * (l2 - m2) * dds + (l2 + m2 - (l2 - m2) * (l2 - m2)) * ddp
             + (n2 + 0.25 * (l2 - m2) * (l2 - m2)) * ddd;
    dd[3][4] = s3 * (0.5 * (l2 - m2) * (n2 - 0.5 * (l2 + m2)) * dds + n2 * (m2 - l2) * ddp
                     + 0.25 * (1.0 + n2) * (l2 - m2) * ddd);
    dd[4][4] = (n2 - 0.5 * (l2 + m2)) * (n2 - 0.5 * (l2 + m2)) * dds + 3.0 * n2 * (l2 + m2) * ddp
             + 0.75 * (l2 + m2) * (l2 + m2) * ddd;
    for (int a = 0; a < 5; ++a) {
        E[0][4 + a] = sdrow[a];
        for (int b = 0; b < 3; ++b) E[1 + b][4 + a] = pd[b][a];
        for (int b = a; b < 5; ++b) E[4 + a][4 + b] = dd[a][b];
    }
    /* lower blocks by parity: E[b][a] = (-1)^(l_a + l_b) E[a][b] */
    for (int a = 0; a < 9; ++a)
        for (int b = 0; b < 9; ++b)
            if (lq[b] > lq[a] || (lq[b] == lq[a] && b > a))
                E[b][a] = ((lq[a] + lq[b]) & 1) ? -E[a][b] : E[a][b];
}

/*
 * Block of a bond between atoms of species A (row) and B (column): the blocks
 * with l_a <= l_b from the integrals v_ab of the ordered pair (A, B) (for a
 * mixed integral the lower angular momentum sits on A), the blocks with
 * l_a > l_b from those of (B, A): <a_i|H|b_j> = <b_j|H|a_i> is the table's
 * block of the reversed bond, (-1)^(l_a + l_b) times its entry at c.
 */
static void orc_sk_table_pair(const double c[3], const double v_ab[10], const double v_ba[10], double E[9][9])
{
    double Eb[9][9];
    orc_sk_table(c, v_ab, E);
    orc_sk_table(c, v_ba, Eb);
    for (int a = 0; a < 9; ++a)
        for (int b = 0; b < 9; ++b)
            if (lq[a] > lq[b]) E[a][b] = Eb[a][b];
}

/*
 * Orbital Hamiltonian of one species with norb = 4 (s, p) or 9 (s, p, d)
 * orbitals per atom: orbital index norb i + a.  For every pair {i, j} of
 * orc_neighbor_pairs the bond vector d = x_j - x_i (minimum image), r = |d|,
 * f = exp(-beta (r/r0 - 1)) give H[norb i + a][norb j + b] = f E(d/r)[a][b]
 * and H[norb j + b][norb i + a] = the same number (E(-c) = E(c)^T).  v holds
 * the ten integrals of orc_sk_table at r0 (only the first four enter when
 * norb = 4); onsite e = {e_s, e_p, e_d}.  With scale (NULL = none, else
 * [npairs][10]) pair p uses the integrals v[l] scale[p][l] instead of v[l]:
 * the learned form of Eq. (2), where each bond's two-centre integrals are
 * network outputs (here v[l] (1 + y_l) with y_l the output of network l), the
 * angular factors unchanged.  Several species (pair_v != NULL): atom i has
 * species[i] in [0, n_species); a bond i -> j uses pair_v[(s_i n_species +
 * s_j) 10 + l] for the blocks with l_a <= l_b and those of (s_j, s_i) for the
 * others (orc_sk_table_pair); onsite energies species_e[3 s_i + shell]; v and
 * e are then unused.  CSR of the off-diagonal part (row_ptr [norb n + 1],
 * col/val [2 norb^2 npairs], columns ascending); diag [norb n].
 * Returns 0, -1 on a bad norb, -2 when out of memory.
 */
int orc_assemble_sk(int64_t n, const double *pos, const double box[3], const int32_t periodic[3],
                    int64_t npairs, const int32_t *pi, const int32_t *pj, int32_t norb, const double v[10],
                    const double *scale, const double e[3], const int32_t *species, int32_t n_species,
                    const double *pair_v, const double *species_e, double r0, double beta,
                    int64_t *row_ptr, int32_t *col, double *val, double *diag)
{
    if (norb != 4 && norb != 9) return -1;
    const int64_t nr = norb * n;
    int64_t *deg = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    if (!deg) return -2;
    for (int64_t p = 0; p < npairs; ++p) { deg[pi[p]]++; deg[pj[p]]++; }
    row_ptr[0] = 0;
    for (int64_t r = 0; r < nr; ++r) row_ptr[r + 1] = row_ptr[r] + norb * deg[r / norb];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nr > 0 ? nr : 1));
    if (!fill) { free(deg); return -2; }
    for (int64_t r = 0; r < nr; ++r) fill[r] = row_ptr[r];
    for (int64_t p = 0; p < npairs; ++p) {
        int32_t i = pi[p], j = pj[p];
        double d[3], E[9][9], c[3];
        double r = orc_displacement(pos, i, j, box, periodic, d);
        for (int k = 0; k < 3; ++k) c[k] = d[k] / r;
        double vab[10], vba[10];
        const double *tab = pair_v ? pair_v + 10 * ((int64_t)species[i] * n_species + species[j]) : v;
        const double *tba = pair_v ? pair_v + 10 * ((int64_t)species[j] * n_species + species[i]) : v;
        for (int l = 0; l < 10; ++l) {
            vab[l] = scale ? tab[l] * scale[10 * p + l] : tab[l];
            vba[l] = scale ? tba[l] * scale[10 * p + l] : tba[l];
        }
        orc_sk_table_pair(c, vab, vba, E);
        double f = exp(-beta * (r / r0 - 1.0));
        for (int a = 0; a < norb; ++a)
            for (int b = 0; b < norb; ++b) {
                double h = f * E[a][b];
                int64_t q = fill[norb * (int64_t)i + a]++;
                col[q] = norb * j + b; val[q] = h;
                q = fill[norb * (int64_t)j + b]++;
                col[q] = norb * i + a; val[q] = h;
            }
    }
    /* sort each row by column (values travel with their columns) */
    for (int64_t r = 0; r < nr; ++r)
        for (int64_t q = row_ptr[r] + 1; q < row_ptr[r + 1]; ++q) {
            int32_t cq = col[q];
            double vq = val[q];
            int64_t t = q - 1;
            while (t >= row_ptr[r] && col[t] > cq) { col[t + 1] = col[t]; val[t + 1] = val[t]; --t; }
            col[t + 1] = cq; val[t + 1] = vq;
        }
    for (int64_t r = 0; r < nr; ++r) {
        int a = (int)(r % norb);
        const double *es = pair_v ? species_e + 3 * (int64_t)species[r / norb] : e;
        diag[r] = a == 0 ? es[0] : (a < 4 ? es[1] : es[2]);
    }
    free(deg); free(fill);
    return 0;
}
