/*
 * ENUFFT reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU implementation of what the hot path computes, written
 * from the paper's definitions.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the product path never
 * does.  It shares no code, header, table or constant with the GPU library.
 *
 * Contents
 *   oracle_hann          radial Hann taper and its gradient (the per-cell window).
 *   oracle_type1         direct quadrature sum: the windowed, weighted type-1
 *                        non-uniform DFT, Section 2.1.1 eq. (quad) and
 *                        Appendix A2 eq. (discrete_quadrature), evaluated term by
 *                        term -- the exact result the NUFFT approximates
 *                        (Section 2.1.2, eqs. spreading..deconv).
 *   oracle_type1_modes   the same sum at an arbitrary list of integer modes.
 *   oracle_type1_axes    the same sum on a product set of listed modes per axis.
 *   oracle_ems           Elastic Mode Selection, Section 2.2 eqs. (energy),
 *                        (sorted_energy), (n_eff), (s_delta), (c_score),
 *                        (alpha_c), (f_cum), (k_elastic), in the paper's order.
 *   oracle_mw_weight,    EMS per timestep with the flow-dependent launch weight of
 *   oracle_ems_flow      Appendix A7 (eqs. mountain_omega, mw_dispersion, mw_action)
 *                        folded into eq. (weighted_e), on fixed coefficients.
 *   oracle_type1_vjp     the exact adjoint (a direct type-2 sum with the +i sign
 *                        of eq. (series)) and the chain rule through the window
 *                        and weights: gradients of a real loss with respect to
 *                        heights and point coordinates.
 *   oracle_reconstruct   the truncated series of eq. (series) over the retained
 *                        modes evaluated at every sample (a direct type-2 sum),
 *                        and the per-cell diagnostics of Section 3.2: the relative
 *                        reconstruction RMSE of eq. (alps_relative_rmse) and the
 *                        two sides of Parseval's identity, eq. (spectral_variance).
 *
 * Conventions (readings of points the paper leaves open)
 *   - Local coordinates live on a periodic box of side 2*pi, so wave numbers
 *     are integers (Appendix A1 with L = 2H = 2*pi).
 *   - A mode box of N modes per axis holds k in [-floor(N/2), ceil(N/2) - 1];
 *     outputs are row-major with k_y slow and k_x fast, both ascending.
 *   - The coefficient carries a caller-chosen overall factor `scale` in place of
 *     the 1/|D| of eq. (discrete_quadrature).
 *   - EMS units are +-k pairs (singletons where the partner is outside the
 *     box); the DC mode is excluded by default; ties in energy are broken by
 *     ascending unit id (row-major flat index of the unit's representative).
 *
 * Parity pins: see the test suite (brute force on tiny inputs, the regular-grid
 * reduction to the DFT, single-point closed forms, linearity, Hermitian
 * symmetry, the shift theorem, the Monte Carlo error law of Appendix A3, the
 * Appendix A4 closed forms for EMS, the adjoint identity and finite
 * differences).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------ window */

/* Radial Hann taper centred on (cx, cy) with radius R:
 *   W(r) = (1 + cos(pi r / R)) / 2   for r < R, and 0 otherwise.
 * Gradient: dW/dr = -(pi / 2R) sin(pi r / R), and grad r = (x - cx, y - cy) / r, so
 *   grad W = -(pi^2 / (2 R^2)) * sinc(pi r / R) * (x - cx, y - cy),  sinc(u) = sin(u)/u,
 * which is finite at r = 0.  kind == 0 means no window (W = 1, grad W = 0). */
void oracle_hann(int kind, double x, double y, double cx, double cy, double R,
                 double *W, double *dWdx, double *dWdy)
{
    if (kind == 0) { *W = 1.0; *dWdx = 0.0; *dWdy = 0.0; return; }
    double dx = x - cx, dy = y - cy;
    double r = sqrt(dx * dx + dy * dy);
    if (!(r < R)) { *W = 0.0; *dWdx = 0.0; *dWdy = 0.0; return; }
    double u = M_PI * r / R;
    *W = 0.5 * (1.0 + cos(u));
    double sinc = (u == 0.0) ? 1.0 : sin(u) / u;
    double g = -(M_PI * M_PI) / (2.0 * R * R) * sinc;
    *dWdx = g * dx;
    *dWdy = g * dy;
}

/* ------------------------------------------------------------------ type 1 */

static int mode_lo(int N) { return -(N / 2); }

/* Point strength c_j = w_j * W(x_j, y_j) * h_j: the quadrature weight of
 * eq. (discrete_quadrature) times the window times the height. */
static double strength(int kind, const double *win, double x, double y, double h, double w)
{
    double W, a, b;
    oracle_hann(kind, x, y, win[0], win[1], win[2], &W, &a, &b);
    return w * W * h;
}

/* f[c][ky][kx] = scale * sum_{j in c} c_j exp(-i (kx x_j + ky y_j)).
 *
 * The exponential of a sum is evaluated as the product of the per-axis
 * exponentials exp(-i kx x) exp(-i ky y), each from a direct sin/cos of the
 * product k * x.  Points are summed in blocks of BLK; block partial sums are
 * added in block order, so the result does not depend on the thread count.
 * f_out holds interleaved (re, im) pairs. */
#define BLK 2048
#define PART_BYTES_MAX ((int64_t)1 << 30)
void oracle_type1(int64_t n_cells, const int64_t *off,
                  const double *x, const double *y, const double *h, const double *w,
                  const double *windows, int kind, int N1, int N2, double scale,
                  double *f_out)
{
    const int64_t M = (int64_t)N1 * N2;
    int64_t group = PART_BYTES_MAX / (int64_t)(sizeof(double) * 2 * M);
    if (group < 1) group = 1;
    for (int64_t c = 0; c < n_cells; ++c) {
        const int64_t a = off[c], b = off[c + 1];
        const int64_t nb = (b - a + BLK - 1) / BLK;
        double *out = f_out + 2 * M * c;
        memset(out, 0, sizeof(double) * 2 * M);
        for (int64_t g0 = 0; g0 < nb; g0 += group) {
            const int64_t g1 = (g0 + group < nb) ? g0 + group : nb;
            double *part = (double *)calloc((size_t)((g1 - g0) * 2 * M), sizeof(double));
            #pragma omp parallel
            {
                double *ex = (double *)malloc(sizeof(double) * 2 * N1);
                double *ey = (double *)malloc(sizeof(double) * 2 * N2);
                #pragma omp for schedule(dynamic, 1)
                for (int64_t blk = g0; blk < g1; ++blk) {
                    double *acc = part + (blk - g0) * 2 * M;
                    const int64_t j0 = a + blk * BLK;
                    const int64_t j1 = (j0 + BLK < b) ? j0 + BLK : b;
                    for (int64_t j = j0; j < j1; ++j) {
                        double cj = strength(kind, windows + 3 * c, x[j], y[j], h[j], w[j]);
                        if (cj == 0.0) continue;
                        for (int i = 0; i < N1; ++i) {
                            double k = (double)(mode_lo(N1) + i);
                            ex[2 * i] = cos(k * x[j]);
                            ex[2 * i + 1] = -sin(k * x[j]);
                        }
                        for (int i = 0; i < N2; ++i) {
                            double k = (double)(mode_lo(N2) + i);
                            ey[2 * i] = cj * cos(k * y[j]);
                            ey[2 * i + 1] = -cj * sin(k * y[j]);
                        }
                        for (int r = 0; r < N2; ++r) {
                            const double yr = ey[2 * r], yi = ey[2 * r + 1];
                            double *row = acc + 2 * (int64_t)r * N1;
                            for (int i = 0; i < N1; ++i) {
                                const double xr = ex[2 * i], xi = ex[2 * i + 1];
                                row[2 * i] += yr * xr - yi * xi;
                                row[2 * i + 1] += yr * xi + yi * xr;
                            }
                        }
                    }
                }
                free(ex);
                free(ey);
            }
            for (int64_t blk = g0; blk < g1; ++blk)
                for (int64_t m = 0; m < 2 * M; ++m) out[m] += part[(blk - g0) * 2 * M + m];
            free(part);
        }
        for (int64_t m = 0; m < 2 * M; ++m) out[m] *= scale;
    }
}

/* Strengths c_j for one cell (exposed so tests can build brute-force sums). */
void oracle_strength(int64_t n, const double *x, const double *y, const double *h, const double *w,
                     int kind, const double *win, double *c_out)
{
    for (int64_t j = 0; j < n; ++j) c_out[j] = strength(kind, win, x[j], y[j], h[j], w[j]);
}

/* f_m = scale * sum_j c_j exp(-i (kx_m x_j + ky_m y_j)) for M listed integer modes,
 * with the strengths c_j given.  Parallel over modes; each mode sums its points in
 * index order. */
void oracle_type1_modes(int64_t n, const double *x, const double *y, const double *c,
                        int64_t M, const int32_t *kx, const int32_t *ky, double scale, double *out)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m) {
        double sr = 0.0, si = 0.0;
        const double ax = (double)kx[m], ay = (double)ky[m];
        for (int64_t j = 0; j < n; ++j) {
            double ph = ax * x[j] + ay * y[j];
            sr += c[j] * cos(ph);
            si -= c[j] * sin(ph);
        }
        out[2 * m] = scale * sr;
        out[2 * m + 1] = scale * si;
    }
}

/* The same sum on a product set of listed integer modes: for every ky in ky_list
 * (n2 entries) and kx in kx_list (n1 entries),
 *   out[r][i] = scale * sum_j c_j exp(-i (kx_list[i] x_j + ky_list[r] y_j)),
 * interleaved (re, im), row-major with ky slow.  Per point the per-axis exponentials
 * are direct sin/cos of k * x; points are summed in blocks of BLK whose partial sums
 * are added in block order (independent of the thread count). */
void oracle_type1_axes(int64_t n, const double *x, const double *y, const double *c,
                       int n1, const int32_t *kx_list, int n2, const int32_t *ky_list,
                       double scale, double *out)
{
    const int64_t M = (int64_t)n1 * n2;
    const int64_t nb = (n + BLK - 1) / BLK;
    memset(out, 0, sizeof(double) * 2 * M);
    int64_t group = PART_BYTES_MAX / (int64_t)(sizeof(double) * 2 * M);
    if (group < 1) group = 1;
    for (int64_t g0 = 0; g0 < nb; g0 += group) {
        const int64_t g1 = (g0 + group < nb) ? g0 + group : nb;
        double *part = (double *)calloc((size_t)((g1 - g0) * 2 * M), sizeof(double));
        #pragma omp parallel
        {
            double *ex = (double *)malloc(sizeof(double) * 2 * n1);
            double *ey = (double *)malloc(sizeof(double) * 2 * n2);
            #pragma omp for schedule(dynamic, 1)
            for (int64_t blk = g0; blk < g1; ++blk) {
                double *acc = part + (blk - g0) * 2 * M;
                const int64_t j0 = blk * BLK;
                const int64_t j1 = (j0 + BLK < n) ? j0 + BLK : n;
                for (int64_t j = j0; j < j1; ++j) {
                    if (c[j] == 0.0) continue;
                    for (int i = 0; i < n1; ++i) {
                        const double ph = (double)kx_list[i] * x[j];
                        ex[2 * i] = cos(ph);
                        ex[2 * i + 1] = -sin(ph);
                    }
                    for (int r = 0; r < n2; ++r) {
                        const double ph = (double)ky_list[r] * y[j];
                        ey[2 * r] = c[j] * cos(ph);
                        ey[2 * r + 1] = -c[j] * sin(ph);
                    }
                    for (int r = 0; r < n2; ++r) {
                        const double yr = ey[2 * r], yi = ey[2 * r + 1];
                        double *dst = acc + 2 * (int64_t)r * n1;
                        for (int i = 0; i < n1; ++i) {
                            const double xr = ex[2 * i], xi = ex[2 * i + 1];
                            dst[2 * i] += yr * xr - yi * xi;
                            dst[2 * i + 1] += yr * xi + yi * xr;
                        }
                    }
                }
            }
            free(ex);
            free(ey);
        }
        for (int64_t blk = g0; blk < g1; ++blk)
            for (int64_t m = 0; m < 2 * M; ++m) out[m] += part[(blk - g0) * 2 * M + m];
        free(part);
    }
    for (int64_t q = 0; q < 2 * M; ++q) out[q] *= scale;
}

/* --------------------------------------------------------------------- EMS */

typedef struct { double e; int32_t id; int32_t rep; int32_t partner; } unit_t;

/* Descending energy, then ascending unit id: the order of eq. (sorted_energy). */
static int cmp_unit(const void *pa, const void *pb)
{
    const unit_t *a = (const unit_t *)pa, *b = (const unit_t *)pb;
    if (a->e > b->e) return -1;
    if (a->e < b->e) return 1;
    return (a->id < b->id) ? -1 : (a->id > b->id);
}

/* Neumaier compensated accumulation. */
typedef struct { double s, c; } ksum_t;
static void kadd(ksum_t *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}
static double kval(const ksum_t *k) { return k->s + k->c; }

/* Elastic Mode Selection for one cell's N2 x N1 coefficients f (interleaved complex).
 *
 *  1. Units: with use_pairs, the pair {k, -k} when both lie in the box (the pair
 *     energy below eq. (energy)), otherwise the single mode; without use_pairs every
 *     signed mode is a unit.  The DC mode is skipped when exclude_dc is set.
 *  2. E_u = sum over the unit's modes of omega_k |f_k|^2 (eq. (energy), weighted as
 *     in eq. (weighted_e) when mode_weight is given, else omega = 1).
 *  3. Sort descending, eq. (sorted_energy); ties by ascending unit id.
 *  4. J* = number of units, J_max = min(J*, K_max) (footnote to eq. (alpha_c)).
 *  5. N_eff = (sum E)^2 / sum E^2 over all J* units, eq. (n_eff).
 *  6. N_clip = min(N_eff, J_max).
 *  7. S_delta = mean over j = 1..J_max-1 of exp(-(G_j - 1)/delta), G_j = E_(j)/E_(j+1),
 *     eq. (s_delta); a zero successor under a positive entry gives a zero term, 0/0
 *     gives G = 1, and J_max < 2 gives S_delta = 1.
 *  8. C = w1 N_clip / J_max + w2 S_delta, eq. (c_score).
 *  9. alpha_C = alpha_min + (alpha_max - alpha_min) C, eq. (alpha_c).
 * 10. theta(K) = sum_{j<=K} E_(j) / sum_r E_(r), eq. (f_cum), accumulated in sorted order;
 *     K_c = min{K : theta(K) >= alpha_C}, or J* if never reached.
 * 11. K* = min(J_max, max(K_min, K_c)), eq. (k_elastic); with zero total power
 *     K* = min(K_min, J*).
 * 12. keep = all modes of the first K* units; P = sum over kept modes of |f_k|^2.
 *
 * stats[8] = (T, P, N_eff, S_delta, C, alpha_C, theta(K*), J*).
 * sorted_id / sorted_e (each J* long, may be NULL) receive the sorted unit ids
 * and energies.  Returns J*, or -1 on bad arguments. */
int oracle_ems(int N1, int N2, const double *f, int k_min, int k_max,
               double alpha_min, double alpha_max, double delta, double w1, double w2,
               int use_pairs, int exclude_dc, const double *mode_weight,
               uint8_t *keep, int32_t *k_star, double *stats,
               int32_t *sorted_id, double *sorted_e)
{
    if (N1 <= 0 || N2 <= 0 || k_min < 0 || k_max < 1 || delta <= 0.0) return -1;
    const int lo1 = mode_lo(N1), lo2 = mode_lo(N2);
    const int hi1 = lo1 + N1 - 1, hi2 = lo2 + N2 - 1;
    const int M = N1 * N2;
    unit_t *u = (unit_t *)malloc(sizeof(unit_t) * (size_t)M);
    int J = 0;
    for (int r = 0; r < N2; ++r) {
        for (int i = 0; i < N1; ++i) {
            const int kx = lo1 + i, ky = lo2 + r;
            const int idx = r * N1 + i;
            if (exclude_dc && kx == 0 && ky == 0) continue;
            int partner = -1;
            if (use_pairs && !(kx == 0 && ky == 0)) {
                const int px = -kx, py = -ky;
                if (px >= lo1 && px <= hi1 && py >= lo2 && py <= hi2) partner = (py - lo2) * N1 + (px - lo1);
            }
            if (partner >= 0) {
                /* representative: k_y > 0, or k_y == 0 and k_x > 0 */
                const int is_rep = (ky > 0) || (ky == 0 && kx > 0);
                if (!is_rep) continue;
            }
            u[J].rep = idx;
            u[J].partner = partner;
            u[J].id = idx;
            double e = 0.0;
            const double om = mode_weight ? mode_weight[idx] : 1.0;
            e += om * (f[2 * idx] * f[2 * idx] + f[2 * idx + 1] * f[2 * idx + 1]);
            if (partner >= 0) {
                const double op = mode_weight ? mode_weight[partner] : 1.0;
                e += op * (f[2 * partner] * f[2 * partner] + f[2 * partner + 1] * f[2 * partner + 1]);
            }
            u[J].e = e;
            ++J;
        }
    }
    /* step 2: totals (before sorting, in unit-id order) */
    ksum_t T = {0, 0}, T2 = {0, 0};
    for (int j = 0; j < J; ++j) { kadd(&T, u[j].e); kadd(&T2, u[j].e * u[j].e); }
    const double tot = kval(&T), tot2 = kval(&T2);
    /* step 3 */
    qsort(u, (size_t)J, sizeof(unit_t), cmp_unit);
    /* step 4 */
    const int Jmax = (J < k_max) ? J : k_max;
    /* step 5, 6 */
    const double neff = (tot2 > 0.0) ? tot * tot / tot2 : 0.0;
    const double nclip = (neff < (double)Jmax) ? neff : (double)Jmax;
    /* step 7 */
    double sdel;
    if (Jmax < 2) {
        sdel = 1.0;
    } else {
        double acc = 0.0;
        for (int j = 0; j < Jmax - 1; ++j) {
            const double a = u[j].e, b = u[j + 1].e;
            double term;
            if (b == 0.0 && a == 0.0) term = 1.0;            /* 0/0: G = 1 */
            else if (b == 0.0) term = 0.0;                    /* infinite gap */
            else term = exp(-(a / b - 1.0) / delta);
            acc += term;
        }
        sdel = acc / (double)(Jmax - 1);
    }
    /* step 8, 9 */
    const double C = (Jmax > 0 ? w1 * nclip / (double)Jmax : 0.0) + w2 * sdel;
    const double alphaC = alpha_min + (alpha_max - alpha_min) * C;
    /* step 10, 11 */
    int kstar;
    double theta_k = 0.0;
    if (!(tot > 0.0)) {
        kstar = (k_min < J) ? k_min : J;
    } else {
        int kc = J;
        double run = 0.0;
        for (int j = 0; j < J; ++j) {
            run += u[j].e;
            if (run / tot >= alphaC) { kc = j + 1; break; }
        }
        int k = (kc > k_min) ? kc : k_min;
        kstar = (k < Jmax) ? k : Jmax;
    }
    /* step 12 */
    memset(keep, 0, (size_t)M);
    double run = 0.0;
    ksum_t P = {0, 0};
    for (int j = 0; j < kstar; ++j) {
        run += u[j].e;
        keep[u[j].rep] = 1;
        kadd(&P, f[2 * u[j].rep] * f[2 * u[j].rep] + f[2 * u[j].rep + 1] * f[2 * u[j].rep + 1]);
        if (u[j].partner >= 0) {
            const int p = u[j].partner;
            keep[p] = 1;
            kadd(&P, f[2 * p] * f[2 * p] + f[2 * p + 1] * f[2 * p + 1]);
        }
    }
    theta_k = (tot > 0.0) ? run / tot : 0.0;
    *k_star = kstar;
    stats[0] = tot; stats[1] = kval(&P); stats[2] = neff; stats[3] = sdel;
    stats[4] = C; stats[5] = alphaC; stats[6] = theta_k; stats[7] = (double)J;
    if (sorted_id) for (int j = 0; j < J; ++j) sorted_id[j] = u[j].id;
    if (sorted_e) for (int j = 0; j < J; ++j) sorted_e[j] = u[j].e;
    free(u);
    return J;
}

/* Batched EMS over n_cells cells (f contiguous per cell); parallel over cells. */
void oracle_ems_batched(int64_t n_cells, int N1, int N2, const double *f, int k_min, int k_max,
                        double alpha_min, double alpha_max, double delta, double w1, double w2,
                        int use_pairs, int exclude_dc, const double *mode_weight,
                        uint8_t *keep, int32_t *k_star, double *stats)
{
    const int64_t M = (int64_t)N1 * N2;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < n_cells; ++c)
        oracle_ems(N1, N2, f + 2 * M * c, k_min, k_max, alpha_min, alpha_max, delta, w1, w2,
                   use_pairs, exclude_dc, mode_weight, keep + M * c, k_star + c, stats + 8 * c,
                   NULL, NULL);
}

/* ------------------------------------------------------ flow-dependent EMS */

/* Launch weight of one mode for an orographic gravity wave (Appendix A7), in the
 * paper's order.  k = kscale (kx, ky) is the physical wave vector, u = (ux, uy)
 * the background wind, N the buoyancy frequency, fc the Coriolis parameter and
 * rho the background density.
 *   intrinsic frequency      omega = -k . u                               (eq. mountain_omega)
 *   vertical wave number     m^2 = |k|^2 (N^2 - omega^2) / (omega^2 - fc^2) (eq. mw_dispersion)
 *   wave action              A = -(rho / 2) (k . u) (|k|^2 + m^2) / |k|^2 |h|^2  (eq. mw_action)
 * The weight is |A| / |h|^2: the magnitude of the action density per unit modal power
 * (the action and the intrinsic frequency are taken on the same signed branch, so the
 * wave energy A omega is positive).  A mode that does not propagate vertically
 * (|omega| <= fc or |omega| >= N, the bounds of eq. mw_dispersion) and the k = 0 mode
 * have weight 0. */
double oracle_mw_weight(int kx, int ky, double kscale, double ux, double uy, double N, double fc, double rho)
{
    const double k1 = kscale * (double)kx, k2 = kscale * (double)ky;
    const double kk = k1 * k1 + k2 * k2;
    if (!(kk > 0.0)) return 0.0;
    const double omega = -(k1 * ux + k2 * uy);
    const double aw = fabs(omega);
    if (!(aw > fabs(fc) && aw < N)) return 0.0;
    const double m2 = kk * (N * N - omega * omega) / (omega * omega - fc * fc);
    const double A = -(rho / 2.0) * (k1 * ux + k2 * uy) * (kk + m2) / kk;
    return fabs(A);
}

/* EMS per timestep on fixed coefficients: for step s and cell c the mode weights of
 * eq. (weighted_e) are the launch weights of oracle_mw_weight under the flow record
 * flow[6 (s n_cells + c) + (0..5)] = (ux, uy, N, fc, rho, kscale), then oracle_ems.
 * Outputs are indexed by s n_cells + c; keep may be NULL. */
void oracle_ems_flow(int n_steps, int64_t n_cells, int N1, int N2, const double *f, int k_min, int k_max,
                     double alpha_min, double alpha_max, double delta, double w1, double w2,
                     int use_pairs, int exclude_dc, const double *flow,
                     uint8_t *keep, int32_t *k_star, double *stats)
{
    const int64_t M = (int64_t)N1 * N2;
    const int64_t total = (int64_t)n_steps * n_cells;
    #pragma omp parallel
    {
        double *om = (double *)malloc(sizeof(double) * (size_t)M);
        uint8_t *kp = (uint8_t *)malloc((size_t)M);
        #pragma omp for schedule(dynamic, 1)
        for (int64_t v = 0; v < total; ++v) {
            const int64_t c = v % n_cells;
            const double *fl = flow + 6 * v;
            for (int r = 0; r < N2; ++r)
                for (int i = 0; i < N1; ++i)
                    om[(int64_t)r * N1 + i] = oracle_mw_weight(mode_lo(N1) + i, mode_lo(N2) + r, fl[5], fl[0],
                                                               fl[1], fl[2], fl[3], fl[4]);
            oracle_ems(N1, N2, f + 2 * M * c, k_min, k_max, alpha_min, alpha_max, delta, w1, w2, use_pairs,
                       exclude_dc, om, keep ? keep + M * v : kp, k_star + v, stats + 8 * v, NULL, NULL);
        }
        free(om);
        free(kp);
    }
}

/* ---------------------------------------------------------------- adjoint */

/* Real adjoint of the type-1 map and the chain rule to heights and coordinates.
 *
 * For a real loss L of the coefficients with cotangent g_k = dL/dRe f_k + i dL/dIm f_k,
 * and f_k = scale * sum_j c_j exp(-i k.x_j) with c_j = w_j W(x_j) h_j:
 *   u_j  = dL/dc_j          = scale * Re sum_k g_k exp(+i k.x_j)       (type-2 sum, +i sign)
 *   ux_j = scale * Re sum_k (i kx) g_k exp(+i k.x_j),  uy_j likewise with ky,
 *   dL/dh_j = w_j W_j u_j,
 *   dL/dx_j = w_j h_j (dW/dx_j u_j + W_j ux_j),   dL/dy_j likewise.
 * The weights and the window parameters are held fixed.  Any output may be NULL. */
void oracle_type1_vjp(int64_t n_cells, const int64_t *off,
                      const double *x, const double *y, const double *h, const double *w,
                      const double *windows, int kind, int N1, int N2, double scale,
                      const double *g, double *grad_h, double *grad_x, double *grad_y)
{
    const int64_t M = (int64_t)N1 * N2;
    for (int64_t c = 0; c < n_cells; ++c) {
        const int64_t a = off[c], b = off[c + 1];
        const double *gc = g + 2 * M * c;
        const double *win = windows + 3 * c;
        #pragma omp parallel
        {
        double *ex = (double *)malloc(sizeof(double) * 2 * N1);
        double *ey = (double *)malloc(sizeof(double) * 2 * N2);
        #pragma omp for schedule(dynamic, 64)
        for (int64_t j = a; j < b; ++j) {
            for (int i = 0; i < N1; ++i) {
                const double k = (double)(mode_lo(N1) + i);
                ex[2 * i] = cos(k * x[j]);
                ex[2 * i + 1] = sin(k * x[j]);
            }
            for (int i = 0; i < N2; ++i) {
                const double k = (double)(mode_lo(N2) + i);
                ey[2 * i] = cos(k * y[j]);
                ey[2 * i + 1] = sin(k * y[j]);
            }
            double u = 0.0, ux = 0.0, uy = 0.0;
            for (int r = 0; r < N2; ++r) {
                const double kyv = (double)(mode_lo(N2) + r);
                double su = 0.0, sx = 0.0;
                for (int i = 0; i < N1; ++i) {
                    const double kxv = (double)(mode_lo(N1) + i);
                    const double gr = gc[2 * (r * N1 + i)], gi = gc[2 * (r * N1 + i) + 1];
                    /* e = exp(+i (kx x + ky y)) */
                    const double er = ex[2 * i] * ey[2 * r] - ex[2 * i + 1] * ey[2 * r + 1];
                    const double ei = ex[2 * i] * ey[2 * r + 1] + ex[2 * i + 1] * ey[2 * r];
                    const double re = gr * er - gi * ei;      /* Re(g e) */
                    const double im = gr * ei + gi * er;      /* Im(g e) */
                    su += re;
                    sx += -kxv * im;                          /* Re(i kx g e) = -kx Im(g e) */
                    uy += -kyv * im;
                }
                u += su;
                ux += sx;
            }
            u *= scale; ux *= scale; uy *= scale;
            double W, dWx, dWy;
            oracle_hann(kind, x[j], y[j], win[0], win[1], win[2], &W, &dWx, &dWy);
            if (grad_h) grad_h[j] = w[j] * W * u;
            if (grad_x) grad_x[j] = w[j] * h[j] * (dWx * u + W * ux);
            if (grad_y) grad_y[j] = w[j] * h[j] * (dWy * u + W * uy);
        }
        free(ex);
        free(ey);
        }
    }
}

/* ------------------------------------------------------------ reconstruction */

/* Reconstruction from retained coefficients and the Section 3.2 diagnostics.
 *
 * For cell c with coefficients coef (interleaved complex, N2 x N1, as oracle_type1
 * writes them) and a keep mask (NULL: every mode):
 *   h_rec(x_q) = Re sum_{k kept} coef_k exp(+i (kx x_q + ky y_q))      (eq. series)
 * The coefficients represent the windowed heights, so the target at sample q is
 *   t_q = W_c(x_q, y_q) h_q   (= h_q without a window, kind == 0).
 * diag[8 c + i]:
 *   0  Q_c, the number of samples
 *   1  sum_q (t_q - h_rec(x_q))^2
 *   2  sum_q t_q^2
 *   3  sigma^2_phys = (1 / |D_c|) sum_q w_q t_q^2                 (eq. spectral_variance, left)
 *   4  sigma^2_spec = sum over all modes k != 0 of |coef_k|^2      (eq. spectral_variance, right)
 *   5  the same sum over the kept modes only
 *   6  eps_rel = sqrt(diag[1] / diag[2])                           (eq. alps_relative_rmse)
 *   7  sigma^2_spec / sigma^2_phys (the Parseval ratio)
 * area[c] = |D_c|.  Sums over samples are compensated (Neumaier), in sample order.
 * h_rec may be NULL. */
void oracle_reconstruct(int64_t n_cells, const int64_t *off,
                        const double *x, const double *y, const double *h, const double *w,
                        const double *windows, int kind, int N1, int N2,
                        const double *coef, const uint8_t *keep, const double *area,
                        double *h_rec, double *diag)
{
    const int64_t M = (int64_t)N1 * N2;
    for (int64_t c = 0; c < n_cells; ++c) {
        const int64_t a = off[c], b = off[c + 1];
        const double *cc = coef + 2 * M * c;
        const uint8_t *kc = keep ? keep + M * c : NULL;
        const double *win = windows + 3 * c;
        double *rec = (double *)malloc(sizeof(double) * (size_t)((b - a) > 0 ? (b - a) : 1));
        #pragma omp parallel for schedule(dynamic, 64)
        for (int64_t j = a; j < b; ++j) {
            double s = 0.0;
            for (int r = 0; r < N2; ++r) {
                const double ky = (double)(mode_lo(N2) + r);
                for (int i = 0; i < N1; ++i) {
                    const int64_t m = (int64_t)r * N1 + i;
                    if (kc && !kc[m]) continue;
                    const double kx = (double)(mode_lo(N1) + i);
                    const double ph = kx * x[j] + ky * y[j];
                    /* Re(coef e^{+i ph}) */
                    s += cc[2 * m] * cos(ph) - cc[2 * m + 1] * sin(ph);
                }
            }
            rec[j - a] = s;
        }
        ksum_t e2 = {0, 0}, t2 = {0, 0}, wt2 = {0, 0}, sall = {0, 0}, skept = {0, 0};
        for (int64_t j = a; j < b; ++j) {
            double W, gx, gy;
            oracle_hann(kind, x[j], y[j], win[0], win[1], win[2], &W, &gx, &gy);
            const double t = W * h[j];
            const double d = t - rec[j - a];
            kadd(&e2, d * d);
            kadd(&t2, t * t);
            kadd(&wt2, w[j] * t * t);
            if (h_rec) h_rec[j] = rec[j - a];
        }
        for (int r = 0; r < N2; ++r)
            for (int i = 0; i < N1; ++i) {
                if (mode_lo(N1) + i == 0 && mode_lo(N2) + r == 0) continue;
                const int64_t m = (int64_t)r * N1 + i;
                const double p2 = cc[2 * m] * cc[2 * m] + cc[2 * m + 1] * cc[2 * m + 1];
                kadd(&sall, p2);
                if (!kc || kc[m]) kadd(&skept, p2);
            }
        double *dg = diag + 8 * c;
        dg[0] = (double)(b - a);
        dg[1] = kval(&e2);
        dg[2] = kval(&t2);
        dg[3] = kval(&wt2) / area[c];
        dg[4] = kval(&sall);
        dg[5] = kval(&skept);
        dg[6] = dg[2] > 0.0 ? sqrt(dg[1] / dg[2]) : 0.0;
        dg[7] = dg[3] > 0.0 ? dg[4] / dg[3] : 0.0;
        free(rec);
    }
}

/* ---------------------------------------------------------- cell geometry */

/* Local frame, support mask, quadrature weights and deplaning of Appendices A1, A2 and
 * A6 for triangular cells, in the paper's order.
 *
 * tri[6 c .. 6 c + 5] = (v1x, v1y, v2x, v2y, v3x, v3y), in the plane of the samples.
 *   centroid        xbar = (v1 + v2 + v3) / 3
 *   orientation     frame 0: R = I (centroid-aligned); frame 1: the rotation of
 *                   eq. (rotation_matrix) that takes the longest of the edges
 *                   e1 = v2 - v1, e2 = v3 - v2, e3 = v1 - v3 onto the +x axis
 *                   (the first of equal longest edges)
 *   local coords    u = R (x - xbar)
 *   half-width      H = (eta / 2) max(extent of the rotated vertices along x, along y)
 *   box coordinates (u_x, u_y) pi / H: the square [-H, H]^2 of period 2H mapped onto the
 *                   2 pi box, so the integer wave numbers are k_m = 2 pi m / (2H)
 *   mask            0 square (|u_x|, |u_y| <= H), 1 triangle (u inside the rotated
 *                   triangle, edges included, and inside the square: the square is
 *                   centred on the centroid, so it can cut the triangle), 2 circle
 *                   (|u| <= H); |D| the area of the mask within the square
 *   weights         0 uniform: w_q = |D| / Q_in (eq. uniform_weights) for the Q_in
 *                   samples inside the mask;
 *                   1 Voronoi by raster sampling (eqs. raster_grid .. voronoi_weights):
 *                   raster N_g x N_g cell centres over the square, those inside the
 *                   mask each assigned to the nearest inside sample (the lowest index
 *                   among equally near ones), A_q = n_q |D| / |G|; a sample with no
 *                   raster point gets floor_frac |D| / |G| and all areas are then
 *                   scaled so that they sum to |D|
 *   deplaning       h' = h - hbar, hbar = (1 / |D|) sum_{inside} w_q h_q (eq.
 *                   alps_deplaning), when deplane is set; else h' = h
 * Outputs per sample: xb, yb (box coordinates), hb (h'), wb = w_q / |D| (0 outside
 * the mask: the factor eq. (discrete_quadrature) puts on h_q), inside (0 / 1) and, when
 * counts is not NULL, n_q.  Per cell, info[8 c ..] = (xbar_x, xbar_y, cos, sin, H, |D|,
 * Q_in, hbar).  Returns 0, or -1 on bad arguments. */
static int point_in_triangle(double px, double py, const double *t)
{
    /* signs of the three edge cross products; inside (or on an edge) when none of
     * them has the opposite sign of another */
    double d1 = (px - t[2]) * (t[1] - t[3]) - (t[0] - t[2]) * (py - t[3]);
    double d2 = (px - t[4]) * (t[3] - t[5]) - (t[2] - t[4]) * (py - t[5]);
    double d3 = (px - t[0]) * (t[5] - t[1]) - (t[4] - t[0]) * (py - t[1]);
    int neg = (d1 < 0) || (d2 < 0) || (d3 < 0);
    int pos = (d1 > 0) || (d2 > 0) || (d3 > 0);
    return !(neg && pos);
}

static int in_mask(int mask, double ux, double uy, double H, const double *ut)
{
    if (mask == 0) return fabs(ux) <= H && fabs(uy) <= H;
    if (mask == 2) return ux * ux + uy * uy <= H * H;
    return fabs(ux) <= H && fabs(uy) <= H && point_in_triangle(ux, uy, ut);
}

/* Area of the triangle ut clipped to the square [-H, H]^2: the polygon cut by the four
 * half-planes one after the other, then the shoelace formula. */
static double clipped_triangle_area(const double *ut, double H)
{
    double P[16][2], Qp[16][2];
    int n = 3;
    for (int i = 0; i < 3; ++i) { P[i][0] = ut[2 * i]; P[i][1] = ut[2 * i + 1]; }
    for (int side = 0; side < 4; ++side) {
        /* keep s * coordinate <= H, coordinate axis = side / 2, s = +-1 */
        const int ax = side >> 1;
        const double sg = (side & 1) ? -1.0 : 1.0;
        int m = 0;
        for (int i = 0; i < n; ++i) {
            const double *A = P[i], *B = P[(i + 1) % n];
            const double da = sg * A[ax] - H, db = sg * B[ax] - H;
            if (da <= 0) { Qp[m][0] = A[0]; Qp[m][1] = A[1]; ++m; }
            if ((da < 0 && db > 0) || (da > 0 && db < 0)) {
                const double t = da / (da - db);
                Qp[m][0] = A[0] + t * (B[0] - A[0]);
                Qp[m][1] = A[1] + t * (B[1] - A[1]);
                ++m;
            }
        }
        n = m;
        for (int i = 0; i < n; ++i) { P[i][0] = Qp[i][0]; P[i][1] = Qp[i][1]; }
    }
    double s2 = 0.0;
    for (int i = 0; i < n; ++i) s2 += P[i][0] * P[(i + 1) % n][1] - P[(i + 1) % n][0] * P[i][1];
    return 0.5 * fabs(s2);
}

int oracle_cell_geometry(int64_t n_cells, const int64_t *off, const double *tri,
                         const double *x, const double *y, const double *h,
                         int frame, int mask, int weights, int raster, double eta, double floor_frac, int deplane,
                         double *xb, double *yb, double *hb, double *wb, uint8_t *inside, double *info,
                         int32_t *counts)
{
    if (frame < 0 || frame > 1 || mask < 0 || mask > 2 || weights < 0 || weights > 1) return -1;
    if (!(eta >= 1.0) || (weights == 1 && raster < 1) || !(floor_frac >= 0.0)) return -1;
    for (int64_t c = 0; c < n_cells; ++c) {
        const double *v = tri + 6 * c;
        const double cx = (v[0] + v[2] + v[4]) / 3.0, cy = (v[1] + v[3] + v[5]) / 3.0;
        double cs = 1.0, sn = 0.0;
        if (frame == 1) {
            const double e[3][2] = {{v[2] - v[0], v[3] - v[1]}, {v[4] - v[2], v[5] - v[3]}, {v[0] - v[4], v[1] - v[5]}};
            int m = 0;
            double best = -1.0;
            for (int i = 0; i < 3; ++i) {
                const double L = sqrt(e[i][0] * e[i][0] + e[i][1] * e[i][1]);
                if (L > best) { best = L; m = i; }
            }
            cs = e[m][0] / best;
            sn = e[m][1] / best;
        }
        /* rotated vertices and the half-width */
        double ut[6];
        for (int i = 0; i < 3; ++i) {
            const double dx = v[2 * i] - cx, dy = v[2 * i + 1] - cy;
            ut[2 * i] = cs * dx + sn * dy;
            ut[2 * i + 1] = -sn * dx + cs * dy;
        }
        const double ex = fmax(fmax(ut[0], ut[2]), ut[4]) - fmin(fmin(ut[0], ut[2]), ut[4]);
        const double ey = fmax(fmax(ut[1], ut[3]), ut[5]) - fmin(fmin(ut[1], ut[3]), ut[5]);
        const double H = 0.5 * eta * fmax(ex, ey);
        double area;
        if (mask == 0) area = 4.0 * H * H;
        else if (mask == 2) area = M_PI * H * H;
        else area = clipped_triangle_area(ut, H);
        const int64_t a = off[c], b = off[c + 1];
        int64_t qin = 0;
        for (int64_t j = a; j < b; ++j) {
            const double dx = x[j] - cx, dy = y[j] - cy;
            const double ux = cs * dx + sn * dy, uy = -sn * dx + cs * dy;
            xb[j] = ux * M_PI / H;
            yb[j] = uy * M_PI / H;
            inside[j] = (uint8_t)in_mask(mask, ux, uy, H, ut);
            qin += inside[j];
            wb[j] = 0.0;
            if (counts) counts[j] = 0;
        }
        if (weights == 0) {
            for (int64_t j = a; j < b; ++j) wb[j] = inside[j] ? 1.0 / (double)qin : 0.0;
        } else if (qin > 0) {
            /* raster cell centres over the square [-H, H]^2, nearest inside sample */
            int64_t *n = (int64_t *)calloc((size_t)(b - a), sizeof(int64_t));
            int64_t ng = 0;
            const double step = 2.0 * H / raster;
            for (int ib = 0; ib < raster; ++ib) {
                const double gy = -H + step * (ib + 0.5);
                for (int ia = 0; ia < raster; ++ia) {
                    const double gx = -H + step * (ia + 0.5);
                    if (!in_mask(mask, gx, gy, H, ut)) continue;
                    ++ng;
                    int64_t arg = -1;
                    double bd = 0.0;
                    for (int64_t j = a; j < b; ++j) {
                        if (!inside[j]) continue;
                        const double dx = x[j] - cx, dy = y[j] - cy;
                        const double ux = cs * dx + sn * dy, uy = -sn * dx + cs * dy;
                        const double d = (ux - gx) * (ux - gx) + (uy - gy) * (uy - gy);
                        if (arg < 0 || d < bd) { bd = d; arg = j; }
                    }
                    n[arg - a] += 1;
                }
            }
            double tot = 0.0;
            for (int64_t j = a; j < b; ++j) {
                if (!inside[j]) continue;
                const double A = ng > 0 ? area * (n[j - a] > 0 ? (double)n[j - a] : floor_frac) / (double)ng : 0.0;
                wb[j] = A;
                tot += A;
                if (counts) counts[j] = (int32_t)n[j - a];
            }
            for (int64_t j = a; j < b; ++j) wb[j] = tot > 0.0 ? wb[j] / tot : 0.0;
            free(n);
        }
        /* wb now holds w_q / |D|; deplaning by the weighted mean over the mask */
        double hbar = 0.0;
        for (int64_t j = a; j < b; ++j) hbar += wb[j] * h[j];
        for (int64_t j = a; j < b; ++j) hb[j] = deplane ? h[j] - hbar : h[j];
        double *ci = info + 8 * c;
        ci[0] = cx; ci[1] = cy; ci[2] = cs; ci[3] = sn; ci[4] = H; ci[5] = area; ci[6] = (double)qin;
        ci[7] = deplane ? hbar : 0.0;
    }
    return 0;
}
