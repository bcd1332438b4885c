/*
 * oracle.c -- reference solver for staggered-grid leapfrog wave propagation
 * with reduced-precision storage and compensated updates.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can check the GPU library against a slow,
 * plain implementation written directly from the paper.  It shares no code
 * with the GPU library.
 *
 * What it computes (Gao & Harms, "Half precision wave simulation"):
 *   - 2D acoustic system, Eq. (1) of Sec. 3, with the + signs as printed,
 *     discretised on a staggered grid with the 4th-order staggered stencil
 *     [1/24, -9/8, 9/8, -1/24] of Sec. 3 (or its 2nd-order [-1, 1] form),
 *     periodic wrap in both directions, 2nd-order staggered leapfrog in time.
 *   - The per-step procedure of Alg. 1 (plain update) and Alg. 2
 *     (compensated update): all vx points, then all vy points, then all p
 *     points; at each point stencil -> scale by the material -> update.
 *   - The two compensated sums of Sec. 4: the 3-operation form (Code 1,
 *     Fast2Sum) and the 6-operation form (Code 2, TwoSum).
 *   - The 3D velocity-stress elastic system, the 3D extension of Eq. (A1)
 *     of App. A, on the standard staggered (Virieux) layout.
 *   - The 2D velocity-stress elastic system of Eq. (A1), App. A, periodic
 *     in x and bounded in y by free surfaces, with the point source on the
 *     vertical velocity (the s^{vy} term) and receivers.
 *   - The discrete energy of the staggered leapfrog scheme (Sec. 3 uses it
 *     as the diagnosis tool but defers its formula; the form used here is
 *     derived from the scheme and conserved exactly in exact arithmetic).
 *
 * Precision emulation: every arithmetic operation is evaluated in double
 * and then rounded to the precision it is specified in ("stencil" format
 * for derivative/scaling arithmetic, "storage" format for the update).  An
 * op on two p-bit numbers evaluated in double (53 bits >= 2p+2 for p <= 24)
 * and then rounded to p bits equals the correctly rounded p-bit op, so this
 * reproduces IEEE arithmetic in fp32, fp16 and bf16 (Table 1 lists the
 * formats; bf16 has 8 significand bits and the fp32 exponent range).  With
 * the storage and stencil formats set to fp64 nothing is rounded and the
 * solver is the plain FP64 reference.
 *
 * Readings of the paper that are not fixed by its text (they are the ones
 * the GPU library implements as well):
 *   - Grid: p[j][i] at (i, j), vx[j][i] at (i+1/2, j), vy[j][i] at (i, j+1/2);
 *     arrays row-major [ny][nx], x fastest.  State at the top of a step is
 *     (v^{n-1/2}, p^n).
 *   - dt and dx are folded into the stencil weights w_k = fp32(c_k*(dt/dx)).
 *   - Material enters as b = fp32(1/rho) and kappa = fp32(kappa) at p points
 *     (kappa = 1/beta); staggered buoyancy is the mean of the two adjacent b.
 *     Scaling multiplies by b instead of dividing by rho.
 *   - Compensation is added after scaling: y = RN_T(inc + c), then the
 *     compensated sum of (v, y) gives the new (v, c).
 *   - The stencil is evaluated in fp32 from the stored values.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Loops over fewer cells than this run on one thread: a parallel region
 * costs more than the work, and many oracle processes side by side would
 * otherwise contend for the cores at every step.  Every loop computes each
 * cell (or row partial) on its own, so the thread count never changes a
 * result. */
#define PAR_MIN (1L << 15)

enum { FMT_F64 = 0, FMT_F32 = 1, FMT_F16 = 2, FMT_BF16 = 3 };
enum { COMP_NONE = 0, COMP_FAST2SUM = 1, COMP_TWOSUM = 2, COMP_TWOSUM8 = 3 };

/* ------------------------------------------------------------------------ */
/* Rounding to a binary floating-point format (Sec. 2, Table 1).            */
/* ------------------------------------------------------------------------ */

/* Round x to the nearest number with `prec` significand bits (hidden bit
 * included), smallest normal exponent `emin` (subnormals are kept: below
 * 2^emin the spacing stays 2^(emin-prec+1)) and largest finite value
 * `maxfin`; ties go to the even neighbour, magnitudes that round beyond
 * maxfin become infinity. */
static double round_to_format(double x, int prec, int emin, double maxfin)
{
    if (x == 0.0 || isnan(x) || isinf(x))
        return x;
    int e;
    frexp(x, &e);               /* x = m * 2^e with 0.5 <= |m| < 1 */
    int lead = e - 1;           /* exponent of the leading bit */
    if (lead < emin)
        lead = emin;
    double quantum = ldexp(1.0, lead - prec + 1);
    double r = nearbyint(x / quantum) * quantum; /* x/quantum is exact */
    if (fabs(r) > maxfin)
        r = copysign(INFINITY, x);
    return r;
}

double orc_round(double x, int fmt)
{
    switch (fmt) {
    case FMT_F32:
        return round_to_format(x, 24, -126, 0x1.fffffep127);
    case FMT_F16:
        return round_to_format(x, 11, -14, 65504.0);
    case FMT_BF16:
        return round_to_format(x, 8, -126, 0x1.fep127);
    default:
        return x;
    }
}

void orc_round_array(const double *x, double *y, long n, int fmt)
{
    for (long i = 0; i < n; ++i)
        y[i] = orc_round(x[i], fmt);
}

/* ------------------------------------------------------------------------ */
/* Compensated sums (Sec. 4, Code 1 and Code 2), in format fmt.             */
/* ------------------------------------------------------------------------ */

/* 3-operation form (Code 1; Dekker's Fast2Sum): the sum s and the part t
 * of b lost in forming it.  Error free when |a| >= |b|. */
void orc_fast2sum(double a, double b, int fmt, double *s, double *t)
{
    double ss = orc_round(a + b, fmt);
    double z = orc_round(ss - a, fmt);
    *t = orc_round(b - z, fmt);
    *s = ss;
}

/* 6-operation form (Code 2; the TwoSum of Knuth and Moller): error free
 * for any ordering of |a| and |b|. */
void orc_twosum(double a, double b, int fmt, double *s, double *t)
{
    double ss = orc_round(a + b, fmt);
    double pa = orc_round(ss - b, fmt);
    double pb = orc_round(ss - pa, fmt);
    double da = orc_round(a - pa, fmt);
    double db = orc_round(b - pb, fmt);
    *t = orc_round(da + db, fmt);
    *s = ss;
}

/* Spacing of the values of format fmt in the binade of s (for zero and
 * subnormal s, the subnormal spacing). */
static double ulp_of(double s, int fmt)
{
    int prec, emin;
    switch (fmt) {
    case FMT_F16: prec = 11; emin = -14; break;
    case FMT_BF16: prec = 8; emin = -126; break;
    case FMT_F32: prec = 24; emin = -126; break;
    default: prec = 53; emin = -1022; break;
    }
    int lead = emin;
    if (s != 0.0 && isfinite(s)) {
        int e;
        frexp(fabs(s), &e);          /* |s| = m 2^e, m in [1/2, 1) */
        if (e - 1 > emin)
            lead = e - 1;
    }
    return ldexp(1.0, lead - prec + 1);
}

/* The compensation term of a sum s held in 8 bits (the compensated sum
 * with a narrow compensation word): t, whose magnitude is at most half the
 * spacing of s's binade, is stored as the integer q = round(t / ulp(s) *
 * 2^7) (ties to even, |q| <= 64) and read back as q * ulp(s) / 2^7; a
 * zero word reads back as +0.  Returns the value read back (0 when s or t
 * is not finite). */
double orc_quantize_comp(double t, double s, int fmt)
{
    if (!isfinite(s) || !isfinite(t))
        return 0.0;
    double u = ulp_of(s, fmt);
    double q = nearbyint(ldexp(t / u, 7));
    if (q == 0.0)
        q = 0.0;                     /* the word is an integer: no -0 */
    return ldexp(q * u, -7);
}

/* Whether the pair (s, t) holds exactly the sum x + y.  Two exact sums of
 * doubles are equal iff their canonical double-double forms (fp64 TwoSum:
 * the rounded sum and the exact remainder) are equal; exact for all the
 * formats here because their values are multiples of 2^-149. */
static int sum_is_exact(double x, double y, double s, double t)
{
    double h1, l1, h2, l2;
    orc_twosum(x, y, FMT_F64, &h1, &l1);
    orc_twosum(s, t, FMT_F64, &h2, &l2);
    return h1 == h2 && l1 == l2;
}

/* Value of a 16-bit pattern: fp16 (1 sign, 5 exponent and 10 fraction
 * bits, exponent bias 15, subnormals below 2^-14) or bf16 (the upper half
 * of an fp32 pattern: 1 sign, 8 exponent, 7 fraction bits, bias 127).
 * *finite is 0 for infinities and NaNs. */
static double decode16(unsigned bits, int fmt, int *finite)
{
    const int sign = (bits >> 15) & 1;
    int ebits, fbits, bias;
    if (fmt == FMT_F16) {
        ebits = 5; fbits = 10; bias = 15;
    } else {
        ebits = 8; fbits = 7; bias = 127;
    }
    const unsigned e = (bits >> fbits) & ((1u << ebits) - 1);
    const unsigned f = bits & ((1u << fbits) - 1);
    *finite = e != (1u << ebits) - 1;
    double v;
    if (e == 0)
        v = ldexp((double)f, 1 - bias - fbits);           /* zero, subnormal */
    else
        v = ldexp((double)(f | (1u << fbits)), (int)e - bias - fbits);
    return sign ? -v : v;
}

/* Exhaustive exactness of the two compensated sums (Sec. 4) in a 16-bit
 * format (fp16 or bf16): every pair (a, b) of finite values, a's bit
 * pattern in [a_lo, a_hi), b over all 2^16 patterns.  counts (8 entries):
 *   [0] pairs checked
 *   [1] pairs where the 6-operation sum is not error free
 *   [2] pairs where an operation of the 6-operation sum overflows (s or t
 *       not finite; there is then no finite split)
 *   [3] ordered pairs (|a| >= |b|), the condition of the 3-operation sum
 *   [4] ordered pairs where the 3-operation sum is not error free
 *   [5] ordered pairs where the 3-operation sum overflows
 *   [6] unordered pairs (|a| < |b|) where the 3-operation sum is finite
 *       and not error free
 *   [7] pairs where the rounded sum a + b itself overflows */
void orc_eft_exhaustive(int fmt, long a_lo, long a_hi, long *counts)
{
    long c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0, c6 = 0, c7 = 0;
#pragma omp parallel for schedule(dynamic, 16) \
    reduction(+ : c0, c1, c2, c3, c4, c5, c6, c7)
    for (long ia = a_lo; ia < a_hi; ++ia) {
        int fa;
        const double x = decode16((unsigned)ia, fmt, &fa);
        if (!fa)
            continue;
        for (unsigned ib = 0; ib < 65536u; ++ib) {
            int fb;
            const double y = decode16(ib, fmt, &fb);
            if (!fb)
                continue;
            ++c0;
            if (!isfinite(orc_round(x + y, fmt)))
                ++c7;
            double s, t;
            orc_twosum(x, y, fmt, &s, &t);
            if (!isfinite(s) || !isfinite(t))
                ++c2;
            else if (!sum_is_exact(x, y, s, t))
                ++c1;
            orc_fast2sum(x, y, fmt, &s, &t);
            const int finite = isfinite(s) && isfinite(t);
            if (fabs(x) >= fabs(y)) {
                ++c3;
                if (!finite)
                    ++c5;
                else if (!sum_is_exact(x, y, s, t))
                    ++c4;
            } else if (finite && !sum_is_exact(x, y, s, t)) {
                ++c6;
            }
        }
    }
    counts[0] = c0; counts[1] = c1; counts[2] = c2; counts[3] = c3;
    counts[4] = c4; counts[5] = c5; counts[6] = c6; counts[7] = c7;
}

/* Exactness check used by the tests: counts pairs (a[i], b[j]) with
 * a + b != s + t.  Equality of two exact sums of doubles is decided by
 * comparing their canonical double-double forms (fp64 TwoSum yields the
 * rounded sum and the exact remainder), which is exact for all the formats
 * here because their values are multiples of 2^-149.  Pairs for which one
 * of the operations overflows (s or t not finite) are skipped: near the top
 * of the range s - b may round to infinity.  If require_order is set, only
 * pairs with |a| >= |b| are checked. */
long orc_eft_check(int fmt, int which, const double *a, long na,
                   const double *b, long nb, int require_order)
{
    long bad = 0;
    for (long i = 0; i < na; ++i) {
        for (long j = 0; j < nb; ++j) {
            double x = a[i], y = b[j];
            if (require_order && fabs(x) < fabs(y))
                continue;
            double s, t;
            if (which == 3)
                orc_fast2sum(x, y, fmt, &s, &t);
            else
                orc_twosum(x, y, fmt, &s, &t);
            if (!isfinite(s) || !isfinite(t))
                continue;   /* an operation overflowed: no finite split */
            if (!sum_is_exact(x, y, s, t))
                ++bad;
        }
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Shared pieces of the solvers.                                            */
/* ------------------------------------------------------------------------ */

static long wrap(long i, long n)
{
    return ((i % n) + n) % n;
}

typedef struct {
    int sf;    /* format of stencil and scaling arithmetic */
    int tf;    /* storage format of fields and compensation terms */
    int comp;  /* COMP_NONE / COMP_FAST2SUM / COMP_TWOSUM */
} arith;

/* Solution update of Alg. 1 (plain, V += R with R held in the storage
 * format) and Alg. 2 (compensated, R carries the bits lost last time). */
static void update(const arith *A, double *v, double *c, double inc)
{
    if (A->comp == COMP_NONE) {
        double r = orc_round(inc, A->tf);
        *v = orc_round(*v + r, A->tf);
        return;
    }
    double y = orc_round(orc_round(inc + *c, A->sf), A->tf);
    double s, t;
    if (A->comp == COMP_FAST2SUM)
        orc_fast2sum(*v, y, A->tf, &s, &t);
    else
        orc_twosum(*v, y, A->tf, &s, &t);
    *v = s;
    /* 8-bit compensation word: keep the part of t that 7 bits below s's
     * last place hold */
    *c = A->comp == COMP_TWOSUM8 ? orc_quantize_comp(t, s, A->tf) : t;
}

/* Neumaier's compensated summation in fp64, used for the energy. */
typedef struct { double s, c; } nsum;

static void nsum_add(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double f32v(double x) { return orc_round(x, FMT_F32); }

/* Stencil coefficients of the staggered first derivative (Sec. 3): order 4
 * uses 9/8 and -1/24 (Levander), order 2 uses 1. */
static void weights(int order, double dt, double dx, double *w1, double *w2)
{
    double r = dt / dx;
    if (order == 4) {
        *w1 = f32v((9.0 / 8.0) * r);
        *w2 = f32v((-1.0 / 24.0) * r);
    } else {
        *w1 = f32v(1.0 * r);
        *w2 = 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* 2D acoustic.                                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    long nx, ny;
    int order;
    double w1, w2;
    double *b, *k;   /* fp32-valued buoyancy 1/rho and modulus kappa */
} ac2d;

#define IX(j, i) (wrap((j), G->ny) * G->nx + wrap((i), G->nx))

/* Coefficients of the step in the stencil format sf: the fp32 values,
 * rounded once more when the stencil runs in a format narrower than fp32
 * (the all-fp16 / all-bf16 step of Alg. 1 taken literally: weights and
 * material are then values of that format as well). */
static double narrow(double x, int sf)
{
    return (sf == FMT_F16 || sf == FMT_BF16) ? orc_round(x, sf) : x;
}

static void ac2d_setup(ac2d *G, long nx, long ny, int order, double dx,
                       double dt, const double *rho, const double *kappa,
                       int sf)
{
    G->nx = nx;
    G->ny = ny;
    G->order = order;
    weights(order, dt, dx, &G->w1, &G->w2);
    G->w1 = narrow(G->w1, sf);
    G->w2 = narrow(G->w2, sf);
    long n = nx * ny;
    G->b = malloc(sizeof(double) * n);
    G->k = malloc(sizeof(double) * n);
#pragma omp parallel for schedule(static) if (n >= PAR_MIN)
    for (long i = 0; i < n; ++i) {
        G->b[i] = narrow(f32v(1.0 / rho[i]), sf);
        G->k[i] = narrow(f32v(kappa[i]), sf);
    }
}

static void ac2d_free(ac2d *G)
{
    free(G->b);
    free(G->k);
}

/* One leapfrog step: v^{n-1/2} -> v^{n+1/2} from p^n, then p^n -> p^{n+1}
 * from v^{n+1/2}.  In place, as in Alg. 1/2: the velocity loops read only
 * p, and the pressure loop reads only the new velocities and p itself. */
static void ac2d_step(const ac2d *G, const arith *A, double *vx, double *vy,
                      double *p, double *cvx, double *cvy, double *cp,
                      long src_q, double src_val)
{
    const int sf = A->sf;
    const long nx = G->nx, ny = G->ny;
    const double w1 = G->w1, w2 = G->w2;
#define S(x) orc_round((x), sf)

    /* vx at (i+1/2, j): dp/dx */
#pragma omp parallel for schedule(static) if (nx * ny >= PAR_MIN)
    for (long j = 0; j < ny; ++j)
        for (long i = 0; i < nx; ++i) {
            double a0 = S(p[IX(j, i + 1)] - p[IX(j, i)]);
            double g;
            if (G->order == 4) {
                double a1 = S(p[IX(j, i + 2)] - p[IX(j, i - 1)]);
                g = S(S(w1 * a0) + S(w2 * a1));
            } else {
                g = S(w1 * a0);
            }
            double bx = S(0.5 * S(G->b[IX(j, i)] + G->b[IX(j, i + 1)]));
            double inc = S(bx * g);
            long q = j * nx + i;
            update(A, &vx[q], cvx ? &cvx[q] : NULL, inc);
        }

    /* vy at (i, j+1/2): dp/dy */
#pragma omp parallel for schedule(static) if (nx * ny >= PAR_MIN)
    for (long j = 0; j < ny; ++j)
        for (long i = 0; i < nx; ++i) {
            double a0 = S(p[IX(j + 1, i)] - p[IX(j, i)]);
            double g;
            if (G->order == 4) {
                double a1 = S(p[IX(j + 2, i)] - p[IX(j - 1, i)]);
                g = S(S(w1 * a0) + S(w2 * a1));
            } else {
                g = S(w1 * a0);
            }
            double by = S(0.5 * S(G->b[IX(j, i)] + G->b[IX(j + 1, i)]));
            double inc = S(by * g);
            long q = j * nx + i;
            update(A, &vy[q], cvy ? &cvy[q] : NULL, inc);
        }

    /* p at (i, j): dvx/dx + dvy/dy */
#pragma omp parallel for schedule(static) if (nx * ny >= PAR_MIN)
    for (long j = 0; j < ny; ++j)
        for (long i = 0; i < nx; ++i) {
            double ax0 = S(vx[IX(j, i)] - vx[IX(j, i - 1)]);
            double ay0 = S(vy[IX(j, i)] - vy[IX(j - 1, i)]);
            double gx, gy;
            if (G->order == 4) {
                double ax1 = S(vx[IX(j, i + 1)] - vx[IX(j, i - 2)]);
                double ay1 = S(vy[IX(j + 1, i)] - vy[IX(j - 2, i)]);
                gx = S(S(w1 * ax0) + S(w2 * ax1));
                gy = S(S(w1 * ay0) + S(w2 * ay1));
            } else {
                gx = S(w1 * ax0);
                gy = S(w1 * ay0);
            }
            double d = S(gx + gy);
            long q = j * nx + i;
            /* point source (Eq. 1, s_p): the sample joins the right-hand
             * side before the division by beta, as in the source line of
             * Alg. 1/2; it is held in the stencil format */
            if (q == src_q)
                d = S(d + S(src_val));
            double inc = S(G->k[q] * d);
            update(A, &p[q], cp ? &cp[q] : NULL, inc);
        }
#undef S
}

/* Discrete energy of the state (v^{n-1/2}, p^n), in fp64:
 *   E^n = dx*dy/2 * sum[ p^2/kappa + vx^- vx^+ / bx + vy^- vy^+ / by ],
 * where v^+ = v^{n+1/2} is recomputed exactly in fp64 from the state.  Per
 * point the terms are formed in the order written; the sum over points is
 * compensated. */
static double ac2d_energy(const ac2d *G, double dx, const double *vx,
                          const double *vy, const double *p)
{
    const long nx = G->nx, ny = G->ny;
    const double w1 = G->w1, w2 = G->w2;
    double *rows = malloc(sizeof(double) * 2 * ny);
#pragma omp parallel for schedule(static) if (nx * ny >= PAR_MIN)
    for (long j = 0; j < ny; ++j) {
        nsum acc = {0.0, 0.0};
        for (long i = 0; i < nx; ++i) {
            long q = j * nx + i;
            double gx = w1 * (p[IX(j, i + 1)] - p[IX(j, i)]);
            double gy = w1 * (p[IX(j + 1, i)] - p[IX(j, i)]);
            if (G->order == 4) {
                gx = gx + w2 * (p[IX(j, i + 2)] - p[IX(j, i - 1)]);
                gy = gy + w2 * (p[IX(j + 2, i)] - p[IX(j - 1, i)]);
            }
            double bx = 0.5 * (G->b[q] + G->b[IX(j, i + 1)]);
            double by = 0.5 * (G->b[q] + G->b[IX(j + 1, i)]);
            double vxp = vx[q] + bx * gx;
            double vyp = vy[q] + by * gy;
            double e = (p[q] * p[q]) / G->k[q] + (vx[q] * vxp) / bx;
            e = e + (vy[q] * vyp) / by;
            nsum_add(&acc, e);
        }
        rows[2 * j] = acc.s;
        rows[2 * j + 1] = acc.c;
    }
    nsum tot = {0.0, 0.0};
    for (long j = 0; j < ny; ++j) {
        nsum_add(&tot, rows[2 * j]);
        nsum_add(&tot, rows[2 * j + 1]);
    }
    free(rows);
    return 0.5 * dx * dx * (tot.s + tot.c);
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Run nsteps leapfrog steps of the 2D acoustic system in place.
 * Fields vx, vy, p (and the compensation arrays, which may be NULL when
 * comp == COMP_NONE) hold values of the storage format on entry.  If
 * energy_every > 0, energy[m] receives E at step m*energy_every for
 * m = 0 .. nsteps/energy_every.
 * Point source: if nsrc > 0, step n (n = 0 .. nsteps-1, counted from this
 * call) adds src[n] (for n < nsrc) to the pressure right-hand side at cell
 * (src_x, src_y).  Receivers: if nrec > 0, after step n the values p^{n+1},
 * vx^{n+1/2}, vy^{n+1/2} at cell (rec_x[r], rec_y[r]) are written to
 * rec_out[(n*nrec + r)*3 + 0, 1, 2].  Returns 0, or -1 on bad arguments. */
int orc_acoustic2d(long nx, long ny, int order, double dx, double dt,
                   const double *rho, const double *kappa, double *vx,
                   double *vy, double *p, double *cvx, double *cvy,
                   double *cp, int storage, int stencil, int comp,
                   long nsteps, long energy_every, double *energy,
                   int nthreads, long src_x, long src_y, const double *src,
                   long nsrc, long nrec, const long *rec_x,
                   const long *rec_y, double *rec_out)
{
    if (nx < 1 || ny < 1 || (order != 2 && order != 4) || nsteps < 0)
        return -1;
    if (comp != COMP_NONE && (!cvx || !cvy || !cp))
        return -1;
    if (nsrc > 0 && (!src || src_x < 0 || src_x >= nx || src_y < 0 ||
                     src_y >= ny))
        return -1;
    if (nrec > 0 && (!rec_x || !rec_y || !rec_out))
        return -1;
    for (long r = 0; r < nrec; ++r)
        if (rec_x[r] < 0 || rec_x[r] >= nx || rec_y[r] < 0 || rec_y[r] >= ny)
            return -1;
    set_threads(nthreads);
    ac2d G, GE;   /* the step's coefficients; the energy's (fp32 values) */
    ac2d_setup(&G, nx, ny, order, dx, dt, rho, kappa, stencil);
    if (energy_every > 0)
        ac2d_setup(&GE, nx, ny, order, dx, dt, rho, kappa, FMT_F32);
    arith A = {stencil, storage, comp};
    long m = 0;
    if (energy_every > 0)
        energy[m++] = ac2d_energy(&GE, dx, vx, vy, p);
    for (long n = 1; n <= nsteps; ++n) {
        const long src_q = n - 1 < nsrc ? src_y * nx + src_x : -1;
        ac2d_step(&G, &A, vx, vy, p, cvx, cvy, cp, src_q,
                  src_q >= 0 ? src[n - 1] : 0.0);
        for (long r = 0; r < nrec; ++r) {
            const long q = rec_y[r] * nx + rec_x[r];
            double *o = rec_out + ((n - 1) * nrec + r) * 3;
            o[0] = p[q];
            o[1] = vx[q];
            o[2] = vy[q];
        }
        if (energy_every > 0 && n % energy_every == 0)
            energy[m++] = ac2d_energy(&GE, dx, vx, vy, p);
    }
    ac2d_free(&G);
    if (energy_every > 0)
        ac2d_free(&GE);
    return 0;
}

double orc_acoustic2d_energy(long nx, long ny, int order, double dx,
                             double dt, const double *rho,
                             const double *kappa, const double *vx,
                             const double *vy, const double *p)
{
    ac2d G;
    ac2d_setup(&G, nx, ny, order, dx, dt, rho, kappa, FMT_F32);
    double e = ac2d_energy(&G, dx, vx, vy, p);
    ac2d_free(&G);
    return e;
}

#undef IX

/* ------------------------------------------------------------------------ */
/* 3D elastic (velocity-stress), 2nd order.                                 */
/*                                                                          */
/* Layout (arrays [nz][ny][nx], x fastest):                                 */
/*   sxx, syy, szz, material      at (i,     j,     k    )                  */
/*   vx at (i+1/2, j, k), vy at (i, j+1/2, k), vz at (i, j, k+1/2)          */
/*   sxy at (i+1/2, j+1/2, k), sxz at (i+1/2, j, k+1/2),                    */
/*   syz at (i, j+1/2, k+1/2)                                               */
/* Field order everywhere: vx, vy, vz, sxx, syy, szz, sxy, sxz, syz.        */
/* ------------------------------------------------------------------------ */

typedef struct {
    long nx, ny, nz;
    double w;
    double *b, *lam, *mu;  /* fp32-valued 1/rho, lambda, mu at cells */
} el3d;

#define IX3(k, j, i)                                                      \
    ((wrap((k), G->nz) * G->ny + wrap((j), G->ny)) * G->nx + wrap((i), G->nx))

static void el3d_setup(el3d *G, long nx, long ny, long nz, double dx,
                       double dt, const double *rho, const double *lam,
                       const double *mu)
{
    G->nx = nx;
    G->ny = ny;
    G->nz = nz;
    G->w = f32v(1.0 * (dt / dx));
    long n = nx * ny * nz;
    G->b = malloc(sizeof(double) * n);
    G->lam = malloc(sizeof(double) * n);
    G->mu = malloc(sizeof(double) * n);
    for (long i = 0; i < n; ++i) {
        G->b[i] = f32v(1.0 / rho[i]);
        G->lam[i] = f32v(lam[i]);
        G->mu[i] = f32v(mu[i]);
    }
}

static void el3d_free(el3d *G)
{
    free(G->b);
    free(G->lam);
    free(G->mu);
}

static void el3d_step(const el3d *G, const arith *A, double *const *f,
                      double *const *c)
{
    const int sf = A->sf;
    const long nx = G->nx, ny = G->ny, nz = G->nz;
    const double w = G->w;
    double *vx = f[0], *vy = f[1], *vz = f[2];
    double *sxx = f[3], *syy = f[4], *szz = f[5];
    double *sxy = f[6], *sxz = f[7], *syz = f[8];
    const double *B = G->b, *L = G->lam, *M = G->mu;
#define S(x) orc_round((x), sf)
#define CP(a, q) ((a) ? &(a)[q] : NULL)

    /* velocities: rho dv/dt = div sigma */
#pragma omp parallel for collapse(2) schedule(static) if (nx * ny * nz >= PAR_MIN)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long q = (k * ny + j) * nx + i;
                {   /* vx at (i+1/2, j, k) */
                    double d1 = S(sxx[IX3(k, j, i + 1)] - sxx[IX3(k, j, i)]);
                    double d2 = S(sxy[IX3(k, j, i)] - sxy[IX3(k, j - 1, i)]);
                    double d3 = S(sxz[IX3(k, j, i)] - sxz[IX3(k - 1, j, i)]);
                    double g = S(w * S(S(d1 + d2) + d3));
                    double bb = S(0.5 * S(B[IX3(k, j, i)] + B[IX3(k, j, i + 1)]));
                    update(A, &vx[q], CP(c[0], q), S(bb * g));
                }
                {   /* vy at (i, j+1/2, k) */
                    double d1 = S(sxy[IX3(k, j, i)] - sxy[IX3(k, j, i - 1)]);
                    double d2 = S(syy[IX3(k, j + 1, i)] - syy[IX3(k, j, i)]);
                    double d3 = S(syz[IX3(k, j, i)] - syz[IX3(k - 1, j, i)]);
                    double g = S(w * S(S(d1 + d2) + d3));
                    double bb = S(0.5 * S(B[IX3(k, j, i)] + B[IX3(k, j + 1, i)]));
                    update(A, &vy[q], CP(c[1], q), S(bb * g));
                }
                {   /* vz at (i, j, k+1/2) */
                    double d1 = S(sxz[IX3(k, j, i)] - sxz[IX3(k, j, i - 1)]);
                    double d2 = S(syz[IX3(k, j, i)] - syz[IX3(k, j - 1, i)]);
                    double d3 = S(szz[IX3(k + 1, j, i)] - szz[IX3(k, j, i)]);
                    double g = S(w * S(S(d1 + d2) + d3));
                    double bb = S(0.5 * S(B[IX3(k, j, i)] + B[IX3(k + 1, j, i)]));
                    update(A, &vz[q], CP(c[2], q), S(bb * g));
                }
            }

    /* stresses: dsigma/dt = lambda tr(e) I + 2 mu e, e the strain rate */
#pragma omp parallel for collapse(2) schedule(static) if (nx * ny * nz >= PAR_MIN)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long q = (k * ny + j) * nx + i;
                double ex = S(w * S(vx[IX3(k, j, i)] - vx[IX3(k, j, i - 1)]));
                double ey = S(w * S(vy[IX3(k, j, i)] - vy[IX3(k, j - 1, i)]));
                double ez = S(w * S(vz[IX3(k, j, i)] - vz[IX3(k - 1, j, i)]));
                double lam = L[q];
                double l2m = S(lam + S(2.0 * M[q]));
                update(A, &sxx[q], CP(c[3], q),
                       S(S(l2m * ex) + S(lam * S(ey + ez))));
                update(A, &syy[q], CP(c[4], q),
                       S(S(l2m * ey) + S(lam * S(ex + ez))));
                update(A, &szz[q], CP(c[5], q),
                       S(S(l2m * ez) + S(lam * S(ex + ey))));
                {   /* sxy at (i+1/2, j+1/2, k) */
                    double a = S(vy[IX3(k, j, i + 1)] - vy[IX3(k, j, i)]);
                    double bq = S(vx[IX3(k, j + 1, i)] - vx[IX3(k, j, i)]);
                    double g = S(w * S(a + bq));
                    double m = S(0.25 * S(S(M[IX3(k, j, i)] + M[IX3(k, j, i + 1)]) +
                                          S(M[IX3(k, j + 1, i)] + M[IX3(k, j + 1, i + 1)])));
                    update(A, &sxy[q], CP(c[6], q), S(m * g));
                }
                {   /* sxz at (i+1/2, j, k+1/2) */
                    double a = S(vz[IX3(k, j, i + 1)] - vz[IX3(k, j, i)]);
                    double bq = S(vx[IX3(k + 1, j, i)] - vx[IX3(k, j, i)]);
                    double g = S(w * S(a + bq));
                    double m = S(0.25 * S(S(M[IX3(k, j, i)] + M[IX3(k, j, i + 1)]) +
                                          S(M[IX3(k + 1, j, i)] + M[IX3(k + 1, j, i + 1)])));
                    update(A, &sxz[q], CP(c[7], q), S(m * g));
                }
                {   /* syz at (i, j+1/2, k+1/2) */
                    double a = S(vz[IX3(k, j + 1, i)] - vz[IX3(k, j, i)]);
                    double bq = S(vy[IX3(k + 1, j, i)] - vy[IX3(k, j, i)]);
                    double g = S(w * S(a + bq));
                    double m = S(0.25 * S(S(M[IX3(k, j, i)] + M[IX3(k, j + 1, i)]) +
                                          S(M[IX3(k + 1, j, i)] + M[IX3(k + 1, j + 1, i)])));
                    update(A, &syz[q], CP(c[8], q), S(m * g));
                }
            }
#undef CP
#undef S
}

/* Discrete energy of the elastic state (v^{n-1/2}, sigma^n), fp64:
 *   E^n = dx^3/2 * sum[ v^- . v^+ / b  +  s_n^T C^{-1} s_n  +  s_ij^2 / mu_ij ]
 * with C = lambda 1 1^T + 2 mu I on the normal stresses, so
 *   s_n^T C^{-1} s_n = (|s_n|^2 - lambda/(3 lambda + 2 mu) (tr s)^2) / (2 mu). */
static double el3d_energy(const el3d *G, double dx, double *const *f)
{
    const long nx = G->nx, ny = G->ny, nz = G->nz;
    const double w = G->w;
    const double *vx = f[0], *vy = f[1], *vz = f[2];
    const double *sxx = f[3], *syy = f[4], *szz = f[5];
    const double *sxy = f[6], *sxz = f[7], *syz = f[8];
    const double *B = G->b, *L = G->lam, *M = G->mu;
    long nrows = ny * nz;
    double *rows = malloc(sizeof(double) * 2 * nrows);
#pragma omp parallel for schedule(static) if (nrows * nx >= PAR_MIN)
    for (long r = 0; r < nrows; ++r) {
        long k = r / ny, j = r % ny;
        nsum acc = {0.0, 0.0};
        for (long i = 0; i < nx; ++i) {
            long q = (k * ny + j) * nx + i;
            double gx = w * ((sxx[IX3(k, j, i + 1)] - sxx[IX3(k, j, i)]) +
                             (sxy[q] - sxy[IX3(k, j - 1, i)]) +
                             (sxz[q] - sxz[IX3(k - 1, j, i)]));
            double gy = w * ((sxy[q] - sxy[IX3(k, j, i - 1)]) +
                             (syy[IX3(k, j + 1, i)] - syy[q]) +
                             (syz[q] - syz[IX3(k - 1, j, i)]));
            double gz = w * ((sxz[q] - sxz[IX3(k, j, i - 1)]) +
                             (syz[q] - syz[IX3(k, j - 1, i)]) +
                             (szz[IX3(k + 1, j, i)] - szz[q]));
            double bx = 0.5 * (B[q] + B[IX3(k, j, i + 1)]);
            double by = 0.5 * (B[q] + B[IX3(k, j + 1, i)]);
            double bz = 0.5 * (B[q] + B[IX3(k + 1, j, i)]);
            double vxp = vx[q] + bx * gx;
            double vyp = vy[q] + by * gy;
            double vzp = vz[q] + bz * gz;
            double ev = (vx[q] * vxp) / bx + (vy[q] * vyp) / by;
            ev = ev + (vz[q] * vzp) / bz;
            double lam = L[q], mu = M[q];
            double tr = (sxx[q] + syy[q]) + szz[q];
            double sq = (sxx[q] * sxx[q] + syy[q] * syy[q]) + szz[q] * szz[q];
            double en = (sq - (lam / (3.0 * lam + 2.0 * mu)) * (tr * tr)) /
                        (2.0 * mu);
            double mxy = 0.25 * ((M[q] + M[IX3(k, j, i + 1)]) +
                                 (M[IX3(k, j + 1, i)] + M[IX3(k, j + 1, i + 1)]));
            double mxz = 0.25 * ((M[q] + M[IX3(k, j, i + 1)]) +
                                 (M[IX3(k + 1, j, i)] + M[IX3(k + 1, j, i + 1)]));
            double myz = 0.25 * ((M[q] + M[IX3(k, j + 1, i)]) +
                                 (M[IX3(k + 1, j, i)] + M[IX3(k + 1, j + 1, i)]));
            double es = (sxy[q] * sxy[q]) / mxy + (sxz[q] * sxz[q]) / mxz;
            es = es + (syz[q] * syz[q]) / myz;
            nsum_add(&acc, (ev + en) + es);
        }
        rows[2 * r] = acc.s;
        rows[2 * r + 1] = acc.c;
    }
    nsum tot = {0.0, 0.0};
    for (long r = 0; r < nrows; ++r) {
        nsum_add(&tot, rows[2 * r]);
        nsum_add(&tot, rows[2 * r + 1]);
    }
    free(rows);
    return 0.5 * dx * dx * dx * (tot.s + tot.c);
}

/* Run nsteps of the 3D elastic system in place.  fields[9] and comps[9]
 * (comps may be NULL when comp == COMP_NONE) are [nz][ny][nx] arrays in the
 * field order above; material is rho, lambda, mu at cell centres. */
int orc_elastic3d(long nx, long ny, long nz, double dx, double dt,
                  const double *rho, const double *lam, const double *mu,
                  double *const *fields, double *const *comps, int storage,
                  int stencil, int comp, long nsteps, long energy_every,
                  double *energy, int nthreads)
{
    if (nx < 1 || ny < 1 || nz < 1 || nsteps < 0)
        return -1;
    double *none[9] = {0};
    if (comp != COMP_NONE) {
        if (!comps)
            return -1;
        for (int f = 0; f < 9; ++f)
            if (!comps[f])
                return -1;
    } else {
        comps = none;
    }
    set_threads(nthreads);
    el3d G;
    el3d_setup(&G, nx, ny, nz, dx, dt, rho, lam, mu);
    arith A = {stencil, storage, comp};
    long m = 0;
    if (energy_every > 0)
        energy[m++] = el3d_energy(&G, dx, fields);
    for (long n = 1; n <= nsteps; ++n) {
        el3d_step(&G, &A, fields, comps);
        if (energy_every > 0 && n % energy_every == 0)
            energy[m++] = el3d_energy(&G, dx, fields);
    }
    el3d_free(&G);
    return 0;
}

double orc_elastic3d_energy(long nx, long ny, long nz, double dx, double dt,
                            const double *rho, const double *lam,
                            const double *mu, double *const *fields)
{
    el3d G;
    el3d_setup(&G, nx, ny, nz, dx, dt, rho, lam, mu);
    double e = el3d_energy(&G, dx, fields);
    el3d_free(&G);
    return e;
}

#undef IX3

/* ------------------------------------------------------------------------ */
/* 2D elastic (velocity-stress, Eq. A1 of App. A), 2nd order, periodic in x */
/* and bounded in y by two free surfaces.                                   */
/*                                                                          */
/* Layout (arrays [ny][nx], x fastest):                                     */
/*   sxx, syy, material  at (i,     j    ),  j = 0 .. ny-1                  */
/*   vx                  at (i+1/2, j    ),  j = 0 .. ny-1                  */
/*   vy                  at (i,     j+1/2),  j = 0 .. ny-2                  */
/*   sxy                 at (i+1/2, j+1/2),  j = 0 .. ny-2                  */
/* Field order everywhere: vx, vy, sxx, syy, sxy.  Row ny-1 of vy and sxy   */
/* lies outside the body; it is held at zero and never updated.             */
/*                                                                          */
/* The surfaces are the normal-stress rows j = 0 and j = ny-1, where the    */
/* traction vanishes: syy is held at zero, sxy is odd about the surface     */
/* (the value half a cell outside is minus the value half a cell inside),   */
/* and sxx, with the vertical strain rate eliminated through syy = 0,       */
/* changes by the plate modulus 4 mu (lambda + mu) / (lambda + 2 mu) times  */
/* the horizontal strain rate.  With half weights on the two surface rows   */
/* the discrete divergence is minus the adjoint of the discrete gradient,   */
/* so the leapfrog energy below is conserved exactly in exact arithmetic.   */
/* ------------------------------------------------------------------------ */

enum { EL2D_NF = 5 };

typedef struct {
    long nx, ny;
    double w;
    double *b;     /* fp32 1/rho at cells */
    double *l2m;   /* fp32 lambda + 2 mu; the plate modulus on surface rows */
    double *lam;   /* fp32 lambda; 0 on surface rows */
    double *mxy;   /* fp32 mean of the four mu around each sxy point */
} el2d;

#define IX2(j, i) ((j) * G->nx + wrap((i), G->nx))

static void el2d_setup(el2d *G, long nx, long ny, double dx, double dt,
                       const double *rho, const double *lam, const double *mu)
{
    G->nx = nx;
    G->ny = ny;
    G->w = f32v(1.0 * (dt / dx));
    long n = nx * ny;
    G->b = malloc(sizeof(double) * n);
    G->l2m = malloc(sizeof(double) * n);
    G->lam = malloc(sizeof(double) * n);
    G->mxy = malloc(sizeof(double) * n);
    for (long j = 0; j < ny; ++j)
        for (long i = 0; i < nx; ++i) {
            long q = j * nx + i;
            int surface = j == 0 || j == ny - 1;
            G->b[q] = f32v(1.0 / rho[q]);
            if (surface) {
                G->l2m[q] = f32v((4.0 * mu[q] * (lam[q] + mu[q])) /
                                 (lam[q] + 2.0 * mu[q]));
                G->lam[q] = 0.0;
            } else {
                G->l2m[q] = f32v(lam[q] + 2.0 * mu[q]);
                G->lam[q] = f32v(lam[q]);
            }
            G->mxy[q] = j < ny - 1
                ? f32v(0.25 * ((mu[q] + mu[IX2(j, i + 1)]) +
                               (mu[IX2(j + 1, i)] + mu[IX2(j + 1, i + 1)])))
                : 0.0;
        }
}

static void el2d_free(el2d *G)
{
    free(G->b);
    free(G->l2m);
    free(G->lam);
    free(G->mxy);
}

/* sxy just below and just above the vx point (i+1/2, j), the images across
 * the surfaces included. */
static double sxy_lo(const el2d *G, const double *sxy, long j, long i)
{
    return j == 0 ? -sxy[IX2(0, i)] : sxy[IX2(j - 1, i)];
}

static double sxy_hi(const el2d *G, const double *sxy, long j, long i)
{
    return j == G->ny - 1 ? -sxy[IX2(G->ny - 2, i)] : sxy[IX2(j, i)];
}

/* One step: velocities from the old stresses (and the v_y point source),
 * then stresses from the new velocities; in place (the velocity loop reads
 * only stresses, the stress loop only velocities and each cell's own
 * stresses). */
static void el2d_step(const el2d *G, const arith *A, double *const *f,
                      double *const *c, long src_q, double src_val)
{
    const int sf = A->sf;
    const long nx = G->nx, ny = G->ny;
    const double w = G->w;
    double *vx = f[0], *vy = f[1], *sxx = f[2], *syy = f[3], *sxy = f[4];
    const double *B = G->b;
#define S(x) orc_round((x), sf)
#define CP(a, q) ((a) ? &(a)[q] : NULL)

#pragma omp parallel for schedule(static) if (nx * ny >= PAR_MIN)
    for (long j = 0; j < ny; ++j)
        for (long i = 0; i < nx; ++i) {
            long q = j * nx + i;
            {   /* vx at (i+1/2, j) */
                double d1 = S(sxx[IX2(j, i + 1)] - sxx[q]);
                double d2 = S(sxy_hi(G, sxy, j, i) - sxy_lo(G, sxy, j, i));
                double g = S(w * S(d1 + d2));
                double bb = S(0.5 * S(B[q] + B[IX2(j, i + 1)]));
                update(A, &vx[q], CP(c[0], q), S(bb * g));
            }
            if (j < ny - 1) {   /* vy at (i, j+1/2) */
                double d1 = S(sxy[q] - sxy[IX2(j, i - 1)]);
                double d2 = S(syy[IX2(j + 1, i)] - syy[q]);
                double g = S(w * S(d1 + d2));
                double bb = S(0.5 * S(B[q] + B[IX2(j + 1, i)]));
                double inc = S(bb * g);
                /* the s^{vy} source of Eq. A1 acts on the velocity itself,
                 * after the division by rho; the sample is held in the
                 * stencil format */
                if (q == src_q)
                    inc = S(inc + S(src_val));
                update(A, &vy[q], CP(c[1], q), inc);
            }
        }

#pragma omp parallel for schedule(static) if (nx * ny >= PAR_MIN)
    for (long j = 0; j < ny; ++j)
        for (long i = 0; i < nx; ++i) {
            long q = j * nx + i;
            int surface = j == 0 || j == ny - 1;
            double ex = S(w * S(vx[q] - vx[IX2(j, i - 1)]));
            double ey = surface ? 0.0 : S(w * S(vy[q] - vy[IX2(j - 1, i)]));
            double l2m = G->l2m[q], lam = G->lam[q];
            update(A, &sxx[q], CP(c[2], q), S(S(l2m * ex) + S(lam * ey)));
            if (!surface)
                update(A, &syy[q], CP(c[3], q), S(S(l2m * ey) + S(lam * ex)));
            if (j < ny - 1) {   /* sxy at (i+1/2, j+1/2) */
                double a1 = S(vy[IX2(j, i + 1)] - vy[q]);
                double a2 = S(vx[IX2(j + 1, i)] - vx[q]);
                double g = S(w * S(a1 + a2));
                update(A, &sxy[q], CP(c[4], q), S(G->mxy[q] * g));
            }
        }
#undef CP
#undef S
}

/* Discrete energy of the state (v^{n-1/2}, sigma^n), fp64:
 *   E^n = dx^2/2 * sum_i [ sum_j h_j ( vx^- vx^+ / bx + s^T C^{-1} s )
 *                        + sum_{j < ny-1} ( vy^- vy^+ / by + sxy^2 / mu_xy ) ]
 * with h_j = 1/2 on the two surface rows and 1 elsewhere, v^+ recomputed in
 * fp64 from the state (no source term), and C the 2x2 stiffness
 * [[l2m, lam], [lam, l2m]] of the normal stresses, so
 *   s^T C^{-1} s = (l2m (sxx^2 + syy^2) - 2 lam sxx syy) / (l2m^2 - lam^2)
 * (on a surface row lam = 0 and syy = 0, leaving sxx^2 / l2m). */
static double el2d_energy(const el2d *G, double dx, double *const *f)
{
    const long nx = G->nx, ny = G->ny;
    const double w = G->w;
    const double *vx = f[0], *vy = f[1], *sxx = f[2], *syy = f[3], *sxy = f[4];
    const double *B = G->b;
    double *rows = malloc(sizeof(double) * 2 * ny);
#pragma omp parallel for schedule(static) if (nx * ny >= PAR_MIN)
    for (long j = 0; j < ny; ++j) {
        nsum acc = {0.0, 0.0};
        const double h = (j == 0 || j == ny - 1) ? 0.5 : 1.0;
        for (long i = 0; i < nx; ++i) {
            long q = j * nx + i;
            double gx = w * ((sxx[IX2(j, i + 1)] - sxx[q]) +
                             (sxy_hi(G, sxy, j, i) - sxy_lo(G, sxy, j, i)));
            double bx = 0.5 * (B[q] + B[IX2(j, i + 1)]);
            double vxp = vx[q] + bx * gx;
            double l2m = G->l2m[q], lam = G->lam[q];
            double en = (l2m * (sxx[q] * sxx[q] + syy[q] * syy[q]) -
                         2.0 * lam * (sxx[q] * syy[q])) /
                        (l2m * l2m - lam * lam);
            double e = h * ((vx[q] * vxp) / bx + en);
            if (j < ny - 1) {
                double gy = w * ((sxy[q] - sxy[IX2(j, i - 1)]) +
                                 (syy[IX2(j + 1, i)] - syy[q]));
                double by = 0.5 * (B[q] + B[IX2(j + 1, i)]);
                double vyp = vy[q] + by * gy;
                e = e + ((vy[q] * vyp) / by + (sxy[q] * sxy[q]) / G->mxy[q]);
            }
            nsum_add(&acc, e);
        }
        rows[2 * j] = acc.s;
        rows[2 * j + 1] = acc.c;
    }
    nsum tot = {0.0, 0.0};
    for (long j = 0; j < ny; ++j) {
        nsum_add(&tot, rows[2 * j]);
        nsum_add(&tot, rows[2 * j + 1]);
    }
    free(rows);
    return 0.5 * dx * dx * (tot.s + tot.c);
}

/* Run nsteps of the 2D elastic free-surface system in place.  fields[5]
 * and comps[5] (comps may be NULL when comp == COMP_NONE) are [ny][nx]
 * arrays in the order vx, vy, sxx, syy, sxy; material rho, lambda, mu at
 * cells.  Requires ny >= 3, syy zero on both surface rows and vy, sxy zero
 * on row ny-1.  Point source: step n adds src[n] (n < nsrc) to vy at
 * (src_x, src_y + 1/2), src_y <= ny-2.  Receivers: after step n, the five
 * fields at cell (rec_x[r], rec_y[r]) go to rec_out[(n*nrec + r)*5 + f].
 * The stencil format is fp64 or fp32.  Returns 0, or -1 on bad arguments. */
int orc_elastic2d(long nx, long ny, double dx, double dt, const double *rho,
                  const double *lam, const double *mu, double *const *fields,
                  double *const *comps, int storage, int stencil, int comp,
                  long nsteps, long energy_every, double *energy, int nthreads,
                  long src_x, long src_y, const double *src, long nsrc,
                  long nrec, const long *rec_x, const long *rec_y,
                  double *rec_out)
{
    if (nx < 1 || ny < 3 || nsteps < 0 ||
        (stencil != FMT_F64 && stencil != FMT_F32))
        return -1;
    double *none[EL2D_NF] = {0};
    if (comp != COMP_NONE) {
        if (!comps)
            return -1;
        for (int f = 0; f < EL2D_NF; ++f)
            if (!comps[f])
                return -1;
    } else {
        comps = none;
    }
    for (long i = 0; i < nx; ++i)
        if (fields[3][i] != 0.0 || fields[3][(ny - 1) * nx + i] != 0.0 ||
            fields[1][(ny - 1) * nx + i] != 0.0 ||
            fields[4][(ny - 1) * nx + i] != 0.0)
            return -1;
    if (nsrc > 0 && (!src || src_x < 0 || src_x >= nx || src_y < 0 ||
                     src_y > ny - 2))
        return -1;
    if (nrec > 0 && (!rec_x || !rec_y || !rec_out))
        return -1;
    for (long r = 0; r < nrec; ++r)
        if (rec_x[r] < 0 || rec_x[r] >= nx || rec_y[r] < 0 || rec_y[r] >= ny)
            return -1;
    set_threads(nthreads);
    el2d G;
    el2d_setup(&G, nx, ny, dx, dt, rho, lam, mu);
    arith A = {stencil, storage, comp};
    long m = 0;
    if (energy_every > 0)
        energy[m++] = el2d_energy(&G, dx, fields);
    for (long n = 1; n <= nsteps; ++n) {
        const long src_q = n - 1 < nsrc ? src_y * nx + src_x : -1;
        el2d_step(&G, &A, fields, comps, src_q, src_q >= 0 ? src[n - 1] : 0.0);
        for (long r = 0; r < nrec; ++r) {
            const long q = rec_y[r] * nx + rec_x[r];
            for (int f = 0; f < EL2D_NF; ++f)
                rec_out[((n - 1) * nrec + r) * EL2D_NF + f] = fields[f][q];
        }
        if (energy_every > 0 && n % energy_every == 0)
            energy[m++] = el2d_energy(&G, dx, fields);
    }
    el2d_free(&G);
    return 0;
}

double orc_elastic2d_energy(long nx, long ny, double dx, double dt,
                            const double *rho, const double *lam,
                            const double *mu, double *const *fields)
{
    if (nx < 1 || ny < 3)
        return NAN;
    el2d G;
    el2d_setup(&G, nx, ny, dx, dt, rho, lam, mu);
    double e = el2d_energy(&G, dx, fields);
    el2d_free(&G);
    return e;
}

#undef IX2
