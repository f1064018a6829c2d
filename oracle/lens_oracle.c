/*
 * Plain FP64 CPU oracle for the image-plane chi^2 of
 *   Rexroth, Schaefer, Fourestey & Kneib (2019), "High Performance Computing
 *   for gravitational lens modeling: single vs double precision on GPUs and
 *   CPUs", Astronomy and Computing (arXiv:1902.03252).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  It shares no code,
 * header, table or constant with the GPU library; only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * Every function follows the paper's steps in the paper's order and notation:
 *   - deflection: the pseudo-elliptical potential of Sec. 2.2.2 (the
 *     potential's own frame, the coordinates theta_{i,eps} = sqrt(1 -/+ eps)
 *     theta_i with their polar form (R, phi), the deflection components
 *     |alpha(R)| sqrt(1 -/+ eps) (cos phi, sin phi), the frame turned back,
 *     superposition over potentials), with the singular isothermal radial
 *     profile generalised to the cored and cut isothermal (dPIE) profile that
 *     the paper names as the next model in Sec. 5.  With r_core = 0 and
 *     r_cut = inf it is the SIE gradient that Algorithm 1 computes.
 *   - lens equation in the form of Sec. 2.2.2 (beta = theta - (D_LS/D_OS) grad Psi,
 *     the distance ratio computed once per source).
 *   - chi^2 re-lensing of Sec. 2.2.1 / 2.2.2 and Fig. 1: observed images to the
 *     source plane, barycentre, two triangles per grid cell, containment test,
 *     predicted images, chi^2 sum.
 * Readings of points the paper leaves open are marked READING where they are
 * taken.
 *
 * Compiled with -O2 -ffp-contract=off: no fused multiply-adds, so every
 * operation rounds exactly as written.
 *
 * Parity pins: every exported function is pinned by tests that do not re-use
 * this code (closed forms, invariants, exact rational arithmetic, brute force).
 */
#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_C_KMS 299792.458                        /* speed of light, km/s */
#define ORC_ARCSEC_PER_RAD (180.0 * 3600.0 / ORC_PI) /* 206264.806... */

/* ----------------------------------------------------------------------- */
/* Normalisation and cosmology                                             */
/* ----------------------------------------------------------------------- */

/* b0 = 4 pi (sigma_v / c)^2 (Sec. 2.2.2, the SIE normalisation; equal to the
 * SIS Einstein angle of Sec. 2.1 for D_LS/D_OS = 1), converted to arcsec. */
double orc_b0(double sigma_v)
{
    double ratio = sigma_v / ORC_C_KMS;
    return 4.0 * ORC_PI * ratio * ratio * ORC_ARCSEC_PER_RAD;
}

/* 1/E(z) for a flat LambdaCDM universe (the cosmology of Sec. 4:
 * H0 = 70, Omega_m = 0.3, Omega_Lambda = 0.7).  READING: radiation neglected,
 * curvature Omega_k = 1 - Omega_m - Omega_Lambda assumed zero. */
static double orc_inv_E(double z, double om, double ol)
{
    double a = 1.0 + z;
    return 1.0 / sqrt(om * a * a * a + ol);
}

/* Line-of-sight comoving distance in units of c/H0, composite Simpson rule. */
double orc_comoving(double z, double om, double ol)
{
    const int n = 200000; /* even number of panels */
    double h = z / n, s = orc_inv_E(0.0, om, ol) + orc_inv_E(z, om, ol);
    for (int k = 1; k < n; k++)
        s += (k & 1 ? 4.0 : 2.0) * orc_inv_E(k * h, om, ol);
    return s * h / 3.0;
}

/* D_LS / D_OS for a flat universe: angular diameter distances are comoving
 * distances over (1+z_s), so the ratio is (chi_s - chi_l) / chi_s.  A source in
 * front of the lens is not lensed (ratio 0). */
double orc_dls_dos(double zl, double zs, double om, double ol)
{
    if (zs <= zl) return 0.0;
    double cl = orc_comoving(zl, om, ol), cs = orc_comoving(zs, om, ol);
    return (cs - cl) / cs;
}

/* ----------------------------------------------------------------------- */
/* Deflection: Algorithm 1, generalised to the cored/cut isothermal profile */
/* ----------------------------------------------------------------------- */

/* Radial profile of the circular cored/cut isothermal potential:
 *   |alpha(R)| = K [ (sqrt(a^2+R^2) - a) - (sqrt(s^2+R^2) - s) ] / R
 * written as |alpha(R)| = K * R * f(R) with
 *   f(R) = 1/(sqrt(a^2+R^2) + a) - 1/(sqrt(s^2+R^2) + s),
 * which follows from (q - a) = R^2 / (q + a) and avoids the cancellation the
 * paper warns about in Sec. 3.1.  For a = 0 and s = inf, f = 1/R and
 * |alpha| = K = b0: the SIS of Sec. 2.1.  K = b0 s / (s - a) (READING: the
 * normalisation that keeps the a -> 0, s -> inf limit equal to Algorithm 1).
 * READING: at the centre of a singular profile (a = 0, R = 0) the
 * contribution is 0. */
static double orc_profile_f(double R2, double a, double s)
{
    if (a == 0.0 && R2 == 0.0) return 0.0;
    double f = 1.0 / (sqrt(a * a + R2) + a);
    if (isfinite(s)) f -= 1.0 / (sqrt(s * s + R2) + s);
    return f;
}

static double orc_profile_K(double sigma_v, double a, double s)
{
    double b0 = orc_b0(sigma_v);
    return isfinite(s) ? b0 * s / (s - a) : b0;
}

/* Turns the vector (x, y) by the angle whose cosine and sine are (c, s):
 * (c x - s y, s x + c y).  A potential's own frame has its first axis along
 * the semi-major axis, at angle Phi counter-clockwise from theta_1 (Sec. 2.2.2);
 * sky -> own frame is the turn by -Phi, own frame -> sky the turn by +Phi. */
static void orc_turn(double c, double s, double x, double y, double *ox, double *oy)
{
    *ox = c * x - s * y;
    *oy = s * x + c * y;
}

/* grad Psi_eps at one point theta = (t1, t2), summed over np potentials given
 * as structure of arrays prm[7][np] (rows x, y, eps, phi, r_core, r_cut,
 * sigma_v).  For each potential, from the equations of Sec. 2.2.2: the offset
 * from its centre in its own frame; the pseudo-elliptical coordinates
 * theta_{1,eps} = sqrt(a_1) theta_1, theta_{2,eps} = sqrt(a_2) theta_2
 * (a_{1,2} = 1 -/+ eps) and their polar form (R, phi); the deflection of the
 * circular profile at R, |alpha(R)|, split into the pseudo-elliptical
 * components |alpha(R)| sqrt(a_1) cos(phi) and |alpha(R)| sqrt(a_2) sin(phi);
 * that vector turned back to the sky frame; the contributions of all
 * potentials added (superposition).  For the SIS profile this is the SIE
 * gradient ((1 - eps) b0 theta_1 / R, (1 + eps) b0 theta_2 / R) of the same
 * section. */
void orc_alpha(const double *prm, int np, double t1, double t2, double *a1, double *a2)
{
    const double *xc = prm, *yc = prm + np, *eps = prm + 2 * np, *phi = prm + 3 * np;
    const double *rc = prm + 4 * np, *rcut = prm + 5 * np, *sig = prm + 6 * np;
    double sum1 = 0.0, sum2 = 0.0;
    for (int i = 0; i < np; i++) {
        double c = cos(phi[i]), s = sin(phi[i]);
        double u, v;                          /* offset in the potential's frame */
        orc_turn(c, -s, t1 - xc[i], t2 - yc[i], &u, &v);
        double sq1 = sqrt(1.0 - eps[i]), sq2 = sqrt(1.0 + eps[i]);
        double e1 = sq1 * u, e2 = sq2 * v;   /* theta_{1,eps}, theta_{2,eps} */
        double R2 = e1 * e1 + e2 * e2;
        double f = orc_profile_f(R2, rc[i], rcut[i]);
        if (f == 0.0) continue;               /* centre of a singular profile */
        double R = sqrt(R2), ang = atan2(e2, e1);
        double mag = orc_profile_K(sig[i], rc[i], rcut[i]) * R * f;   /* |alpha(R)| */
        double g1, g2;
        orc_turn(c, s, mag * sq1 * cos(ang), mag * sq2 * sin(ang), &g1, &g2);
        sum1 += g1;
        sum2 += g2;
    }
    *a1 = sum1;
    *a2 = sum2;
}

/* The same equations in complex arithmetic, used only for complex-step
 * derivatives (Squire & Trapp 1998): every operation is analytic away from
 * R = 0, so Im(f(x + i h)) / h = f'(x) to rounding for tiny h.  The polar
 * angle enters through cos(phi) = theta_{1,eps} / R, sin(phi) =
 * theta_{2,eps} / R (analytic, unlike atan2), with R cancelled against the
 * profile's |alpha(R)| = K R f(R). */
static double complex orc_profile_f_c(double complex R2, double complex a, double complex s, int s_inf)
{
    if (creal(a) == 0.0 && cimag(a) == 0.0 && creal(R2) == 0.0 && cimag(R2) == 0.0) return 0.0;
    double complex f = 1.0 / (csqrt(a * a + R2) + a);
    if (!s_inf) f -= 1.0 / (csqrt(s * s + R2) + s);
    return f;
}

static void orc_turn_c(double complex c, double complex s, double complex x, double complex y,
                       double complex *ox, double complex *oy)
{
    *ox = c * x - s * y;
    *oy = s * x + c * y;
}

/* Deflection of a single potential with complex parameters p[7] at complex
 * position (t1, t2). */
static void orc_alpha1_c(const double complex *p, double complex t1, double complex t2,
                         double complex *a1, double complex *a2)
{
    double complex xc = p[0], yc = p[1], eps = p[2], phi = p[3], rc = p[4], rcut = p[5], sig = p[6];
    int s_inf = !isfinite(creal(rcut));
    double complex c = ccos(phi), s = csin(phi), u, v;
    orc_turn_c(c, -s, t1 - xc, t2 - yc, &u, &v);
    double complex sq1 = csqrt(1.0 - eps), sq2 = csqrt(1.0 + eps);
    double complex e1 = sq1 * u, e2 = sq2 * v;
    double complex R2 = e1 * e1 + e2 * e2;
    double complex f = orc_profile_f_c(R2, rc, rcut, s_inf);
    if (f == 0.0) { *a1 = 0.0; *a2 = 0.0; return; }
    double complex ratio = sig / ORC_C_KMS;
    double complex b0 = 4.0 * ORC_PI * ratio * ratio * ORC_ARCSEC_PER_RAD;
    double complex K = s_inf ? b0 : b0 * rcut / (rcut - rc);
    /* |alpha(R)| cos(phi) = (K R f) (theta_{1,eps} / R) = K f theta_{1,eps}, and
     * likewise for sin(phi): the same quantity, analytic also at R = 0 (the
     * centre of a cored profile) */
    double complex Kf = K * f;
    orc_turn_c(c, s, Kf * sq1 * e1, Kf * sq2 * e2, a1, a2);
}

/* Complex deflection summed over all potentials; parameter (kq, pq) of the
 * list carries an imaginary part ih (kq < 0: none). */
static void orc_alpha_c(const double *prm, int np, double complex t1, double complex t2,
                        int kq, int pq, double ih, double complex *a1, double complex *a2)
{
    double complex s1 = 0.0, s2 = 0.0;
    for (int i = 0; i < np; i++) {
        double complex p[7];
        for (int k = 0; k < 7; k++) p[k] = prm[k * np + i];
        if (i == pq && kq >= 0) p[kq] += ih * I;
        double complex g1, g2;
        orc_alpha1_c(p, t1, t2, &g1, &g2);
        s1 += g1;
        s2 += g2;
    }
    *a1 = s1;
    *a2 = s2;
}

/* Exported complex-step helpers. */
void orc_alpha_cplx(const double *prm, int np, double t1, double t1i, double t2, double t2i,
                    int kq, int pq, double ih, double *out /* re1, im1, re2, im2 */)
{
    double complex a1, a2;
    orc_alpha_c(prm, np, t1 + t1i * I, t2 + t2i * I, kq, pq, ih, &a1, &a2);
    out[0] = creal(a1); out[1] = cimag(a1); out[2] = creal(a2); out[3] = cimag(a2);
}

/* ----------------------------------------------------------------------- */
/* Deflection field on the grid (threads over rows)                        */
/* ----------------------------------------------------------------------- */

/* Every threaded job starts with this header: the half-open range of rows
 * [j0, j1) it owns. */
typedef struct { int j0, j1; } orc_rows;

typedef struct {
    orc_rows rows;
    const double *prm; int np;
    double x0, y0, h; int nx, ny;
    double *ax, *ay;
} orc_field_job;

static void *orc_field_rows(void *arg)
{
    orc_field_job *jb = (orc_field_job *)arg;
    for (int j = jb->rows.j0; j < jb->rows.j1; j++)
        for (int i = 0; i < jb->nx; i++) {
            double t1 = jb->x0 + i * jb->h, t2 = jb->y0 + j * jb->h;
            orc_alpha(jb->prm, jb->np, t1, t2, &jb->ax[(size_t)j * jb->nx + i], &jb->ay[(size_t)j * jb->nx + i]);
        }
    return NULL;
}

static void orc_run_rows(void *(*fn)(void *), void *jobs, size_t job_size, int ny, int nthreads)
{
    pthread_t th[256];
    for (int t = 0; t < nthreads; t++) {
        orc_rows *r = (orc_rows *)((char *)jobs + t * job_size);
        r->j0 = (int)((long)ny * t / nthreads);
        r->j1 = (int)((long)ny * (t + 1) / nthreads);
    }
    for (int t = 1; t < nthreads; t++) pthread_create(&th[t], NULL, fn, (char *)jobs + t * job_size);
    fn(jobs);
    for (int t = 1; t < nthreads; t++) pthread_join(th[t], NULL);
}

static int orc_clamp_threads(int nthreads, int ny)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (ny >= 1 && nthreads > ny) nthreads = ny;
    return nthreads;
}

/* Node (i, j) sits at (x0 + i h, y0 + j h); output arrays are row-major
 * [ny][nx].  READING: the grid is made of nodes (pixel corners), not pixel
 * centres. */
void orc_alpha_grid(const double *prm, int np, double x0, double y0, double h, int nx, int ny,
                    double *ax, double *ay, int nthreads)
{
    orc_field_job jobs[256];
    nthreads = orc_clamp_threads(nthreads, ny);
    for (int t = 0; t < nthreads; t++) {
        orc_field_job jb = {{0, 0}, prm, np, x0, y0, h, nx, ny, ax, ay};
        jobs[t] = jb;
    }
    orc_run_rows(orc_field_rows, jobs, sizeof(orc_field_job), ny, nthreads);
}

/* ----------------------------------------------------------------------- */
/* Sources and barycentres (Sec. 2.2.2)                                    */
/* ----------------------------------------------------------------------- */

/* beta_ij = theta_obs,ij - (D_LS/D_OS)_i alpha(theta_obs,ij) with alpha
 * evaluated at the observed position itself (READING), and the barycentre of
 * system i as the plain mean of its beta_ij (READING: unweighted). */
void orc_source_positions(const double *prm, int np, int nsys, const int32_t *sys_off,
                          const double *ox, const double *oy, const double *dls,
                          double *bx, double *by, double *barx, double *bary)
{
    for (int i = 0; i < nsys; i++) {
        double sx = 0.0, sy = 0.0;
        for (int j = sys_off[i]; j < sys_off[i + 1]; j++) {
            double a1, a2;
            orc_alpha(prm, np, ox[j], oy[j], &a1, &a2);
            bx[j] = ox[j] - dls[i] * a1;
            by[j] = oy[j] - dls[i] * a2;
            sx += bx[j];
            sy += by[j];
        }
        int n = sys_off[i + 1] - sys_off[i];
        barx[i] = n > 0 ? sx / n : 0.0;
        bary[i] = n > 0 ? sy / n : 0.0;
    }
}

/* ----------------------------------------------------------------------- */
/* Exact orientation sign with plain multi-precision integers              */
/* ----------------------------------------------------------------------- */

/* Every finite double is an integer multiple of 2^-1074, so after scaling by
 * 2^1074 all inputs are integers of at most 2099 bits, their differences fit
 * in 2100 bits and products in 4200 bits.  Schoolbook arithmetic on 32-bit
 * limbs gives the exact sign of the 2x2 determinant. */
#define ORC_NW 136

typedef struct { int neg; uint32_t w[ORC_NW]; } orc_big;

static void orc_big_from_double(orc_big *r, double x)
{
    memset(r, 0, sizeof *r);
    if (x == 0.0) return;
    r->neg = x < 0.0;
    int e;
    double f = frexp(fabs(x), &e);              /* |x| = f 2^e, 0.5 <= f < 1 */
    uint64_t m = (uint64_t)ldexp(f, 53);        /* exact integer             */
    int shift = e - 53 + 1074;                  /* |x| 2^1074 = m 2^shift    */
    while (shift < 0) { m >>= 1; shift++; }     /* subnormals: exact zeros   */
    int limb = shift / 32, bit = shift % 32;
    unsigned __int128 v = (unsigned __int128)m << bit;
    for (int k = 0; k < 4 && limb + k < ORC_NW; k++) r->w[limb + k] = (uint32_t)(v >> (32 * k));
}

static int orc_mag_cmp(const uint32_t *a, const uint32_t *b)
{
    for (int k = ORC_NW - 1; k >= 0; k--)
        if (a[k] != b[k]) return a[k] > b[k] ? 1 : -1;
    return 0;
}

static void orc_mag_add(uint32_t *r, const uint32_t *a, const uint32_t *b)
{
    uint64_t c = 0;
    for (int k = 0; k < ORC_NW; k++) { c += (uint64_t)a[k] + b[k]; r[k] = (uint32_t)c; c >>= 32; }
}

static void orc_mag_sub(uint32_t *r, const uint32_t *a, const uint32_t *b) /* a >= b */
{
    int64_t c = 0;
    for (int k = 0; k < ORC_NW; k++) {
        c += (int64_t)a[k] - b[k];
        r[k] = (uint32_t)c;
        c = c < 0 ? -1 : 0;
    }
}

static void orc_big_sub(orc_big *r, const orc_big *a, const orc_big *b)
{
    orc_big out;
    memset(&out, 0, sizeof out);
    if (a->neg != b->neg) {                 /* a - b = a + (-b), same sign as a */
        orc_mag_add(out.w, a->w, b->w);
        out.neg = a->neg;
    } else {
        int c = orc_mag_cmp(a->w, b->w);
        if (c >= 0) { orc_mag_sub(out.w, a->w, b->w); out.neg = c == 0 ? 0 : a->neg; }
        else        { orc_mag_sub(out.w, b->w, a->w); out.neg = !a->neg; }
    }
    *r = out;
}

static void orc_big_mul(orc_big *r, const orc_big *a, const orc_big *b)
{
    uint32_t out[ORC_NW];
    memset(out, 0, sizeof out);
    for (int i = 0; i < ORC_NW; i++) {
        if (!a->w[i]) continue;
        uint64_t c = 0;
        for (int j = 0; i + j < ORC_NW; j++) {
            c += (uint64_t)a->w[i] * b->w[j] + out[i + j];
            out[i + j] = (uint32_t)c;
            c >>= 32;
        }
    }
    memcpy(r->w, out, sizeof out);
    int zero = 1;
    for (int k = 0; k < ORC_NW; k++) if (out[k]) { zero = 0; break; }
    r->neg = zero ? 0 : (a->neg != b->neg);
}

/* Exact sign of (a - c) x (b - c) = (ax-cx)(by-cy) - (ay-cy)(bx-cx):
 * +1 if c lies to the left of the directed line a -> b, -1 right, 0 on it. */
int orc_orient(double ax, double ay, double bx, double by, double cx, double cy)
{
    orc_big A, B, C, D, E, F, P, Q, T;
    orc_big_from_double(&A, ax); orc_big_from_double(&C, cx); orc_big_sub(&A, &A, &C); /* ax-cx */
    orc_big_from_double(&B, by); orc_big_from_double(&D, cy); orc_big_sub(&B, &B, &D); /* by-cy */
    orc_big_from_double(&E, ay); orc_big_sub(&E, &E, &D);                              /* ay-cy */
    orc_big_from_double(&F, bx); orc_big_sub(&F, &F, &C);                              /* bx-cx */
    orc_big_mul(&P, &A, &B);
    orc_big_mul(&Q, &E, &F);
    orc_big_sub(&T, &P, &Q);
    int zero = 1;
    for (int k = 0; k < ORC_NW; k++) if (T.w[k]) { zero = 0; break; }
    return zero ? 0 : (T.neg ? -1 : 1);
}

/* ----------------------------------------------------------------------- */
/* Triangles of the grid (Fig. 1)                                          */
/* ----------------------------------------------------------------------- */

/* READING: cell (i, j), 0 <= i < nx-1, 0 <= j < ny-1, is split along its
 * anti-diagonal into triangle k = 0 with vertices (i,j), (i+1,j), (i,j+1) and
 * triangle k = 1 with vertices (i+1,j+1), (i,j+1), (i+1,j); both are
 * counter-clockwise in the image plane.  Triangle id t = 2 (j (nx-1) + i) + k. */
static void orc_triangle_nodes(int nx, int i, int j, int k, int *ni, int *nj)
{
    if (k == 0) { ni[0] = i;     nj[0] = j;     ni[1] = i + 1; nj[1] = j;     ni[2] = i;     nj[2] = j + 1; }
    else        { ni[0] = i + 1; nj[0] = j + 1; ni[1] = i;     nj[1] = j + 1; ni[2] = i + 1; nj[2] = j;     }
    (void)nx;
}

/* Containment of the barycentre (px, py) in the source-plane triangle with
 * vertices (vx[k], vy[k]) (Sec. 2.2.2).  An exact bounding-box rejection,
 * then the three exact edge signs; hit iff all three are strictly positive
 * or all strictly negative (lensing may flip the orientation).  READING:
 * points exactly on an edge are misses.  Returns 1 for a hit. */
static int orc_contains(const double *vx, const double *vy, double px, double py, int *n_bbox)
{
    double xmin = vx[0], xmax = vx[0], ymin = vy[0], ymax = vy[0];
    for (int k = 1; k < 3; k++) {
        if (vx[k] < xmin) xmin = vx[k];
        if (vx[k] > xmax) xmax = vx[k];
        if (vy[k] < ymin) ymin = vy[k];
        if (vy[k] > ymax) ymax = vy[k];
    }
    if (px < xmin || px > xmax || py < ymin || py > ymax) return 0;
    (*n_bbox)++;
    int s0 = orc_orient(vx[0], vy[0], vx[1], vy[1], px, py);
    int s1 = orc_orient(vx[1], vy[1], vx[2], vy[2], px, py);
    int s2 = orc_orient(vx[2], vy[2], vx[0], vy[0], px, py);
    return (s0 > 0 && s1 > 0 && s2 > 0) || (s0 < 0 && s1 < 0 && s2 < 0);
}

typedef struct {
    orc_rows rows;
    const double *ax, *ay;
    double x0, y0, h; int nx, ny;
    int nsys; const double *barx, *bary, *dls;
    int cap, n; int32_t *sys, *tid;
    long n_bbox;
} orc_tri_job;

static void *orc_tri_rows(void *arg)
{
    orc_tri_job *jb = (orc_tri_job *)arg;
    int nx = jb->nx;
    for (int s = 0; s < jb->nsys; s++) {
        double r = jb->dls[s];
        for (int j = jb->rows.j0; j < jb->rows.j1; j++)
            for (int i = 0; i < nx - 1; i++)
                for (int k = 0; k < 2; k++) {
                    int ni[3], nj[3];
                    double vx[3], vy[3];
                    orc_triangle_nodes(nx, i, j, k, ni, nj);
                    for (int v = 0; v < 3; v++) {
                        size_t n = (size_t)nj[v] * nx + ni[v];
                        double t1 = jb->x0 + ni[v] * jb->h, t2 = jb->y0 + nj[v] * jb->h;
                        vx[v] = t1 - r * jb->ax[n];   /* lens equation, Sec. 2.2.2 */
                        vy[v] = t2 - r * jb->ay[n];
                    }
                    int nb = 0;
                    if (orc_contains(vx, vy, jb->barx[s], jb->bary[s], &nb)) {
                        if (jb->n < jb->cap) {
                            jb->sys[jb->n] = s;
                            jb->tid[jb->n] = 2 * (j * (nx - 1) + i) + k;
                        }
                        jb->n++;
                    }
                    jb->n_bbox += nb;
                }
    }
    return NULL;
}

static int orc_cmp_hit(const void *pa, const void *pb)
{
    const int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    return a < b ? -1 : a > b;
}

/* Predicted image position for hit (system s, triangle t): barycentric
 * interpolation of the image-plane vertices with weights from the
 * source-plane triangle (READING: the exact inverse of the linear map of the
 * triangle).  lambda_k = c_{k+1} / (c_0 + c_1 + c_2) with
 * c_k = (B_k - p) x (B_{k+1} - p). */
static void orc_image_position(const double *ax, const double *ay, double x0, double y0, double h,
                               int nx, int t, double r, double px, double py, double *xo, double *yo)
{
    int cell = t / 2, k = t % 2, i = cell % (nx - 1), j = cell / (nx - 1);
    int ni[3], nj[3];
    double vx[3], vy[3], tx[3], ty[3], c[3];
    orc_triangle_nodes(nx, i, j, k, ni, nj);
    for (int v = 0; v < 3; v++) {
        size_t n = (size_t)nj[v] * nx + ni[v];
        tx[v] = x0 + ni[v] * h;
        ty[v] = y0 + nj[v] * h;
        vx[v] = tx[v] - r * ax[n];
        vy[v] = ty[v] - r * ay[n];
    }
    for (int v = 0; v < 3; v++) {
        int w = (v + 1) % 3;
        c[v] = (vx[v] - px) * (vy[w] - py) - (vy[v] - py) * (vx[w] - px);
    }
    double sum = c[0] + c[1] + c[2];
    double l0 = c[1] / sum, l1 = c[2] / sum, l2 = c[0] / sum;
    *xo = l0 * tx[0] + l1 * tx[1] + l2 * tx[2];
    *yo = l0 * ty[0] + l1 * ty[1] + l2 * ty[2];
}

/* Triangle stage on a given deflection field ax, ay [ny][nx]: every triangle
 * of the grid is mapped to the source plane of every system (lens equation
 * with that system's D_LS/D_OS) and tested for containment of the system's
 * barycentre (barx, bary).  Hits are returned sorted by (system, triangle
 * id); at most cap are stored; the return value is the total number. */
int orc_hits_from_field(const double *ax, const double *ay, double x0, double y0, double h,
                        int nx, int ny, int nsys, const double *barx, const double *bary,
                        const double *dls, int nthreads, int cap, int32_t *hit_sys, int32_t *hit_tid,
                        int64_t *n_bbox_pass)
{
    int ncell_rows = ny - 1;
    nthreads = orc_clamp_threads(nthreads, ncell_rows);
    int per_cap = cap + 1;
    orc_tri_job *jobs = (orc_tri_job *)calloc(nthreads, sizeof(orc_tri_job));
    for (int t = 0; t < nthreads; t++) {
        orc_tri_job jb = {{0, 0}, ax, ay, x0, y0, h, nx, ny, nsys, barx, bary, dls, per_cap, 0,
                          (int32_t *)malloc(per_cap * sizeof(int32_t)),
                          (int32_t *)malloc(per_cap * sizeof(int32_t)), 0};
        jobs[t] = jb;
    }
    orc_run_rows(orc_tri_rows, jobs, sizeof(orc_tri_job), ncell_rows, nthreads);
    long total = 0, nbbox = 0;
    for (int t = 0; t < nthreads; t++) { total += jobs[t].n; nbbox += jobs[t].n_bbox; }
    int64_t *keys = (int64_t *)malloc((total + 1) * sizeof(int64_t));
    long nk = 0;
    for (int t = 0; t < nthreads; t++)
        for (int q = 0; q < jobs[t].n && q < per_cap; q++)
            keys[nk++] = ((int64_t)jobs[t].sys[q] << 32) | (uint32_t)jobs[t].tid[q];
    qsort(keys, nk, sizeof(int64_t), orc_cmp_hit);
    for (long q = 0; q < nk && q < cap; q++) {
        hit_sys[q] = (int32_t)(keys[q] >> 32);
        hit_tid[q] = (int32_t)(keys[q] & 0xffffffff);
    }
    if (n_bbox_pass) *n_bbox_pass = nbbox;
    for (int t = 0; t < nthreads; t++) { free(jobs[t].sys); free(jobs[t].tid); }
    free(jobs);
    free(keys);
    return (int)total;
}

/* Predicted positions of nh hits (sorted by system) on a given field. */
void orc_positions_from_field(const double *ax, const double *ay, double x0, double y0, double h,
                              int nx, int nh, const int32_t *hit_sys, const int32_t *hit_tid,
                              const double *barx, const double *bary, const double *dls,
                              double *hit_x, double *hit_y)
{
    for (int q = 0; q < nh; q++) {
        int s = hit_sys[q];
        orc_image_position(ax, ay, x0, y0, h, nx, hit_tid[q], dls[s], barx[s], bary[s], &hit_x[q], &hit_y[q]);
    }
}

/* Matching and chi^2 (Sec. 2.2.1) for hits sorted by system.
 * READING (the paper leaves the pairing open): each observed image is paired
 * with the nearest predicted image of its own system (Euclidean distance, ties
 * to the lower triangle id, i.e. the earlier hit); chi2_i = sum_j
 * |x_obs,ij - x_ij|^2 / sigma_ij^2; a system without any predicted image has
 * chi2_i = +inf.  Sums run in index order. */
double orc_match_chi2(int nsys, const int32_t *sys_off, const double *ox, const double *oy,
                      const double *osig, int nh, const int32_t *hit_sys, const double *hit_x,
                      const double *hit_y, int32_t *n_pred, double *chi2_sys, int32_t *match)
{
    for (int s = 0; s < nsys; s++) n_pred[s] = 0;
    for (int q = 0; q < nh; q++) n_pred[hit_sys[q]]++;
    double tot = 0.0;
    long first = 0;
    for (int s = 0; s < nsys; s++) {
        long lo = first, hi = first + n_pred[s];
        double cs = 0.0;
        for (int j = sys_off[s]; j < sys_off[s + 1]; j++) {
            long best = -1;
            double bd = 0.0;
            for (long q = lo; q < hi; q++) {
                double dx = ox[j] - hit_x[q], dy = oy[j] - hit_y[q];
                double d2 = dx * dx + dy * dy;
                if (best < 0 || d2 < bd) { best = q; bd = d2; }
            }
            match[j] = (int32_t)best;
            if (best >= 0) cs += bd / (osig[j] * osig[j]);
        }
        if (n_pred[s] == 0) cs = INFINITY;
        chi2_sys[s] = cs;
        tot += cs;
        first = hi;
    }
    return tot;
}

/* Full chi^2 evaluation (Sec. 2.2.1 and 2.2.2, Fig. 1).
 *
 * Inputs: potentials prm[7][np]; grid (x0, y0, h, nx, ny); nsys systems in CSR
 * form sys_off[nsys+1] over observed images (ox, oy, osig); D_LS/D_OS per
 * system.  Outputs (caller-allocated):
 *   hit_sys, hit_tid [cap]  predicted-image triangles sorted by (system, id)
 *   hit_x, hit_y [cap]      predicted image positions
 *   n_pred [nsys], chi2_sys [nsys], *chi2
 *   match [n_img]           index (into the hit list) of the predicted image
 *                           matched to each observed image, -1 if none
 *   stats [4]               n_hits, n_bbox_pass, n_tests, reserved
 *   barx, bary [nsys]       barycentres of the systems' sources
 * Returns the number of hits; if it exceeds cap, only the first cap are
 * stored and positions/chi^2 are not computed. */
int orc_image_chi2(const double *prm, int np, double x0, double y0, double h, int nx, int ny,
                   int nsys, const int32_t *sys_off, const double *ox, const double *oy,
                   const double *osig, const double *dls, int nthreads, int cap,
                   int32_t *hit_sys, int32_t *hit_tid, double *hit_x, double *hit_y,
                   int32_t *n_pred, double *chi2_sys, double *chi2, int32_t *match, int64_t *stats,
                   double *barx, double *bary)
{
    size_t nn = (size_t)nx * ny;
    double *ax = (double *)malloc(nn * sizeof(double));
    double *ay = (double *)malloc(nn * sizeof(double));
    int nimg = sys_off[nsys];
    double *bx = (double *)malloc((nimg + 1) * sizeof(double));
    double *by = (double *)malloc((nimg + 1) * sizeof(double));

    /* 1. gradient field at every node (Algorithm 1) */
    orc_alpha_grid(prm, np, x0, y0, h, nx, ny, ax, ay, nthreads);
    /* 2. observed images -> sources -> barycentre */
    orc_source_positions(prm, np, nsys, sys_off, ox, oy, dls, bx, by, barx, bary);
    /* 3. triangles -> source plane -> containment of the barycentre */
    int64_t nbbox = 0;
    int total = orc_hits_from_field(ax, ay, x0, y0, h, nx, ny, nsys, barx, bary, dls, nthreads, cap,
                                    hit_sys, hit_tid, &nbbox);
    stats[0] = total;
    stats[1] = nbbox;
    stats[2] = (int64_t)2 * (nx - 1) * (ny - 1) * nsys;
    stats[3] = 0;
    if (total <= cap) {
        /* 4. predicted positions; 5. matching and chi^2 */
        orc_positions_from_field(ax, ay, x0, y0, h, nx, total, hit_sys, hit_tid, barx, bary, dls, hit_x, hit_y);
        *chi2 = orc_match_chi2(nsys, sys_off, ox, oy, osig, total, hit_sys, hit_x, hit_y, n_pred, chi2_sys, match);
    }
    free(ax); free(ay); free(bx); free(by);
    return total;
}

/* ----------------------------------------------------------------------- */
/* Brute-force image finder (Newton on the lens equation)                  */
/* ----------------------------------------------------------------------- */

/* Newton-Raphson on F(theta) = theta - r alpha(theta) - beta = 0 starting at
 * (tx, ty); the Jacobian dF/dtheta = I - r d(alpha)/d(theta) comes from the
 * complex step in theta_1 and theta_2.  Returns 1 if |F| < tol within maxit
 * iterations, with the root in (*rx, *ry). */
int orc_newton(const double *prm, int np, double r, double bx, double by, double tx, double ty,
               int maxit, double tol, double *rx, double *ry)
{
    const double ih = 1e-30;
    for (int it = 0; it < maxit; it++) {
        double complex a1, a2, b1, b2;
        orc_alpha_c(prm, np, tx + ih * I, ty, -1, -1, 0.0, &a1, &a2);
        orc_alpha_c(prm, np, tx, ty + ih * I, -1, -1, 0.0, &b1, &b2);
        double F1 = tx - r * creal(a1) - bx, F2 = ty - r * creal(a2) - by;
        if (!isfinite(F1) || !isfinite(F2)) return 0;
        if (sqrt(F1 * F1 + F2 * F2) < tol) { *rx = tx; *ry = ty; return 1; }
        double J11 = 1.0 - r * cimag(a1) / ih, J21 = -r * cimag(a2) / ih;
        double J12 = -r * cimag(b1) / ih, J22 = 1.0 - r * cimag(b2) / ih;
        double det = J11 * J22 - J12 * J21;
        if (det == 0.0 || !isfinite(det)) return 0;
        double d1 = (J22 * F1 - J12 * F2) / det, d2 = (J11 * F2 - J21 * F1) / det;
        /* damp very long steps (they only happen near critical curves) */
        double step = sqrt(d1 * d1 + d2 * d2);
        if (step > 5.0) { d1 *= 5.0 / step; d2 *= 5.0 / step; }
        tx -= d1;
        ty -= d2;
    }
    return 0;
}

/* Seeds at every node of a (nx, ny) grid; converged roots inside
 * [xlo, xhi] x [ylo, yhi] are de-duplicated within dedup arcsec.  Returns
 * the number of distinct roots (at most cap are stored). */
int orc_find_images(const double *prm, int np, double r, double bx, double by,
                    double x0, double y0, double h, int nx, int ny,
                    double xlo, double xhi, double ylo, double yhi,
                    double tol, double dedup, int cap, double *out_x, double *out_y)
{
    int n = 0;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            double rx, ry;
            if (!orc_newton(prm, np, r, bx, by, x0 + i * h, y0 + j * h, 60, tol, &rx, &ry)) continue;
            if (rx < xlo || rx > xhi || ry < ylo || ry > yhi) continue;
            int dup = 0;
            for (int q = 0; q < n && q < cap; q++) {
                double dx = rx - out_x[q], dy = ry - out_y[q];
                if (sqrt(dx * dx + dy * dy) < dedup) { dup = 1; break; }
            }
            if (dup) continue;
            if (n < cap) { out_x[n] = rx; out_y[n] = ry; }
            n++;
        }
    return n;
}

/* ----------------------------------------------------------------------- */
/* Source-plane chi^2 and complex-step gradients                           */
/* ----------------------------------------------------------------------- */

/* READING of the smooth source-plane chi^2 (not defined in the paper):
 *   chi2_src = sum_i sum_j |beta_ij - bar(beta)_i|^2 / sigma_ij^2
 * with beta_ij from the lens equation at the observed images and
 * bar(beta)_i their unweighted mean.  Complex version: parameter (kq, pq)
 * carries an imaginary part ih. */
static double complex orc_src_chi2_c(const double *prm, int np, int nsys, const int32_t *sys_off,
                                     const double *ox, const double *oy, const double *osig,
                                     const double *dls, int kq, int pq, double ih)
{
    double complex total = 0.0;
    for (int i = 0; i < nsys; i++) {
        int n = sys_off[i + 1] - sys_off[i];
        if (n <= 0) continue;
        double complex *b1 = (double complex *)malloc(n * sizeof(double complex));
        double complex *b2 = (double complex *)malloc(n * sizeof(double complex));
        double complex m1 = 0.0, m2 = 0.0;
        for (int j = 0; j < n; j++) {
            double complex a1, a2;
            int q = sys_off[i] + j;
            orc_alpha_c(prm, np, ox[q], oy[q], kq, pq, ih, &a1, &a2);
            b1[j] = ox[q] - dls[i] * a1;
            b2[j] = oy[q] - dls[i] * a2;
            m1 += b1[j];
            m2 += b2[j];
        }
        m1 /= n;
        m2 /= n;
        double complex cs = 0.0;
        for (int j = 0; j < n; j++) {
            int q = sys_off[i] + j;
            double complex d1 = b1[j] - m1, d2 = b2[j] - m2;
            cs += (d1 * d1 + d2 * d2) / (osig[q] * osig[q]);
        }
        total += cs;
        free(b1);
        free(b2);
    }
    return total;
}

double orc_src_chi2(const double *prm, int np, int nsys, const int32_t *sys_off, const double *ox,
                    const double *oy, const double *osig, const double *dls)
{
    return creal(orc_src_chi2_c(prm, np, nsys, sys_off, ox, oy, osig, dls, -1, -1, 0.0));
}

/* d chi2_src / d q for all 7 np parameters, complex step 1e-30; grad[k*np+p]. */
void orc_src_chi2_grad(const double *prm, int np, int nsys, const int32_t *sys_off, const double *ox,
                       const double *oy, const double *osig, const double *dls, double *grad)
{
    const double ih = 1e-30;
    for (int k = 0; k < 7; k++)
        for (int p = 0; p < np; p++) {
            double v = prm[k * np + p];
            if (k == 5 && !isfinite(v)) { grad[k * np + p] = 0.0; continue; }
            grad[k * np + p] = cimag(orc_src_chi2_c(prm, np, nsys, sys_off, ox, oy, osig, dls, k, p, ih)) / ih;
        }
}

/* Vector-Jacobian product of the deflection field: grad[k*np+p] =
 * sum over nodes of gx * d alpha_1/d q + gy * d alpha_2 / d q, q = parameter k
 * of potential p.  Only potential p depends on its own parameters, so each
 * derivative is the complex step of that one potential's deflection. */
typedef struct {
    orc_rows rows;
    const double *prm; int np;
    double x0, y0, h; int nx, ny;
    const double *gx, *gy;
    int absval;            /* 1: sum |gx d alpha_1/dq| + |gy d alpha_2/dq| instead */
    double *part;          /* [7*np] partial sums of this thread */
} orc_vjp_job;

static void *orc_vjp_rows(void *arg)
{
    orc_vjp_job *jb = (orc_vjp_job *)arg;
    const double ih = 1e-30;
    int np = jb->np;
    for (int j = jb->rows.j0; j < jb->rows.j1; j++)
        for (int i = 0; i < jb->nx; i++) {
            size_t n = (size_t)j * jb->nx + i;
            double t1 = jb->x0 + i * jb->h, t2 = jb->y0 + j * jb->h;
            for (int p = 0; p < np; p++)
                for (int k = 0; k < 7; k++) {
                    double complex q[7], a1, a2;
                    for (int m = 0; m < 7; m++) q[m] = jb->prm[m * np + p];
                    if (k == 5 && !isfinite(creal(q[5]))) continue;
                    q[k] += ih * I;
                    orc_alpha1_c(q, t1, t2, &a1, &a2);
                    double t1v = jb->gx[n] * (cimag(a1) / ih), t2v = jb->gy[n] * (cimag(a2) / ih);
                    if (jb->absval) { t1v = fabs(t1v); t2v = fabs(t2v); }
                    jb->part[k * np + p] += t1v + t2v;
                }
        }
    return NULL;
}

/* absval = 1 gives the magnitude sum over nodes of |gx d alpha_1/dq| +
 * |gy d alpha_2/dq| (the scale of the rounding error of any evaluation order). */
void orc_alpha_vjp(const double *prm, int np, double x0, double y0, double h, int nx, int ny,
                   const double *gx, const double *gy, double *grad, int nthreads, int absval)
{
    nthreads = orc_clamp_threads(nthreads, ny);
    orc_vjp_job *jobs = (orc_vjp_job *)calloc(nthreads, sizeof(orc_vjp_job));
    for (int t = 0; t < nthreads; t++) {
        orc_vjp_job jb = {{0, 0}, prm, np, x0, y0, h, nx, ny, gx, gy, absval,
                          (double *)calloc(7 * np, sizeof(double))};
        jobs[t] = jb;
    }
    orc_run_rows(orc_vjp_rows, jobs, sizeof(orc_vjp_job), ny, nthreads);
    for (int q = 0; q < 7 * np; q++) grad[q] = 0.0;
    for (int t = 0; t < nthreads; t++) {
        for (int q = 0; q < 7 * np; q++) grad[q] += jobs[t].part[q];
        free(jobs[t].part);
    }
    free(jobs);
}

/* ----------------------------------------------------------------------- */
/* The paper's mixed-precision gradient (Sec. 3.2, Sec. 3.3, Appendix A.3) */
/* ----------------------------------------------------------------------- */

/* Double-precision patches (Sec. 3.2, Appendix A.3): a block of pc x pc pixels
 * centred on each of the first n_cluster potentials (the cluster-scale halos)
 * and of pg x pg pixels centred on every other potential (galaxy-scale halos).
 * READING: the block centred on a halo spans node indices [k - p/2, k - p/2 + p)
 * along each axis, k = the node nearest the centre, (x_c - x0)/h rounded with
 * halves away from zero; blocks are clipped to the grid.  mask[j*nx + i] = 1
 * inside any block, 0 elsewhere. */
void orc_dp_patches(const double *prm, int np, int n_cluster, int pc, int pg, double x0, double y0, double h,
                    int nx, int ny, uint8_t *mask)
{
    memset(mask, 0, (size_t)nx * ny);
    for (int p = 0; p < np; p++) {
        long size = p < n_cluster ? pc : pg;
        long ki = lround((prm[p] - x0) / h), kj = lround((prm[np + p] - y0) / h);
        long i0 = ki - size / 2, j0 = kj - size / 2;
        for (long j = j0; j < j0 + size; j++) {
            if (j < 0 || j >= ny) continue;
            for (long i = i0; i < i0 + size; i++) {
                if (i < 0 || i >= nx) continue;
                mask[(size_t)j * nx + i] = 1;
            }
        }
    }
}

/* The criteria of Sec. 3.3 on a gradient field (ax, ay) whose pixels have
 * length dx along both axes:
 *     d1 = ax(i, j) - ax(i-1, j),   d2 = ay(i, j) - ay(i, j-1),
 *     d3 = ax(i, j) - ax(i, j-1),   d4 = ay(i, j) - ay(i-1, j),
 * pixel (i, j) needs double precision when |dx - d1| < t12 or |dx - d2| < t12
 * (the source-plane pixel length below t12, eq. Criterion_delta_1_2) or
 * |d3| > t34 or |d4| > t34 (eq. Criterion_delta_3_4).  READING: a difference
 * whose neighbour lies outside the image (i = 0 for d1 and d4, j = 0 for d2 and
 * d3) is not evaluated.  flags[j*nx + i] = 1 for such pixels, else 0. */
void orc_criteria(const double *ax, const double *ay, int nx, int ny, double dx, double t12, double t34,
                  uint8_t *flags)
{
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            size_t n = (size_t)j * nx + i;
            int need = 0;
            if (i > 0) {
                double d1 = ax[n] - ax[n - 1];
                double d4 = ay[n] - ay[n - 1];
                if (fabs(dx - d1) < t12 || fabs(d4) > t34) need = 1;
            }
            if (j > 0) {
                double d2 = ay[n] - ay[n - nx];
                double d3 = ax[n] - ax[n - nx];
                if (fabs(dx - d2) < t12 || fabs(d3) > t34) need = 1;
            }
            flags[n] = (uint8_t)need;
        }
}

/* ----------------------------------------------------------------------- */
/* Pseudo-elliptical NFW deflection (the second family named in Sec. 5)    */
/* ----------------------------------------------------------------------- */

/* The NFW convergence kappa(x) = 2 kappa_s (1 - F(x)) / (x^2 - 1), x = R / r_s,
 * encloses the mean convergence kbar(x) = 4 kappa_s g(x) / x^2 with
 *     g(x) = ln(x/2) + F(x),
 *     F(x) = arccosh(1/x) / sqrt(1 - x^2)   (x < 1),
 *            1                              (x = 1),
 *            arccos(1/x) / sqrt(x^2 - 1)    (x > 1)
 * (Bartelmann 1996; Wright & Brainerd 2000).  The circular deflection is
 * alpha(R) = R kbar = 4 kappa_s r_s g(x) / x.  The pseudo-elliptical form
 * replaces R by the R of Algorithm 1 exactly as for the SIE (Sec. 2.2.2): the
 * lens-frame gradient is alpha(R)/R * ((1 - eps) dt1', (1 + eps) dt2').
 * Evaluated in long double (the textbook forms lose digits to cancellation at
 * small x); the centre contributes 0.  prm: [6][np] rows x, y, eps, phi, r_s,
 * kappa_s. */
static long double orc_nfw_g(long double x)
{
    long double F;
    if (x < 1.0L) F = acoshl(1.0L / x) / sqrtl(1.0L - x * x);
    else if (x > 1.0L) F = acosl(1.0L / x) / sqrtl(x * x - 1.0L);
    else F = 1.0L;
    return logl(x / 2.0L) + F;
}

void orc_nfw_alpha(const double *prm, int np, double t1, double t2, double *a1, double *a2)
{
    const double *xc = prm, *yc = prm + np, *eps = prm + 2 * np, *phi = prm + 3 * np;
    const double *rs = prm + 4 * np, *ks = prm + 5 * np;
    long double sum1 = 0.0L, sum2 = 0.0L;
    for (int i = 0; i < np; i++) {
        long double dt1 = (long double)t1 - xc[i];
        long double dt2 = (long double)t2 - yc[i];
        long double c = cosl(phi[i]), s = sinl(phi[i]);
        long double dt1r = dt1 * c + dt2 * s;
        long double dt2r = dt2 * c - dt1 * s;
        long double R2 = dt1r * dt1r * (1.0L - eps[i]) + dt2r * dt2r * (1.0L + eps[i]);
        if (R2 == 0.0L) continue;
        long double R = sqrtl(R2), x = R / rs[i];
        long double aR = 4.0L * ks[i] * rs[i] * orc_nfw_g(x) / x;   /* circular deflection */
        long double g1 = (1.0L - eps[i]) * aR * dt1r / R;
        long double g2 = (1.0L + eps[i]) * aR * dt2r / R;
        sum1 += g1 * c - g2 * s;                                      /* rotate back by +Phi */
        sum2 += g2 * c + g1 * s;
    }
    *a1 = (double)sum1;
    *a2 = (double)sum2;
}

typedef struct {
    orc_rows rows;
    const double *prm; int np;
    double x0, y0, h; int nx, ny;
    double *ax, *ay;
} orc_nfw_job;

static void *orc_nfw_rows(void *arg)
{
    orc_nfw_job *jb = (orc_nfw_job *)arg;
    for (int j = jb->rows.j0; j < jb->rows.j1; j++)
        for (int i = 0; i < jb->nx; i++) {
            double t1 = jb->x0 + i * jb->h, t2 = jb->y0 + j * jb->h;
            orc_nfw_alpha(jb->prm, jb->np, t1, t2, &jb->ax[(size_t)j * jb->nx + i], &jb->ay[(size_t)j * jb->nx + i]);
        }
    return NULL;
}

void orc_nfw_alpha_grid(const double *prm, int np, double x0, double y0, double h, int nx, int ny, double *ax,
                        double *ay, int nthreads)
{
    orc_nfw_job jobs[256];
    nthreads = orc_clamp_threads(nthreads, ny);
    for (int t = 0; t < nthreads; t++) {
        orc_nfw_job jb = {{0, 0}, prm, np, x0, y0, h, nx, ny, ax, ay};
        jobs[t] = jb;
    }
    orc_run_rows(orc_nfw_rows, jobs, sizeof(orc_nfw_job), ny, nthreads);
}
