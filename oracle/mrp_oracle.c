/*
 * Plain FP64 CPU oracle for the spectral kinetic simulation of the ideal
 * Multipole Resonance Probe (Gong, Friedrichs, Oberrath, Brinkmann,
 * arXiv:2111.13072).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the
 * HIP library.
 *
 * What it computes is the plain definition, written out pair by pair:
 *
 *   Phi(x) = (1/nt) sum_{i != k} q G~_L(x, x_i) + (1/nt) Q_S / (4 pi r)
 *            + Phi_ion(r) + u_asy Psi_anti,L(x)
 *
 * (modified potential of Sec. 3 with the projection P^ taken as "l <= L",
 * super-particle scaling of Sec. 4), where the truncated modified Green's
 * function of Sec. 3 (R^(p,p)_l of App. A summed over m with the spherical
 * harmonic addition theorem, plus the floating-potential term that removes
 * the l = 0 image) is
 *
 *   G~_L(x,y) = 1/(4 pi) [ 1/r_> + sum_{l=1..L} ( r_<^l / r_>^(l+1)
 *                                   - f_l / (r_x r_y)^(l+1) ) P_l(xhat.yhat) ].
 *
 * In the axisymmetric mode (m = 0 only, the paper's dipole kernel of Sec. 3)
 * P_l(xhat.yhat) becomes P_l(cos th_x) P_l(cos th_y).
 *
 * No sorting is needed: for each pair the smaller radius is decided by the
 * key (r^2, id) with r^2 = (x*x + y*y) + z*z evaluated without contraction
 * (build with -ffp-contract=off).
 *
 * Parity pins live in tests/test_oracle_pins.py, among them the diffuse wall
 * law (Kolmogorov-Smirnov tests of its angular distribution) and its
 * random-number generator (numpy's Philox).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_PIL 3.14159265358979323846264338327950288L

/* Electrons: charge -1 (units of e), mass 1 (units of m_e), Sec. 4.  A
 * particle whose id has bit 31 set is an ion: charge +1, mass ion_mass. */
#define ORC_Q (-1.0)
#define ORC_M (1.0)
#define ORC_ION_BIT 0x80000000u

enum { ORC_M_FULL = 0, ORC_M_AXISYM = 1 };
enum { ORC_BC_ABSORB = 0, ORC_BC_SPECULAR = 1, ORC_BC_DIFFUSE = 2 };

typedef struct {
    double d;            /* dielectric thickness / R; electrode radius a = 1 - d */
    double eps_r;        /* dielectric permittivity */
    double r_out;        /* outer particle wall, units of R */
    double dt;           /* time step, units of 1/omega_pe */
    double ntilde;       /* super-particles per unit volume R^3 */
    double ion_density;  /* immobile uniform ion background, units of n_inf */
    int32_t l_max;
    int32_t m_mode;
    int32_t probe_bc;
    int32_t wall_bc;
    uint64_t seed;       /* diffuse reflection only */
    /* Optional immobile ion profile (replaces ion_density when non-NULL):
     * density at ion_prof_len >= 2 equally spaced radii from 1 to r_out,
     * linear in between. */
    const double *ion_prof;
    int64_t ion_prof_len;
    double ion_mass;     /* m_i / m_e of particles whose id has bit 31 set */
} orc_params;

static double charge_of(uint32_t id) { return (id & ORC_ION_BIT) ? 1.0 : ORC_Q; }

static double mass_of(const orc_params *p, uint32_t id)
{
    return (id & ORC_ION_BIT) ? p->ion_mass : ORC_M;
}

/* ------------------------------------------------------------------------ */
/* Coefficients                                                              */
/* ------------------------------------------------------------------------ */

/* Image coefficient f_l of R^(p,p)_l (App. A, closed form for R = 1,
 * R_E = a). */
static double coef_f(double eps, double a, int l)
{
    double a2l1 = pow(a, 2.0 * l + 1.0);
    double num = l * (eps - 1.0) + (l + eps + l * eps) * a2l1;
    double den = (l + 1.0 + l * eps) + (l + 1.0) * (eps - 1.0) * a2l1;
    return num / den;
}

/* Plasma-side coefficient b^P_l of the electrode influence function psi_l
 * (Sec. 3, the a^D, b^D, b^P system). */
static double coef_bP(double eps, double a, int l)
{
    double den = (l + 1.0) * (eps - 1.0) * pow(a, 2.0 * l + 1.0) + l * eps + l + 1.0;
    return (2.0 * l + 1.0) * eps * pow(a, l + 1.0) / den;
}

/* Legendre coefficient c of the antisymmetric electrode data for odd l,
 * l = 2l' - 1 (Sec. 3, Psi_anti series):
 * c_{l'} = (-1/2)^{l'+1} (4l'-1) (2l'-3)!! / l'!, with (-1)!! = 1. */
static double coef_c(int l)
{
    if (l % 2 == 0) return 0.0;
    int lp = (l + 1) / 2;
    double dfact = 1.0;
    for (int j = 2 * lp - 3; j > 1; j -= 2) dfact *= j;
    double fact = 1.0;
    for (int j = 2; j <= lp; ++j) fact *= j;
    return pow(-0.5, lp + 1) * (4.0 * lp - 1.0) * dfact / fact;
}

void orc_coeffs(double eps_r, double d, int l_max, double *f, double *bP, double *c)
{
    double a = 1.0 - d;
    for (int l = 0; l <= l_max; ++l) {
        f[l] = coef_f(eps_r, a, l);
        bP[l] = coef_bP(eps_r, a, l);
        c[l] = coef_c(l);
    }
}

/* ------------------------------------------------------------------------ */
/* Geometry helpers                                                          */
/* ------------------------------------------------------------------------ */

/* Radial sort key of the method: r^2 evaluated as (x*x + y*y) + z*z. */
static double key_r2(const double *x)
{
    double xx = x[0] * x[0];
    double yy = x[1] * x[1];
    double zz = x[2] * x[2];
    return (xx + yy) + zz;
}

/* |x| in long double; the radial order still comes from the double key. */
static long double norm_ld(const double *x)
{
    long double a = x[0], b = x[1], c = x[2];
    return sqrtl(a * a + b * b + c * c);
}

static int key_less(double r2a, uint32_t ida, double r2b, uint32_t idb)
{
    return (r2a < r2b) || (r2a == r2b && ida < idb);
}

/* P_l(u) and P'_l(u) for l = 0..L (Bonnet recurrence and its derivative). */
static void legendre(long double u, int L, long double *P, long double *dP)
{
    P[0] = 1.0L;
    dP[0] = 0.0L;
    if (L >= 1) {
        P[1] = u;
        dP[1] = 1.0L;
    }
    for (int l = 1; l < L; ++l) {
        P[l + 1] = ((2.0L * l + 1.0L) * u * P[l] - l * P[l - 1]) / (l + 1.0L);
        dP[l + 1] = dP[l - 1] + (2.0L * l + 1.0L) * P[l];
    }
}

#define ORC_LMAX_CAP 128

/* ------------------------------------------------------------------------ */
/* Truncated modified Green's function G~_L and its gradient in x            */
/* ------------------------------------------------------------------------ */

/*
 * Value of G~_L(x, y) and gradient with respect to x.  x_outer says which of
 * the two is r_> (it matters only for the gradient at an exact radius tie).
 * f[] are the image coefficients (f[0] unused: the l = 0 image cancels
 * against the floating-potential term Psi_sym(r) / (4 pi r'), Sec. 3).
 *
 * Every step runs in long double.  With the super-particle weight of Sec. 4
 * the field a particle feels is what is left after the pair sum and the ion
 * background cancel, and that remainder falls as N^-1/2 while the rounding
 * of each pair term does not; near-coincident pairs (r_x ~ r_y, xhat.yhat
 * ~ 1) carry the largest terms and the largest recurrence error, and in
 * double their rounding reaches 1e-12 of the RMS field at 1.6e7 particles.
 */
static void greens(const orc_params *p, const double *f, const double *x, const double *y,
                   int x_outer, long double *G, long double *grad)
{
    int L = p->l_max;
    long double rx = norm_ld(x);
    long double ry = norm_ld(y);
    long double xh[3] = {x[0] / rx, x[1] / rx, x[2] / rx};
    long double yh[3] = {y[0] / ry, y[1] / ry, y[2] / ry};
    long double P[ORC_LMAX_CAP + 1], dP[ORC_LMAX_CAP + 1];
    long double Py[ORC_LMAX_CAP + 1], dPy[ORC_LMAX_CAP + 1];
    long double gu[3];     /* gradient in x of the angular argument */
    int axisym = (p->m_mode == ORC_M_AXISYM);

    if (!axisym) {
        long double u = xh[0] * yh[0] + xh[1] * yh[1] + xh[2] * yh[2];
        legendre(u, L, P, dP);
        for (int j = 0; j < 3; ++j) gu[j] = (yh[j] - u * xh[j]) / rx;
    } else {
        long double cx = xh[2], cy = yh[2];
        legendre(cx, L, P, dP);
        legendre(cy, L, Py, dPy);
        for (int j = 0; j < 3; ++j) gu[j] = ((j == 2 ? 1.0L : 0.0L) - cx * xh[j]) / rx;
    }

    /* Radial factors by running products:
     *   x outer: r_<^l / r_>^(l+1) = rho^l / r_x,  d/dr_x = -(l+1) rho^l / r_x^2, rho = r_y/r_x
     *   x inner: r_<^l / r_>^(l+1) = rho^l / r_y,  d/dr_x = l rho^(l-1) / r_y^2,  rho = r_x/r_y
     *   image:   -f_l w^(l+1),  d/dr_x = (l+1) f_l w^(l+1) / r_x,               w = 1/(r_x r_y) */
    long double rho = x_outer ? ry / rx : rx / ry;
    long double w = 1.0L / (rx * ry);
    long double rho_l = 1.0L;      /* rho^l */
    long double rho_lm1 = 0.0L;    /* rho^(l-1), zero for l = 0 */
    long double w_l1 = w;          /* w^(l+1) */
    long double g = 0.0L;
    long double gr = 0.0L;   /* coefficient of xhat */
    long double ga = 0.0L;   /* coefficient of gu */
    for (int l = 0; l <= L; ++l) {
        long double ang, dang;
        if (!axisym) {
            ang = P[l];
            dang = dP[l];
        } else {
            ang = P[l] * Py[l];
            dang = dP[l] * Py[l];
        }
        long double dir, ddir;  /* direct term r_<^l / r_>^(l+1): value and d/d r_x */
        if (x_outer) {
            dir = rho_l / rx;
            ddir = -(l + 1.0L) * rho_l / (rx * rx);
        } else {
            dir = rho_l / ry;
            ddir = l * rho_lm1 / (ry * ry);
        }
        long double img = 0.0L, dimg = 0.0L;
        if (l >= 1) {
            img = -f[l] * w_l1;
            dimg = (l + 1.0L) * f[l] * w_l1 / rx;
        }
        g += (dir + img) * ang;
        gr += (ddir + dimg) * ang;
        ga += (dir + img) * dang;
        rho_lm1 = rho_l;
        rho_l *= rho;
        w_l1 *= w;
    }
    const long double four_pi = 4.0L * ORC_PIL;
    *G = g / four_pi;
    for (int j = 0; j < 3; ++j) grad[j] = (gr * xh[j] + ga * gu[j]) / four_pi;
}

/* Psi_anti,L and its gradient: sum over odd l <= L of c_l b^P_l r^-(l+1)
 * P_l(cos th) (Sec. 3; plasma region r >= R). */
static void psi_anti(const orc_params *p, const double *bP, const double *c, const double *x,
                     double *psi, double *grad)
{
    int L = p->l_max;
    double r = sqrt(key_r2(x));
    double xh[3] = {x[0] / r, x[1] / r, x[2] / r};
    double ct = xh[2];
    long double Pl[ORC_LMAX_CAP + 1], dPl[ORC_LMAX_CAP + 1];
    double P[ORC_LMAX_CAP + 1], dP[ORC_LMAX_CAP + 1];
    legendre(ct, L, Pl, dPl);
    for (int l = 0; l <= L; ++l) {
        P[l] = (double)Pl[l];
        dP[l] = (double)dPl[l];
    }
    double s = 0.0, sr = 0.0, sa = 0.0;
    for (int l = 1; l <= L; l += 2) {
        double w = c[l] * bP[l];
        s += w * P[l] / pow(r, l + 1);
        sr += -(l + 1.0) * w * P[l] / pow(r, l + 2);
        sa += w * dP[l] / pow(r, l + 1);
    }
    *psi = s;
    if (grad) {
        for (int j = 0; j < 3; ++j) {
            double gct = ((j == 2 ? 1.0 : 0.0) - ct * xh[j]) / r;
            grad[j] = sr * xh[j] + sa * gct;
        }
    }
}

/* int_a^b n(s) s^k ds over the profile, segment by segment with 3-point
 * Gauss-Legendre quadrature (exact: the integrand is a polynomial of degree
 * at most 3 on each segment). */
static double prof_moment(const orc_params *p, double a, double b, int k)
{
    static const double xg[3] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};
    static const double wg[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
    if (!(b > a)) return 0.0;
    const int64_t K = p->ion_prof_len - 1;
    const double h = (p->r_out - 1.0) / (double)K;
    long double acc = 0.0L;
    double lo = a;
    while (lo < b) {
        int64_t j = (int64_t)floor((lo - 1.0) / h);
        if (j < 0) j = 0;
        if (j > K - 1) j = K - 1;
        double hi = 1.0 + (double)(j + 1) * h;
        if (j == K - 1 || hi > b) hi = b;
        if (!(hi > lo)) hi = b;   /* guard against a node rounding onto lo */
        const double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
        for (int g = 0; g < 3; ++g) {
            const double s = mid + half * xg[g];
            const double t = (s - (1.0 + (double)j * h)) / h;
            const double n = p->ion_prof[j] * (1.0 - t) + p->ion_prof[j + 1] * t;
            acc += (long double)(wg[g] * half * n * (k == 2 ? s * s : s));
        }
        lo = hi;
    }
    return (double)acc;
}

/* Potential and field of the immobile ion background through the l = 0 part
 * of G~ (1/(4 pi r_>)): uniform density n_i on 1 < r < r_out, or the profile. */
static double phi_ion(const orc_params *p, double r)
{
    if (p->ion_prof)
        return prof_moment(p, 1.0, r, 2) / r + prof_moment(p, r, p->r_out, 1);
    double ni = p->ion_density, ro = p->r_out;
    return ni * ((r * r * r - 1.0) / (3.0 * r) + (ro * ro - r * r) / 2.0);
}

static double eion_r(const orc_params *p, double r)
{
    if (p->ion_prof) return prof_moment(p, 1.0, r, 2) / (r * r);
    return p->ion_density * (r * r * r - 1.0) / (3.0 * r * r);
}

/* ------------------------------------------------------------------------ */
/* Exported building blocks (used by the parity pins)                        */
/* ------------------------------------------------------------------------ */

int orc_greens(const orc_params *p, const double *x, const double *y, int x_outer,
               double *G, double *grad)
{
    if (p->l_max < 0 || p->l_max > ORC_LMAX_CAP) return -1;
    double f[ORC_LMAX_CAP + 1], bP[ORC_LMAX_CAP + 1], c[ORC_LMAX_CAP + 1];
    orc_coeffs(p->eps_r, p->d, p->l_max, f, bP, c);
    long double Gl, gl[3];
    greens(p, f, x, y, x_outer, &Gl, gl);
    *G = (double)Gl;
    for (int j = 0; j < 3; ++j) grad[j] = (double)gl[j];
    return 0;
}

/* Radial field and potential of the ion background at radius r. */
double orc_ion_field(const orc_params *p, double r, double *phi)
{
    if (phi) *phi = phi_ion(p, r);
    return eion_r(p, r);
}

int orc_psi_anti(const orc_params *p, const double *x, double *psi, double *grad)
{
    if (p->l_max < 0 || p->l_max > ORC_LMAX_CAP) return -1;
    double f[ORC_LMAX_CAP + 1], bP[ORC_LMAX_CAP + 1], c[ORC_LMAX_CAP + 1];
    orc_coeffs(p->eps_r, p->d, p->l_max, f, bP, c);
    psi_anti(p, bP, c, x, psi, grad);
    return 0;
}

/*
 * Field E_k = -grad Phi at every target k (targets == NULL: all particles),
 * equations of motion of Sec. 4 with the pair sum over alive i != k.
 * phi_out (optional) receives Phi at x_k without the self term.
 */
int orc_field(const orc_params *p, int64_t n, const double *pos, const uint32_t *ids,
              const uint8_t *alive, double q_surface, double u_asy,
              int64_t n_targets, const int64_t *targets, double *E_out, double *phi_out)
{
    if (p->l_max < 0 || p->l_max > ORC_LMAX_CAP) return -1;
    double f[ORC_LMAX_CAP + 1], bP[ORC_LMAX_CAP + 1], c[ORC_LMAX_CAP + 1];
    orc_coeffs(p->eps_r, p->d, p->l_max, f, bP, c);
    int64_t nt = targets ? n_targets : n;
    double inv_nt = 1.0 / p->ntilde;

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t k = targets ? targets[t] : t;
        double *E = E_out + 3 * t;
        if (alive && !alive[k]) {
            E[0] = E[1] = E[2] = 0.0;
            if (phi_out) phi_out[t] = 0.0;
            continue;
        }
        const double *xk = pos + 3 * k;
        double r2k = key_r2(xk);
        /* Extended-precision accumulators keep the oracle's own rounding far
         * below the parity tolerance when ~1e6 pair terms cancel against the
         * ion background. */
        long double gsum[3] = {0.0L, 0.0L, 0.0L};
        long double phi = 0.0L;
        for (int64_t i = 0; i < n; ++i) {
            if (i == k) continue;
            if (alive && !alive[i]) continue;
            const double *xi = pos + 3 * i;
            int k_outer = key_less(key_r2(xi), ids[i], r2k, ids[k]);
            long double G, g[3];
            greens(p, f, xk, xi, k_outer, &G, g);
            const double qi = charge_of(ids[i]);
            phi += qi * G;
            for (int j = 0; j < 3; ++j) gsum[j] += qi * g[j];
        }
        double rk = sqrt(r2k);
        long double rkl = norm_ld(xk);
        long double xh[3] = {xk[0] / rkl, xk[1] / rkl, xk[2] / rkl};
        double psi, gpsi[3];
        psi_anti(p, bP, c, xk, &psi, gpsi);
        /* Radial field of the surface charge and of the ions, also in long
         * double: it cancels the l = 0 part of the pair sum. */
        long double e_rad = (long double)q_surface / (p->ntilde * 4.0L * ORC_PIL * rkl * rkl);
        if (p->ion_prof)
            e_rad += (long double)eion_r(p, rk);
        else
            e_rad += p->ion_density * (rkl * rkl * rkl - 1.0L) / (3.0L * rkl * rkl);
        for (int j = 0; j < 3; ++j)
            E[j] = (double)(-gsum[j] / p->ntilde + e_rad * xh[j] -
                            (long double)(u_asy * gpsi[j]));
        if (phi_out)
            phi_out[t] = (double)((long double)inv_nt * phi +
                                  (long double)(inv_nt * q_surface / (4.0 * ORC_PI * rk)) +
                                  (long double)phi_ion(p, rk) + (long double)(u_asy * psi));
    }
    return 0;
}

/* Q_diff = -(1/nt) sum_i q_i Psi_anti,L(x_i)  (Sec. 4, truncated to odd l <= L). */
double orc_qdiff(const orc_params *p, int64_t n, const double *pos, const uint32_t *ids,
                 const uint8_t *alive)
{
    double f[ORC_LMAX_CAP + 1], bP[ORC_LMAX_CAP + 1], c[ORC_LMAX_CAP + 1];
    orc_coeffs(p->eps_r, p->d, p->l_max, f, bP, c);
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (alive && !alive[i]) continue;
        double psi;
        psi_anti(p, bP, c, pos + 3 * i, &psi, NULL);
        s += (ids ? charge_of(ids[i]) : ORC_Q) * psi;
    }
    return -s / p->ntilde;
}

/* ------------------------------------------------------------------------ */
/* Philox-4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) for diffuse walls      */
/* ------------------------------------------------------------------------ */

void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform double in (0, 1) from the top 53 bits of a 64-bit word. */
static double u01(uint64_t w)
{
    return ((double)(w >> 11) + 0.5) / 9007199254740992.0;
}

/*
 * Diffuse reflection (Sec. 4: same speed, random direction back into the
 * domain).  The angular law is not stated; the reading taken is uniform on
 * the hemisphere that points back into the domain.  Counter = (step, id,
 * wall, 0), key = (seed, 0).
 */
static void diffuse_dir(uint64_t seed, uint32_t id, int64_t step, int wall,
                        const double *nrm_in, double *dir)
{
    uint64_t ctr[4] = {(uint64_t)step, (uint64_t)id, (uint64_t)wall, 0};
    uint64_t key[2] = {seed, 0};
    uint64_t o[4];
    orc_philox4x64_10(ctr, key, o);
    double ct = u01(o[0]);               /* cos of the angle to the inward normal */
    double st = sqrt(1.0 - ct * ct);
    double ph = 2.0 * ORC_PI * u01(o[1]);
    /* orthonormal frame around the inward normal */
    const double *nz = nrm_in;
    double t[3];
    if (fabs(nz[2]) < 0.9) { t[0] = 0.0; t[1] = 0.0; t[2] = 1.0; }
    else { t[0] = 1.0; t[1] = 0.0; t[2] = 0.0; }
    double ex[3] = {t[1] * nz[2] - t[2] * nz[1], t[2] * nz[0] - t[0] * nz[2],
                    t[0] * nz[1] - t[1] * nz[0]};
    double ne = sqrt(ex[0] * ex[0] + ex[1] * ex[1] + ex[2] * ex[2]);
    for (int j = 0; j < 3; ++j) ex[j] /= ne;
    double ey[3] = {nz[1] * ex[2] - nz[2] * ex[1], nz[2] * ex[0] - nz[0] * ex[2],
                    nz[0] * ex[1] - nz[1] * ex[0]};
    for (int j = 0; j < 3; ++j)
        dir[j] = ct * nz[j] + st * (cos(ph) * ex[j] + sin(ph) * ey[j]);
}

/* Threads of the oracle's parallel loops (its CPU timing uses 1 and all). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* The diffuse-wall direction for a given inward unit normal, exported so
 * that its angular law can be checked on its own. */
void orc_diffuse_dir(uint64_t seed, uint32_t id, int64_t step, int wall, const double *nrm_in,
                     double *dir)
{
    diffuse_dir(seed, id, step, wall, nrm_in, dir);
}

/* ------------------------------------------------------------------------ */
/* Time stepping                                                             */
/* ------------------------------------------------------------------------ */

/*
 * One step n of the scheme (Sec. 4 equations of motion, leapfrog):
 *   Q_diff[n] at x^n; E at x^n with u_asy(t_n) and the current Q_S;
 *   v^{n+1/2} = v^{n-1/2} + (q/m) E dt;  x^{n+1} = x^n + v^{n+1/2} dt;
 *   boundaries tested on x^{n+1}: r <= 1 probe, r >= r_out wall.
 * E_scratch must hold 3 n doubles.  Returns the number absorbed.
 */
int64_t orc_step(const orc_params *p, int64_t n, double *pos, double *vel, const uint32_t *ids,
                 uint8_t *alive, double *q_surface, double u_asy, int64_t step,
                 double *qdiff_out, double *E_scratch)
{
    *qdiff_out = orc_qdiff(p, n, pos, ids, alive);
    orc_field(p, n, pos, ids, alive, *q_surface, u_asy, 0, NULL, E_scratch, NULL);
    int64_t absorbed = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (alive && !alive[k]) continue;
        double *x = pos + 3 * k, *v = vel + 3 * k;
        const double *E = E_scratch + 3 * k;
        const double qk = charge_of(ids[k]), qm = qk / mass_of(p, ids[k]);
        for (int j = 0; j < 3; ++j) v[j] = v[j] + qm * E[j] * p->dt;
        for (int j = 0; j < 3; ++j) x[j] = x[j] + v[j] * p->dt;
        double r = sqrt(key_r2(x));
        if (r <= 1.0) {
            if (p->probe_bc == ORC_BC_ABSORB) {
                alive[k] = 0;
                *q_surface += qk;
                ++absorbed;
            } else {
                double s = (2.0 - r) / r;
                double nrm[3] = {x[0] / r, x[1] / r, x[2] / r};
                for (int j = 0; j < 3; ++j) x[j] *= s;
                if (p->probe_bc == ORC_BC_SPECULAR) {
                    double vn = v[0] * nrm[0] + v[1] * nrm[1] + v[2] * nrm[2];
                    for (int j = 0; j < 3; ++j) v[j] = v[j] - 2.0 * vn * nrm[j];
                } else {
                    double sp = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                    double dir[3];
                    diffuse_dir(p->seed, ids[k], step, 0, nrm, dir);  /* inward = +rhat */
                    for (int j = 0; j < 3; ++j) v[j] = sp * dir[j];
                }
            }
        } else if (r >= p->r_out) {
            double s = (2.0 * p->r_out - r) / r;
            double nrm[3] = {x[0] / r, x[1] / r, x[2] / r};
            for (int j = 0; j < 3; ++j) x[j] *= s;
            if (p->wall_bc == ORC_BC_DIFFUSE) {
                double sp = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                double inw[3] = {-nrm[0], -nrm[1], -nrm[2]};
                double dir[3];
                diffuse_dir(p->seed, ids[k], step, 1, inw, dir);
                for (int j = 0; j < 3; ++j) v[j] = sp * dir[j];
            } else {
                double vn = v[0] * nrm[0] + v[1] * nrm[1] + v[2] * nrm[2];
                for (int j = 0; j < 3; ++j) v[j] = v[j] - 2.0 * vn * nrm[j];
            }
        }
    }
    return absorbed;
}

/* n_steps steps starting at absolute step start_step; u_asy and qdiff are
 * indexed by the absolute step.  Returns total absorbed or -1. */
int64_t orc_run(const orc_params *p, int64_t n, double *pos, double *vel, const uint32_t *ids,
                uint8_t *alive, double *q_surface, const double *u_asy, int64_t start_step,
                int64_t n_steps, double *qdiff)
{
    if (p->l_max < 0 || p->l_max > ORC_LMAX_CAP) return -1;
    double *E = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!E) return -1;
    int64_t tot = 0;
    for (int64_t s = start_step; s < start_step + n_steps; ++s)
        tot += orc_step(p, n, pos, vel, ids, alive, q_surface, u_asy[s], s, qdiff + s, E);
    free(E);
    return tot;
}

/*
 * Total energy H = sum 1/2 m v^2 + (1/2nt) sum_k sum_{i!=k} q q G~ + sum_k q
 * [ (1/nt) Q_S / (4 pi r_k) + Phi_ion(r_k) ] + sum_k q u Psi_anti (Sec. 2
 * Hamiltonian in the scaling of Sec. 4).  v2 holds per-particle v.v (the
 * caller forms the leapfrog average).
 */
double orc_energy(const orc_params *p, int64_t n, const double *pos, const double *v2,
                  const uint32_t *ids, const uint8_t *alive, double q_surface, double u_asy,
                  double *kinetic_out, double *potential_out)
{
    double *phi = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *E = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    orc_field(p, n, pos, ids, alive, 0.0, 0.0, 0, NULL, E, phi);
    double f[ORC_LMAX_CAP + 1], bP[ORC_LMAX_CAP + 1], c[ORC_LMAX_CAP + 1];
    orc_coeffs(p->eps_r, p->d, p->l_max, f, bP, c);
    double ke = 0.0, pe = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        if (alive && !alive[k]) continue;
        double r = sqrt(key_r2(pos + 3 * k));
        double pair = phi[k] - phi_ion(p, r);   /* phi was built with Q_S = u = 0 */
        double psi;
        psi_anti(p, bP, c, pos + 3 * k, &psi, NULL);
        const double qk = charge_of(ids[k]);
        ke += 0.5 * mass_of(p, ids[k]) * v2[k];
        pe += 0.5 * qk * pair +
              qk * (q_surface / (p->ntilde * 4.0 * ORC_PI * r) + phi_ion(p, r) + u_asy * psi);
    }
    free(phi);
    free(E);
    if (kinetic_out) *kinetic_out = ke;
    if (potential_out) *potential_out = pe;
    return ke + pe;
}
