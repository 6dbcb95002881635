/*
 * qed_oracle.c -- FP64 CPU oracle for the per-particle QED event generator of a
 * QED-PIC step (Volokitin et al., "Optimized routines for event generators in
 * QED-PIC codes", arXiv:2008.10468).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which only
 * the test suite, the package smoke check and the CPU-baseline leg of the
 * benchmark load.  The GPU library never links, includes or calls it, and it
 * shares no code, header, table or constant generator with the GPU library.
 *
 * Everything is plain, slow and written to be checked against the paper by eye:
 *   - Philox4x32-10 from its published definition (Salmon et al., SC'11);
 *   - synchrotron functions F(x) = x * int_x^inf K_{5/3} and G(x) = x K_{2/3}
 *     (Sec. 3.2.1) by the trapezoid rule on the integral representation
 *     K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt (DLMF 10.32.9);
 *   - the emission density P(delta) of eq. (1) and the pair density P_p of
 *     eq. (2) with its bracket sign corrected (see orc_pp);
 *   - the sub-step bounds f(b) of Sec. 3.1.1 exactly as printed;
 *   - Algorithm 1 (charged particles) and Algorithm 2 (photons) in the order
 *     push -> chi -> sample (x, y) -> accept test -> event.
 *
 * Units: time in hbar/(m c^2), lengths in hbar/(m c), momenta u = p/(m c) for
 * e-/e+ and k = hbar k/(m c) for photons, E and B in units of the Schwinger
 * field.  The prefactor [dt e^2 m c / hbar^2] of eqs. (1)-(2) becomes alpha*dt.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ALPHA 7.2973525693e-3 /* fine-structure constant, CODATA 2018 */
#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  One round maps the     */
/* counter (c0,c1,c2,c3) with round key (k0,k1) to                            */
/*   (hi(M1*c2)^c1^k0, lo(M1*c2), hi(M0*c0)^c3^k1, lo(M0*c0));                */
/* the key is bumped by the Weyl constants between rounds.                    */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Uniform in (0,1), 53-bit: k = top 52 bits of (hi:lo), value (2k+1) 2^-53. */
double orc_u53(uint32_t hi, uint32_t lo)
{
    uint64_t k = (((uint64_t)hi << 32) | (uint64_t)lo) >> 12;
    return ((double)(2 * k + 1)) * 0x1p-53;
}

/* Uniform in (0,1), 24-bit: k = top 23 bits of w, value (2k+1) 2^-24. */
double orc_u24(uint32_t w)
{
    uint32_t k = w >> 9;
    return ((double)(2 * k + 1)) * 0x1p-24;
}

/* Random-number layout of the generator (an interface of this library, not of
 * the paper): the counter is (id_lo, id_hi, step, j) under key (seed_lo, seed_hi).
 *   53-bit mode (FP64 path):  j = i, x from words (0,1), y from words (2,3);
 *   24-bit mode (mixed path): j = i/2; even i takes x=w0, y=w1, odd i x=w2, y=w3. */
void orc_draw_xy(uint64_t seed, uint64_t id, uint32_t step, uint32_t i, int rng_bits,
                 double *x, double *y)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    if (rng_bits == 53) {
        uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), step, i};
        orc_philox4x32_10(ctr, key, w);
        *x = orc_u53(w[0], w[1]);
        *y = orc_u53(w[2], w[3]);
    } else {
        uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), step, i / 2};
        orc_philox4x32_10(ctr, key, w);
        if ((i % 2) == 0) {
            *x = orc_u24(w[0]);
            *y = orc_u24(w[1]);
        } else {
            *x = orc_u24(w[2]);
            *y = orc_u24(w[3]);
        }
    }
}

/* Identity of a child particle: Philox under the seed key xor'ed with the fixed
 * tag (0x5851F42D, 0x4C957F2D), counter (parent_lo, parent_hi, step, 2 i + slot);
 * the id is words 0 (low half) and 1 (high half).  slot 0 = emitted photon or
 * pair electron, slot 1 = pair positron. */
uint64_t orc_child_id(uint64_t seed, uint64_t parent, uint32_t step, uint32_t i, uint32_t slot)
{
    uint32_t key[2] = {(uint32_t)seed ^ 0x5851F42Du, (uint32_t)(seed >> 32) ^ 0x4C957F2Du};
    uint32_t ctr[4] = {(uint32_t)parent, (uint32_t)(parent >> 32), step, 2 * i + slot};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    return ((uint64_t)w[1] << 32) | (uint64_t)w[0];
}

/* ------------------------------------------------------------------------- */
/* Synchrotron functions (Sec. 3.2.1).                                        */
/*   F(x) = x int_x^inf K_{5/3}(s) ds = x int_0^inf e^{-x cosh t} cosh(5t/3)/cosh t dt
 *   G(x) = x K_{2/3}(x)            = x int_0^inf e^{-x cosh t} cosh(2t/3) dt
 * (the first by exchanging the order of integration in DLMF 10.32.9).
 * Both integrands are even and analytic in a strip around the real axis, so the
 * trapezoid rule on [0, inf) converges exponentially (Trefethen & Weideman,
 * SIAM Review 2014).  The factor e^{-x} is taken out and cosh t - 1 is written
 * as 2 sinh^2(t/2) so that large x keeps full relative accuracy.  The step
 * h = min(0.2, 0.4/sqrt(x)) follows the width of the peak at t = 0.          */
/* ------------------------------------------------------------------------- */
void orc_synchrotron(double x, double *F, double *G)
{
    if (isnan(x) || x < 0.0) {
        *F = NAN;
        *G = NAN;
        return;
    }
    if (x == 0.0 || isinf(x)) {
        *F = 0.0;
        *G = 0.0;
        return;
    }
    double h = 0.2;
    if (0.4 / sqrt(x) < h) h = 0.4 / sqrt(x);
    /* t = 0 term, half weight */
    double sF = 0.5, sG = 0.5;
    for (int k = 1; k < 100000; ++k) {
        double t = k * h;
        double sh = sinh(0.5 * t);
        double damp = exp(-x * 2.0 * sh * sh);
        double tF = damp * cosh(5.0 * t / 3.0) / cosh(t);
        double tG = damp * cosh(2.0 * t / 3.0);
        sF += tF;
        sG += tG;
        if (x * 2.0 * sh * sh > 40.0 && tF < 1e-19 * sF && tG < 1e-19 * sG) break;
    }
    double pre = x * exp(-x) * h;
    *F = pre * sF;
    *G = pre * sG;
}

double orc_F1(double x)
{
    double F, G;
    orc_synchrotron(x, &F, &G);
    return F;
}

double orc_F2(double x)
{
    double F, G;
    orc_synchrotron(x, &F, &G);
    return G;
}

/* ------------------------------------------------------------------------- */
/* Quantum parameters (eq. (1) text and eq. (2) text).                        */
/*   chi   = sqrt((gamma E + u x B)^2 - (u . E)^2)        for e-/e+            */
/*   chi_g = sqrt((eps E + k x B)^2 - (k . E)^2), eps=|k|  for photons         */
/* ------------------------------------------------------------------------- */
static double chi_generic(double energy, const double p[3], const double E[3], const double B[3])
{
    double cx = p[1] * B[2] - p[2] * B[1];
    double cy = p[2] * B[0] - p[0] * B[2];
    double cz = p[0] * B[1] - p[1] * B[0];
    double ax = energy * E[0] + cx;
    double ay = energy * E[1] + cy;
    double az = energy * E[2] + cz;
    double pe = p[0] * E[0] + p[1] * E[1] + p[2] * E[2];
    double s = ax * ax + ay * ay + az * az - pe * pe;
    return s > 0.0 ? sqrt(s) : 0.0;
}

double orc_chi_lepton(const double u[3], const double E[3], const double B[3])
{
    double gamma = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    return chi_generic(gamma, u, E, B);
}

double orc_chi_photon(const double k[3], const double E[3], const double B[3])
{
    double eps = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    return chi_generic(eps, k, E, B);
}

/* ------------------------------------------------------------------------- */
/* Sub-step bounds (Sec. 3.1.1).                                              */
/* Emission: b = 3 chi / 2, c = sqrt(3) alpha dt / (pi gamma), and the four-   */
/* piece f(b).  The printed ranges leave b = 0.1, 0.5, 10 unassigned; each    */
/* breakpoint is given to the piece above it.                                 */
/* ------------------------------------------------------------------------- */
double orc_bound_emission(double chi, double gamma, double dt)
{
    double b = 1.5 * chi;
    double c = sqrt(3.0) * ORC_ALPHA * dt / (ORC_PI * gamma);
    double f;
    if (b < 0.1)
        f = 0.56 * ORC_PI * c * b + 0.1 * c * b;
    else if (b < 0.5)
        f = 0.45 * ORC_PI * c * pow(b, 11.0 / 12.0) + 0.1 * c * b;
    else if (b < 10.0)
        f = 0.42 * ORC_PI * c * pow(b, 19.0 / 24.0) + 0.1 * c * b;
    else
        f = 0.55 * ORC_PI * c * pow(b, 2.0 / 3.0) + 0.1 * c * b;
    return f;
}

/* Pair bound f = coef * c * b (printed with coef = 0.1), with b = 3 chi_g / 2
 * and c = sqrt(3) alpha dt / (pi eps_g): the emission definitions with the
 * photon energy in place of gamma. */
double orc_bound_pair(double chi_g, double eps_g, double dt, double coef)
{
    double b = 1.5 * chi_g;
    double c = sqrt(3.0) * ORC_ALPHA * dt / (ORC_PI * eps_g);
    return coef * c * b;
}

/* Number of sub-steps: the smallest N >= 1 with f / N <= p_max, capped. */
uint32_t orc_nsub(double f, double p_max, uint32_t n_cap)
{
    double r = ceil(f / p_max);
    if (!(r >= 1.0)) r = 1.0;
    if (r > (double)n_cap) r = (double)n_cap;
    return (uint32_t)r;
}

/* ------------------------------------------------------------------------- */
/* Rates.                                                                     */
/* Emission, eq. (1):                                                         */
/*   P(delta) = alpha dt sqrt(3)/(2 pi) (chi/gamma) (1-delta)/delta            */
/*              * (F(z_q) + 3/2 delta chi z_q G(z_q)),  z_q = 2/3 delta/(chi (1-delta)),
 * and Algorithm 1 accepts y < P_m(x) = 3 x^2 P(x^3).                          */
/* 1 - x^3 is formed as (1-x)(1+x+x^2) so that it keeps relative accuracy.     */
/* ------------------------------------------------------------------------- */
double orc_pm(double x, double chi, double gamma, double dt)
{
    if (!(chi > 0.0)) return 0.0;
    double delta = x * x * x;
    double omd = (1.0 - x) * (1.0 + x + x * x);
    double zq = (2.0 / 3.0) * delta / (chi * omd);
    double F, G;
    orc_synchrotron(zq, &F, &G);
    double P = ORC_ALPHA * dt * sqrt(3.0) / (2.0 * ORC_PI) * (chi / gamma) * (omd / delta) *
               (F + 1.5 * delta * chi * zq * G);
    return 3.0 * x * x * P;
}

/* Pair creation, eq. (2):
 *   P_p(d) = alpha dt sqrt(3)/(2 pi) (chi_g/eps_g) (1-d) d * (3/2 chi_g z_p G(z_p) - F(z_p)),
 *   z_p = 2/3 / (chi_g (1-d) d).
 * As printed the bracket reads F - 3/2 chi_g z_p G.  Since 3/2 chi_g z_p =
 * 1/(d(1-d)) >= 4 and F(z) = 2 G(z) - z int_z^inf K_{1/3} < 2 G(z) (DLMF 10.29.1),
 * that order is negative for every d; the two terms are swapped here.  With
 * this order the density equals the Baier-Katkov pair spectrum (checked in the
 * tests). */
double orc_pp(double x, double chi_g, double eps_g, double dt)
{
    if (!(chi_g > 0.0) || !(eps_g > 0.0)) return 0.0;
    double d = x;
    double zp = (2.0 / 3.0) / (chi_g * (1.0 - d) * d);
    double F, G;
    orc_synchrotron(zp, &F, &G);
    return ORC_ALPHA * dt * sqrt(3.0) / (2.0 * ORC_PI) * (chi_g / eps_g) * (1.0 - d) * d *
           (1.5 * chi_g * zp * G - F);
}

/* ------------------------------------------------------------------------- */
/* Boris pusher (Boris 1970; textbook form), du/dt = q (E + u x B / gamma).   */
/* ------------------------------------------------------------------------- */
void orc_boris(double u[3], const double E[3], const double B[3], double q, double dt)
{
    double h = 0.5 * q * dt;
    double um[3] = {u[0] + h * E[0], u[1] + h * E[1], u[2] + h * E[2]};
    double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    double t[3] = {h * B[0] / gm, h * B[1] / gm, h * B[2] / gm};
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    double s[3] = {2.0 * t[0] / (1.0 + t2), 2.0 * t[1] / (1.0 + t2), 2.0 * t[2] / (1.0 + t2)};
    double up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]), um[1] + (um[2] * t[0] - um[0] * t[2]),
                    um[2] + (um[0] * t[1] - um[1] * t[0])};
    double pl[3] = {um[0] + (up[1] * s[2] - up[2] * s[1]), um[1] + (up[2] * s[0] - up[0] * s[2]),
                    um[2] + (up[0] * s[1] - up[1] * s[0])};
    u[0] = pl[0] + h * E[0];
    u[1] = pl[1] + h * E[1];
    u[2] = pl[2] + h * E[2];
}

/* ------------------------------------------------------------------------- */
/* One global step of Algorithm 1 for a batch of e- (q=-1) or e+ (q=+1).       */
/* ------------------------------------------------------------------------- */
typedef struct {
    double dt;        /* global step */
    double p_max;     /* target event probability per sub-step */
    double pair_coef; /* coefficient of the pair bound (0.1 as printed) */
    uint64_t seed;
    uint32_t step;    /* global step index, Philox counter word 2 */
    uint32_t n_cap;   /* cap on the number of sub-steps */
    int32_t rng_bits; /* 53 or 24 */
    int32_t pad;
} orc_params;

typedef struct {
    int64_t cap; /* capacity of the child arrays */
    int64_t n;   /* children written (or needed, if > cap) */
    double *x, *y, *z, *px, *py, *pz, *w;
    uint64_t *id, *parent;
    uint32_t *sub;  /* sub-step index of the event */
    int32_t *kind;  /* 0 photon, 1 electron, 2 positron */
    double *tb;     /* birth time within the step (end of the event's sub-step) */
} orc_children;

typedef struct {
    uint64_t substeps, events, clips;
    double max_p;
} orc_tally;

static void push_child(orc_children *c, const double pos[3], const double p[3], double w,
                       uint64_t id, uint64_t parent, uint32_t sub, int kind, double tb)
{
    int64_t j = c->n++;
    if (j >= c->cap) return;
    c->tb[j] = tb;
    c->x[j] = pos[0];
    c->y[j] = pos[1];
    c->z[j] = pos[2];
    c->px[j] = p[0];
    c->py[j] = p[1];
    c->pz[j] = p[2];
    c->w[j] = w;
    c->id[j] = id;
    c->parent[j] = parent;
    c->sub[j] = sub;
    c->kind[j] = kind;
}

static int all_finite(const double *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Returns 0, or -1 if the particle had non-finite input and was left alone.
 * t0: the time within the step at which the particle starts (0 for particles
 * present at the step start; the birth time of a child in a cascade pass); it
 * runs Algorithm 1 over the remaining time dt - t0.  nforce: 0, or the number of
 * sub-steps to take instead of the particle's own (a sub-step chosen for the
 * particle's cell). */
static int lepton_one(const orc_params *P, double t0, double q, double u[3], double pos[3], double w,
                      uint64_t id, const double E[3], const double B[3], uint32_t nforce, uint32_t *nsub_out,
                      uint32_t *nev_out, orc_children *ch, orc_tally *tl)
{
    if (!all_finite(u, 3) || !all_finite(E, 3) || !all_finite(B, 3)) {
        *nsub_out = 0;
        *nev_out = 0;
        return -1;
    }
    /* Algorithm 1: sub-step from the bound at the step start. */
    double gamma0 = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double chi0 = orc_chi_lepton(u, E, B);
    double dt = P->dt - t0;
    uint32_t N = orc_nsub(orc_bound_emission(chi0, gamma0, dt), P->p_max, P->n_cap);
    if (nforce) N = nforce;
    double st = dt / (double)N;
    uint32_t nev = 0;
    for (uint32_t i = 0; i < N; ++i) {
        /* push: Boris rotation by st in the frozen field, then move */
        orc_boris(u, E, B, q, st);
        double gamma = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        pos[0] += u[0] / gamma * st;
        pos[1] += u[1] / gamma * st;
        pos[2] += u[2] / gamma * st;
        /* quantum parameter after the push */
        double chi = orc_chi_lepton(u, E, B);
        /* draw the candidate x and the test value y */
        double x, y;
        orc_draw_xy(P->seed, id, P->step, i, P->rng_bits, &x, &y);
        /* acceptance test against eq. (1) */
        double pm = orc_pm(x, chi, gamma, st);
        if (pm > tl->max_p) tl->max_p = pm;
        if (pm > 1.0) tl->clips++;
        if (y < pm) {
            /* emission: photon of energy fraction delta = x^3 along u, same weight;
             * the parent keeps its direction and loses the photon energy. */
            double delta = x * x * x;
            double umag = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            double dir[3] = {0.0, 0.0, 0.0};
            if (umag > 0.0) {
                dir[0] = u[0] / umag;
                dir[1] = u[1] / umag;
                dir[2] = u[2] / umag;
            }
            double eph = delta * gamma;
            double k[3] = {eph * dir[0], eph * dir[1], eph * dir[2]};
            push_child(ch, pos, k, w, orc_child_id(P->seed, id, P->step, i, 0), id, i, 0,
                       t0 + (double)(i + 1) * st);
            double g1 = (1.0 - delta) * gamma;
            double u1 = g1 * g1 - 1.0;
            u1 = u1 > 0.0 ? sqrt(u1) : 0.0;
            u[0] = u1 * dir[0];
            u[1] = u1 * dir[1];
            u[2] = u1 * dir[2];
            nev++;
        }
    }
    tl->substeps += N;
    tl->events += nev;
    *nsub_out = N;
    *nev_out = nev;
    return 0;
}

/* Algorithm 2 for one photon.  Returns 1 if it decayed, 0 if it survived,
 * -1 for non-finite input (left alone, alive).  nforce as for lepton_one. */
static int photon_one(const orc_params *P, double t0, double k[3], double pos[3], double w, uint64_t id,
                      const double E[3], const double B[3], uint32_t nforce, uint32_t *nsub_out,
                      uint32_t *nev_out, orc_children *ch, orc_tally *tl)
{
    if (!all_finite(k, 3) || !all_finite(E, 3) || !all_finite(B, 3)) {
        *nsub_out = 0;
        *nev_out = 0;
        return -1;
    }
    double eps = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    double chi0 = orc_chi_photon(k, E, B);
    double dt = P->dt - t0;
    uint32_t N = 1;
    if (eps > 0.0) N = orc_nsub(orc_bound_pair(chi0, eps, dt, P->pair_coef), P->p_max, P->n_cap);
    if (nforce) N = nforce;
    double st = dt / (double)N;
    double dir[3] = {0.0, 0.0, 0.0};
    if (eps > 0.0) {
        dir[0] = k[0] / eps;
        dir[1] = k[1] / eps;
        dir[2] = k[2] / eps;
    }
    uint32_t used = 0;
    int decayed = 0;
    for (uint32_t i = 0; i < N; ++i) {
        used++;
        /* move: straight line at the speed of light */
        pos[0] += dir[0] * st;
        pos[1] += dir[1] * st;
        pos[2] += dir[2] * st;
        /* photon quantum parameter */
        double chi = orc_chi_photon(k, E, B);
        /* draw the candidate x and the test value y */
        double x, y;
        orc_draw_xy(P->seed, id, P->step, i, P->rng_bits, &x, &y);
        /* acceptance test against eq. (2) */
        double pp = orc_pp(x, chi, eps, st);
        if (pp > tl->max_p) tl->max_p = pp;
        if (pp > 1.0) tl->clips++;
        if (y < pp) {
            /* pair creation: electron takes energy fraction x, positron 1-x, both
             * along the photon, same weight; the photon is deleted. */
            double ge = x * eps, gp = (1.0 - x) * eps;
            double ue = ge * ge - 1.0, up = gp * gp - 1.0;
            ue = ue > 0.0 ? sqrt(ue) : 0.0;
            up = up > 0.0 ? sqrt(up) : 0.0;
            double pe[3] = {ue * dir[0], ue * dir[1], ue * dir[2]};
            double pq[3] = {up * dir[0], up * dir[1], up * dir[2]};
            double tb = t0 + (double)(i + 1) * st;
            push_child(ch, pos, pe, w, orc_child_id(P->seed, id, P->step, i, 0), id, i, 1, tb);
            push_child(ch, pos, pq, w, orc_child_id(P->seed, id, P->step, i, 1), id, i, 2, tb);
            decayed = 1;
            break;
        }
    }
    tl->substeps += used;
    tl->events += (uint64_t)decayed;
    *nsub_out = used;
    *nev_out = (uint32_t)decayed;
    return decayed;
}

/* Batch drivers.  Fields are six arrays (Ex,Ey,Ez,Bx,By,Bz) read at index
 * i*fstride (fstride 0: one field for all).  t0 (may be NULL: all zero) gives each
 * particle's start time within the step; nforce (may be NULL: all zero) forced
 * sub-step counts (0: the particle's own).  Children are appended in particle
 * order, then sub-step order.  Return value: number of non-finite particles. */
int64_t orc_lepton_batch(const orc_params *P, double q, int64_t n, double *ux, double *uy, double *uz,
                         double *x, double *y, double *z, const double *w, const uint64_t *id,
                         const double *t0, const double *const fld[6], int64_t fstride, uint32_t *nsub,
                         uint32_t *nev, orc_children *ch, orc_tally *tl, const uint32_t *nforce)
{
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t f = i * fstride;
        double E[3] = {fld[0][f], fld[1][f], fld[2][f]};
        double B[3] = {fld[3][f], fld[4][f], fld[5][f]};
        double u[3] = {ux[i], uy[i], uz[i]};
        double pos[3] = {x[i], y[i], z[i]};
        if (lepton_one(P, t0 ? t0[i] : 0.0, q, u, pos, w[i], id[i], E, B, nforce ? nforce[i] : 0u, &nsub[i],
                       &nev[i], ch, tl) < 0) {
            bad++;
            continue;
        }
        ux[i] = u[0];
        uy[i] = u[1];
        uz[i] = u[2];
        x[i] = pos[0];
        y[i] = pos[1];
        z[i] = pos[2];
    }
    return bad;
}

int64_t orc_photon_batch(const orc_params *P, int64_t n, double *kx, double *ky, double *kz, double *x,
                         double *y, double *z, const double *w, const uint64_t *id, const double *t0,
                         const double *const fld[6], int64_t fstride, uint8_t *alive, uint32_t *nsub,
                         uint32_t *nev, orc_children *ch, orc_tally *tl, const uint32_t *nforce)
{
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t f = i * fstride;
        double E[3] = {fld[0][f], fld[1][f], fld[2][f]};
        double B[3] = {fld[3][f], fld[4][f], fld[5][f]};
        double k[3] = {kx[i], ky[i], kz[i]};
        double pos[3] = {x[i], y[i], z[i]};
        int r = photon_one(P, t0 ? t0[i] : 0.0, k, pos, w[i], id[i], E, B, nforce ? nforce[i] : 0u, &nsub[i],
                           &nev[i], ch, tl);
        if (r < 0) {
            bad++;
            alive[i] = 1;
            continue;
        }
        alive[i] = (uint8_t)(r == 0);
        x[i] = pos[0];
        y[i] = pos[1];
        z[i] = pos[2];
    }
    return bad;
}

/* ------------------------------------------------------------------------- */
/* Integrals over the candidate variable x in (0,1), by adaptive Gauss-       */
/* Legendre: a panel is accepted when the 24-point rule on it agrees with the */
/* sum of the rules on its halves.  Nodes come from Newton's iteration on     */
/* P_24 (textbook construction, computed once).                               */
/* ------------------------------------------------------------------------- */
#define GL_N 24
static double gl_x[GL_N], gl_w[GL_N];
static int gl_ready = 0;

static void gl_init(void)
{
    if (gl_ready) return;
    for (int i = 0; i < GL_N; ++i) {
        double z = cos(ORC_PI * (i + 0.75) / (GL_N + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int j = 1; j <= GL_N; ++j) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
            }
            double dp = GL_N * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) {
                gl_x[i] = z;
                gl_w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
                break;
            }
        }
    }
    gl_ready = 1;
}

typedef double (*orc_fx)(double x, const double *par);

static double gl_panel(orc_fx f, const double *par, double a, double b)
{
    double m = 0.5 * (a + b), r = 0.5 * (b - a), s = 0.0;
    for (int i = 0; i < GL_N; ++i) s += gl_w[i] * f(m + r * gl_x[i], par);
    return s * r;
}

static double gl_adapt(orc_fx f, const double *par, double a, double b, double whole, double tol, int depth)
{
    double m = 0.5 * (a + b);
    double l = gl_panel(f, par, a, m), r = gl_panel(f, par, m, b);
    if (depth >= 40 || fabs(l + r - whole) <= tol) return l + r;
    return gl_adapt(f, par, a, m, l, 0.5 * tol, depth + 1) + gl_adapt(f, par, m, b, r, 0.5 * tol, depth + 1);
}

static double integrate01(orc_fx f, const double *par, double lo, double hi, double rel)
{
    gl_init();
    /* start from 16 panels so the adaptivity sees features near x -> 1 */
    double total = 0.0;
    double est = 0.0;
    for (int j = 0; j < 16; ++j) est += fabs(gl_panel(f, par, lo + (hi - lo) * j / 16.0, lo + (hi - lo) * (j + 1) / 16.0));
    double tol = rel * est / 16.0 + 1e-300;
    for (int j = 0; j < 16; ++j) {
        double a = lo + (hi - lo) * j / 16.0, b = lo + (hi - lo) * (j + 1) / 16.0;
        total += gl_adapt(f, par, a, b, gl_panel(f, par, a, b), tol, 0);
    }
    return total;
}

static double f_pm(double x, const double *p) { return orc_pm(x, p[0], p[1], p[2]); }
static double f_pm_clip(double x, const double *p)
{
    double v = orc_pm(x, p[0], p[1], p[2]);
    return v < 1.0 ? v : 1.0;
}
static double f_pm_energy(double x, const double *p) { return x * x * x * orc_pm(x, p[0], p[1], p[2]); }
static double f_pp(double x, const double *p) { return orc_pp(x, p[0], p[1], p[2]); }
static double f_pp_clip(double x, const double *p)
{
    double v = orc_pp(x, p[0], p[1], p[2]);
    return v < 1.0 ? v : 1.0;
}

/* Per-(sub)step emission probability int_0^1 P_m(x) dx (the left side of the
 * bound of Sec. 3.1.1), and the same with P_m clipped at 1 (the acceptance
 * probability of one sub-step of Algorithm 1). */
double orc_emission_prob(double chi, double gamma, double dt, int clip)
{
    double par[3] = {chi, gamma, dt};
    return integrate01(clip ? f_pm_clip : f_pm, par, 0.0, 1.0, 1e-13);
}

/* Mean energy fraction times probability: int_0^1 x^3 P_m(x) dx. */
double orc_emission_energy(double chi, double gamma, double dt)
{
    double par[3] = {chi, gamma, dt};
    return integrate01(f_pm_energy, par, 0.0, 1.0, 1e-13);
}

/* Normalised emission spectrum CDF in delta: C(delta) = int_0^{delta^(1/3)} P_m / int_0^1 P_m. */
double orc_emission_cdf(double chi, double delta)
{
    double par[3] = {chi, 1.0, 1.0};
    double tot = integrate01(f_pm, par, 0.0, 1.0, 1e-13);
    double xc = cbrt(delta);
    if (xc <= 0.0) return 0.0;
    if (xc >= 1.0) return 1.0;
    return integrate01(f_pm, par, 0.0, xc, 1e-13) / tot;
}

double orc_pair_prob(double chi_g, double eps_g, double dt, int clip)
{
    double par[3] = {chi_g, eps_g, dt};
    return integrate01(clip ? f_pp_clip : f_pp, par, 0.0, 1.0, 1e-13);
}

/* Normalised energy-split CDF of pair creation (eq. (2)): the probability that the
 * electron takes an energy fraction below x, int_0^x P_p / int_0^1 P_p. */
double orc_pair_cdf(double chi_g, double x)
{
    double par[3] = {chi_g, 1.0, 1.0};
    if (x <= 0.0) return 0.0;
    if (x >= 1.0) return 1.0;
    double tot = integrate01(f_pp, par, 0.0, 1.0, 1e-13);
    return integrate01(f_pp, par, 0.0, x, 1e-13) / tot;
}

/* Vectorised helpers for the Python side. */
void orc_synchrotron_vec(int64_t n, const double *x, double *F, double *G)
{
    for (int64_t i = 0; i < n; ++i) orc_synchrotron(x[i], &F[i], &G[i]);
}

void orc_philox_vec(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}
