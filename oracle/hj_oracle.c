/*
 * hj_oracle.c -- plain FP64 CPU reference solver for the explicit level-set
 * time step of arXiv 2507.11542 (LevelSetPy).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library: every formula below is
 * written out again from the paper (and, where the paper defers to it, from
 * Osher & Fedkiw, "Level Set Methods and Dynamic Implicit Surfaces").
 *
 * What it computes (paper section in brackets):
 *   - grid nodes and ghost values                        [Sec. 2.1, Fig. 3]
 *   - one-sided derivatives p-/p+ per axis:
 *       first order upwind                               [Sec. 3, eq. (fwd_bck_differencing), Sec. 3.1]
 *       ENO2 from the divided-difference table           [Sec. 3.2]
 *       ENO3 (third divided differences, the c* choice)  [Sec. 3.2, ENO3 paragraph]
 *       WENO5 (Jiang-Peng weights)                       [Sec. 3.3]
 *   - Lax-Friedrichs numerical Hamiltonian               [Sec. 4, LF equation]
 *     with the dissipation coefficients of reading R4 (LF), or per node over
 *     the node's own costate box (LLF) or the grid-wide box (GLF)
 *                                                        [Sec. 4, dissFunc(dL, dR)]
 *   - dissipation alpha_i = max over nodes of |dH/dp_i| bound, CFL dt [Sec. 4]
 *   - TVD Runge-Kutta 1/2/3 and the CFL time loop        [Sec. 5, odeCFL3 listing]
 *   - tube update V <- min(V, V0) after each step        [Sec. 6.1 BRT]
 *   - tube as the variational inequality: the update of every stage
 *     restricted to non-increasing values                [Sec. 6.1, the min[0,H] form]
 *   - tube update at output times only, output times    [Sec. 6.1, the global steps]
 *   - the rockets launch game (x, z, theta)              [Sec. 6.1, eq. ham_def]
 *   - implicit-surface initial value functions: sphere, cylinder, box,
 *     ellipsoid, combined by union / intersection / difference  [Sec. 2.2, Fig. 4]
 *
 * Readings where the paper is silent or garbled (all are also listed in the
 * design notes):
 *   R1  D- v_i = (v_i - v_{i-1})/dx, D+ v_i = (v_{i+1} - v_i)/dx; the printed
 *       difference equation has the labels swapped, the upwind rule of Sec. 3.1
 *       (use D- when the speed is positive) fixes the direction.
 *   R2  ENO2: D1_{k+1/2} = (v_{k+1}-v_k)/dx, D2_k = (D1_{k+1/2}-D1_{k-1/2})/(2dx)
 *       (computed with the reciprocals 1/dx and 1/(2dx));
 *       p- = D1_{i-1/2} + dx*m(D2_{i-1}, D2_i), p+ = D1_{i+1/2} - dx*m(D2_i, D2_{i+1}),
 *       m(a,b) = a if |a| <= |b| else b (the <= tie rule printed for ENO3).
 *   R3  WENO5: Jiang-Peng with eps = 1e-6*max(v_k^2) + 1e-99.
 *   R25 dissipation variants: alpha_d(x) = max over p in a costate box B and
 *       over the controls of |dH/dp_d(x, p)|, with B the node's own
 *       [min(p-, p+), max(p-, p+)] per axis (LLF) or the same over the whole
 *       grid and both one-sided derivatives (GLF, the box of the dissFunc
 *       (dL, dR) arguments); a switching function s = a.p (+ const) may take
 *       the sign +1 where its interval's upper end is >= 0 and -1 where its
 *       lower end is <= 0 (interval ends in axis order); the step size keeps
 *       the control-set bound of R4, which bounds every box value, so the
 *       schedule stays independent of V.
 *   R24 ENO3 (Osher-Fedkiw's HJ ENO3, which the paper follows):
 *       D3_{j+1/2} = (D2_{j+1} - D2_j)/(3dx) (with the reciprocal 1/(3dx));
 *       k = i-1 for p-, k = i for p+; Q1' = D1_{k+1/2};
 *       c = D2_k, k* = k-1 if |D2_k| <= |D2_{k+1}|, else c = D2_{k+1}, k* = k;
 *       Q2' = c (2(i-k)-1) dx;
 *       c* = D3_{k*+1/2} if |D3_{k*+1/2}| <= |D3_{k*+3/2}| else D3_{k*+3/2};
 *       Q3' = c* (3(i-k*)^2 - 6(i-k*) + 2) dx^2; p = (Q1' + Q2') + Q3'.
 *   R4  alpha_i = max over grid nodes of max over controls |f_i(x,u,d)|;
 *       computed once per solve (it does not depend on V).
 *   R5  dt = cfl / sum_i alpha_i/dx_i, fixed for all stages of a step.
 *   R6  loop while (tf - t) >= eps*(tf - t0), eps = 100*2^-52, h = min(dt, tf-t).
 *   R7  RK2 = Shu-Osher TVD-RK2 (Heun): V1 = V + h L(V); V+ = (V + V1 + h L(V1))/2.
 *   R8  RK3 as the odeCFL3 listing: V1 = V + hL(V); V2 = V1 + hL(V1);
 *       Vh = (3V + V2)/4; V3 = Vh + hL(Vh); V+ = (V + 2 V3)/3.
 *   R9  V_t + H(x, grad V) = 0 integrated forward from V0; H = -opt p.f.
 *   R11 tube: V <- min(V, V0) after every full step.
 *   R12 non-periodic ghosts: linear extrapolation v_{-k} = v_0 + k (v_0 - v_1).
 *   R14 non-periodic axis: dx = (hi-lo)/(N-1), both ends are nodes;
 *       periodic axis: dx = (hi-lo)/N, hi is not a node.
 *   R20 rockets: the vector field is the one inside the Hamiltonian's
 *       definition, f = (a cos th + ue x, a sin th + a + up x - g, up - ue)
 *       with a_p = a_e = a and |ue|, |up| <= umax, the evader maximising
 *       and the pursuer minimising, so
 *       H = -a p1 cos th - p2 (a sin th + a - g) - umax |p1 x - p3|
 *           + umax |p2 x + p3|;
 *       the relative equations of motion print ue x in zdot and the closed
 *       form printed after the definition has other signs, so neither is used.
 *   R21 variational-inequality tube (the min[0,H] form): with V_t + H = 0
 *       integrated forward, the zero sublevel set may only grow, so every
 *       stage uses L = min(-Hhat, 0) (V never increases); no min with V0.
 *   R22 output times: an output time is hit exactly; each interval
 *       [t_{k-1}, t_k] runs the loop of R6 on its own (rule relative to the
 *       interval).  The tube-at-outputs mode takes V <- min(V, V0) at the
 *       output times only.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXD 4

/* scheme, integrator and dynamics codes of this file (the Python shim maps
 * names to them; nothing outside this file shares them) */
enum { ORC_UPWIND1 = 1, ORC_ENO2 = 2, ORC_ENO3 = 3, ORC_WENO5 = 5 };
enum { ORC_TRANSLATION = 0, ORC_BALL = 1, ORC_DOUBLE_INTEGRATOR = 2,
       ORC_REL_DUBINS = 3, ORC_DUBINS4D = 4, ORC_ROCKETS = 5 };
enum { ORC_SET = 0, ORC_TUBE = 1, ORC_TUBE_VI = 2, ORC_TUBE_OUT = 3 };
enum { ORC_LF = 0, ORC_LLF = 1, ORC_GLF = 2 };

/* dissipation variant of the solver entry points (reading R25); set with
 * orc_set_dissipation before a call */
static int g_diss = ORC_LF;

/* FP32 storage model of orc_steps (a measurement aid for the single-precision
 * form of the method, not part of the method; 0 = plain FP64, the default).
 * ORC_ROUND_STAGES rounds every stage result of an RK step, and so the state,
 * to the nearest single-precision value as it is stored.
 * ORC_ROUND_INPUTS rounds what a single-precision evaluation holds in single
 * precision: the node coordinates and their cos/sin, the dynamics parameters,
 * the cell sizes and their reciprocals, alpha as the Lax-Friedrichs
 * coefficient, and the step size.  The arithmetic itself stays FP64. */
enum { ORC_ROUND_STAGES = 1, ORC_ROUND_INPUTS = 2 };
static int g_store = 0;

/* nearest single-precision value (round to nearest even) */
static double round32(double x)
{
    return (double)(float)x;
}

typedef struct {
    int nd;
    long n[ORC_MAXD];
    long stride[ORC_MAXD];
    long total;
    double lo[ORC_MAXD], hi[ORC_MAXD], dx[ORC_MAXD];
    double inv_dx[ORC_MAXD];  /* 1/dx */
    double inv_2dx[ORC_MAXD]; /* 1/(2 dx) */
    double inv_3dx[ORC_MAXD]; /* 1/(3 dx) */
    int periodic[ORC_MAXD];
    double *x[ORC_MAXD]; /* node coordinates per axis */
    double *cs[ORC_MAXD]; /* cos of the node coordinates */
    double *sn[ORC_MAXD]; /* sin of the node coordinates */
} ogrid;

typedef struct {
    int kind;
    double prm[8];
} odyn;

/* ---------------------------------------------------------------- grid */

/* Sec. 2.1 (createGrid): nodes lo + k*dx per axis; reading R14 for dx. */
static int grid_init(ogrid *g, int nd, const long *n, const double *lo,
                     const double *hi, unsigned periodic_mask)
{
    if (nd < 1 || nd > ORC_MAXD) return -1;
    g->nd = nd;
    g->total = 1;
    for (int d = 0; d < nd; ++d) {
        g->n[d] = n[d];
        g->lo[d] = lo[d];
        g->hi[d] = hi[d];
        g->periodic[d] = (periodic_mask >> d) & 1u;
        if (n[d] < 2) return -1;
        g->dx[d] = g->periodic[d] ? (hi[d] - lo[d]) / (double)n[d]
                                  : (hi[d] - lo[d]) / (double)(n[d] - 1);
        g->inv_dx[d] = 1.0 / g->dx[d];
        g->inv_2dx[d] = 1.0 / (2.0 * g->dx[d]);
        g->inv_3dx[d] = 1.0 / (3.0 * g->dx[d]);
        g->total *= n[d];
    }
    /* C order: the last axis is the fastest */
    long s = 1;
    for (int d = nd - 1; d >= 0; --d) {
        g->stride[d] = s;
        s *= n[d];
    }
    for (int d = 0; d < nd; ++d) {
        g->x[d] = (double *)malloc(sizeof(double) * (size_t)n[d]);
        g->cs[d] = (double *)malloc(sizeof(double) * (size_t)n[d]);
        g->sn[d] = (double *)malloc(sizeof(double) * (size_t)n[d]);
        if (!g->x[d] || !g->cs[d] || !g->sn[d]) return -2;
        for (long k = 0; k < n[d]; ++k) {
            g->x[d][k] = lo[d] + (double)k * g->dx[d];
            g->cs[d][k] = cos(g->x[d][k]);
            g->sn[d][k] = sin(g->x[d][k]);
        }
    }
    return 0;
}

static void grid_free(ogrid *g)
{
    for (int d = 0; d < ORC_MAXD; ++d) {
        free(g->x[d]);
        free(g->cs[d]);
        free(g->sn[d]);
    }
}

static long axis_index(const ogrid *g, long node, int d)
{
    return (node / g->stride[d]) % g->n[d];
}

/* Fig. 3 / reading R12: value at axis-d index j (possibly a ghost index) on
 * the grid line through `node`. */
static double line_value(const ogrid *g, const double *v, long node, int d, long j)
{
    long n = g->n[d];
    long base = node - axis_index(g, node, d) * g->stride[d];
    if (j >= 0 && j < n) return v[base + j * g->stride[d]];
    if (g->periodic[d]) {
        long jj = ((j % n) + n) % n;
        return v[base + jj * g->stride[d]];
    }
    if (j < 0) {
        double v0 = v[base];
        double v1 = v[base + g->stride[d]];
        return v0 + (double)(-j) * (v0 - v1);
    }
    {
        double va = v[base + (n - 1) * g->stride[d]];
        double vb = v[base + (n - 2) * g->stride[d]];
        return va + (double)(j - (n - 1)) * (va - vb);
    }
}

/* ------------------------------------------------- one-sided derivatives */

/* Sec. 3.3, Jiang-Peng WENO5 (Osher-Fedkiw eqs. 3.28-3.39), reading R3 for
 * eps.  The left-biased approximation at node i uses the five consecutive
 * differences D1 at i-5/2 .. i+3/2; the right-biased one at node i-1 uses the
 * same five differences in reverse order.  Both are written here on the
 * window w0..w4 (increasing grid order):
 *   smoothness on the three triples, with e = (a + c) - 2b:
 *     SA = 13/12 e^2 + 1/4 ((a + 3c) - 4b)^2   on (w0, w1, w2)
 *     SB = 13/12 e^2 + 1/4 (a - c)^2           on (w1, w2, w3)
 *     SC = 13/12 e^2 + 1/4 ((3a + c) - 4b)^2   on (w2, w3, w4)
 *   (the left-biased S1, S2, S3 are SA, SB, SC; the right-biased S1, S2, S3
 *   are SC, SB, SA: the same values),
 *   eps = 1e-6 max_k w_k^2 + 1e-99, r_X = 1/(S_X + eps)^2,
 *   weights gamma = (0.1, 0.6, 0.3) on (rA, rB, rC) for the left-biased and on
 *   (rC, rB, rA) for the right-biased approximation, normalised by one
 *   division of the weighted sum of the third-order candidates.
 * The constant fractions are multiplied as precomputed doubles.  Every
 * quantity shared by the two approximations of a window is rounded the same
 * way in both, so a device implementation may evaluate it once. */
static const double C1_3 = 1.0 / 3.0, C1_6 = 1.0 / 6.0, C5_6 = 5.0 / 6.0,
                    C7_6 = 7.0 / 6.0, C11_6 = 11.0 / 6.0, C13_12 = 13.0 / 12.0;

typedef struct {
    double ra, rb, rc; /* reciprocal squared regularised smoothness */
} wweights;

static wweights weno_window(const double *w)
{
    double ea = (w[0] + w[2]) - 2.0 * w[1];
    double eb = (w[1] + w[3]) - 2.0 * w[2];
    double ec = (w[2] + w[4]) - 2.0 * w[3];
    double fa = (w[0] + 3.0 * w[2]) - 4.0 * w[1];
    double fb = w[1] - w[3];
    double fc = (3.0 * w[2] + w[4]) - 4.0 * w[3];
    double sa = C13_12 * ea * ea + 0.25 * fa * fa;
    double sb = C13_12 * eb * eb + 0.25 * fb * fb;
    double sc = C13_12 * ec * ec + 0.25 * fc * fc;

    double mx = w[0] * w[0];
    for (int k = 1; k < 5; ++k)
        if (w[k] * w[k] > mx) mx = w[k] * w[k];
    double eps = 1e-6 * mx + 1e-99;

    wweights r;
    r.ra = 1.0 / ((sa + eps) * (sa + eps));
    r.rb = 1.0 / ((sb + eps) * (sb + eps));
    r.rc = 1.0 / ((sc + eps) * (sc + eps));
    return r;
}

/* WENO5 blend of the candidates on v1..v5 with the reciprocal weights
 * r1, r2, r3 of their substencils */
static double weno_blend(double v1, double v2, double v3, double v4, double v5,
                         double r1, double r2, double r3)
{
    double phi1 = v1 * C1_3 - v2 * C7_6 + v3 * C11_6;
    double phi2 = -v2 * C1_6 + v3 * C5_6 + v4 * C1_3;
    double phi3 = v3 * C1_3 + v4 * C5_6 - v5 * C1_6;
    double a1 = 0.1 * r1, a2 = 0.6 * r2, a3 = 0.3 * r3;
    return (a1 * phi1 + a2 * phi2 + a3 * phi3) / (a1 + a2 + a3);
}

/* left-biased approximation (p- of the node right of the window centre) */
static double weno_left(const double *w)
{
    wweights r = weno_window(w);
    return weno_blend(w[0], w[1], w[2], w[3], w[4], r.ra, r.rb, r.rc);
}

/* right-biased approximation (p+ of the node left of the window centre) */
static double weno_right(const double *w)
{
    wweights r = weno_window(w);
    return weno_blend(w[4], w[3], w[2], w[1], w[0], r.rc, r.rb, r.ra);
}

/* ENO choice of the smaller second difference, tie to the first argument
 * (reading R2). */
static double eno_pick(double a, double b)
{
    return fabs(a) <= fabs(b) ? a : b;
}

/* Sec. 3 (upwinding): left (p-) and right (p+) approximations of dV/dx_d at
 * one node.  The local stencil is patched with ghost values, then the
 * divided-difference table of that stencil is formed. */
static void derivs_at(const ogrid *g, const double *v, long node, int d,
                      int scheme, double *pm, double *pp)
{
    long i = axis_index(g, node, d);
    double dx = g->dx[d];
    double inv_dx = g->inv_dx[d];
    if (scheme == ORC_UPWIND1) {
        double vm = line_value(g, v, node, d, i - 1);
        double vc = line_value(g, v, node, d, i);
        double vp = line_value(g, v, node, d, i + 1);
        *pm = (vc - vm) * inv_dx;
        *pp = (vp - vc) * inv_dx;
        return;
    }
    if (scheme == ORC_ENO2) {
        /* s[0..4] = v_{i-2} .. v_{i+2} */
        double s[5];
        for (int k = 0; k < 5; ++k) s[k] = line_value(g, v, node, d, i - 2 + k);
        /* first divided differences at half points i-3/2 .. i+3/2 */
        double d1[4];
        for (int k = 0; k < 4; ++k) d1[k] = (s[k + 1] - s[k]) * inv_dx;
        /* second divided differences at nodes i-1, i, i+1 */
        double d2[3];
        for (int k = 0; k < 3; ++k) d2[k] = (d1[k + 1] - d1[k]) * g->inv_2dx[d];
        *pm = d1[1] + dx * eno_pick(d2[0], d2[1]);
        *pp = d1[2] - dx * eno_pick(d2[1], d2[2]);
        return;
    }
    if (scheme == ORC_ENO3) {
        /* s[0..6] = v_{i-3} .. v_{i+3}; the table of reading R24:
         * d1[j] = D1 at i-5/2+j, d2[j] = D2 at i-2+j, d3[j] = D3 at i-3/2+j */
        double s[7], d1[6], d2[5], d3[4];
        for (int k = 0; k < 7; ++k) s[k] = line_value(g, v, node, d, i - 3 + k);
        for (int k = 0; k < 6; ++k) d1[k] = (s[k + 1] - s[k]) * inv_dx;
        for (int k = 0; k < 5; ++k) d2[k] = (d1[k + 1] - d1[k]) * g->inv_2dx[d];
        for (int k = 0; k < 4; ++k) d3[k] = (d2[k + 1] - d2[k]) * g->inv_3dx[d];
        double dxx = dx * dx;
        /* p-: k = i-1, so i-k = 1 and Q2' = c dx; k* = i-2 (factor 2) or i-1 (-1) */
        double c, cs, f;
        if (fabs(d2[1]) <= fabs(d2[2])) {
            c = d2[1];
            cs = eno_pick(d3[0], d3[1]);
            f = 2.0;
        } else {
            c = d2[2];
            cs = eno_pick(d3[1], d3[2]);
            f = -1.0;
        }
        *pm = (d1[2] + c * dx) + cs * (f * dxx);
        /* p+: k = i, so i-k = 0 and Q2' = -c dx; k* = i-1 (factor -1) or i (2) */
        if (fabs(d2[2]) <= fabs(d2[3])) {
            c = d2[2];
            cs = eno_pick(d3[1], d3[2]);
            f = -1.0;
        } else {
            c = d2[3];
            cs = eno_pick(d3[2], d3[3]);
            f = 2.0;
        }
        *pp = (d1[3] - c * dx) + cs * (f * dxx);
        return;
    }
    /* WENO5: s[0..6] = v_{i-3} .. v_{i+3}; D1 at half points i-5/2 .. i+5/2 */
    double s[7];
    for (int k = 0; k < 7; ++k) s[k] = line_value(g, v, node, d, i - 3 + k);
    double d1[6];
    for (int k = 0; k < 6; ++k) d1[k] = (s[k + 1] - s[k]) * inv_dx;
    /* p-: D-v at i-2..i+2 = D1 at i-5/2..i+3/2 */
    *pm = weno_left(&d1[0]);
    /* p+: D+v at i+2..i-2 = D1 at i+5/2..i-3/2, the window d1[1..5] reversed */
    *pp = weno_right(&d1[1]);
}

/* ------------------------------------------------------------ dynamics */

/* Hamiltonian H(x, p) with the sign convention of reading R9.
 *  TRANSLATION  xdot = b               H = -b.p
 *  BALL         xdot = s u, |u|_2<=1   H = s |p|_2 (s < 0: the set shrinks)
 *  DOUBLE_INT.  x1dot = x2, x2dot = u, |u|<=umax, control minimises:
 *               H = -(p1 x2 + min_u p2 u) = -p1 x2 + umax |p2|
 *  REL_DUBINS   (x, y, psi): xdot = -ve + vp cos psi + we y,
 *               ydot = vp sin psi - we x, psidot = wp - we; evader (we)
 *               maximises, pursuer (wp) minimises:
 *               H = -max_we min_wp p.f
 *                 = -p1(-ve + vp cos psi) - p2 vp sin psi
 *                   - wemax |p1 y - p2 x - p3| + wpmax |p3|
 *  DUBINS4D     (x, y, th, v): xdot = v cos th, ydot = v sin th, thdot = w,
 *               vdot = a; control minimises:
 *               H = -p1 v cos th - p2 v sin th + wmax |p3| + amax |p4|
 *  ROCKETS      (x, z, th), reading R20: p.f = p1 a cos th
 *               + p2 (a sin th + a - g) + ue (p1 x - p3) + up (p2 x + p3);
 *               the evader's max gives umax |p1 x - p3|, the pursuer's min
 *               -umax |p2 x + p3|, and H = -(max min p.f)
 */
static double hamiltonian(const ogrid *g, const odyn *dy, long node, const double *p)
{
    switch (dy->kind) {
    case ORC_TRANSLATION: {
        double h = 0.0;
        for (int d = 0; d < g->nd; ++d) h -= dy->prm[d] * p[d];
        return h;
    }
    case ORC_BALL: {
        double s = 0.0;
        for (int d = 0; d < g->nd; ++d) s += p[d] * p[d];
        return dy->prm[0] * sqrt(s);
    }
    case ORC_DOUBLE_INTEGRATOR: {
        double x2 = g->x[1][axis_index(g, node, 1)];
        return -p[0] * x2 + dy->prm[0] * fabs(p[1]);
    }
    case ORC_REL_DUBINS: {
        double ve = dy->prm[0], vp = dy->prm[1], we = dy->prm[2], wp = dy->prm[3];
        double x = g->x[0][axis_index(g, node, 0)];
        double y = g->x[1][axis_index(g, node, 1)];
        long k = axis_index(g, node, 2);
        double c = g->cs[2][k], s = g->sn[2][k];
        return -p[0] * (-ve + vp * c) - p[1] * (vp * s)
               - we * fabs(p[0] * y - p[1] * x - p[2]) + wp * fabs(p[2]);
    }
    case ORC_DUBINS4D: {
        double wm = dy->prm[0], am = dy->prm[1];
        long k = axis_index(g, node, 2);
        double v = g->x[3][axis_index(g, node, 3)];
        return -p[0] * (v * g->cs[2][k]) - p[1] * (v * g->sn[2][k])
               + wm * fabs(p[2]) + am * fabs(p[3]);
    }
    case ORC_ROCKETS: {
        double a = dy->prm[0], grav = dy->prm[1], um = dy->prm[2];
        double x = g->x[0][axis_index(g, node, 0)];
        long k = axis_index(g, node, 2);
        double drift1 = a * g->cs[2][k];
        double drift2 = a * g->sn[2][k] + a - grav;
        return -p[0] * drift1 - p[1] * drift2 - um * fabs(p[0] * x - p[2])
               + um * fabs(p[1] * x + p[2]);
    }
    }
    return 0.0;
}

/* Reading R4: bound over the control sets of |f_d(x, u, d)| = |dH/dp_d| at
 * one node. */
static double speed_bound(const ogrid *g, const odyn *dy, long node, int d)
{
    switch (dy->kind) {
    case ORC_TRANSLATION:
        return fabs(dy->prm[d]);
    case ORC_BALL:
        return fabs(dy->prm[0]);
    case ORC_DOUBLE_INTEGRATOR:
        if (d == 0) return fabs(g->x[1][axis_index(g, node, 1)]);
        return dy->prm[0];
    case ORC_REL_DUBINS: {
        double ve = dy->prm[0], vp = dy->prm[1], we = dy->prm[2], wp = dy->prm[3];
        double x = g->x[0][axis_index(g, node, 0)];
        double y = g->x[1][axis_index(g, node, 1)];
        long k = axis_index(g, node, 2);
        if (d == 0) return fabs(-ve + vp * g->cs[2][k]) + we * fabs(y);
        if (d == 1) return fabs(vp * g->sn[2][k]) + we * fabs(x);
        return we + wp;
    }
    case ORC_DUBINS4D: {
        long k = axis_index(g, node, 2);
        double v = g->x[3][axis_index(g, node, 3)];
        if (d == 0) return fabs(v * g->cs[2][k]);
        if (d == 1) return fabs(v * g->sn[2][k]);
        if (d == 2) return dy->prm[0];
        return dy->prm[1];
    }
    case ORC_ROCKETS: {
        /* |f1| <= |a cos th| + umax |x|, |f2| <= |a sin th + a - g| + umax |x|,
         * |f3| <= 2 umax */
        double a = dy->prm[0], grav = dy->prm[1], um = dy->prm[2];
        double x = g->x[0][axis_index(g, node, 0)];
        long k = axis_index(g, node, 2);
        if (d == 0) return fabs(a * g->cs[2][k]) + um * fabs(x);
        if (d == 1) return fabs(a * g->sn[2][k] + a - grav) + um * fabs(x);
        return 2.0 * um;
    }
    }
    return 0.0;
}

/* Reading R25: the interval of s = sum_j a_j p_j over the box lo..hi (axes
 * in order), and the signs s may take there. */
static void lin_interval(int nd, const double *a, const double *lo, const double *hi,
                         double *smin, double *smax)
{
    double l = 0.0, h = 0.0;
    for (int j = 0; j < nd; ++j) {
        double u = a[j] * lo[j], w = a[j] * hi[j];
        l = l + (u < w ? u : w);
        h = h + (u < w ? w : u);
    }
    *smin = l;
    *smax = h;
}

/* max over sign choices of |base + k * sigma| with sigma in the signs the
 * interval [smin, smax] allows */
static double sign_max(double base, double k, double smin, double smax)
{
    double m = 0.0;
    if (smax >= 0.0) {
        double v = fabs(base + k);
        if (v > m) m = v;
    }
    if (smin <= 0.0) {
        double v = fabs(base - k);
        if (v > m) m = v;
    }
    return m;
}

/* Reading R25: max over p in the box lo..hi of |dH/dp_d| at one node. */
static double box_bound(const ogrid *g, const odyn *dy, long node, int d, const double *lo,
                        const double *hi)
{
    int nd = g->nd;
    switch (dy->kind) {
    case ORC_BALL: {
        /* H = s|p|: |dH/dp_d| = |s| |p_d| / |p|, largest at the largest |p_d|
         * and the smallest |p_j| (j != d) of the box */
        double big = fabs(lo[d]) > fabs(hi[d]) ? fabs(lo[d]) : fabs(hi[d]);
        double rest = 0.0;
        int all_zero = big == 0.0;
        for (int j = 0; j < nd; ++j) {
            if (j == d) continue;
            double m = (lo[j] <= 0.0 && hi[j] >= 0.0) ? 0.0
                       : (fabs(lo[j]) < fabs(hi[j]) ? fabs(lo[j]) : fabs(hi[j]));
            if (m != 0.0) all_zero = 0;
            rest = rest + m * m;
        }
        if (big == 0.0) return all_zero ? fabs(dy->prm[0]) : 0.0;
        return fabs(dy->prm[0]) * (big / sqrt(big * big + rest));
    }
    case ORC_REL_DUBINS: {
        double ve = dy->prm[0], vp = dy->prm[1], we = dy->prm[2], wp = dy->prm[3];
        double x = g->x[0][axis_index(g, node, 0)];
        double y = g->x[1][axis_index(g, node, 1)];
        long k = axis_index(g, node, 2);
        double a[3] = {y, -x, -1.0}, smin, smax;
        lin_interval(3, a, lo, hi, &smin, &smax);
        /* dH/dp1 = (ve - vp cos) - we y sgn s, dH/dp2 = -vp sin + we x sgn s,
         * dH/dp3 = we sgn s + wp sgn p3 */
        if (d == 0) return sign_max(ve - vp * g->cs[2][k], -we * y, smin, smax);
        if (d == 1) return sign_max(-(vp * g->sn[2][k]), we * x, smin, smax);
        {
            double m = 0.0;
            if (smax >= 0.0) {
                double v = sign_max(we, wp, lo[2], hi[2]);
                if (v > m) m = v;
            }
            if (smin <= 0.0) {
                double v = sign_max(-we, wp, lo[2], hi[2]);
                if (v > m) m = v;
            }
            return m;
        }
    }
    case ORC_ROCKETS: {
        double am = dy->prm[0], grav = dy->prm[1], um = dy->prm[2];
        double x = g->x[0][axis_index(g, node, 0)];
        long k = axis_index(g, node, 2);
        double a1[3] = {x, 0.0, -1.0}, a2[3] = {0.0, x, 1.0};
        double l1, h1, l2, h2;
        lin_interval(3, a1, lo, hi, &l1, &h1);
        lin_interval(3, a2, lo, hi, &l2, &h2);
        /* dH/dp1 = -a cos - um x sgn s1, dH/dp2 = -(a sin + a - g) + um x sgn s2,
         * dH/dp3 = um sgn s1 - um sgn s2 */
        if (d == 0) return sign_max(-(am * g->cs[2][k]), -um * x, l1, h1);
        if (d == 1) return sign_max(-(am * g->sn[2][k] + am - grav), um * x, l2, h2);
        {
            double m = 0.0;
            if (h1 >= 0.0) {
                double v = sign_max(um, um, l2, h2);
                if (v > m) m = v;
            }
            if (l1 <= 0.0) {
                double v = sign_max(-um, um, l2, h2);
                if (v > m) m = v;
            }
            return m;
        }
    }
    default:
        /* translation, double integrator, 4-D Dubins: |dH/dp_d| does not
         * depend on p beyond the control bound */
        return speed_bound(g, dy, node, d);
    }
}

/* Sec. 4: global Lax-Friedrichs dissipation coefficients. */
static void compute_alpha(const ogrid *g, const odyn *dy, double *alpha)
{
    for (int d = 0; d < g->nd; ++d) {
        double m = 0.0;
        /* a maximum is exact whatever the order, so the threads may split it */
#pragma omp parallel for schedule(static) reduction(max : m)
        for (long node = 0; node < g->total; ++node) {
            double b = speed_bound(g, dy, node, d);
            if (b > m) m = b;
        }
        alpha[d] = m;
    }
}

/* Sec. 4 CFL condition, reading R5: the step that makes
 * dt * sum_d alpha_d/dx_d equal to cfl. */
static double cfl_dt(const ogrid *g, const double *alpha, double cfl)
{
    double rate = 0.0;
    for (int d = 0; d < g->nd; ++d) rate += alpha[d] / g->dx[d];
    if (rate <= 0.0) return INFINITY;
    return cfl / rate;
}

/* Sec. 4, Lax-Friedrichs:
 *   Hhat = H(x, (p+ + p-)/2) - sum_d alpha_d (p+_d - p-_d)/2,
 * (the dissipation summed over the axes in order, then subtracted) and the
 * semi-discrete right-hand side L(V) = -Hhat (from V_t + H = 0). */
static double rhs_at(const ogrid *g, const odyn *dy, int scheme,
                     const double *alpha, const double *v, long node, const double *gbox)
{
    double pm[ORC_MAXD], pp[ORC_MAXD], pbar[ORC_MAXD];
    for (int d = 0; d < g->nd; ++d) derivs_at(g, v, node, d, scheme, &pm[d], &pp[d]);
    /* reading R25: the costate box of the dissipation coefficients */
    double lo[ORC_MAXD], hi[ORC_MAXD];
    for (int d = 0; d < g->nd; ++d) {
        if (g_diss == ORC_GLF) {
            lo[d] = gbox[2 * d];
            hi[d] = gbox[2 * d + 1];
        } else {
            lo[d] = pm[d] < pp[d] ? pm[d] : pp[d];
            hi[d] = pm[d] < pp[d] ? pp[d] : pm[d];
        }
    }
    double diss = 0.0;
    for (int d = 0; d < g->nd; ++d) {
        double a = g_diss == ORC_LF ? alpha[d] : box_bound(g, dy, node, d, lo, hi);
        pbar[d] = (pp[d] + pm[d]) / 2.0;
        diss += a * ((pp[d] - pm[d]) / 2.0);
    }
    double hhat = hamiltonian(g, dy, node, pbar) - diss;
    return -hhat;
}

/* Reading R25, GLF: the grid-wide box of both one-sided derivatives, per axis
 * [min, max] into box[2d], box[2d+1]. */
static void global_box(const ogrid *g, int scheme, const double *v, double *box)
{
    for (int d = 0; d < g->nd; ++d) {
        double lo = INFINITY, hi = -INFINITY;
        /* min and max are exact: any grouping of the nodes gives the same box */
#pragma omp parallel for schedule(static) reduction(min : lo) reduction(max : hi)
        for (long node = 0; node < g->total; ++node) {
            double pm, pp;
            derivs_at(g, v, node, d, scheme, &pm, &pp);
            if (pm < lo) lo = pm;
            if (pp < lo) lo = pp;
            if (pm > hi) hi = pm;
            if (pp > hi) hi = pp;
        }
        box[2 * d] = lo;
        box[2 * d + 1] = hi;
    }
}

/* L(V) at every node; in the variational-inequality tube (reading R21) the
 * update is restricted to L <= 0. */
static void rhs_all(const ogrid *g, const odyn *dy, int scheme,
                    const double *alpha, const double *v, double *out, int mode)
{
    double box[2 * ORC_MAXD] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (g_diss == ORC_GLF) global_box(g, scheme, v, box);
#pragma omp parallel for schedule(static)
    for (long node = 0; node < g->total; ++node) {
        double l = rhs_at(g, dy, scheme, alpha, v, node, box);
        if (mode == ORC_TUBE_VI && l > 0.0) l = 0.0;
        out[node] = l;
    }
}

/* the FP32 storage model: a stage result as it is stored */
static void store_stage(const ogrid *g, double *w, int store)
{
    if (!(store & ORC_ROUND_STAGES)) return;
    for (long k = 0; k < g->total; ++k) w[k] = round32(w[k]);
}

/* the FP32 storage model: the grid's tables and the dynamics parameters as
 * a single-precision evaluation holds them */
static void round_inputs(ogrid *g, odyn *dy)
{
    for (int d = 0; d < g->nd; ++d) {
        g->dx[d] = round32(g->dx[d]);
        g->inv_dx[d] = round32(g->inv_dx[d]);
        g->inv_2dx[d] = round32(g->inv_2dx[d]);
        g->inv_3dx[d] = round32(g->inv_3dx[d]);
        for (long k = 0; k < g->n[d]; ++k) {
            g->x[d][k] = round32(g->x[d][k]);
            g->cs[d][k] = round32(g->cs[d][k]);
            g->sn[d][k] = round32(g->sn[d][k]);
        }
    }
    for (int k = 0; k < 8; ++k) dy->prm[k] = round32(dy->prm[k]);
}

/* Sec. 5 (odeCFL listing) and readings R7, R8, R11: one TVD-RK step of size h
 * applied in place to v.  w1, w2, l are scratch arrays of the grid size.
 * store: the FP32 storage model's flags (0 in every solve entry point). */
static void rk_step(const ogrid *g, const odyn *dy, int scheme, int order,
                    const double *alpha, double h, double *v, const double *v0,
                    int mode, double *w1, double *w2, double *l, int store)
{
    long n = g->total;
    if (order == 1) {
        rhs_all(g, dy, scheme, alpha, v, l, mode);
        for (long k = 0; k < n; ++k) v[k] = v[k] + h * l[k];
    } else if (order == 2) {
        rhs_all(g, dy, scheme, alpha, v, l, mode);
        for (long k = 0; k < n; ++k) w1[k] = v[k] + h * l[k];
        store_stage(g, w1, store);
        rhs_all(g, dy, scheme, alpha, w1, l, mode);
        for (long k = 0; k < n; ++k) {
            double v2 = w1[k] + h * l[k];
            v[k] = (v[k] + v2) / 2.0;
        }
    } else {
        rhs_all(g, dy, scheme, alpha, v, l, mode);
        for (long k = 0; k < n; ++k) w1[k] = v[k] + h * l[k];
        store_stage(g, w1, store);
        rhs_all(g, dy, scheme, alpha, w1, l, mode);
        for (long k = 0; k < n; ++k) {
            double v2 = w1[k] + h * l[k];
            w2[k] = (3.0 * v[k] + v2) / 4.0;
        }
        store_stage(g, w2, store);
        rhs_all(g, dy, scheme, alpha, w2, l, mode);
        for (long k = 0; k < n; ++k) {
            double v3 = w2[k] + h * l[k];
            v[k] = (v[k] + 2.0 * v3) / 3.0;
        }
    }
    store_stage(g, v, store);
    if (mode == ORC_TUBE)
        for (long k = 0; k < n; ++k)
            if (v0[k] < v[k]) v[k] = v0[k];
}

static int setup(ogrid *g, odyn *dy, int nd, const long *n, const double *lo,
                 const double *hi, unsigned pmask, int dyn, const double *prm,
                 int nprm)
{
    if (grid_init(g, nd, n, lo, hi, pmask) != 0) return -1;
    dy->kind = dyn;
    memset(dy->prm, 0, sizeof(dy->prm));
    for (int k = 0; k < nprm && k < 8; ++k) dy->prm[k] = prm[k];
    return 0;
}

/* --------------------------------------------------------- exported API */

/* alpha per axis, the CFL step and the step count of a solve over [t0, tf]
 * (readings R4-R6). */
int orc_schedule(int nd, const long *n, const double *lo, const double *hi,
                 unsigned pmask, int dyn, const double *prm, int nprm,
                 double cfl, double t0, double tf, double *alpha_out,
                 double *dt_out, long *nsteps_out, double *tend_out)
{
    ogrid g;
    odyn dy;
    memset(&g, 0, sizeof(g));
    if (setup(&g, &dy, nd, n, lo, hi, pmask, dyn, prm, nprm) != 0) {
        grid_free(&g);
        return -1;
    }
    compute_alpha(&g, &dy, alpha_out);
    double dt = cfl_dt(&g, alpha_out, cfl);
    *dt_out = dt;
    long steps = 0;
    double t = t0;
    const double eps = 100.0 * 2.220446049250313e-16;
    if (tf > t0) {
        while (tf - t >= eps * (tf - t0)) {
            double h = dt < tf - t ? dt : tf - t;
            t = t + h;
            ++steps;
        }
    }
    *nsteps_out = steps;
    *tend_out = t;
    grid_free(&g);
    return 0;
}

/* p- and p+ along axis `axis` at every node of v (Sec. 3). */
int orc_derivs(int nd, const long *n, const double *lo, const double *hi,
               unsigned pmask, int scheme, int axis, const double *v,
               double *pm, double *pp)
{
    ogrid g;
    memset(&g, 0, sizeof(g));
    if (grid_init(&g, nd, n, lo, hi, pmask) != 0) {
        grid_free(&g);
        return -1;
    }
    for (long node = 0; node < g.total; ++node)
        derivs_at(&g, v, node, axis, scheme, &pm[node], &pp[node]);
    grid_free(&g);
    return 0;
}

/* L(V) = -Hhat at the listed nodes (Sec. 4), for a given alpha. */
int orc_rhs_at(int nd, const long *n, const double *lo, const double *hi,
               unsigned pmask, int dyn, const double *prm, int nprm,
               int scheme, const double *alpha, const double *v, long count,
               const long *nodes, double *out)
{
    ogrid g;
    odyn dy;
    memset(&g, 0, sizeof(g));
    if (setup(&g, &dy, nd, n, lo, hi, pmask, dyn, prm, nprm) != 0) {
        grid_free(&g);
        return -1;
    }
    double box[2 * ORC_MAXD] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (g_diss == ORC_GLF) global_box(&g, scheme, v, box);
    for (long k = 0; k < count; ++k)
        out[k] = rhs_at(&g, &dy, scheme, alpha, v, nodes[k], box);
    grid_free(&g);
    return 0;
}

/* Advance v in place by `nsteps` TVD-RK steps of size h each (h is used as
 * given), with the tube update when mode is ORC_TUBE. alpha is supplied.
 * The FP32 storage model (orc_set_storage_model) applies to this entry point
 * only. */
int orc_steps(int nd, const long *n, const double *lo, const double *hi,
              unsigned pmask, int dyn, const double *prm, int nprm,
              int scheme, int order, const double *alpha, double h, long nsteps,
              double *v, const double *v0, int mode)
{
    ogrid g;
    odyn dy;
    memset(&g, 0, sizeof(g));
    if (setup(&g, &dy, nd, n, lo, hi, pmask, dyn, prm, nprm) != 0) {
        grid_free(&g);
        return -1;
    }
    double a[ORC_MAXD] = {0, 0, 0, 0};
    for (int d = 0; d < nd; ++d) a[d] = alpha[d];
    if (g_store & ORC_ROUND_INPUTS) {
        round_inputs(&g, &dy);
        for (int d = 0; d < nd; ++d) a[d] = round32(a[d]);
        h = round32(h);
    }
    size_t bytes = sizeof(double) * (size_t)g.total;
    double *w1 = (double *)malloc(bytes), *w2 = (double *)malloc(bytes),
           *l = (double *)malloc(bytes);
    int rc = 0;
    if (!w1 || !w2 || !l) {
        rc = -2;
    } else {
        for (long s = 0; s < nsteps; ++s)
            rk_step(&g, &dy, scheme, order, a, h, v, v0, mode, w1, w2, l, g_store);
    }
    free(w1);
    free(w2);
    free(l);
    grid_free(&g);
    return rc;
}

/* Full solve over [t0, tf] from V0 (Sec. 5 time loop with readings R4-R6,
 * R11).  v_out receives V(tf).  Returns the step count or a negative code. */
long orc_solve(int nd, const long *n, const double *lo, const double *hi,
               unsigned pmask, int dyn, const double *prm, int nprm,
               int scheme, int order, double cfl, const double *v0,
               double *v_out, double t0, double tf, int mode,
               double *alpha_out, double *dt_out)
{
    ogrid g;
    odyn dy;
    memset(&g, 0, sizeof(g));
    if (setup(&g, &dy, nd, n, lo, hi, pmask, dyn, prm, nprm) != 0) {
        grid_free(&g);
        return -1;
    }
    double alpha[ORC_MAXD] = {0, 0, 0, 0};
    compute_alpha(&g, &dy, alpha);
    double dt = cfl_dt(&g, alpha, cfl);
    for (int d = 0; d < nd; ++d) alpha_out[d] = alpha[d];
    *dt_out = dt;

    size_t bytes = sizeof(double) * (size_t)g.total;
    memcpy(v_out, v0, bytes);
    double *w1 = (double *)malloc(bytes), *w2 = (double *)malloc(bytes),
           *l = (double *)malloc(bytes);
    if (!w1 || !w2 || !l) {
        free(w1);
        free(w2);
        free(l);
        grid_free(&g);
        return -2;
    }
    long steps = 0;
    double t = t0;
    const double eps = 100.0 * 2.220446049250313e-16;
    if (tf > t0) {
        while (tf - t >= eps * (tf - t0)) {
            double h = dt < tf - t ? dt : tf - t;
            rk_step(&g, &dy, scheme, order, alpha, h, v_out, v0, mode, w1, w2, l, 0);
            t = t + h;
            ++steps;
        }
    }
    if (mode == ORC_TUBE_OUT) /* reading R22: the one output time is tf */
        for (long q = 0; q < g.total; ++q)
            if (v0[q] < v_out[q]) v_out[q] = v0[q];
    free(w1);
    free(w2);
    free(l);
    grid_free(&g);
    return steps;
}

/* Solve from V0 at t0 through the output times times[0..ntimes) (ascending,
 * times[0] >= t0), writing V at each into v_outs[k * total ...] (readings
 * R22 and R11/R21; in the tube-at-outputs mode V <- min(V, V0) is taken at
 * each output time only).  Returns the total step count or a negative code. */
long orc_solve_outputs(int nd, const long *n, const double *lo, const double *hi,
                       unsigned pmask, int dyn, const double *prm, int nprm,
                       int scheme, int order, double cfl, const double *v0,
                       double t0, const double *times, long ntimes, int mode,
                       double *v_outs)
{
    ogrid g;
    odyn dy;
    memset(&g, 0, sizeof(g));
    if (setup(&g, &dy, nd, n, lo, hi, pmask, dyn, prm, nprm) != 0) {
        grid_free(&g);
        return -1;
    }
    double alpha[ORC_MAXD] = {0, 0, 0, 0};
    compute_alpha(&g, &dy, alpha);
    double dt = cfl_dt(&g, alpha, cfl);
    size_t bytes = sizeof(double) * (size_t)g.total;
    double *v = (double *)malloc(bytes);
    double *w1 = (double *)malloc(bytes), *w2 = (double *)malloc(bytes),
           *l = (double *)malloc(bytes);
    if (!v || !w1 || !w2 || !l) {
        free(v);
        free(w1);
        free(w2);
        free(l);
        grid_free(&g);
        return -2;
    }
    memcpy(v, v0, bytes);
    /* the per-step update: none in the tube-at-outputs mode */
    const int step_mode = mode == ORC_TUBE_OUT ? ORC_SET : mode;
    const double eps = 100.0 * 2.220446049250313e-16;
    long steps = 0;
    double t = t0;
    for (long k = 0; k < ntimes; ++k) {
        double ta = t, tb = times[k];
        if (tb > ta) {
            while (tb - t >= eps * (tb - ta)) {
                double h = dt < tb - t ? dt : tb - t;
                rk_step(&g, &dy, scheme, order, alpha, h, v, v0, step_mode, w1, w2, l, 0);
                t = t + h;
                ++steps;
            }
        }
        t = tb;
        if (mode == ORC_TUBE_OUT)
            for (long q = 0; q < g.total; ++q)
                if (v0[q] < v[q]) v[q] = v0[q];
        memcpy(v_outs + (size_t)k * (size_t)g.total, v, bytes);
    }
    free(v);
    free(w1);
    free(w2);
    free(l);
    grid_free(&g);
    return steps;
}

/* ------------------------------------------------- implicit surfaces */

/* Sec. 2.2: V0 as a function of the node coordinates, negative inside the
 * shape.  A shape takes part along the axes of its mask (all axes for a
 * sphere or a zero mask); coordinate differences are plain (no wrap on a
 * periodic axis).
 *   SPHERE, CYLINDER  sqrt(sum (x_d - c_d)^2) - r           (signed distance)
 *   BOX               |max(q, 0)|_2 + min(max_d q_d, 0),
 *                     q_d = |x_d - c_d| - h_d                (signed distance)
 *   ELLIPSOID         sum w_d (x_d - c_d)^2 - r              (the quadratic
 *                     form of the ellipsoid listing, weights w = (1, 4, 9))
 * Shapes combine left to right (Fig. 4): union min(v, s), intersection
 * max(v, s), difference max(v, -s). */
enum { ORC_SPHERE = 0, ORC_CYLINDER = 1, ORC_BOX = 2, ORC_ELLIPSOID = 3 };
enum { ORC_UNION = 0, ORC_INTERSECT = 1, ORC_SUBTRACT = 2 };

static double shape_value(int nd, int kind, unsigned mask, const double *c,
                          const double *size, double r, const double *x)
{
    if (kind == ORC_SPHERE || mask == 0) mask = (1u << nd) - 1u;
    if (kind == ORC_BOX) {
        double outside = 0.0, inside = -INFINITY;
        for (int d = 0; d < nd; ++d) {
            if (!((mask >> d) & 1u)) continue;
            double q = fabs(x[d] - c[d]) - size[d];
            if (q > 0.0) outside = outside + q * q;
            if (q > inside) inside = q;
        }
        return sqrt(outside) + (inside < 0.0 ? inside : 0.0);
    }
    double acc = 0.0;
    for (int d = 0; d < nd; ++d) {
        if (!((mask >> d) & 1u)) continue;
        double t = x[d] - c[d];
        if (kind == ORC_ELLIPSOID)
            acc = acc + size[d] * (t * t);
        else
            acc = acc + t * t;
    }
    if (kind == ORC_ELLIPSOID) return acc - r;
    return sqrt(acc) - r;
}

/* V at every node from nshapes shapes (kinds, ops, masks, centers and sizes
 * as nshapes x 4 arrays, radii). */
int orc_shapes(int nd, const long *n, const double *lo, const double *hi,
               unsigned pmask, int nshapes, const int *kinds, const int *ops,
               const unsigned *masks, const double *centers, const double *sizes,
               const double *radii, double *out)
{
    ogrid g;
    memset(&g, 0, sizeof(g));
    if (nshapes < 1 || grid_init(&g, nd, n, lo, hi, pmask) != 0) {
        grid_free(&g);
        return -1;
    }
    for (long node = 0; node < g.total; ++node) {
        double x[ORC_MAXD] = {0, 0, 0, 0};
        for (int d = 0; d < nd; ++d) x[d] = g.x[d][axis_index(&g, node, d)];
        double v = 0.0;
        for (int k = 0; k < nshapes; ++k) {
            double sv = shape_value(nd, kinds[k], masks[k], &centers[4 * k], &sizes[4 * k],
                                    radii[k], x);
            if (k == 0)
                v = sv;
            else if (ops[k] == ORC_UNION)
                v = sv < v ? sv : v;
            else if (ops[k] == ORC_INTERSECT)
                v = sv > v ? sv : v;
            else
                v = -sv > v ? -sv : v;
        }
        out[node] = v;
    }
    grid_free(&g);
    return 0;
}

/* Reading R25 at one node: max over p in the box blo..bhi of |dH/dp_d|. */
double orc_box_bound(int nd, const long *n, const double *lo, const double *hi,
                     unsigned pmask, int dyn, const double *prm, int nprm, long node, int d,
                     const double *blo, const double *bhi)
{
    ogrid g;
    odyn dy;
    memset(&g, 0, sizeof(g));
    if (setup(&g, &dy, nd, n, lo, hi, pmask, dyn, prm, nprm) != 0) {
        grid_free(&g);
        return -1.0;
    }
    double r = box_bound(&g, &dy, node, d, blo, bhi);
    grid_free(&g);
    return r;
}

/* dissipation variant of later calls (reading R25): 0 LF, 1 LLF, 2 GLF;
 * returns the previous one */
int orc_set_dissipation(int kind)
{
    int old = g_diss;
    g_diss = kind;
    return old;
}

/* FP32 storage model of orc_steps (ORC_ROUND_STAGES | ORC_ROUND_INPUTS, or
 * 0 for plain FP64); returns the previous setting */
int orc_set_storage_model(int flags)
{
    int old = g_store;
    g_store = flags;
    return old;
}

/* number of host threads used by the node loops (0 or less: all cores) */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
