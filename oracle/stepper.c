/*
 * Oracle for the swept-rule hot path: a plain, slow, obviously correct CPU
 * stepper.
 *
 * TEST INFRASTRUCTURE ONLY. It exists to check the GPU library. Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the product path never calls it and shares no code with it.
 *
 * What it computes. The swept rule of space-time decomposition reaches
 * exactly the values of plain step-by-step time advancing: every space-time
 * point is computed once, from its complete 3x3 neighbourhood one level below
 * (abstract: no redundant computation; Sec. 4, first paragraph). The oracle is
 * that plain definition written out: on a doubly periodic grid (Sec. 2,
 * assumption 1), for every global sub-step T, every point receives the
 * sub-step operation St_{T mod m} applied to its 3x3 neighbourhood at level T
 * (Sec. 2, assumption 2; the stencil list St of Algorithms 1-5).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (x86-64 SSE2 arithmetic,
 * IEEE binary64 / binary32, round to nearest even). The OpenMP loop over rows
 * does not change any bit: there is no reduction.
 *
 * Layout: state[v][j][i] (structure of arrays), i = x fastest, j = 0 is the
 * north row. Neighbour k = 3*(dj+1) + (di+1): 0 NW, 1 N, 2 NE, 3 W, 4 centre,
 * 5 E, 6 SW, 7 S, 8 SE.
 *
 * The per-point operations below are the canonical expressions of the heat,
 * wave, Euler and test stencils, evaluated left to right as written. The
 * paper fixes none of these (its experiments use a wave and an Euler solver
 * whose code is not part of the text); the expressions are this project's
 * definitions and are restated, not shared, on the GPU side.
 *
 * In the wave's velocity form for FP32 with the compensation confined to
 * residencies (st_wave_f32v), the sign with which the new velocity's
 * compensation enters the displacement's increment is pinned on one point
 * with dyadic values, where the compensated form must give exact leapfrog.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PDE_HEAT5 1
#define PDE_WAVE_LF 2
#define PDE_EULER_RUS_RK2 3
#define PDE_EULER_FD_RK4 4
#define PDE_TEST_HASH 100
#define PDE_TEST_INCR 101
#define PDE_TEST_PUSH5 102

#define MAXV 12

/* ---------------------------------------------------------------- FP64 */

/* Heat, 5-point forward-time centred-space: u' = u + r * lap(u). */
static void st_heat(const double nb[9][MAXV], double *out, const double *prm)
{
    double r = prm[0];
    double u = nb[4][0];
    double t1 = nb[3][0] + nb[5][0];
    double t2 = nb[1][0] + nb[7][0];
    double lap = (t1 + t2) - 4.0 * u;
    out[0] = u + r * lap;
}

/* Wave, leapfrog with the previous level carried as a second variable:
 * (u, p) -> ((2u - p) + C2 lap(u), u). */
static void st_wave(const double nb[9][MAXV], double *out, const double *prm)
{
    double c2 = prm[0];
    double u = nb[4][0];
    double p = nb[4][1];
    double t1 = nb[3][0] + nb[5][0];
    double t2 = nb[1][0] + nb[7][0];
    double lap = (t1 + t2) - 4.0 * u;
    out[0] = (2.0 * u - p) + c2 * lap;
    out[1] = u;
}

/* Order-sensitive 64-bit mix of the 9 neighbours and the sub-step index.
 * Values are integers below 2^52 held exactly in doubles. Any neighbour taken
 * from the wrong place or the wrong level changes the result. */
static void st_hash(long long T, const double nb[9][MAXV], double *out)
{
    uint64_t h = 0x9E3779B97F4A7C15ull ^ (uint64_t)T;
    for (int k = 0; k < 9; ++k) {
        h ^= (uint64_t)nb[k][0];
        h *= 0xFF51AFD7ED558CCDull;
        h ^= h >> 32;
    }
    out[0] = (double)(h >> 12);
}

/* The paper's worked example (Sec. 3.1): increment by one. A point whose
 * neighbours are not all at its own level becomes NaN, so a swept schedule
 * that mixes levels is caught. */
static void st_incr(const double nb[9][MAXV], double *out)
{
    double u = nb[4][0];
    int same = 1;
    for (int k = 0; k < 9; ++k)
        if (nb[k][0] != u) same = 0;
    out[0] = same ? u + 1.0 : NAN;
}

/* Sub-step decomposition of Eq. (1) into Eq. (2) (push the four neighbours)
 * and Eq. (3) (combine the pushed values). 0-based slots: slot 0 holds u,
 * slots 1..4 hold the pushed west, east, north (j-1) and south (j+1) values. */
static void st_push5(long long T, const double nb[9][MAXV], double *out)
{
    if ((T & 1) == 0) {
        out[0] = nb[4][0];
        out[1] = nb[3][0];
        out[2] = nb[5][0];
        out[3] = nb[1][0];
        out[4] = nb[7][0];
    } else {
        out[0] = nb[3][1] + nb[5][2] + nb[1][3] + nb[7][4] - 4.0 * nb[4][0];
        out[1] = 0.0;
        out[2] = 0.0;
        out[3] = 0.0;
        out[4] = 0.0;
    }
}

/* Euler: physical flux along direction d (0 = x, 1 = y) of U = (rho, mx, my, E)
 * and the largest signal speed |u_n| + c. */
static void euler_phys(const double *U, int d, double gamma, double *F, double *speed)
{
    double rho = U[0], mx = U[1], my = U[2], en = U[3];
    double ke = 0.5 * ((mx * mx + my * my) / rho);
    double p = (gamma - 1.0) * (en - ke);
    double c = sqrt((gamma * p) / rho);
    if (d == 0) {
        double un = mx / rho;
        F[0] = mx;
        F[1] = mx * un + p;
        F[2] = my * un;
        F[3] = (en + p) * un;
        *speed = fabs(un) + c;
    } else {
        double un = my / rho;
        F[0] = my;
        F[1] = mx * un;
        F[2] = my * un + p;
        F[3] = (en + p) * un;
        *speed = fabs(un) + c;
    }
}

/* Rusanov (local Lax-Friedrichs) flux through the face between the left /
 * lower state L and the right / upper state R. The arguments are always
 * passed in (left, right) order, so both cells sharing a face see the same
 * bits and the update telescopes exactly. */
static void euler_rusanov(const double *L, const double *R, int d, double gamma, double *Fh)
{
    double FL[4], FR[4], aL, aR;
    euler_phys(L, d, gamma, FL, &aL);
    euler_phys(R, d, gamma, FR, &aR);
    double a = fmax(aL, aR);
    for (int k = 0; k < 4; ++k)
        Fh[k] = 0.5 * (FL[k] + FR[k]) - 0.5 * (a * (R[k] - L[k]));
}

/* dt * L(U) at the centre, from the slots starting at off of the 5-point
 * neighbourhood; j increases southward, so the south face is j + 1/2. */
static void euler_increment(const double nb[9][MAXV], int off, double gamma, double dtoh, double *du)
{
    double Fw[4], Fe[4], Gn[4], Gs[4];
    euler_rusanov(nb[3] + off, nb[4] + off, 0, gamma, Fw);
    euler_rusanov(nb[4] + off, nb[5] + off, 0, gamma, Fe);
    euler_rusanov(nb[1] + off, nb[4] + off, 1, gamma, Gn);
    euler_rusanov(nb[4] + off, nb[7] + off, 1, gamma, Gs);
    for (int k = 0; k < 4; ++k) {
        double div = (Fe[k] - Fw[k]) + (Gs[k] - Gn[k]);
        du[k] = -(dtoh * div);
    }
}

/* Two-stage strong-stability-preserving Runge-Kutta (Heun) as two sub-steps.
 * Slots 0..3 hold U^n, slots 4..7 the stage U*.
 * sub-step 0: U* = U + dt L(U)                 (slots 0..3 carried along)
 * sub-step 1: U' = 0.5 U + 0.5 (U* + dt L(U*)) (slots 4..7 := slots 0..3) */
static void st_euler(long long T, const double nb[9][MAXV], double *out, const double *prm)
{
    double gamma = prm[0], dtoh = prm[1];
    double du[4];
    const double *C = nb[4];
    if ((T & 1) == 0) {
        euler_increment(nb, 0, gamma, dtoh, du);
        for (int k = 0; k < 4; ++k) {
            out[k] = C[k];
            out[4 + k] = C[k] + du[k];
        }
    } else {
        euler_increment(nb, 4, gamma, dtoh, du);
        for (int k = 0; k < 4; ++k) {
            double v = 0.5 * C[k] + 0.5 * (C[4 + k] + du[k]);
            out[k] = v;
            out[4 + k] = v;
        }
    }
}

/* Euler in the paper's own discretisation (Sec. 8): conservative,
 * skew-symmetric central finite differences and a four-stage Runge-Kutta
 * step. The split (skew-symmetric) form of a convective derivative
 * d(m phi)/dx, with m the mass flux component and phi in {1, u, v, H},
 * H = (E + p) / rho, is half the sum of d(m phi), m d(phi) and phi d(m).
 * With central differences it is conservative: it equals the difference of
 * the face fluxes (m_L + m_R)(phi_L + phi_R) / 4; the pressure term takes
 * (p_L + p_R) / 2 on the face. Points are (rho, mx, my, E). */
/* Primitives from (rho, mx, my, E) through one reciprocal of the density
 * (the paper fixes no evaluation order; this is the order used here). */
static void eulerfd_prim(const double *U, double gamma, double *u, double *v, double *p, double *H)
{
    double rho = U[0], mx = U[1], my = U[2], en = U[3];
    double ri = 1.0 / rho;
    *u = mx * ri;
    *v = my * ri;
    *p = (gamma - 1.0) * (en - 0.5 * ((mx * mx + my * my) * ri));
    *H = (en + *p) * ri;
}

/* Face flux between the left / lower point L and the right / upper point R
 * along d (0 = x, 1 = y), arguments always in (left, right) order. */
static void eulerfd_face(const double *L, const double *R, int d, double gamma, double *F)
{
    double uL, vL, pL, HL, uR, vR, pR, HR;
    eulerfd_prim(L, gamma, &uL, &vL, &pL, &HL);
    eulerfd_prim(R, gamma, &uR, &vR, &pR, &HR);
    double a = 0.25 * (L[1 + d] + R[1 + d]);
    double pf = 0.5 * (pL + pR);
    F[0] = 2.0 * a;
    if (d == 0) {
        F[1] = a * (uL + uR) + pf;
        F[2] = a * (vL + vR);
    } else {
        F[1] = a * (uL + uR);
        F[2] = a * (vL + vR) + pf;
    }
    F[3] = a * (HL + HR);
}

/* The classical four-stage Runge-Kutta step as four sub-steps on the stage
 * values Y (slots 4..7): sub-step s forms r = h div F(Y) at the point (so
 * that dt L(Y) = -(dt/h) r) and, with U^n in slots 0..3 and the sum of the
 * stage derivatives K (slots 8..11, in units of -r):
 *   s = 0: K = -r;        Y = U - (dt/2h) r
 *   s = 1: K = K - 2 r;   Y = U - (dt/2h) r
 *   s = 2: K = K - 2 r;   Y = U - (dt/h) r
 *   s = 3: U = U + (dt/6h) (K - r);  Y = U;  K = 0
 * A state enters with Y = U and K = 0. Parameters: gamma, dt/h. */
static void st_eulerfd(long long T, const double nb[9][MAXV], double *out, const double *prm)
{
    double gamma = prm[0], dth = prm[1];
    const double *C = nb[4];
    double Fw[4], Fe[4], Gn[4], Gs[4];
    eulerfd_face(nb[3] + 4, C + 4, 0, gamma, Fw);
    eulerfd_face(C + 4, nb[5] + 4, 0, gamma, Fe);
    eulerfd_face(nb[1] + 4, C + 4, 1, gamma, Gn);
    eulerfd_face(C + 4, nb[7] + 4, 1, gamma, Gs);
    int s = (int)(T & 3);
    for (int k = 0; k < 4; ++k) {
        double r = (Fe[k] - Fw[k]) + (Gs[k] - Gn[k]);
        double U = C[k], K = C[8 + k];
        if (s == 0) {
            out[k] = U;
            out[8 + k] = -r;
            out[4 + k] = U - (0.5 * dth) * r;
        } else if (s == 1) {
            out[k] = U;
            out[8 + k] = K - 2.0 * r;
            out[4 + k] = U - (0.5 * dth) * r;
        } else if (s == 2) {
            out[k] = U;
            out[8 + k] = K - 2.0 * r;
            out[4 + k] = U - dth * r;
        } else {
            double v = U + (dth / 6.0) * (K - r);
            out[k] = v;
            out[4 + k] = v;
            out[8 + k] = 0.0;
        }
    }
}

static int pde_shape_ok(int pde, int nvars)
{
    switch (pde) {
    case PDE_HEAT5: return nvars == 1;
    case PDE_WAVE_LF: return nvars == 2;
    case PDE_EULER_RUS_RK2: return nvars == 8;
    case PDE_EULER_FD_RK4: return nvars == 12;
    case PDE_TEST_HASH: return nvars == 1;
    case PDE_TEST_INCR: return nvars == 1;
    case PDE_TEST_PUSH5: return nvars == 5;
    default: return 0;
    }
}

static int nparams_needed(int pde)
{
    switch (pde) {
    case PDE_HEAT5: return 1;
    case PDE_WAVE_LF: return 1;
    case PDE_EULER_RUS_RK2: return 2;
    case PDE_EULER_FD_RK4: return 2;
    default: return 0;
    }
}

/* Advance a doubly periodic FP64 state by nsub sub-steps, starting at global
 * sub-step index t0. Returns 0, or -1 on invalid arguments, -3 when out of
 * memory. */
int oracle_advance_f64(int pde, int nx, int ny, int nvars, const double *params, int nparams,
                       double *state, long long t0, long long nsub, int nthreads)
{
    if (nx < 1 || ny < 1 || nsub < 0 || t0 < 0 || !state || !pde_shape_ok(pde, nvars))
        return -1;
    if (nparams < nparams_needed(pde) || (nparams_needed(pde) > 0 && !params))
        return -1;
    if (nthreads < 1) nthreads = 1;
    size_t plane = (size_t)nx * (size_t)ny;
    double *tmp = (double *)malloc(plane * (size_t)nvars * sizeof(double));
    if (!tmp) return -3;
    double *cur = state, *nxt = tmp;
    for (long long s = 0; s < nsub; ++s) {
        long long T = t0 + s;
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int j = 0; j < ny; ++j) {
            double nb[9][MAXV];
            double out[MAXV];
            for (int i = 0; i < nx; ++i) {
                for (int dj = -1; dj <= 1; ++dj) {
                    int jj = (j + dj + ny) % ny;
                    for (int di = -1; di <= 1; ++di) {
                        int ii = (i + di + nx) % nx;
                        int k = 3 * (dj + 1) + (di + 1);
                        for (int v = 0; v < nvars; ++v)
                            nb[k][v] = cur[(size_t)v * plane + (size_t)jj * nx + ii];
                    }
                }
                switch (pde) {
                case PDE_HEAT5: st_heat(nb, out, params); break;
                case PDE_WAVE_LF: st_wave(nb, out, params); break;
                case PDE_EULER_RUS_RK2: st_euler(T, nb, out, params); break;
                case PDE_EULER_FD_RK4: st_eulerfd(T, nb, out, params); break;
                case PDE_TEST_HASH: st_hash(T, nb, out); break;
                case PDE_TEST_INCR: st_incr(nb, out); break;
                case PDE_TEST_PUSH5: st_push5(T, nb, out); break;
                }
                for (int v = 0; v < nvars; ++v)
                    nxt[(size_t)v * plane + (size_t)j * nx + i] = out[v];
            }
        }
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != state)
        memcpy(state, cur, plane * (size_t)nvars * sizeof(double));
    free(tmp);
    return 0;
}

/* ------------------------------------------------- FP32, compensated update
 *
 * The state is FP32 values u with, per value, an FP32 compensation term c
 * that is part of the state (it travels with the point).
 *
 * Heat and wave use Kahan's summation for the time update u += delta: with
 * y = delta - c, t = u + y, the new compensation is c = (t - u) - y (the
 * negative of the part of y that did not make it into t) and u = t.
 * Differences of neighbours are formed against the centre first, so for a
 * smooth field they are exact (Sterbenz).
 *
 * Euler keeps the flux and pressure arithmetic in FP64: the compensated value
 * (double)u - (double)c of every input is formed exactly in FP64, the whole
 * FP64 update is applied, and the FP64 result t is split back into
 * u = (float)t and c = (float)((double)u - t).
 *
 * In all three the pair (u, c) stands for the value u - c. */

static void st_heat_f32c(const float nu[9][MAXV], const float *cc, float *ou, float *oc, const double *prm)
{
    float r = (float)prm[0];
    float u = nu[4][0];
    float lap = ((nu[3][0] - u) + (nu[5][0] - u)) + ((nu[1][0] - u) + (nu[7][0] - u));
    float y = r * lap - cc[0];
    float t = u + y;
    oc[0] = (t - u) - y;
    ou[0] = t;
}

/* Leapfrog as u' = u + v with v = (u - p) + C2 lap; the compensated previous
 * difference (u - p) - (c_u - c_p) keeps the velocity accurate.
 *
 * The Laplacian is that of the compensated values u - c_u: the Laplacian of
 * the u's (Sterbenz-exact differences against the centre) minus the
 * Laplacian of the compensations, which are a rounding error in size, so
 * their own sum is accurate far below the FP32 unit of u. Leapfrog
 * integrates any error of lap into the velocity, so the Laplacian of the
 * uncompensated u's alone lets a per-step rounding of u accumulate. */
static void st_wave_f32c(const float nu[9][MAXV], const float nc[9][MAXV], float *ou, float *oc,
                         const double *prm)
{
    float c2 = (float)prm[0];
    float u = nu[4][0];
    float p = nu[4][1];
    float cu = nc[4][0], cp = nc[4][1];
    float lapu = ((nu[3][0] - u) + (nu[5][0] - u)) + ((nu[1][0] - u) + (nu[7][0] - u));
    float lapc = ((nc[3][0] + nc[5][0]) + (nc[1][0] + nc[7][0])) - 4.0f * cu;
    float lap = lapu - lapc;
    float v = ((u - p) - (cu - cp)) + c2 * lap;
    float y = v - cu;
    float t = u + y;
    oc[0] = (t - u) - y;
    ou[0] = t;
    ou[1] = u;
    oc[1] = cu;
}

static void split_f64(double t, float *u, float *c)
{
    float hi = (float)t;
    *u = hi;
    *c = (float)((double)hi - t);
}

static void st_euler_f32c(long long T, const float nu[9][MAXV], const float nc[9][MAXV], float *ou,
                          float *oc, const double *prm)
{
    double gamma = prm[0], dtoh = prm[1];
    double nb[9][MAXV];
    for (int k = 0; k < 9; ++k)
        for (int v = 0; v < 8; ++v)
            nb[k][v] = (double)nu[k][v] - (double)nc[k][v];
    double du[4];
    if ((T & 1) == 0) {
        euler_increment(nb, 0, gamma, dtoh, du);
        for (int k = 0; k < 4; ++k) {
            ou[k] = nu[4][k];
            oc[k] = nc[4][k];
            split_f64(nb[4][k] + du[k], &ou[4 + k], &oc[4 + k]);
        }
    } else {
        euler_increment(nb, 4, gamma, dtoh, du);
        for (int k = 0; k < 4; ++k) {
            double v = 0.5 * nb[4][k] + 0.5 * (nb[4][4 + k] + du[k]);
            split_f64(v, &ou[k], &oc[k]);
            ou[4 + k] = ou[k];
            oc[4 + k] = oc[k];
        }
    }
}

/* The paper's Euler discretisation (st_eulerfd) on FP32-compensated slots:
 * every input widened to the FP64 value u - c, the FP64 sub-step applied,
 * each slot the sub-step changes split back; slots it carries unchanged (the
 * conserved values U before the last stage) keep their pair as it is, and
 * the zeroed derivative sum is the pair (0, 0). */
static void st_eulerfd_f32c(long long T, const float nu[9][MAXV], const float nc[9][MAXV], float *ou,
                            float *oc, const double *prm)
{
    double nb[9][MAXV], out[MAXV];
    for (int k = 0; k < 9; ++k)
        for (int v = 0; v < 12; ++v)
            nb[k][v] = (double)nu[k][v] - (double)nc[k][v];
    st_eulerfd(T, nb, out, prm);
    const int last = (int)(T & 3) == 3;
    for (int v = 0; v < 12; ++v) {
        if (v < 4 && !last) {
            ou[v] = nu[4][v];
            oc[v] = nc[4][v];
        } else if (v >= 8 && last) {
            ou[v] = 0.0f;
            oc[v] = 0.0f;
        } else {
            split_f64(out[v], &ou[v], &oc[v]);
        }
    }
}

/* Advance an FP32-compensated state (u and c planes, each [nvars][ny][nx]).
 * Heat, wave and both Euler schemes have a compensated form. */
int oracle_advance_f32c(int pde, int nx, int ny, int nvars, const double *params, int nparams,
                        float *u, float *c, long long t0, long long nsub, int nthreads)
{
    if (nx < 1 || ny < 1 || nsub < 0 || t0 < 0 || !u || !c || !pde_shape_ok(pde, nvars))
        return -1;
    if (pde != PDE_HEAT5 && pde != PDE_WAVE_LF && pde != PDE_EULER_RUS_RK2 && pde != PDE_EULER_FD_RK4)
        return -1;
    if (nparams < nparams_needed(pde) || !params)
        return -1;
    if (nthreads < 1) nthreads = 1;
    size_t plane = (size_t)nx * (size_t)ny;
    size_t tot = plane * (size_t)nvars;
    float *tu = (float *)malloc(tot * sizeof(float));
    float *tc = (float *)malloc(tot * sizeof(float));
    if (!tu || !tc) {
        free(tu);
        free(tc);
        return -3;
    }
    float *cu = u, *cc = c, *xu = tu, *xc = tc;
    for (long long s = 0; s < nsub; ++s) {
        long long T = t0 + s;
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int j = 0; j < ny; ++j) {
            float nu[9][MAXV], ncp[9][MAXV];
            float ou[MAXV], oc[MAXV];
            for (int i = 0; i < nx; ++i) {
                for (int dj = -1; dj <= 1; ++dj) {
                    int jj = (j + dj + ny) % ny;
                    for (int di = -1; di <= 1; ++di) {
                        int ii = (i + di + nx) % nx;
                        int k = 3 * (dj + 1) + (di + 1);
                        for (int v = 0; v < nvars; ++v) {
                            nu[k][v] = cu[(size_t)v * plane + (size_t)jj * nx + ii];
                            ncp[k][v] = cc[(size_t)v * plane + (size_t)jj * nx + ii];
                        }
                    }
                }
                switch (pde) {
                case PDE_HEAT5: st_heat_f32c(nu, ncp[4], ou, oc, params); break;
                case PDE_WAVE_LF: st_wave_f32c(nu, ncp, ou, oc, params); break;
                case PDE_EULER_RUS_RK2: st_euler_f32c(T, nu, ncp, ou, oc, params); break;
                case PDE_EULER_FD_RK4: st_eulerfd_f32c(T, nu, ncp, ou, oc, params); break;
                }
                for (int v = 0; v < nvars; ++v) {
                    xu[(size_t)v * plane + (size_t)j * nx + i] = ou[v];
                    xc[(size_t)v * plane + (size_t)j * nx + i] = oc[v];
                }
            }
        }
        float *t = cu;
        cu = xu;
        xu = t;
        t = cc;
        cc = xc;
        xc = t;
    }
    if (cu != u) {
        memcpy(u, cu, tot * sizeof(float));
        memcpy(c, cc, tot * sizeof(float));
    }
    free(tu);
    free(tc);
    return 0;
}

/* ------------------------------- FP32, compensation kept within a residency
 *
 * The same compensated heat and wave updates, with only the values u part of
 * the state: what the swept rule's components exchange (panels) and store is
 * u, and a compensation c lives only while the point's successive levels are
 * computed by one workgroup in one window (a residency). A value that arrives
 * from another component, or from the stored state, comes with c = 0.
 *
 * Residencies of the swept schedule (Sec. 3-4) for an advance of S sub-steps
 * on tiles of side n, h = n/2: half cycle k holds levels L = k h + 1 ..
 * (k + 1) h of the advance (the last one possibly shorter), on the tiling
 * offset by (k mod 2) h in x and y. With dx, dy the point's distances to the
 * nearest tile edge of that tiling and l = L - k h, level L belongs to
 *   the upward pyramid          if dx >= l and dy >= l,
 *   the downward pyramid        if dx <  l and dy <  l,
 *   a bridge                    otherwise.
 * The first upward pyramid (holding level 0 too) is one residency. A downward
 * pyramid continues in its window as the next half cycle's upward pyramid on
 * the shifted tiling (the tile centred on its corner), so the two share one
 * residency; each half cycle's bridges are another. Numbered per point:
 * upward pyramid of half cycle k -> 2k, its bridge -> 2k + 1, its downward
 * pyramid -> 2k + 2. A point at level L reads a neighbour's level L - 1 with
 * its compensation only when both numbers agree (then they are the same
 * workgroup: components of one phase never read each other's points).
 * Tile side 0 stands for the per-step method: every level its own launch, so
 * no compensation survives a sub-step (plain FP32). */

static long long residency(int x, int y, long long L, int n, int nx, int ny)
{
    if (n < 0) return 0;
    if (n == 0) return L;
    if (L == 0) return 0;
    int h = n / 2;
    long long k = (L - 1) / h;
    int l = (int)((L - 1) % h) + 1;
    int off = (k & 1) ? h : 0;
    int lx = ((x - off) % nx + nx) % nx % n;
    int ly = ((y - off) % ny + ny) % ny % n;
    int dx = lx < n - 1 - lx ? lx : n - 1 - lx;
    int dy = ly < n - 1 - ly ? ly : n - 1 - ly;
    if (dx >= l && dy >= l) return 2 * k;
    if (dx < l && dy < l) return 2 * k + 2;
    return 2 * k + 1;
}

/* The wave in velocity form for the residency-confined compensation: slots
 * u and v = u^n - u^(n-1) (both public), compensations c_u and c_v.
 * Leapfrog u^(n+1) = 2u^n - u^(n-1) + C2 lap is, in exact arithmetic,
 * v' = v + C2 lap followed by u' = u + v'. Here v' is a compensated sum (the
 * pair tv, c_v' standing for tv - c_v'), and u' a compensated sum whose
 * increment is that pair, both compensations folded in first; lap as in the
 * FP32C wave (of the compensated values u - c_u). The velocity is the stored
 * variable, so a compensation dropped when a value changes window perturbs
 * u or v by half a unit of its own size, and the velocity's unit is far
 * below the displacement's; in the (u, u_prev) form the displacement's
 * rounding would enter the velocity u - u_prev and be integrated. */
static void st_wave_f32v(const float nu[9][MAXV], const float nc[9][MAXV], float *ou, float *oc,
                         const double *prm)
{
    float c2 = (float)prm[0];
    float u = nu[4][0];
    float v = nu[4][1];
    float cu = nc[4][0];
    float lapu = ((nu[3][0] - u) + (nu[5][0] - u)) + ((nu[1][0] - u) + (nu[7][0] - u));
    float lapc = ((nc[3][0] + nc[5][0]) + (nc[1][0] + nc[7][0])) - 4.0f * cu;
    float lap = lapu - lapc;
    float cv = nc[4][1];
    float yv = c2 * lap - cv;
    float tv = v + yv;
    float cv1 = (tv - v) - yv;
    float y = tv - (cu + cv1);
    float t = u + y;
    oc[0] = (t - u) - y;
    ou[0] = t;
    ou[1] = tv;
    oc[1] = cv1;
}

/* Residency number of point (x, y) at level L of an advance on tile side n
 * (exported for the pins). */
long long oracle_residency(int x, int y, long long L, int n, int nx, int ny)
{
    return residency(x, y, L, n, nx, ny);
}

/* One point of the wave's velocity form (st_wave_f32v) on a given 3x3
 * neighbourhood (exported for the pins): nu, nc are [9][2] (row-major
 * neighbours, north-west first; slots u, v), ou, oc [2]. */
void oracle_point_wave_f32v(const float *nu, const float *nc, float *ou, float *oc, double c2)
{
    float u9[9][MAXV], c9[9][MAXV];
    memset(u9, 0, sizeof u9);
    memset(c9, 0, sizeof c9);
    for (int k = 0; k < 9; ++k)
        for (int v = 0; v < 2; ++v) {
            u9[k][v] = nu[2 * k + v];
            c9[k][v] = nc[2 * k + v];
        }
    st_wave_f32v(u9, c9, ou, oc, &c2);
}

/* Advance u ([nvars][ny][nx] FP32) by nsub sub-steps from global sub-step t0
 * as one advance on tiles of side n (0: the per-step method). Heat (u) and
 * wave (u, v in velocity form) only. Returns 0, or -1 on invalid arguments,
 * -3 when out of memory. */
int oracle_advance_f32r(int pde, int nx, int ny, int nvars, const double *params, int nparams, float *u, int n,
                        long long t0, long long nsub, int nthreads)
{
    if (nx < 1 || ny < 1 || nsub < 0 || t0 < 0 || !u || !pde_shape_ok(pde, nvars))
        return -1;
    if (pde != PDE_HEAT5 && pde != PDE_WAVE_LF)
        return -1;
    if (nparams < nparams_needed(pde) || !params)
        return -1;
    if (n > 0 && ((n & 1) || n < 2 || nx % n || ny % n))
        return -1;
    if (n < -1)
        return -1;
    if (nthreads < 1) nthreads = 1;
    size_t plane = (size_t)nx * (size_t)ny;
    size_t tot = plane * (size_t)nvars;
    float *tu = (float *)malloc(tot * sizeof(float));
    float *c0 = (float *)calloc(tot, sizeof(float));
    float *c1 = (float *)malloc(tot * sizeof(float));
    long long *r0 = (long long *)malloc(plane * sizeof(long long));
    long long *r1 = (long long *)malloc(plane * sizeof(long long));
    if (!tu || !c0 || !c1 || !r0 || !r1) {
        free(tu);
        free(c0);
        free(c1);
        free(r0);
        free(r1);
        return -3;
    }
    float *cu = u, *cc = c0, *xu = tu, *xc = c1;
    long long *rprev = r0, *rcur = r1;  /* residency of every point at levels L - 1 and L */
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            rprev[(size_t)j * nx + i] = residency(i, j, 0, n, nx, ny);
    (void)t0; /* heat and wave apply the same operation at every sub-step */
    for (long long s = 0; s < nsub; ++s) {
        long long L = s + 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                rcur[(size_t)j * nx + i] = residency(i, j, L, n, nx, ny);
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int j = 0; j < ny; ++j) {
            float nu[9][MAXV], ncp[9][MAXV];
            float ou[MAXV], oc[MAXV];
            for (int i = 0; i < nx; ++i) {
                long long rp = rcur[(size_t)j * nx + i];
                for (int dj = -1; dj <= 1; ++dj) {
                    int jj = (j + dj + ny) % ny;
                    for (int di = -1; di <= 1; ++di) {
                        int ii = (i + di + nx) % nx;
                        int k = 3 * (dj + 1) + (di + 1);
                        int same = rprev[(size_t)jj * nx + ii] == rp;
                        for (int v = 0; v < nvars; ++v) {
                            nu[k][v] = cu[(size_t)v * plane + (size_t)jj * nx + ii];
                            ncp[k][v] = same ? cc[(size_t)v * plane + (size_t)jj * nx + ii] : 0.0f;
                        }
                    }
                }
                switch (pde) {
                case PDE_HEAT5: st_heat_f32c(nu, ncp[4], ou, oc, params); break;
                case PDE_WAVE_LF: st_wave_f32v(nu, ncp, ou, oc, params); break;
                }
                for (int v = 0; v < nvars; ++v) {
                    xu[(size_t)v * plane + (size_t)j * nx + i] = ou[v];
                    xc[(size_t)v * plane + (size_t)j * nx + i] = oc[v];
                }
            }
        }
        float *t = cu;
        cu = xu;
        xu = t;
        t = cc;
        cc = xc;
        xc = t;
        long long *tr = rprev;
        rprev = rcur;
        rcur = tr;
    }
    if (cu != u)
        memcpy(u, cu, tot * sizeof(float));
    free(tu);
    free(c0);
    free(c1);
    free(r0);
    free(r1);
    return 0;
}

/* ------------------------------------------ a stencil reaching two rings
 *
 * Sec. 2 asks a stencil that reads beyond its nearest neighbours to be split
 * into nearest-neighbour sub-steps; the split must compute the same values
 * as the stencil itself, so the oracle is the stencil applied directly, one
 * full step at a time: the 25-point test hash, an order-sensitive 64-bit mix
 * of the values at offsets |di|, |dj| <= 2 in row-major order (north west
 * first) seeded with the step index k (integers below 2^52 held in doubles). */
static double st_hash25(long long k, const double *u, int nx, int ny, int i, int j)
{
    uint64_t h = 0xC2B2AE3D27D4EB4Full ^ (uint64_t)k;
    for (int dj = -2; dj <= 2; ++dj) {
        int jj = ((j + dj) % ny + ny) % ny;
        for (int di = -2; di <= 2; ++di) {
            int ii = ((i + di) % nx + nx) % nx;
            h ^= (uint64_t)u[(size_t)jj * nx + ii];
            h *= 0xFF51AFD7ED558CCDull;
            h ^= h >> 32;
        }
    }
    return (double)(h >> 12);
}

/* Advance the scalar field u ([ny][nx]) by nsteps applications of the
 * 25-point hash, the first with step index k0. */
int oracle_advance_hash25(int nx, int ny, double *u, long long k0, long long nsteps, int nthreads)
{
    if (nx < 1 || ny < 1 || nsteps < 0 || k0 < 0 || !u)
        return -1;
    if (nthreads < 1) nthreads = 1;
    size_t plane = (size_t)nx * (size_t)ny;
    double *tmp = (double *)malloc(plane * sizeof(double));
    if (!tmp) return -3;
    double *cur = u, *nxt = tmp;
    for (long long s = 0; s < nsteps; ++s) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                nxt[(size_t)j * nx + i] = st_hash25(k0 + s, cur, nx, ny, i, j);
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != u)
        memcpy(u, cur, plane * sizeof(double));
    free(tmp);
    return 0;
}

/* ------------------------------------------------------------------- 3D
 *
 * The swept rule in three dimensions (Sec. 1 motivates it with 3D grids):
 * the same plain definition on a triply periodic grid, state[z][y][x] with
 * x fastest, one value per point. Neighbour k = 9 (dz + 1) + 3 (dy + 1) +
 * (dx + 1) of the 3x3x3 neighbourhood.
 *   heat, 7 points: t = ((u_W + u_E) + (u_N + u_S)) + (u_B + u_F),
 *     lap = t - 6u, u' = u + r lap (B / F: z - 1 / z + 1); params {r}
 *   test hash, 27 points: an order-sensitive 64-bit mix of the 27 values
 *     (k = 0..26) seeded with the sub-step index; integers below 2^52. */
#define PDE3_HEAT7 1
#define PDE3_TEST_HASH27 100

static double st3_heat(const double nb[27], const double *prm)
{
    double u = nb[13];
    double t = ((nb[12] + nb[14]) + (nb[10] + nb[16])) + (nb[4] + nb[22]);
    double lap = t - 6.0 * u;
    return u + prm[0] * lap;
}

static double st3_hash(long long T, const double nb[27])
{
    uint64_t h = 0x94D049BB133111EBull ^ (uint64_t)T;
    for (int k = 0; k < 27; ++k) {
        h ^= (uint64_t)nb[k];
        h *= 0xFF51AFD7ED558CCDull;
        h ^= h >> 32;
    }
    return (double)(h >> 12);
}

int oracle_advance3d_f64(int pde, int nx, int ny, int nz, const double *params, int nparams, double *state,
                         long long t0, long long nsub, int nthreads)
{
    if (nx < 1 || ny < 1 || nz < 1 || nsub < 0 || t0 < 0 || !state)
        return -1;
    if (pde != PDE3_HEAT7 && pde != PDE3_TEST_HASH27)
        return -1;
    if (pde == PDE3_HEAT7 && (nparams < 1 || !params))
        return -1;
    if (nthreads < 1) nthreads = 1;
    size_t tot = (size_t)nx * ny * nz;
    double *tmp = (double *)malloc(tot * sizeof(double));
    if (!tmp) return -3;
    double *cur = state, *nxt = tmp;
    for (long long s = 0; s < nsub; ++s) {
        long long T = t0 + s;
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int k = 0; k < nz; ++k) {
            double nb[27];
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    for (int dk = -1; dk <= 1; ++dk)
                        for (int dj = -1; dj <= 1; ++dj)
                            for (int di = -1; di <= 1; ++di) {
                                int kk = (k + dk + nz) % nz, jj = (j + dj + ny) % ny, ii = (i + di + nx) % nx;
                                nb[9 * (dk + 1) + 3 * (dj + 1) + (di + 1)] =
                                    cur[((size_t)kk * ny + jj) * nx + ii];
                            }
                    nxt[((size_t)k * ny + j) * nx + i] =
                        pde == PDE3_HEAT7 ? st3_heat(nb, params) : st3_hash(T, nb);
                }
        }
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != state)
        memcpy(state, cur, tot * sizeof(double));
    free(tmp);
    return 0;
}
