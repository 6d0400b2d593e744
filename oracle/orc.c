/*
 * orc.c -- CPU oracle for the DPD solvent step (Mirheo, arXiv 1911.04712).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * reference against which the GPU library is checked.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it.  It
 * shares no source, header, table or helper with the HIP path, and the HIP
 * path never loads it.
 *
 * Everything is FP64.  Each function names the passage it follows:
 *
 *   - equations of motion ................ Sec. 2.1, Eq. (1)
 *   - DPD force sum, C/D/R terms ......... Sec. 2.1, Eqs. (2)-(5), with the
 *                                          fluctuation-dissipation relation
 *                                          w_D = w_R^2, sigma^2 = 2 gamma kT
 *                                          and the kernel w_R = w^k
 *   - cell lists (edge r_c, sort by cell)  Sec. 3.2
 *   - fused velocity-Verlet (kick, drift)  Sec. 3.1, time-stepping step 5
 *   - periodic Poiseuille body force ..... Sec. 4.2, Eq. (11)
 *   - walls: SDF surface, frozen particles, Sec. 2.3; bounce-back at the
 *     SDF's zero along the drift, Sec. 3.3; rotating coaxial cylinders of
 *     the Taylor-Couette test, Sec. 4.3
 *   - several species with their own a, gamma and cutoff per pair of
 *     species (fluids of different viscosity side by side: Sec. 2.3,
 *     Sec. 5.2, Sec. 5.3; several cutoffs: Sec. 3.1); kT, dt and the mass
 *     stay shared; cutoffs stay within the cell edge
 *   - random term: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 *     random numbers: as easy as 1, 2, 3", SC'11) followed by the
 *     Box-Muller transform (Box & Muller 1958).  The paper names no
 *     generator; it requires xi_ij = xi_ji, zero mean, unit variance and
 *     independence per pair and per step (Sec. 2.1).
 *
 * Readings where the paper is silent are listed at each use and in the
 * design notes of the repository (integrator form, which velocity enters
 * the dissipative force, noise discretisation xi/sqrt(dt), coincident
 * particles, body-force tie, time-centred kT estimator).
 *
 * Units: r_c = 1, so the cell edge is 1 and a box of L_x x L_y x L_z cells
 * has edges L_x, L_y, L_z.  Fully periodic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double a;          /* conservative amplitude (alpha in Eq. 3)          */
    double gamma;      /* dissipative coefficient (Eq. 5)                  */
    double kT;         /* k_B T; sigma = sqrt(2 gamma kT)                  */
    double dt;         /* time step                                        */
    double mass;       /* particle mass m (Eq. 1)                          */
    double body_f;     /* periodic-Poiseuille amplitude f (Eq. 11); 0=off  */
    int32_t flow_axis; /* axis the body force acts along                   */
    int32_t grad_axis; /* axis whose coordinate selects the force sign     */
    double kexp;       /* kernel exponent k of w_R = w^k, 0 < k <= 1 (Sec. 2.1);
                          0 means k = 1                                   */
    int32_t ntypes;    /* species; 0 or 1: one species with (a, gamma)     */
    int32_t reserved;
    const int32_t* type; /* species of each particle (row of x), ntypes > 1 */
    const double* a_tab; /* ntypes x ntypes, symmetric: a of species pair  */
    const double* g_tab; /* ntypes x ntypes, symmetric: gamma of the pair  */
    int32_t body_uniform; /* 1: body force +f along flow_axis everywhere (pipe
                             or channel flow); 0: Eq. 11's two halves        */
    int32_t wall_kind;   /* walls (Sec. 2.3): 0 none; 1 two plates normal to
                            grad_axis, fluid where |y - L/2| < wall_h; 2 a pipe
                            along flow_axis through the box centre, fluid
                            where the distance to its axis is < wall_h       */
    double wall_h;       /* plate half-gap or pipe radius                    */
    const uint8_t* frozen; /* per particle: 1 = frozen wall particle, which
                              interacts but never moves; NULL = none         */
    double rc;           /* cutoff of the pair, 0 < rc <= 1 (the cell edge);
                            0 means 1                                        */
    const double* rc_tab; /* ntypes x ntypes, symmetric: cutoff per species
                             pair (NULL: every pair at rc)                   */
    double wall_r_in;    /* wall_kind 3: two coaxial cylinders along
                            flow_axis through the box centre, fluid where
                            wall_r_in < distance to the axis < wall_h     */
    double omega_in, omega_out; /* their angular velocities about the axis
                            (right-handed about +flow_axis); every wall has
                            a velocity field omega x r and frozen particles
                            carry it                                       */
} orc_params;

typedef struct {
    double momentum[3]; /* sum m v^{n+1/2}                                  */
    double ke_half;     /* sum m |v^{n+1/2}|^2 / 2                          */
    double ke_centred;  /* sum m |v^{n-1/2} + dt f^n/(2m)|^2 / 2            */
    double kT_centred;  /* 2 ke_centred / (3 (N-1))                         */
    double virial;      /* sum_{i<j} r_ij . F^C_ij at x^n                   */
    double pressure;    /* rho kT_centred + virial / (3 V)                  */
} orc_diag;

/* ------------------------------------------------------------------ */
/* Philox4x32-10, written from its published definition (SC'11, Sec. 4) */
/* ------------------------------------------------------------------ */

/* Round multipliers and Weyl key increments of Philox4x32. */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {               /* the key is bumped between rounds */
            k0 += ORC_PHILOX_W0;
            k1 += ORC_PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)ORC_PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)ORC_PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_philox_batch(int64_t n, const uint32_t* ctr4, const uint32_t key[2], uint32_t* out4)
{
    for (int64_t i = 0; i < n; ++i)
        orc_philox4x32_10(ctr4 + 4 * i, key, out4 + 4 * i);
}

/* Box-Muller on two 24-bit uniforms: u1 in (0,1], u2 in [0,1). */
double orc_box_muller(uint32_t w0, uint32_t w1)
{
    const double two_m24 = 1.0 / 16777216.0;
    double u1 = ((double)(w0 >> 8) + 1.0) * two_m24;
    double u2 = (double)(w1 >> 8) * two_m24;
    const double two_pi = 6.283185307179586476925286766559;
    return sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
}

void orc_box_muller_batch(int64_t n, const uint32_t* w0, const uint32_t* w1, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = orc_box_muller(w0[i], w1[i]);
}

/* Philox words for the unordered pair {id_a, id_b} at force evaluation
 * `step` of a run with `seed`: counter (min id, max id, step mod 2^32, 0),
 * key (seed mod 2^32, seed >> 32).  Symmetric in (id_a, id_b) by
 * construction, which gives xi_ij = xi_ji (Sec. 2.1). */
void orc_pair_words(uint32_t id_a, uint32_t id_b, uint64_t step, uint64_t seed, uint32_t out[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = id_a < id_b ? id_a : id_b;
    ctr[1] = id_a < id_b ? id_b : id_a;
    ctr[2] = (uint32_t)step;
    ctr[3] = 0u;
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    orc_philox4x32_10(ctr, key, out);
}

double orc_xi(uint32_t id_a, uint32_t id_b, uint64_t step, uint64_t seed)
{
    uint32_t w[4];
    orc_pair_words(id_a, id_b, step, seed, w);
    return orc_box_muller(w[0], w[1]);
}

void orc_xi_batch(int64_t n, const uint32_t* id_a, const uint32_t* id_b, const uint64_t* step,
                  uint64_t seed, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = orc_xi(id_a[i], id_b[i], step[i], seed);
}

/* ------------------------------------------------------------------ */
/* Cell lists (Sec. 3.2)                                                */
/* ------------------------------------------------------------------ */

static int32_t orc_cell_coord(double x, int32_t L)
{
    /* Unit cells: the cell coordinate is floor(x), clamped to [0, L-1] so a
     * coordinate that rounds onto the upper face stays in the box. */
    double f = floor(x);
    int32_t c = (int32_t)f;
    if (f < 0.0) c = 0;
    if (c > L - 1) c = L - 1;
    return c;
}

static int64_t orc_cell_of(const double* r, const int32_t cells[3])
{
    int64_t cx = orc_cell_coord(r[0], cells[0]);
    int64_t cy = orc_cell_coord(r[1], cells[1]);
    int64_t cz = orc_cell_coord(r[2], cells[2]);
    return cx + (int64_t)cells[0] * (cy + (int64_t)cells[1] * cz); /* x fastest */
}

/* Stable counting sort of particles by cell: histogram of cell sizes,
 * exclusive scan into cell starts, then placement in input order, so that
 * inside a cell particles keep their previous relative order.
 * order[k] = input index of the k-th particle in cell order;
 * cell_start has n_cells + 1 entries. */
static int orc_bin_f64(int64_t n, const double* x, const int32_t cells[3], int64_t* order,
                       int32_t* cell_start)
{
    int64_t nc = (int64_t)cells[0] * cells[1] * cells[2];
    int64_t* fill = (int64_t*)calloc((size_t)nc, sizeof(int64_t));
    int64_t* key = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!fill || !key) { free(fill); free(key); return -2; }
    for (int64_t i = 0; i < n; ++i) {
        key[i] = orc_cell_of(x + 3 * i, cells);
        fill[key[i]] += 1;
    }
    int64_t run = 0;
    for (int64_t c = 0; c < nc; ++c) {
        cell_start[c] = (int32_t)run;
        run += fill[c];
        fill[c] = 0;
    }
    cell_start[nc] = (int32_t)run;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = key[i];
        order[cell_start[c] + fill[c]] = i;
        fill[c] += 1;
    }
    free(fill);
    free(key);
    return 0;
}

/* The same binning, taking FP32 coordinates exactly as the GPU stores them.
 * The FP32 value is widened exactly to FP64 before flooring. */
int orc_bin(int64_t n, const float* pos3, const int32_t cells[3], int64_t* order, int32_t* cell_start)
{
    double* x = (double*)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    if (!x) return -2;
    for (int64_t i = 0; i < 3 * n; ++i) x[i] = (double)pos3[i];
    int rc = orc_bin_f64(n, x, cells, order, cell_start);
    free(x);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Pair force (Sec. 2.1, Eqs. 3-5)                                      */
/* ------------------------------------------------------------------ */

/* Force on i from j.  Minimum-image displacement r_ij = r_i - r_j, unit
 * vector e_ij = r_ij / r_ij, weight w = 1 - r / r_c (Eq. 4; r_c = p->rc, 1
 * unless a species pair sets its own) of the conservative term, random-term
 * kernel w_R = w^k and dissipative kernel w_D = w_R^2 (Sec. 2.1),
 * v_ij = v_i - v_j, sigma = sqrt(2 gamma kT), and the white noise
 * discretised as xi / sqrt(dt).  Pairs at r >= r_c, and a pair at r = 0
 * (where e_ij is undefined), contribute nothing.
 * Outputs: F (total pair force on i), Fc (conservative part), mag (sum of
 * the magnitudes of the three terms, the scale of the rounding error).
 * xi_ij is drawn for the pair's ids at force evaluation `step`.
 * Returns 1 when the pair interacts. */
int orc_pair_force(const double ri[3], const double rj[3], const double vi[3], const double vj[3],
                   const double box[3], const orc_params* p, uint32_t id_i, uint32_t id_j,
                   uint64_t step, uint64_t seed, double F[3], double Fc[3], double* mag)
{
    double d[3];
    for (int k = 0; k < 3; ++k) {
        double dk = ri[k] - rj[k];
        d[k] = dk - box[k] * nearbyint(dk / box[k]);
    }
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    F[0] = F[1] = F[2] = 0.0;
    Fc[0] = Fc[1] = Fc[2] = 0.0;
    *mag = 0.0;
    double rc = p->rc > 0.0 ? p->rc : 1.0;
    if (!(r2 < rc * rc) || r2 == 0.0) return 0;
    double r = sqrt(r2);
    double w = 1.0 - r / rc;
    double e[3] = {d[0] / r, d[1] / r, d[2] / r};
    double ev = e[0] * (vi[0] - vj[0]) + e[1] * (vi[1] - vj[1]) + e[2] * (vi[2] - vj[2]);
    double sigma = sqrt(2.0 * p->gamma * p->kT);
    double xi = orc_xi(id_i, id_j, step, seed);
    double wr = (p->kexp == 0.0 || p->kexp == 1.0) ? w : pow(w, p->kexp);
    double fC = p->a * w;
    double fD = -p->gamma * wr * wr * ev;
    double fR = sigma * wr * xi / sqrt(p->dt);
    double fs = fC + fD + fR;
    for (int k = 0; k < 3; ++k) {
        F[k] = fs * e[k];
        Fc[k] = fC * e[k];
    }
    *mag = fabs(fC) + fabs(fD) + fabs(fR);
    return 1;
}

/* Periodic-Poiseuille body force (Sec. 4.2, Eq. 11): -f along the flow
 * axis where the gradient coordinate is <= L/2, +f otherwise; or a uniform
 * +f (body_uniform), the drive of flow between walls. */
static double orc_body_force(const double* r, const int32_t cells[3], const orc_params* p)
{
    if (p->body_f == 0.0) return 0.0;
    if (p->body_uniform) return p->body_f;
    double half = 0.5 * (double)cells[p->grad_axis];
    return r[p->grad_axis] <= half ? -p->body_f : p->body_f;
}

/* Parameters of the pair of particles (rows) i and j: with several species
 * the pair takes a and gamma of its species pair (s, t) from the symmetric
 * tables, so F_ij = -F_ji still holds; everything else is shared. */
static orc_params orc_pair_params(const orc_params* p, int64_t i, int64_t j)
{
    orc_params q = *p;
    if (p->ntypes > 1) {
        int64_t k = (int64_t)p->type[i] * p->ntypes + p->type[j];
        q.a = p->a_tab[k];
        q.gamma = p->g_tab[k];
        if (p->rc_tab) q.rc = p->rc_tab[k];
    }
    return q;
}

/* Force on one particle i, gathering over its 27 neighbour cells (or over
 * all particles when brute != 0).  Writes f[3] (pair sum + body force),
 * *s (error scale) and adds i's half of the conservative virial. */
static void orc_force_on(int64_t i, int64_t n, const double* x, const double* v, const uint32_t* id,
                         const int32_t cells[3], const double box[3], const orc_params* p,
                         uint64_t step, uint64_t seed, int brute, const int64_t* order,
                         const int32_t* cell_start, double f[3], double* s, double* virial_half)
{
    double acc[3] = {0.0, 0.0, 0.0};
    double scale = 0.0, vir = 0.0;
    const double* ri = x + 3 * i;
    const double* vi = v + 3 * i;
    if (brute) {
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double F[3], Fc[3], mag;
            orc_params q = orc_pair_params(p, i, j);
            if (orc_pair_force(ri, x + 3 * j, vi, v + 3 * j, box, &q, id[i], id[j], step, seed, F, Fc,
                               &mag)) {
                double d[3];
                for (int k = 0; k < 3; ++k) {
                    double dk = ri[k] - x[3 * j + k];
                    d[k] = dk - box[k] * nearbyint(dk / box[k]);
                    acc[k] += F[k];
                }
                scale += mag;
                vir += 0.5 * (d[0] * Fc[0] + d[1] * Fc[1] + d[2] * Fc[2]);
            }
        }
    } else {
        int32_t c[3];
        for (int k = 0; k < 3; ++k) c[k] = orc_cell_coord(ri[k], cells[k]);
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int32_t nx = (c[0] + dx + cells[0]) % cells[0];
                    int32_t ny = (c[1] + dy + cells[1]) % cells[1];
                    int32_t nz = (c[2] + dz + cells[2]) % cells[2];
                    int64_t cell = nx + (int64_t)cells[0] * (ny + (int64_t)cells[1] * nz);
                    for (int32_t k = cell_start[cell]; k < cell_start[cell + 1]; ++k) {
                        int64_t j = order[k];
                        if (j == i) continue;
                        double F[3], Fc[3], mag;
                        orc_params q = orc_pair_params(p, i, j);
                        if (orc_pair_force(ri, x + 3 * j, vi, v + 3 * j, box, &q, id[i], id[j], step,
                                           seed, F, Fc, &mag)) {
                            double d[3];
                            for (int q = 0; q < 3; ++q) {
                                double dq = ri[q] - x[3 * j + q];
                                d[q] = dq - box[q] * nearbyint(dq / box[q]);
                                acc[q] += F[q];
                            }
                            scale += mag;
                            vir += 0.5 * (d[0] * Fc[0] + d[1] * Fc[1] + d[2] * Fc[2]);
                        }
                    }
                }
    }
    double fb = orc_body_force(ri, cells, p);
    acc[p->flow_axis] += fb;
    scale += fabs(fb);
    f[0] = acc[0]; f[1] = acc[1]; f[2] = acc[2];
    *s = scale;
    *virial_half = vir;
}

/* Signed distance to the wall surface (Sec. 2.3): negative in the fluid,
 * zero on the wall surface, positive inside the wall. */
double orc_sdf(const double* r, const int32_t cells[3], const orc_params* p)
{
    if (p->wall_kind == 1) {
        double y = r[p->grad_axis] - 0.5 * (double)cells[p->grad_axis];
        return fabs(y) - p->wall_h;
    }
    if (p->wall_kind == 2 || p->wall_kind == 3) {
        double q2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            if (k == p->flow_axis) continue;
            double c = r[k] - 0.5 * (double)cells[k];
            q2 += c * c;
        }
        double q = sqrt(q2);
        if (p->wall_kind == 2) return q - p->wall_h;
        return fmax(p->wall_r_in - q, q - p->wall_h);
    }
    return -1.0;
}

/* Velocity of the wall surface nearest to r: omega x (r - axis), with the
 * inner cylinder's omega inside the mid radius and the outer one's outside
 * (Sec. 4.3); zero for plates and pipes. */
void orc_wall_velocity(const double* r, const int32_t cells[3], const orc_params* p, double u[3])
{
    u[0] = u[1] = u[2] = 0.0;
    if (p->wall_kind != 3) return;
    int a1 = (p->flow_axis + 1) % 3, a2 = (p->flow_axis + 2) % 3;   /* right-handed about the axis */
    double c1 = r[a1] - 0.5 * (double)cells[a1], c2 = r[a2] - 0.5 * (double)cells[a2];
    double q = sqrt(c1 * c1 + c2 * c2);
    double om = q < 0.5 * (p->wall_r_in + p->wall_h) ? p->omega_in : p->omega_out;
    u[a1] = -om * c2;
    u[a2] = om * c1;
}

/* Bounce-back (Sec. 3.3): a particle whose drift from x0 by dx ends inside
 * the wall is placed at the collision point, the zero of the SDF along the
 * drift (found by bisection; the fluid-side end of the final bracket), and
 * its velocity is reversed in the frame of the wall there: v -> 2 u_w - v
 * (v -> -v for walls at rest).  Returns 1 on a bounce. */
static int orc_bounce(const double x0[3], const double dx[3], double x[3], double v[3], const int32_t cells[3],
                      const orc_params* p)
{
    if (!p->wall_kind || orc_sdf(x, cells, p) <= 0.0) return 0;
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 60; ++it) {
        double mid = 0.5 * (lo + hi), m[3];
        for (int k = 0; k < 3; ++k) m[k] = x0[k] + mid * dx[k];
        if (orc_sdf(m, cells, p) > 0.0) hi = mid; else lo = mid;
    }
    for (int k = 0; k < 3; ++k) x[k] = x0[k] + lo * dx[k];
    double u[3];
    orc_wall_velocity(x, cells, p, u);
    for (int k = 0; k < 3; ++k) v[k] = 2.0 * u[k] - v[k];
    return 1;
}

/* A frozen particle of a turning cylinder turns with it: its position is
 * rotated about the axis by omega dt each step (the surface, and so the
 * SDF, is unchanged by the rotation) and its velocity is the wall velocity
 * at the new position.  Frozen particles of resting walls keep position and
 * velocity.  Moving the layer with its wall, rather than only giving it the
 * wall's velocity, keeps the static corrugation of fixed particles from
 * dragging the fluid back towards rest. */
static void orc_move_frozen(double* x, double* v, const int32_t cells[3], const orc_params* p)
{
    if (p->wall_kind != 3) return;
    int a1 = (p->flow_axis + 1) % 3, a2 = (p->flow_axis + 2) % 3;
    double c1 = x[a1] - 0.5 * (double)cells[a1], c2 = x[a2] - 0.5 * (double)cells[a2];
    double q = sqrt(c1 * c1 + c2 * c2);
    double om = q < 0.5 * (p->wall_r_in + p->wall_h) ? p->omega_in : p->omega_out;
    if (om == 0.0) return;
    double ph = om * p->dt, cs = cos(ph), sn = sin(ph);
    x[a1] = 0.5 * (double)cells[a1] + cs * c1 - sn * c2;
    x[a2] = 0.5 * (double)cells[a2] + sn * c1 + cs * c2;
    orc_wall_velocity(x, cells, p, v);
}

static int orc_check(const int32_t cells[3], const orc_params* p)
{
    for (int k = 0; k < 3; ++k)
        if (cells[k] < 3) return -1;      /* 27 distinct neighbour cells need L >= 3 */
    if (!(p->dt > 0.0) || !(p->mass > 0.0) || p->gamma < 0.0 || p->kT < 0.0) return -1;
    if (!(p->kexp >= 0.0 && p->kexp <= 1.0)) return -1;
    if (p->flow_axis < 0 || p->flow_axis > 2 || p->grad_axis < 0 || p->grad_axis > 2) return -1;
    if (p->flow_axis == p->grad_axis) return -1;
    if (p->ntypes < 0 || p->ntypes > 64) return -1;
    if (p->wall_kind < 0 || p->wall_kind > 3 || (p->wall_kind && !(p->wall_h > 0.0))) return -1;
    if (p->wall_kind == 3 && !(p->wall_r_in > 0.0 && p->wall_r_in < p->wall_h)) return -1;
    if (p->ntypes > 1) {
        if (!p->type || !p->a_tab || !p->g_tab) return -1;
        for (int s = 0; s < p->ntypes; ++s)
            for (int t = 0; t < p->ntypes; ++t) {
                double a = p->a_tab[s * p->ntypes + t], g = p->g_tab[s * p->ntypes + t];
                if (!isfinite(a) || !isfinite(g) || g < 0.0) return -1;
                if (a != p->a_tab[t * p->ntypes + s] || g != p->g_tab[t * p->ntypes + s]) return -1;
                if (p->rc_tab) {
                    double c = p->rc_tab[s * p->ntypes + t];
                    if (!(c > 0.0 && c <= 1.0) || c != p->rc_tab[t * p->ntypes + s]) return -1;
                }
            }
    }
    if (!(p->rc >= 0.0 && p->rc <= 1.0)) return -1;
    return 0;
}

/* Every particle's species in [0, ntypes). */
static int orc_check_types(int64_t n, const orc_params* p)
{
    if (p->ntypes <= 1) return 0;
    for (int64_t i = 0; i < n; ++i)
        if (p->type[i] < 0 || p->type[i] >= p->ntypes) return -1;
    return 0;
}

/* Forces at one instant.  If `which` is NULL all n particles are evaluated
 * (outputs n x 3 / n); otherwise only the m listed particles (outputs
 * m x 3 / m).  brute != 0 uses the O(N^2) minimum-image sum instead of
 * cell lists.  *virial (may be NULL) receives sum_{i<j} r_ij . F^C_ij when
 * all particles are evaluated. */
int orc_forces(int64_t n, const double* x, const double* v, const uint32_t* id,
               const int32_t cells[3], const orc_params* p, uint64_t step, uint64_t seed,
               int brute, int64_t m, const int64_t* which, double* f, double* s, double* virial)
{
    if (orc_check(cells, p) || orc_check_types(n, p)) return -1;
    double box[3] = {(double)cells[0], (double)cells[1], (double)cells[2]};
    int64_t nc = (int64_t)cells[0] * cells[1] * cells[2];
    int64_t* order = NULL;
    int32_t* cell_start = NULL;
    if (!brute) {
        order = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
        cell_start = (int32_t*)malloc((size_t)(nc + 1) * sizeof(int32_t));
        if (!order || !cell_start) { free(order); free(cell_start); return -2; }
        if (orc_bin_f64(n, x, cells, order, cell_start)) { free(order); free(cell_start); return -2; }
    }
    int64_t count = which ? m : n;
    double vir_total = 0.0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : vir_total)
    for (int64_t t = 0; t < count; ++t) {
        int64_t i = which ? which[t] : t;
        double vh;
        orc_force_on(i, n, x, v, id, cells, box, p, step, seed, brute, order, cell_start,
                     f + 3 * t, s + t, &vh);
        vir_total += vh;
    }
    if (virial) *virial = which ? 0.0 : vir_total;
    free(order);
    free(cell_start);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Time stepping (Sec. 3.1, step 5; Eq. 1)                             */
/* ------------------------------------------------------------------ */

/* Advance nsteps steps.  State: x (n x 3, wrapped into [0, L)), v (n x 3)
 * holding the half-step velocity v^{n-1/2}, ids, seed and the index step0
 * of the next force evaluation.  Each step:
 *   1. forces f^n at (x^n, v^{n-1/2}) through the cell list, plus the body
 *      force;
 *   2. diagnostics at time level n (time-centred velocity
 *      v^{n-1/2} + dt f^n / (2m)), profile of the flow velocity over
 *      `nbins` slabs along the gradient axis;
 *   3. kick v^{n+1/2} = v^{n-1/2} + dt f^n / m, then drift
 *      x^{n+1} = x^n + dt v^{n+1/2}, bounce-back off the walls (Sec. 3.3),
 *      then periodic wrap;
 *   4. momentum and KE of v^{n+1/2}.
 * Frozen wall particles (Sec. 2.3) take part in the forces, move only with
 * their wall (a turning cylinder turns them, orc_move_frozen) and are not
 * counted in the diagnostics (kT uses 3 (N_fluid - 1) degrees of freedom)
 * or the profile.
 * diag (nsteps entries), prof_sum / prof_cnt (nbins, accumulated) and
 * f_last (n x 3, forces of the last step) may each be NULL. */
int orc_step(int64_t n, double* x, double* v, const uint32_t* id, const int32_t cells[3],
             const orc_params* p, uint64_t seed, uint64_t step0, int64_t nsteps, int32_t nbins,
             orc_diag* diag, double* prof_sum, double* prof_cnt, double* f_last)
{
    if (orc_check(cells, p) || orc_check_types(n, p)) return -1;
    if (n < 2 || nsteps < 0) return -1;
    double box[3] = {(double)cells[0], (double)cells[1], (double)cells[2]};
    double vol = box[0] * box[1] * box[2];
    int64_t nfluid = n;                 /* diagnostics cover the moving particles only */
    if (p->frozen)
        for (int64_t i = 0; i < n; ++i) nfluid -= p->frozen[i] ? 1 : 0;
    if (nfluid < 2) return -1;
    double* f = (double*)malloc((size_t)n * 3 * sizeof(double));
    double* s = (double*)malloc((size_t)n * sizeof(double));
    if (!f || !s) { free(f); free(s); return -2; }
    for (int64_t it = 0; it < nsteps; ++it) {
        uint64_t step = step0 + (uint64_t)it;
        double virial = 0.0;
        int rc = orc_forces(n, x, v, id, cells, p, step, seed, 0, 0, NULL, f, s, &virial);
        if (rc) { free(f); free(s); return rc; }
        double ke_c = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (p->frozen && p->frozen[i]) continue;
            double vc[3];
            for (int k = 0; k < 3; ++k) vc[k] = v[3 * i + k] + 0.5 * p->dt * f[3 * i + k] / p->mass;
            ke_c += 0.5 * p->mass * (vc[0] * vc[0] + vc[1] * vc[1] + vc[2] * vc[2]);
            if (prof_sum && prof_cnt && nbins > 0) {
                double g = x[3 * i + p->grad_axis];
                int32_t b = (int32_t)floor(g * (double)nbins / box[p->grad_axis]);
                if (b < 0) b = 0;
                if (b > nbins - 1) b = nbins - 1;
                prof_sum[b] += vc[p->flow_axis];
                prof_cnt[b] += 1.0;
            }
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            if (p->frozen && p->frozen[i]) {                  /* wall particles move with their wall */
                orc_move_frozen(x + 3 * i, v + 3 * i, cells, p);
                continue;
            }
            double x0[3], dx[3];
            for (int k = 0; k < 3; ++k) {
                v[3 * i + k] += p->dt * f[3 * i + k] / p->mass;
                x0[k] = x[3 * i + k];
                dx[k] = p->dt * v[3 * i + k];
                x[3 * i + k] += dx[k];
            }
            orc_bounce(x0, dx, x + 3 * i, v + 3 * i, cells, p);
            for (int k = 0; k < 3; ++k) x[3 * i + k] -= box[k] * floor(x[3 * i + k] / box[k]);
        }
        if (diag) {
            orc_diag* dg = diag + it;
            double mom[3] = {0.0, 0.0, 0.0}, ke_h = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                if (p->frozen && p->frozen[i]) continue;
                double* vi = v + 3 * i;
                for (int k = 0; k < 3; ++k) mom[k] += p->mass * vi[k];
                ke_h += 0.5 * p->mass * (vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]);
            }
            for (int k = 0; k < 3; ++k) dg->momentum[k] = mom[k];
            dg->ke_half = ke_h;
            dg->ke_centred = ke_c;
            dg->kT_centred = 2.0 * ke_c / (3.0 * (double)(nfluid - 1));
            dg->virial = virial;
            dg->pressure = ((double)n / vol) * dg->kT_centred + virial / (3.0 * vol);
        }
        if (f_last && it == nsteps - 1) memcpy(f_last, f, (size_t)n * 3 * sizeof(double));
    }
    free(f);
    free(s);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
