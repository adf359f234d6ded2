/*
 * flock_oracle.c -- CPU oracle for one timestep of the flock environment.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * statement of what the GPU step computes.  Only the test suite, the smoke
 * check and the benchmark's cpu_baseline leg may load it; the product path
 * (the HIP library and its Python binding) never links, imports or calls it.
 * It shares no code, header, table or constant generator with the HIP path.
 *
 * Source: Langham-Lopez, Schmon, Cannon, "High Performance Simulation for
 * Scalable Multi-Agent Reinforcement Learning" (arXiv:2207.03945).
 *   - Sec. 2.1: agents are updated in discrete time-steps and every
 *     interaction updates all agents simultaneously.
 *   - Sec. 4: each agent's field of view is divided into v sectors; sector k
 *     holds the distance to the nearest other agent seen at that bearing.
 *   - Sec. 4.1: two-dimensional action (accelerate/decelerate with the speed
 *     clamped to [s_min, s_max]; rotate by at most theta_max); reward of agent
 *     i is Eq. (1), a sum of f(d_ij) over the agents j with d_ij < d_v, with a
 *     collision penalty when two agents are closer than 2 d_r (Fig. 4).
 *   - Sec. 4.1, last paragraph: in each update the agents are first rotated
 *     and accelerated by their actions, then the view and reward are updated
 *     for all pairs of agents in spatial proximity.
 *
 * Readings of points the paper leaves open (workload constants; the printed
 * speed update in Sec. 4.1 is garbled and is read as a clamp):
 *   move:  turn = clamp(a0, -max_turn, max_turn); ds = clamp(a1, -max_ds, max_ds)
 *          (clamp(a,lo,hi) = fminf(fmaxf(a,lo),hi), so NaN -> lo)
 *          th' = th + turn, wrapped once into [0, 2pi_f) with 2pi_f = (float)2pi
 *          s'  = clamp(s + ds, s_min, s_max)
 *          x'  = x + s' cos th' ; y' = y + s' sin th'   (dt = 1, new th', s')
 *          wrapped into [0, L): if x' < 0 add L, then if x' >= L subtract L.
 *          The state is FP32: every one of these operations is one IEEE
 *          single-precision operation (no fused multiply-add), and cos/sin of
 *          the FP32 heading are the correctly rounded FP32 values (evaluated
 *          in double precision and rounded once).
 *   sense: evaluated exactly (double precision) on the FP32 post-move state.
 *          Every ordered pair (i, j), j != i by index, uses the minimum image
 *          in the periodic box.  j is a neighbour of i iff d_ij < R (strict);
 *          it is a collision iff d_ij < r_c (strict), and a collision is also
 *          a neighbour.  Bearing phi = (atan2(dy, dx) - th_i) mod 2pi; sector
 *          k = min(v-1, floor(phi v / 2pi)); sector 0 starts at the heading and
 *          sectors advance counter-clockwise; a coincident pair (d = 0) is put
 *          in sector 0 (it is taken to lie on the heading).  obs[i][k] =
 *          1 - d_min(k)/R, or 0 if the sector is empty.
 *          reward = r_nb * n_nb + r_col * n_col.
 *   field of view (Sec. 5 gives the benchmark agents a convex field of view
 *          of about 250 degrees): with fov < 2pi the v sectors split the arc
 *          [-fov/2, fov/2) of bearings relative to the heading (wrapped into
 *          (-pi, pi]), counter-clockwise from its right edge; a neighbour
 *          outside the arc is not seen but still counts in the reward, since
 *          Eq. (1) sums over every agent within the vision range.
 *
 * Tolerance bands.  With eps_d > 0 and eps_phi > 0 the oracle additionally
 * reports, per agent, the lowest and highest neighbour / collision counts and
 * the per-sector smallest distance over unambiguous pairs only ("strict") and
 * over unambiguous plus ambiguous pairs ("loose").  A pair is ambiguous for a
 * radius when |d - radius| <= eps_d and ambiguous for its sector when its
 * bearing lies within eps_phi of a sector edge.  With eps_d = eps_phi = 0 the
 * bands collapse onto the plain values.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#define TWO_PI_D 6.283185307179586476925286766559
#define PI_D 3.1415926535897932384626433832795

/* ------------------------------------------------------------------------ */
/* Step part 1: rotate, accelerate, move (Sec. 4.1).                          */
/* ------------------------------------------------------------------------ */

static float clamp_action(float a, float lo, float hi)
{
    return fminf(fmaxf(a, lo), hi);
}

/* In place: x, y, th, s are [n] FP32 arrays; act is [n][2] (turn, dspeed). */
void oracle_move(int n, float box, float max_turn, float max_dspeed,
                 float s_min, float s_max,
                 float *x, float *y, float *th, float *s, const float *act)
{
    const float two_pi_f = (float)TWO_PI_D;
    for (int i = 0; i < n; ++i) {
        float turn = clamp_action(act[2 * i + 0], -max_turn, max_turn);
        float ds = clamp_action(act[2 * i + 1], -max_dspeed, max_dspeed);

        float h = th[i] + turn;
        if (h < 0.0f) h = h + two_pi_f;
        if (h >= two_pi_f) h = h - two_pi_f;

        float sp = s[i] + ds;
        sp = fminf(fmaxf(sp, s_min), s_max);

        float c = (float)cos((double)h);
        float sn = (float)sin((double)h);
        float stepx = sp * c;
        float stepy = sp * sn;

        float nx = x[i] + stepx;
        if (nx < 0.0f) nx = nx + box;
        if (nx >= box) nx = nx - box;
        float ny = y[i] + stepy;
        if (ny < 0.0f) ny = ny + box;
        if (ny >= box) ny = ny - box;

        x[i] = nx;
        y[i] = ny;
        th[i] = h;
        s[i] = sp;
    }
}

/* ------------------------------------------------------------------------ */
/* Step part 2: view and reward over all pairs (Sec. 4, Sec. 4.1, Eq. (1)).   */
/* ------------------------------------------------------------------------ */

/* Minimum-image displacement along one axis of a periodic box of side L. */
static double min_image(double d, double L)
{
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

/* Bearing of (dx, dy) relative to heading th, reduced into [0, 2pi). */
static double relative_bearing(double dx, double dy, double th)
{
    double phi = atan2(dy, dx) - th;
    phi = fmod(phi, TWO_PI_D);
    if (phi < 0.0) phi += TWO_PI_D;
    if (phi >= TWO_PI_D) phi -= TWO_PI_D;
    return phi;
}

static int sector_of(double phi, int v)
{
    int k = (int)floor(phi * (double)v / TWO_PI_D);
    if (k < 0) k = 0;
    if (k > v - 1) k = v - 1;
    return k;
}

/* Position of bearing phi (in [0, 2pi) from the heading) in sector units:
 * [0, v) when visible.  Full view: phi v / 2pi.  Limited view: the bearing
 * wrapped into (-pi, pi], shifted by fov/2, times v / fov. */
static double view_position(double phi, int v, double fov)
{
    if (fov >= TWO_PI_D) return phi * (double)v / TWO_PI_D;
    double rel = phi > PI_D ? phi - TWO_PI_D : phi;
    return (rel + 0.5 * fov) * (double)v / fov;
}

/*
 * Sense every agent in `list` (or agents 0..n_list-1 when list is NULL)
 * against all n agents.
 *
 * Inputs: FP32 positions x, y in [0, box) and headings th, all [n].
 * Plain outputs (row r corresponds to list[r]):
 *   obs[n_list][v]       1 - d_min/R per sector, 0 for an empty sector
 *   n_nb[n_list]         neighbours (d < R)
 *   n_col[n_list]        collisions (d < r_c)
 *   reward[n_list]       r_nb * n_nb + r_col * n_col
 * Band outputs (any of these pointers may be NULL):
 *   nb_lo/nb_hi, col_lo/col_hi [n_list]    count range over ambiguous pairs
 *   dmin_strict[n_list][v]  min distance over pairs unambiguously inside R
 *                           and unambiguously in the sector (INFINITY if none)
 *   dmin_loose[n_list][v]   min distance over pairs possibly inside R and
 *                           possibly in the sector (INFINITY if none)
 */
void oracle_sense(int n, double box, double radius, double collide, int v, double fov,
                  double r_nb, double r_col,
                  const float *x, const float *y, const float *th,
                  int n_list, const int *list,
                  double eps_d, double eps_phi,
                  double *obs, int *n_nb, int *n_col, double *reward,
                  int *nb_lo, int *nb_hi, int *col_lo, int *col_hi,
                  double *dmin_strict, double *dmin_loose)
{
    const int full = fov >= TWO_PI_D;
    const double eps_sector = eps_phi * (double)v / (full ? TWO_PI_D : fov);
    if (v < 1 || v > 256) return;

#pragma omp parallel for schedule(dynamic, 16)
    for (int r = 0; r < n_list; ++r) {
        const int i = list ? list[r] : r;
        const double xi = (double)x[i], yi = (double)y[i], thi = (double)th[i];

        double dmin[256], dstrict[256], dloose[256];
        for (int k = 0; k < v; ++k) {
            dmin[k] = INFINITY;
            dstrict[k] = INFINITY;
            dloose[k] = INFINITY;
        }
        int nb = 0, col = 0, nbl = 0, nbh = 0, coll = 0, colh = 0;

        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = min_image((double)x[j] - xi, box);
            double dy = min_image((double)y[j] - yi, box);
            double d = sqrt(dx * dx + dy * dy);
            if (d >= radius + eps_d) continue;

            /* plain definition */
            int k = 0, seen = 1;
            double t = 0.0;
            if (d > 0.0) {
                double phi = relative_bearing(dx, dy, thi);
                t = view_position(phi, v, fov);
                if (full) {
                    k = sector_of(phi, v);
                } else {
                    seen = t >= 0.0 && t < (double)v;
                    k = seen ? (int)floor(t) : -1;
                }
            } else if (!full) {
                t = 0.5 * (double)v; /* coincident: straight ahead */
                k = (int)floor(t);
            }
            if (d < radius) {
                nb += 1;
                if (seen && d < dmin[k]) dmin[k] = d;
            }
            if (d < collide) col += 1;

            /* bands */
            int sure_in = d < radius - eps_d;
            nbl += sure_in;
            nbh += 1; /* d < radius + eps_d here */
            coll += d < collide - eps_d;
            colh += d < collide + eps_d;

            int k_lo = k, k_hi = k;
            if (d > 0.0 && eps_sector > 0.0) {
                /* position in sector units; for a full view k_lo = -1 or
                 * k_hi = v wrap round, for a limited view they fall outside */
                k_lo = (int)floor(t - eps_sector);
                k_hi = (int)floor(t + eps_sector);
            }
            if (sure_in && seen && k_lo == k_hi && d < dstrict[k]) dstrict[k] = d;
            for (int kk = k_lo; kk <= k_hi; ++kk) {
                if (!full && (kk < 0 || kk >= v)) continue;
                int kw = ((kk % v) + v) % v;
                if (d < dloose[kw]) dloose[kw] = d;
            }
        }

        for (int k = 0; k < v; ++k) {
            obs[(size_t)r * v + k] = isinf(dmin[k]) ? 0.0 : 1.0 - dmin[k] / radius;
            if (dmin_strict) dmin_strict[(size_t)r * v + k] = dstrict[k];
            if (dmin_loose) dmin_loose[(size_t)r * v + k] = dloose[k];
        }
        n_nb[r] = nb;
        n_col[r] = col;
        reward[r] = r_nb * (double)nb + r_col * (double)col;
        if (nb_lo) nb_lo[r] = nbl;
        if (nb_hi) nb_hi[r] = nbh;
        if (col_lo) col_lo[r] = coll;
        if (col_hi) col_hi[r] = colh;
    }
}

/* ------------------------------------------------------------------------ */
/* Tag environment (Sec. 4.2): runners and chasers.                           */
/* ------------------------------------------------------------------------ */
/*
 * Sec. 4.2: two agent types; chasers are rewarded for touching runners,
 * runners for staying close to other runners and penalised for touching a
 * chaser; the view has two colour channels (runners, chasers) of v = 64
 * sectors each (observation 128 = 2 x 64); the action turns the heading by
 * at most theta_max and moves the agent along it at a speed in [0, s_max].
 * Fig. 6: one agent in eleven is a chaser (a tenth of the runners' number).
 *
 * Readings: agents 0 .. n_chasers-1 are the chasers, the rest runners; the
 * second action component is the speed itself (clamped to [0, s_max]), the
 * rest of the move is the flock's; a touch is d < r_touch (strict), between
 * agents of different types; a runner's reward is r_near per runner within
 * the vision range plus r_caught per chaser touching it; a chaser's is
 * r_catch per runner it touches; both channels use the flock's sector
 * geometry and field of view.
 */

/* In place; act[i] = (turn, speed). */
void oracle_move_tag(int n, float box, float max_turn, float s_max,
                     float *x, float *y, float *th, float *s, const float *act)
{
    const float two_pi_f = (float)TWO_PI_D;
    for (int i = 0; i < n; ++i) {
        float turn = clamp_action(act[2 * i + 0], -max_turn, max_turn);
        float sp = clamp_action(act[2 * i + 1], 0.0f, s_max);

        float h = th[i] + turn;
        if (h < 0.0f) h = h + two_pi_f;
        if (h >= two_pi_f) h = h - two_pi_f;

        float c = (float)cos((double)h);
        float sn = (float)sin((double)h);
        float nx = x[i] + sp * c;
        if (nx < 0.0f) nx = nx + box;
        if (nx >= box) nx = nx - box;
        float ny = y[i] + sp * sn;
        if (ny < 0.0f) ny = ny + box;
        if (ny >= box) ny = ny - box;

        x[i] = nx;
        y[i] = ny;
        th[i] = h;
        s[i] = sp;
    }
}

/*
 * View (two channels), counts and reward of each agent in `list`.
 * obs[n_list][2v]: channel 0 (runners) then channel 1 (chasers).
 * n_near[r]: runners within the vision range (other than i);
 * n_touch[r]: agents of the other type closer than r_touch.
 * Bands as in oracle_sense: near/touch count ranges over pairs within
 * eps_d of the radius, dmin_strict / dmin_loose [n_list][2v].
 */
void oracle_sense_tag(int n, int n_chasers, double box, double radius, double r_touch, int v,
                      double fov, double r_near, double r_caught, double r_catch,
                      const float *x, const float *y, const float *th,
                      int n_list, const int *list, double eps_d, double eps_phi,
                      double *obs, int *n_near, int *n_touch, double *reward,
                      int *near_lo, int *near_hi, int *touch_lo, int *touch_hi,
                      double *dmin_strict, double *dmin_loose)
{
    const int full = fov >= TWO_PI_D;
    const double eps_sector = eps_phi * (double)v / (full ? TWO_PI_D : fov);
    if (v < 1 || v > 256) return;

#pragma omp parallel for schedule(dynamic, 16)
    for (int r = 0; r < n_list; ++r) {
        const int i = list ? list[r] : r;
        const int ti = i < n_chasers;
        const double xi = (double)x[i], yi = (double)y[i], thi = (double)th[i];
        double dmin[512], dstrict[512], dloose[512];
        for (int k = 0; k < 2 * v; ++k) {
            dmin[k] = INFINITY;
            dstrict[k] = INFINITY;
            dloose[k] = INFINITY;
        }
        int nr = 0, nt = 0, nrl = 0, nrh = 0, ntl = 0, nth = 0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            const int tj = j < n_chasers;
            double dx = min_image((double)x[j] - xi, box);
            double dy = min_image((double)y[j] - yi, box);
            double d = sqrt(dx * dx + dy * dy);
            if (d >= radius + eps_d) continue;

            int k = 0, seen = 1;
            double t = 0.0;
            if (d > 0.0) {
                double phi = relative_bearing(dx, dy, thi);
                t = view_position(phi, v, fov);
                if (full) {
                    k = sector_of(phi, v);
                } else {
                    seen = t >= 0.0 && t < (double)v;
                    k = seen ? (int)floor(t) : -1;
                }
            } else if (!full) {
                t = 0.5 * (double)v;
                k = (int)floor(t);
            }
            const int ch = tj * v;  /* channel of j */
            if (d < radius) {
                if (!tj) nr += 1;
                if (seen && d < dmin[ch + k]) dmin[ch + k] = d;
            }
            if (tj != ti && d < r_touch) nt += 1;

            int sure_in = d < radius - eps_d;
            if (!tj) {
                nrl += sure_in;
                nrh += 1;
            }
            if (tj != ti) {
                ntl += d < r_touch - eps_d;
                nth += d < r_touch + eps_d;
            }
            int k_lo = k, k_hi = k;
            if (d > 0.0 && eps_sector > 0.0) {
                k_lo = (int)floor(t - eps_sector);
                k_hi = (int)floor(t + eps_sector);
            }
            if (sure_in && seen && k_lo == k_hi && d < dstrict[ch + k]) dstrict[ch + k] = d;
            for (int kk = k_lo; kk <= k_hi; ++kk) {
                if (!full && (kk < 0 || kk >= v)) continue;
                int kw = ((kk % v) + v) % v;
                if (d < dloose[ch + kw]) dloose[ch + kw] = d;
            }
        }
        for (int k = 0; k < 2 * v; ++k) {
            obs[(size_t)r * 2 * v + k] = isinf(dmin[k]) ? 0.0 : 1.0 - dmin[k] / radius;
            if (dmin_strict) dmin_strict[(size_t)r * 2 * v + k] = dstrict[k];
            if (dmin_loose) dmin_loose[(size_t)r * 2 * v + k] = dloose[k];
        }
        n_near[r] = nr;
        n_touch[r] = nt;
        reward[r] = ti ? r_catch * (double)nt : r_near * (double)nr + r_caught * (double)nt;
        if (near_lo) near_lo[r] = nrl;
        if (near_hi) near_hi[r] = nrh;
        if (touch_lo) touch_lo[r] = ntl;
        if (touch_hi) touch_hi[r] = nth;
    }
}

/* Number of OpenMP threads the sense loop uses (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
