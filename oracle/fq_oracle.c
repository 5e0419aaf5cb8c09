/*
 * fq_oracle.c -- plain FP64 CPU oracle for RF synthesis, RF->IQ demodulation
 * and delay-and-sum beamforming with coherent compounding.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the HIP path and never calls it.
 *
 * Everything is written as the direct definition, in double precision, with no
 * blocking or algebraic rearrangement:
 *
 *  Element e = ix + nx_el*iy at p_e = ((ix-(nx_el-1)/2) pitch_x, (iy-(ny_el-1)/2) pitch_y, 0).
 *  Transmit a (tilted plane wave, Section 2.4.1 / Algorithm 3 "transmit events"):
 *     u_a = (sin tx, sin ty, sqrt(1 - sin^2 tx - sin^2 ty)),
 *     t0_a = min_e (u_a . p_e)/c           (t = 0 when the first element fires),
 *     tau_tx(a, r) = (u_a . r)/c - t0_a.
 *  Receive: rho(e, r) = |r - p_e|, tau_rx = rho/c.
 *  Pulse: g(t) = exp(-t^2/(2 s^2)) cos(2 pi fc t), envelope FWHM = n_cyc/fc,
 *     s = n_cyc / (2 sqrt(2 ln 2) fc), g = 0 for |t| > trunc*s.
 *  RF (weak scattering, linear superposition of point echoes, Section 2.3 and
 *  Algorithm 1's RF_total = RF_phantom + RF_flow):
 *     rf[f,a,e,n] = sum_s A_s (r_ref/rho) g(n/fs - tau_tx(a,r_s(f)) - rho/c).
 *  rf2iq (Algorithm 3, step "convert to IQ"; zero outside the record):
 *     b[n] = 2 sum_{k=-16..16} h_k rf[n-k] exp(-i 2 pi fc (n-k)/fs),
 *     h_k proportional to 0.5 (1 + cos(pi k/17)) sinc(2 fc k/fs), sum h_k = 1.
 *  DAS (Algorithm 3, "apply delays" then "average over transmits"):
 *     x = fs (tau_tx(a, r_v) + tau_rx(e, r_v)), n = floor(x), alpha = x - n,
 *     linear : B = (1-alpha) b[n] + alpha b[n+1]
 *     hermite: B = sum_{j=-1..2} w_j(alpha) b[n+j]   (Catmull-Rom cubic)
 *     IQ[f,v] = (1/A) sum_a sum_e B_{f,a,e} exp(+i 2 pi fc x / fs);
 *     taps outside [0, T) read zero (zero padding).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_ANGLES 64
#define ORC_FIR_HALF 16

typedef struct {
    int32_t nx_el, ny_el;
    double pitch_x, pitch_y;
    double fc, fs, c;
    int32_t n_angles;
    double tilt[ORC_MAX_ANGLES][2]; /* radians (theta_x, theta_y) */
} orc_acq;

typedef struct {
    int32_t nx, ny, nz;
    double x0, y0, z0, dx, dy, dz;
} orc_grid;

typedef struct {
    double n_cycles;     /* envelope FWHM in carrier cycles */
    double trunc_sigmas; /* pulse support +- trunc_sigmas * sigma */
    double r_ref;        /* reference distance of the 1/r amplitude */
} orc_pulse;

static void elem_pos(const orc_acq *q, int e, double p[3]) {
    int ix = e % q->nx_el, iy = e / q->nx_el;
    p[0] = (ix - 0.5 * (q->nx_el - 1)) * q->pitch_x;
    p[1] = (iy - 0.5 * (q->ny_el - 1)) * q->pitch_y;
    p[2] = 0.0;
}

static void tx_dir(const orc_acq *q, int a, double u[3], double *t0) {
    double sx = sin(q->tilt[a][0]), sy = sin(q->tilt[a][1]);
    u[0] = sx;
    u[1] = sy;
    u[2] = sqrt(1.0 - sx * sx - sy * sy);
    double best = INFINITY;
    for (int e = 0; e < q->nx_el * q->ny_el; ++e) {
        double p[3];
        elem_pos(q, e, p);
        double d = (u[0] * p[0] + u[1] * p[1] + u[2] * p[2]) / q->c;
        if (d < best) best = d;
    }
    *t0 = best;
}

static double tau_tx(const double u[3], double t0, double c, const double r[3]) {
    return (u[0] * r[0] + u[1] * r[1] + u[2] * r[2]) / c - t0;
}

static double dist(const double a[3], const double b[3]) {
    double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
    return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

int orc_version(void) { return 1; }

/* ------------------------------------------------------------------------ */
/* RF synthesis for a list of traces (f, a, e).  pos is [n_pos_frames][S][3]
 * float32; n_pos_frames == 1 means static positions.  out: [n_sel][T] double. */
void orc_rf_traces(const orc_acq *q, const orc_pulse *pl, int32_t n_pos_frames, int64_t n_scat,
                   const float *pos, const float *amp, int32_t T, int64_t n_sel,
                   const int32_t *sel /* [n_sel][3] = f, a, e */, double *out) {
    const double sigma = pl->n_cycles / (2.0 * sqrt(2.0 * log(2.0)) * q->fc);
    const double half = pl->trunc_sigmas * sigma;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n_sel; ++i) {
        int f = sel[3 * i], a = sel[3 * i + 1], e = sel[3 * i + 2];
        double u[3], t0, pe[3];
        tx_dir(q, a, u, &t0);
        elem_pos(q, e, pe);
        double *o = out + i * (int64_t)T;
        memset(o, 0, sizeof(double) * (size_t)T);
        const float *pf = pos + (n_pos_frames == 1 ? 0 : (int64_t)f * n_scat * 3);
        for (int64_t s = 0; s < n_scat; ++s) {
            double r[3] = {pf[3 * s], pf[3 * s + 1], pf[3 * s + 2]};
            double rho = dist(r, pe);
            double tau = tau_tx(u, t0, q->c, r) + rho / q->c;
            double A = (double)amp[s] * pl->r_ref / rho;
            /* only samples with |t| <= half can be non-zero */
            int64_t n_lo = (int64_t)ceil((tau - half) * q->fs) - 1;
            int64_t n_hi = (int64_t)floor((tau + half) * q->fs) + 1;
            if (n_lo < 0) n_lo = 0;
            if (n_hi > T - 1) n_hi = T - 1;
            for (int64_t n = n_lo; n <= n_hi; ++n) {
                double t = n / q->fs - tau;
                if (fabs(t) > half) continue;
                o[n] += A * exp(-t * t / (2.0 * sigma * sigma)) * cos(2.0 * M_PI * q->fc * t);
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Low-pass taps h_k, k = -16..16 (33 taps), normalised to unit DC gain. */
void orc_fir_taps(double fc, double fs, double *h /* [33] */) {
    double sum = 0.0;
    for (int k = -ORC_FIR_HALF; k <= ORC_FIR_HALF; ++k) {
        double w = 0.5 * (1.0 + cos(M_PI * k / (ORC_FIR_HALF + 1)));
        double x = 2.0 * fc * k / fs;
        double sn = (k == 0) ? 1.0 : sin(M_PI * x) / (M_PI * x);
        h[k + ORC_FIR_HALF] = w * sn;
        sum += w * sn;
    }
    for (int k = 0; k < 2 * ORC_FIR_HALF + 1; ++k) h[k] /= sum;
}

/* b[n] for one trace at one sample index n (0 outside [0, T)). */
static void iq_sample(const float *rf, int32_t T, int64_t n, const double *h, double fc, double fs,
                      double *re, double *im) {
    double sr = 0.0, si = 0.0;
    if (n >= 0 && n < T) {
        for (int k = -ORC_FIR_HALF; k <= ORC_FIR_HALF; ++k) {
            int64_t m = n - k;
            if (m < 0 || m >= T) continue;
            double ph = -2.0 * M_PI * fc * (double)m / fs;
            double v = 2.0 * h[k + ORC_FIR_HALF] * (double)rf[m];
            sr += v * cos(ph);
            si += v * sin(ph);
        }
    }
    *re = sr;
    *im = si;
}

/* rf: [n_traces][T] float32 -> out: [n_traces][T][2] double */
void orc_rf2iq(int64_t n_traces, int32_t T, double fc, double fs, const float *rf, double *out) {
    double h[2 * ORC_FIR_HALF + 1];
    orc_fir_taps(fc, fs, h);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < n_traces; ++t)
        for (int n = 0; n < T; ++n)
            iq_sample(rf + t * (int64_t)T, T, n, h, fc, fs, &out[(t * T + n) * 2], &out[(t * T + n) * 2 + 1]);
}

/* ------------------------------------------------------------------------ */
static void interp_weights(int interp, double al, double w[4], int *j0, int *nt) {
    if (interp == 0) {
        *j0 = 0;
        *nt = 2;
        w[0] = 1.0 - al;
        w[1] = al;
    } else {
        /* Catmull-Rom (Keys a = -1/2) on taps n-1, n, n+1, n+2 */
        double a2 = al * al, a3 = a2 * al;
        *j0 = -1;
        *nt = 4;
        w[0] = 0.5 * (-a3 + 2.0 * a2 - al);
        w[1] = 0.5 * (3.0 * a3 - 5.0 * a2 + 2.0);
        w[2] = 0.5 * (-3.0 * a3 + 4.0 * a2 + al);
        w[3] = 0.5 * (a3 - a2);
    }
}

static void voxel_pos(const orc_grid *g, int64_t v, double r[3]) {
    int64_t ix = v % g->nx, iy = (v / g->nx) % g->ny, iz = v / ((int64_t)g->nx * g->ny);
    r[0] = g->x0 + ix * g->dx;
    r[1] = g->y0 + iy * g->dy;
    r[2] = g->z0 + iz * g->dz;
}

/* DAS from precomputed baseband for selected voxels.  The baseband is stored
 * with the frame index innermost, bb[a][e][n][f][2] (double), so that the
 * per-voxel loop over frames reads contiguous memory.  out: [n_sel][F][2]. */
void orc_das_bb(const orc_acq *q, const orc_grid *g, int32_t F, int32_t T, const double *bb,
                int32_t interp, int64_t n_sel, const int64_t *sel, double *out) {
    const int A = q->n_angles, E = q->nx_el * q->ny_el;
    double U[ORC_MAX_ANGLES][3], T0[ORC_MAX_ANGLES];
    for (int a = 0; a < A; ++a) tx_dir(q, a, U[a], &T0[a]);
#pragma omp parallel for schedule(dynamic, 2)
    for (int64_t i = 0; i < n_sel; ++i) {
        double r[3];
        voxel_pos(g, sel[i], r);
        double *o = out + i * (int64_t)F * 2;
        memset(o, 0, sizeof(double) * 2 * (size_t)F);
        for (int a = 0; a < A; ++a) {
            double ttx = tau_tx(U[a], T0[a], q->c, r);
            for (int e = 0; e < E; ++e) {
                double pe[3];
                elem_pos(q, e, pe);
                double x = q->fs * (ttx + dist(r, pe) / q->c);
                double n = floor(x), al = x - n;
                double w[4];
                int j0, nt;
                interp_weights(interp, al, w, &j0, &nt);
                double ph = 2.0 * M_PI * q->fc * x / q->fs;
                double cr = cos(ph), ci = sin(ph);
                const double *tr = bb + (((int64_t)a * E + e) * T) * (int64_t)F * 2;
                for (int f = 0; f < F; ++f) {
                    double br = 0.0, bi = 0.0;
                    for (int j = 0; j < nt; ++j) {
                        int64_t m = (int64_t)n + j0 + j;
                        if (m < 0 || m >= T) continue;
                        br += w[j] * tr[(m * F + f) * 2];
                        bi += w[j] * tr[(m * F + f) * 2 + 1];
                    }
                    o[2 * f] += br * cr - bi * ci;
                    o[2 * f + 1] += br * ci + bi * cr;
                }
            }
        }
        for (int f = 0; f < 2 * F; ++f) o[f] /= A;
    }
}

/* DAS straight from RF [F][A][E][T] float32 for selected voxels: each needed
 * baseband tap is demodulated on demand with the rf2iq definition.  Same
 * result as orc_rf2iq followed by orc_das_bb; meant for sampled voxels of
 * volumes too large to demodulate whole.  out: [n_sel][F][2] double. */
void orc_das_rf(const orc_acq *q, const orc_grid *g, int32_t F, int32_t T, const float *rf,
                int32_t interp, int64_t n_sel, const int64_t *sel, double *out) {
    const int A = q->n_angles, E = q->nx_el * q->ny_el;
    double U[ORC_MAX_ANGLES][3], T0[ORC_MAX_ANGLES];
    for (int a = 0; a < A; ++a) tx_dir(q, a, U[a], &T0[a]);
    double h[2 * ORC_FIR_HALF + 1];
    orc_fir_taps(q->fc, q->fs, h);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n_sel; ++i) {
        double r[3];
        voxel_pos(g, sel[i], r);
        double *o = out + i * (int64_t)F * 2;
        memset(o, 0, sizeof(double) * 2 * (size_t)F);
        for (int a = 0; a < A; ++a) {
            double ttx = tau_tx(U[a], T0[a], q->c, r);
            for (int e = 0; e < E; ++e) {
                double pe[3];
                elem_pos(q, e, pe);
                double x = q->fs * (ttx + dist(r, pe) / q->c);
                double n = floor(x), al = x - n;
                double w[4];
                int j0, nt;
                interp_weights(interp, al, w, &j0, &nt);
                double ph = 2.0 * M_PI * q->fc * x / q->fs;
                double cr = cos(ph), ci = sin(ph);
                for (int f = 0; f < F; ++f) {
                    const float *tr = rf + (((int64_t)f * A + a) * E + e) * (int64_t)T;
                    double br = 0.0, bi = 0.0;
                    for (int j = 0; j < nt; ++j) {
                        double sr, si;
                        iq_sample(tr, T, (int64_t)n + j0 + j, h, q->fc, q->fs, &sr, &si);
                        br += w[j] * sr;
                        bi += w[j] * si;
                    }
                    o[2 * f] += br * cr - bi * ci;
                    o[2 * f + 1] += br * ci + bi * cr;
                }
            }
        }
        for (int f = 0; f < 2 * F; ++f) o[f] /= A;
    }
}
