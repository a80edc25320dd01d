/*
 * sonosim_oracle.c -- plain, slow FP64 CPU oracle of the model-based
 * ultrasound simulator (SonoGym, arXiv 2507.01152, App. B.2).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU path; both are written separately
 * from the paper's equations and the readings listed below.
 *
 * What is computed, per environment (volume L (+CT C), tissue table,
 * probe (W, H, dx, dy, f, E0, c_psf, DR), pose [R|t]):
 *
 *   O1 plane geometry (App. B.2 / Sec. 4 "Ultrasound simulation": the image
 *      plane comes from the end-effector pose): pixel (x,y) sits at probe
 *      point (a + x*dx, b, y*dy), a = -0.5*(W-1)*dx, b = the plane's
 *      elevation (0 for a linear probe; a volumetric probe, Sec. 4 surgery
 *      task, is a stack of such planes), mapped by the pose into
 *      volume mm, divided by the voxel spacing and rounded to Q16 fixed point
 *      (rint, half-even) as an origin and two per-pixel steps; every pixel
 *      position is then the exact integer P0 + x*DX + y*DY.
 *   O2 nearest label: i = floor((Q + 2^15) / 2^16); outside the grid -> air.
 *   O3 impedance: per-label table Z, or with a CT volume Z = max(HU+1000, 0)
 *      from trilinear HU (successive linear interpolation along x, y, z;
 *      outside corners -1000 HU).  Z proportional to CT intensity, App. B.2.
 *   O4 interface terms of the reflection equation R (App. B.2): boundary
 *      indicator G = [label(x,y) != label(x,y+1)], amplitude reflection
 *      r = (Z2-Z1)/(Z2+Z1) and intensity transmission t = 1 - r^2 (total
 *      reflection when one side is 0 or +inf).
 *   O5 remaining energy (App. B.2, energy equation, plus transmission):
 *      E(x,y) = E0 * prod_{v<y} t(x,v) * exp(-f * dy_cm * sum_{v<y} alpha).
 *   O6 incidence angle from the label slice: Sobel on [label differs from the
 *      centre label], cos(theta) = |gy'| / |(gx', gy')| in physical units.
 *   O7 scattering pattern T (App. B.2, scattering equations): per voxel
 *      Philox4x32-10 words (key = volume seed, counter = voxel index),
 *      N0 by Box-Muller, gate N1 <= mu1 as the integer test w2 < Phi(mu1)*2^32.
 *      Multi-scale noise (App. B.2, last sentence on the scattering pattern;
 *      reading): with S > 1 scales, scale s draws the same generator on cells
 *      of 2^s voxels per axis (counter = (cell index, 0, s, 0); s = 0 is the
 *      voxel stream above) and
 *        N0 = (1/sqrt(S)) * sum_s BoxMuller(w0_s, w1_s)       (FP64),
 *        gate: N1 = (1/sqrt(S)) * sum_s N1_s <= mu1, with N1_s the quantised
 *        standard normal Q[w2_s >> 20] * 2^-20, Q[k] = rint(Phi^-1((k + 1/2)
 *        / 4096) * 2^20) (int32).  The sum of the Q is an exact integer, so
 *        the gate is the integer test sum_s Q[w2_s >> 20] <= floor(sqrt(S) *
 *        mu1 * 2^20), the threshold rounded once in FP64 in that order.
 *   O8 R' = G * E * cos(theta) * |r|.
 *   O9 separable Gaussian PSF with std c_psf * (image size) per axis, radius
 *      max(1, ceil(3 sigma)), normalised, zero padding (App. B.2).
 *   O10 I = K (x) R' + E * (K (x) T).
 *   O11 display Y = clamp(1 + (20/DR) log10(max(I,0)/E0), 0, 1).
 *
 * Philox4x32-10 follows Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3" (SC'11); Box-Muller follows Box & Muller (1958).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny, nz;
    double sx, sy, sz;        /* voxel spacing, mm */
    const uint8_t* labels;    /* [nz][ny][nx] */
    const int16_t* ct;        /* [nz][ny][nx] or NULL */
    uint64_t seed;            /* noise-field key */
    int32_t scales;           /* noise scales S (<= 1: one) */
    const int32_t* q_lut;     /* [4096] quantised normal Q in units of 2^-20 (used when S > 1) */
} or_volume;

typedef struct {
    float Z, alpha, mu0, sigma0, mu1;
} or_tissue;

typedef struct {
    int32_t W, H;
    double dx, dy, f, E0, psf, dr;
    double elev;              /* elevation b of this image plane, mm (0: single plane) */
} or_probe;

/* Per-pixel planes, each [H][W] row-major (philox [H][W][4], q [H][W][3]).
 * Any pointer may be NULL. */
typedef struct {
    int64_t* q;
    uint8_t* label;
    int64_t* voxel;      /* -1 outside */
    uint32_t* philox;    /* 0 outside */
    double* Z;
    uint8_t* G;
    double* r;
    double* t;
    double* E;
    double* cos_theta;
    double* T;
    double* Rp;
    double* I;
    double* A;           /* magnitude sum K(x)R' + E*(K(x)|T|) */
    double* Y;
} or_planes;

/* ------------------------------------------------------------------------
 * Philox-4xW-10, one generic round structure instantiated at 32 and 64 bits.
 * Round: (c0,c1,c2,c3) -> (hi(M1*c2)^c1^k0, lo(M1*c2), hi(M0*c0)^c3^k1,
 * lo(M0*c0)); the key is bumped by the Weyl constants between rounds.
 */
static void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

#define OR_DEFINE_PHILOX(NAME, T, MULHILO, M0, M1, W0, W1)                 \
    void NAME##_rounds(const T ctr[4], const T key[2], int rounds, T out[4]) \
    {                                                                      \
        T c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];              \
        T k0 = key[0], k1 = key[1];                                        \
        for (int round = 0; round < rounds; ++round) {                     \
            T hi0, lo0, hi1, lo1;                                          \
            if (round > 0) { k0 += (T)(W0); k1 += (T)(W1); }               \
            MULHILO((T)(M0), c0, &hi0, &lo0);                              \
            MULHILO((T)(M1), c2, &hi1, &lo1);                              \
            T n0 = hi1 ^ c1 ^ k0;                                          \
            T n1 = lo1;                                                    \
            T n2 = hi0 ^ c3 ^ k1;                                          \
            T n3 = lo0;                                                    \
            c0 = n0; c1 = n1; c2 = n2; c3 = n3;                            \
        }                                                                  \
        out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;                \
    }                                                                      \
    void NAME##_10(const T ctr[4], const T key[2], T out[4])               \
    {                                                                      \
        NAME##_rounds(ctr, key, 10, out);                                  \
    }

/* 32-bit multipliers from Salmon et al.; Weyl constants are the first
 * 32 / 64 fractional bits of the golden ratio and of sqrt(3). */
OR_DEFINE_PHILOX(or_philox4x32, uint32_t, mulhilo32,
                 0xD2511F53u, 0xCD9E8D57u, 0x9E3779B9u, 0xBB67AE85u)
OR_DEFINE_PHILOX(or_philox4x64, uint64_t, mulhilo64,
                 0xD2E7470EE14C6C93ull, 0xCA5A826395121157ull,
                 0x9E3779B97F4A7C15ull, 0xBB67AE8584CAA73Bull)

/* ------------------------------------------------------------------------ */

static int64_t floordiv(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
    return q;
}

/* O1: Q16 origin and steps (voxel units * 65536), one op at a time. */
void or_geometry(const or_volume* v, const or_probe* p, const double pose[12],
                 int64_t P0[3], int64_t DX[3], int64_t DY[3])
{
    const double s[3] = {v->sx, v->sy, v->sz};
    double a = -0.5 * (double)(p->W - 1);
    a = a * p->dx;
    for (int c = 0; c < 3; ++c) {
        double Rc0 = pose[4 * c + 0];
        double Rc1 = pose[4 * c + 1];
        double Rc2 = pose[4 * c + 2];
        double tc = pose[4 * c + 3];
        double u = Rc0 * a;
        u = tc + u;
        double v = Rc1 * p->elev;
        u = u + v;
        u = u / s[c];
        u = u * 65536.0;
        P0[c] = (int64_t)rint(u);
        double w = Rc0 * p->dx;
        w = w / s[c];
        w = w * 65536.0;
        DX[c] = (int64_t)rint(w);
        double z = Rc2 * p->dy;
        z = z / s[c];
        z = z * 65536.0;
        DY[c] = (int64_t)rint(z);
    }
}

/* O7 gate threshold: floor(Phi(mu1) * 2^32), capped at 2^32. */
uint64_t or_gate_threshold(float mu1)
{
    double m = (double)mu1;
    double phi = 0.5 * erfc(-m / sqrt(2.0));
    double x = floor(phi * 4294967296.0);
    if (x >= 4294967296.0) return 4294967296ull;
    if (x <= 0.0) return 0;
    return (uint64_t)x;
}

/* O9: normalised sampled Gaussian, K[0..2r], returns r. */
int32_t or_psf_kernel(double sigma, double* K, int32_t cap)
{
    int32_t r = (int32_t)ceil(3.0 * sigma);
    if (r < 1) r = 1;
    if (2 * r + 1 > cap) return -1;
    double sum = 0.0;
    for (int32_t k = -r; k <= r; ++k) {
        double e = exp(-((double)k * (double)k) / (2.0 * sigma * sigma));
        K[k + r] = e;
        sum += e;
    }
    for (int32_t k = 0; k < 2 * r + 1; ++k) K[k] /= sum;
    return r;
}

/* O7 multi-scale gate threshold: floor(sqrt(S) * mu1 * 2^20), one FP64
 * rounding per operation in that order, clamped to the int32 range (sums of
 * at most four quantised normals stay far inside it; mu1 = -inf never
 * passes, +inf always). */
int64_t or_multiscale_threshold(int32_t S, float mu1)
{
    double x = sqrt((double)S);
    x = x * (double)mu1;
    x = x * 1048576.0;
    x = floor(x);
    if (!(x > -2147483648.0)) return -2147483648ll;
    if (x > 2147483647.0) return 2147483647ll;
    return (int64_t)x;
}

/* O7 for one voxel (ix, iy, iz) inside the grid: N0 and, with S > 1, the
 * integer sum N1 of the quantised normals (units of 2^-20) and its threshold
 * test; words of scale 0 in w[4].  Returns the gate (1: scatter). */
int or_scatter_voxel(const or_volume* v, float mu1, int64_t ix, int64_t iy, int64_t iz, double* n0, int64_t* n1,
                     uint32_t w[4])
{
    const uint32_t key[2] = {(uint32_t)v->seed, (uint32_t)(v->seed >> 32)};
    const int S = v->scales > 1 ? v->scales : 1;
    double sum0 = 0.0;
    int64_t sum1 = 0;
    int gate = 0;
    for (int s = 0; s < S; ++s) {
        const int64_t mx = ((int64_t)v->nx + ((int64_t)1 << s) - 1) >> s;
        const int64_t my = ((int64_t)v->ny + ((int64_t)1 << s) - 1) >> s;
        const int64_t cell = (((iz >> s) * my) + (iy >> s)) * mx + (ix >> s);
        const uint32_t ctr[4] = {(uint32_t)cell, (uint32_t)(cell >> 32), (uint32_t)s, 0u};
        uint32_t ws[4];
        or_philox4x32_10(ctr, key, ws);
        if (s == 0) memcpy(w, ws, sizeof(ws));
        double u0 = (2.0 * (double)(ws[0] >> 9) + 1.0) / 16777216.0;
        double u1 = (2.0 * (double)(ws[1] >> 9) + 1.0) / 16777216.0;
        sum0 += sqrt(-2.0 * log(u0)) * cos(2.0 * M_PI * u1);
        if (S > 1) sum1 += v->q_lut[ws[2] >> 20];
    }
    if (S == 1) {
        *n0 = sum0;
        *n1 = 0;
        gate = (uint64_t)w[2] < or_gate_threshold(mu1);
    } else {
        *n0 = sum0 / sqrt((double)S);
        *n1 = sum1;
        gate = sum1 <= or_multiscale_threshold(S, mu1);
    }
    return gate;
}

/* O7 over the whole grid: N0, N1 and the gate of every voxel, [nz][ny][nx]. */
void or_scatter_grid(const or_volume* v, float mu1, double* n0, int64_t* n1, uint8_t* gate)
{
    const int64_t n = (int64_t)v->nx * v->ny * v->nz;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        uint32_t w[4];
        const int64_t ix = k % v->nx, iy = (k / v->nx) % v->ny, iz = k / ((int64_t)v->nx * v->ny);
        gate[k] = (uint8_t)or_scatter_voxel(v, mu1, ix, iy, iz, &n0[k], &n1[k], w);
    }
}

static double ct_at(const or_volume* v, int64_t ix, int64_t iy, int64_t iz)
{
    if (ix < 0 || iy < 0 || iz < 0 || ix >= v->nx || iy >= v->ny || iz >= v->nz) return -1000.0;
    return (double)v->ct[((int64_t)iz * v->ny + iy) * v->nx + ix];
}

/* Simulate one environment.  Returns 0, or -1 on bad arguments. */
int or_simulate_env(const or_volume* v, const or_tissue* table, int32_t n_labels,
                    const or_probe* p, const double pose[12], or_planes* out)
{
    const int32_t W = p->W, H = p->H;
    if (W < 1 || H < 1 || n_labels < 1) return -1;
    const int64_t NP = (int64_t)W * H;

    int64_t P0[3], DX[3], DY[3];
    or_geometry(v, p, pose, P0, DX, DY);

    uint8_t* lab = (uint8_t*)malloc(NP);
    int64_t* vox = (int64_t*)malloc(NP * sizeof(int64_t));
    double* Z = (double*)malloc(NP * sizeof(double));
    uint8_t* G = (uint8_t*)malloc(NP);
    double* r = (double*)malloc(NP * sizeof(double));
    double* t = (double*)malloc(NP * sizeof(double));
    double* E = (double*)malloc(NP * sizeof(double));
    double* cs = (double*)malloc(NP * sizeof(double));
    double* T = (double*)malloc(NP * sizeof(double));
    double* Tabs = (double*)malloc(NP * sizeof(double));
    double* Rp = (double*)malloc(NP * sizeof(double));
    uint32_t* ph = (uint32_t*)malloc(NP * 4 * sizeof(uint32_t));
    if (!lab || !vox || !Z || !G || !r || !t || !E || !cs || !T || !Tabs || !Rp || !ph) {
        free(lab); free(vox); free(Z); free(G); free(r); free(t); free(E); free(cs);
        free(T); free(Tabs); free(Rp); free(ph);
        return -1;
    }

    /* O2, O3 */
    for (int32_t y = 0; y < H; ++y) {
        for (int32_t x = 0; x < W; ++x) {
            int64_t k = (int64_t)y * W + x;
            int64_t q[3];
            for (int c = 0; c < 3; ++c) q[c] = P0[c] + (int64_t)x * DX[c] + (int64_t)y * DY[c];
            if (out->q) for (int c = 0; c < 3; ++c) out->q[3 * k + c] = q[c];
            int64_t ix = floordiv(q[0] + 32768, 65536);
            int64_t iy = floordiv(q[1] + 32768, 65536);
            int64_t iz = floordiv(q[2] + 32768, 65536);
            int inside = ix >= 0 && iy >= 0 && iz >= 0 && ix < v->nx && iy < v->ny && iz < v->nz;
            if (inside) {
                vox[k] = (iz * v->ny + iy) * v->nx + ix;
                lab[k] = v->labels[vox[k]];
            } else {
                vox[k] = -1;
                lab[k] = 0;
            }
            if (lab[k] >= n_labels) {
                free(lab); free(vox); free(Z); free(G); free(r); free(t); free(E); free(cs);
                free(T); free(Tabs); free(Rp); free(ph);
                return -1;
            }
            if (v->ct) {
                /* trilinear as successive linear interpolations along x, y, z */
                int64_t b[3];
                double w[3];
                for (int c = 0; c < 3; ++c) {
                    b[c] = floordiv(q[c], 65536);
                    w[c] = (double)(q[c] - 65536 * b[c]) / 65536.0;
                }
                double cy[2];
                for (int dz = 0; dz < 2; ++dz) {
                    double cx[2];
                    for (int dy = 0; dy < 2; ++dy) {
                        double h0 = ct_at(v, b[0], b[1] + dy, b[2] + dz);
                        double h1 = ct_at(v, b[0] + 1, b[1] + dy, b[2] + dz);
                        cx[dy] = h0 + w[0] * (h1 - h0);
                    }
                    cy[dz] = cx[0] + w[1] * (cx[1] - cx[0]);
                }
                double hu = cy[0] + w[2] * (cy[1] - cy[0]);
                double z = hu + 1000.0;
                Z[k] = z > 0.0 ? z : 0.0;
            } else {
                Z[k] = (double)table[lab[k]].Z;
            }
        }
    }

    /* O4 */
    for (int32_t y = 0; y < H; ++y) {
        for (int32_t x = 0; x < W; ++x) {
            int64_t k = (int64_t)y * W + x;
            G[k] = (y < H - 1) && lab[k] != lab[k + W];
            r[k] = 0.0;
            t[k] = 1.0;
            if (!G[k]) continue;
            double Z1 = Z[k], Z2 = Z[k + W];
            if (Z1 == Z2) continue;
            if (Z1 == 0.0 || Z2 == 0.0 || isinf(Z1) || isinf(Z2)) {
                r[k] = (Z2 > Z1) ? 1.0 : -1.0;
                t[k] = 0.0;
            } else {
                r[k] = (Z2 - Z1) / (Z2 + Z1);
                t[k] = (2.0 * Z1 / (Z1 + Z2)) * (2.0 * Z2 / (Z1 + Z2));
            }
        }
    }

    /* O5 */
    const double coef = p->f * (p->dy / 10.0);
    for (int32_t x = 0; x < W; ++x) {
        double prod_t = 1.0, sum_a = 0.0;
        for (int32_t y = 0; y < H; ++y) {
            int64_t k = (int64_t)y * W + x;
            E[k] = p->E0 * prod_t * exp(-coef * sum_a);
            prod_t *= t[k];
            sum_a += (double)table[lab[k]].alpha;
        }
    }

    /* O6 */
    for (int32_t y = 0; y < H; ++y) {
        for (int32_t x = 0; x < W; ++x) {
            int64_t k = (int64_t)y * W + x;
            cs[k] = 1.0;
            if (!G[k]) continue;
            int b[3][3];
            for (int j = -1; j <= 1; ++j)
                for (int i = -1; i <= 1; ++i) {
                    int32_t xx = x + i, yy = y + j;
                    if (xx < 0) xx = 0;
                    if (xx > W - 1) xx = W - 1;
                    if (yy < 0) yy = 0;
                    if (yy > H - 1) yy = H - 1;
                    b[j + 1][i + 1] = lab[(int64_t)yy * W + xx] != lab[k];
                }
            double gx = 0.0, gy = 0.0;
            const double wgt[3] = {1.0, 2.0, 1.0};
            for (int d = 0; d < 3; ++d) {
                gx += wgt[d] * (double)(b[d][2] - b[d][0]);
                gy += wgt[d] * (double)(b[2][d] - b[0][d]);
            }
            gx /= p->dx;
            gy /= p->dy;
            double h = hypot(gx, gy);
            cs[k] = (h == 0.0) ? 1.0 : fabs(gy) / h;
        }
    }

    /* O7, O8 */
    for (int64_t k = 0; k < NP; ++k) {
        T[k] = 0.0;
        ph[4 * k + 0] = ph[4 * k + 1] = ph[4 * k + 2] = ph[4 * k + 3] = 0;
        if (vox[k] >= 0) {
            const int64_t ix = vox[k] % v->nx, iy = (vox[k] / v->nx) % v->ny, iz = vox[k] / ((int64_t)v->nx * v->ny);
            const or_tissue* tt = &table[lab[k]];
            double n0;
            int64_t n1;
            if (or_scatter_voxel(v, tt->mu1, ix, iy, iz, &n0, &n1, &ph[4 * k]))
                T[k] = n0 * (double)tt->sigma0 + (double)tt->mu0;
        }
        Tabs[k] = fabs(T[k]);
        Rp[k] = G[k] ? E[k] * cs[k] * fabs(r[k]) : 0.0;
    }

    /* O9 .. O11 */
    double Kax[4096], Klat[4096];
    int32_t rax = or_psf_kernel(p->psf * (double)H, Kax, 4096);
    int32_t rlat = or_psf_kernel(p->psf * (double)W, Klat, 4096);
    if (rax < 0 || rlat < 0) {
        free(lab); free(vox); free(Z); free(G); free(r); free(t); free(E); free(cs);
        free(T); free(Tabs); free(Rp); free(ph);
        return -1;
    }
    for (int32_t y = 0; y < H; ++y) {
        for (int32_t x = 0; x < W; ++x) {
            int64_t k = (int64_t)y * W + x;
            double kr = 0.0, kt = 0.0, ka = 0.0;
            for (int32_t i = -rlat; i <= rlat; ++i) {
                int32_t xx = x - i;
                if (xx < 0 || xx >= W) continue;
                for (int32_t j = -rax; j <= rax; ++j) {
                    int32_t yy = y - j;
                    if (yy < 0 || yy >= H) continue;
                    double w = Klat[i + rlat] * Kax[j + rax];
                    int64_t kk = (int64_t)yy * W + xx;
                    kr += w * Rp[kk];
                    kt += w * T[kk];
                    ka += w * Tabs[kk];
                }
            }
            double I = kr + E[k] * kt;
            double A = kr + E[k] * ka;
            double Y = 0.0;
            if (I > 0.0) {
                Y = 1.0 + (20.0 / p->dr) * log10(I / p->E0);
                if (Y < 0.0) Y = 0.0;
                if (Y > 1.0) Y = 1.0;
            }
            if (out->I) out->I[k] = I;
            if (out->A) out->A[k] = A;
            if (out->Y) out->Y[k] = Y;
        }
    }

    for (int64_t k = 0; k < NP; ++k) {
        if (out->label) out->label[k] = lab[k];
        if (out->voxel) out->voxel[k] = vox[k];
        if (out->philox) memcpy(&out->philox[4 * k], &ph[4 * k], 4 * sizeof(uint32_t));
        if (out->Z) out->Z[k] = Z[k];
        if (out->G) out->G[k] = G[k];
        if (out->r) out->r[k] = r[k];
        if (out->t) out->t[k] = t[k];
        if (out->E) out->E[k] = E[k];
        if (out->cos_theta) out->cos_theta[k] = cs[k];
        if (out->T) out->T[k] = T[k];
        if (out->Rp) out->Rp[k] = Rp[k];
    }
    free(lab); free(vox); free(Z); free(G); free(r); free(t); free(E); free(cs);
    free(T); free(Tabs); free(Rp); free(ph);
    return 0;
}

/* Many environments, display output only, OpenMP over environments.
 * Y is packed per env at Y + offsets[e] (in doubles).  Returns 0 or -1.
 * *threads_used receives the number of threads of the parallel region. */
int or_simulate_batch(int32_t n_envs, const or_volume* vols, const int32_t* vol_ids,
                      const or_tissue* table, int32_t n_labels, const or_probe* probes,
                      const double* poses, double* Y, const int64_t* offsets,
                      int32_t n_threads, int32_t* threads_used)
{
    int err = 0;
    int used = 1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 1)
        for (int32_t e = 0; e < n_envs; ++e) {
            or_planes pl;
            memset(&pl, 0, sizeof(pl));
            pl.Y = Y + offsets[e];
            if (or_simulate_env(&vols[vol_ids[e]], table, n_labels, &probes[e], &poses[12 * e], &pl)) {
#pragma omp atomic write
                err = -1;
            }
        }
    }
#else
    (void)n_threads;
    for (int32_t e = 0; e < n_envs; ++e) {
        or_planes pl;
        memset(&pl, 0, sizeof(pl));
        pl.Y = Y + offsets[e];
        if (or_simulate_env(&vols[vol_ids[e]], table, n_labels, &probes[e], &poses[12 * e], &pl))
            err = -1;
    }
#endif
    if (threads_used) *threads_used = used;
    return err;
}

/* ------------------------------------------------------------------------
 * Reconstruction observation (Sec. 4 task 2 "Bone surface reconstruction";
 * App. C environment settings; readings):
 *   R1 surface points of a frame: per scanline x of image plane j, the first
 *      pixel (smallest depth y) whose nearest label is a bone label; pixels
 *      below it lie in the acoustic shadow.
 *   R2 segmentation misses each ground-truth point independently with
 *      probability p: Philox4x32-10, key = reconstruction seed, counter =
 *      (x | j << 16, env, step, 0x5245434F); the point is kept when word 0 <
 *      floor((1 - p) * 2^32).
 *   R3 a kept point is stored in volume mm: the pixel's probe point
 *      (a + x*dx, b_j, y*dy) mapped by that step's pose, in FP64 with the
 *      operation order written below (no contraction).
 *   R4 observation at a pose: every stored point, moved into that pose's
 *      probe frame (u = R^T (p - t)), falls in the 40^3 grid of 3 mm cells
 *      indexed (depth floor(u_z / 3), lateral floor((u_x + 60) / 3),
 *      elevation floor((u_y + 60) / 3)); occupied cells read 1.
 */
#define OR_RECON_TAG 0x5245434Fu

/* R1-R3 for one plane; appends kept points (xyz triples) to pts, returns
 * their number, -1 on bad labels. */
int64_t or_recon_points(const or_volume* v, const uint8_t* bone, const or_probe* p, const double pose[12],
                        int32_t plane, int32_t env, int32_t step, uint64_t seed, double p_drop, double* pts)
{
    int64_t P0[3], DX[3], DY[3];
    or_geometry(v, p, pose, P0, DX, DY);
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    double keep = floor((1.0 - p_drop) * 4294967296.0);
    int64_t n = 0;
    for (int32_t x = 0; x < p->W; ++x) {
        int32_t yb = -1;
        for (int32_t y = 0; y < p->H && yb < 0; ++y) {
            int64_t ix = floordiv(P0[0] + (int64_t)x * DX[0] + (int64_t)y * DY[0] + 32768, 65536);
            int64_t iy = floordiv(P0[1] + (int64_t)x * DX[1] + (int64_t)y * DY[1] + 32768, 65536);
            int64_t iz = floordiv(P0[2] + (int64_t)x * DX[2] + (int64_t)y * DY[2] + 32768, 65536);
            int lab = 0;
            if (ix >= 0 && iy >= 0 && iz >= 0 && ix < v->nx && iy < v->ny && iz < v->nz)
                lab = v->labels[(iz * v->ny + iy) * v->nx + ix];
            if (bone[lab]) yb = y;
        }
        if (yb < 0) continue;
        const uint32_t ctr[4] = {(uint32_t)x | ((uint32_t)plane << 16), (uint32_t)env, (uint32_t)step, OR_RECON_TAG};
        uint32_t w[4];
        or_philox4x32_10(ctr, key, w);
        if (!((double)w[0] < keep)) continue;
        double a = -0.5 * (double)(p->W - 1);
        a = a * p->dx;
        double px = (double)x * p->dx;
        px = a + px;
        double pz = (double)yb * p->dy;
        for (int c = 0; c < 3; ++c) {
            double s = pose[4 * c + 0] * px;
            double e = pose[4 * c + 1] * p->elev;
            s = s + e;
            double z = pose[4 * c + 2] * pz;
            s = s + z;
            s = s + pose[4 * c + 3];
            pts[3 * n + c] = s;
        }
        ++n;
    }
    return n;
}

/* R4: occupancy grid [40][40][40] (depth, lateral, elevation) of n points. */
void or_recon_observe(const double* pts, int64_t n, const double pose[12], uint8_t* grid)
{
    memset(grid, 0, 40 * 40 * 40);
    for (int64_t k = 0; k < n; ++k) {
        double d[3], u[3];
        for (int c = 0; c < 3; ++c) d[c] = pts[3 * k + c] - pose[4 * c + 3];
        for (int a = 0; a < 3; ++a) {   /* u_a = column a of R dotted with d */
            double s = pose[0 * 4 + a] * d[0];
            double s1 = pose[1 * 4 + a] * d[1];
            s = s + s1;
            double s2 = pose[2 * 4 + a] * d[2];
            s = s + s2;
            u[a] = s;
        }
        double fh = floor(u[2] / 3.0);
        double fw = floor((u[0] + 60.0) / 3.0);
        double fe = floor((u[1] + 60.0) / 3.0);
        if (fh >= 0.0 && fh < 40.0 && fw >= 0.0 && fw < 40.0 && fe >= 0.0 && fe < 40.0)
            grid[((int)fh * 40 + (int)fw) * 40 + (int)fe] = 1;
    }
}
