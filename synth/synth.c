/*
 * synth.c - seeded synthetic point catalogues.
 *
 * This module is shared input plumbing: it draws random numbers and lays out
 * points, nothing else. It contains none of the counting method's arithmetic
 * (no separations, no bins, no enumeration), so the CPU oracle and the GPU
 * library can both be fed from it without sharing any of the computation that
 * is being checked.
 *
 * Random numbers: xoshiro256** (Blackman & Vigna, "Scrambled linear
 * pseudorandom number generators", 2018), state seeded with SplitMix64
 * (Steele, Lea & Flood, 2014). Uniform doubles in [0,1) are (u >> 11) * 2^-53.
 * Gaussians use the Box-Muller transform.
 *
 * All outputs are AoS float64 xyz (n x 3) inside the periodic box [0, L)^3.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static void rng_seed(rng_t *r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&x);
}

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t rng_next(rng_t *r) {
    uint64_t *s = r->s;
    uint64_t result = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return result;
}

/* uniform in [0,1) */
static double u01(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* uniform in (0,1] (for the logarithm in Box-Muller) */
static double u01_open0(rng_t *r) { return (double)((rng_next(r) >> 11) + 1) * 0x1.0p-53; }

/* coordinate uniform in [0,L) */
static double ucoord(rng_t *r, double L) {
    double x = u01(r) * L;
    if (x >= L) x -= L;
    return x;
}

/* map any finite x to [0,L) by whole periods */
static double wrap(double x, double L) {
    if (x >= L || x < 0.0) {
        x = x - L * floor(x / L);
        if (x >= L) x -= L;
        if (x < 0.0) x += L;
        if (x >= L || x < 0.0) x = 0.0;
    }
    return x;
}

typedef struct { rng_t r; int have; double spare; } gauss_t;

static double gauss(gauss_t *g) {
    if (g->have) { g->have = 0; return g->spare; }
    double u1 = u01_open0(&g->r), u2 = u01(&g->r);
    double rad = sqrt(-2.0 * log(u1));
    double ang = 6.283185307179586 * u2;
    g->spare = rad * sin(ang);
    g->have = 1;
    return rad * cos(ang);
}

/* n points uniform in [0,L)^3 */
int synth_uniform(double *xyz, int64_t n, double L, uint64_t seed) {
    if (n < 0 || !(L > 0)) return -1;
    rng_t r;
    rng_seed(&r, seed);
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) xyz[3 * i + c] = ucoord(&r, L);
    return 0;
}

/*
 * Neyman-Scott process: ceil(n / per_parent) parent centres uniform in the
 * box; each parent gets per_parent offspring (the last one the remainder),
 * offset by N(0, sigma^2) per axis and wrapped into the box. Parents are not
 * themselves points.
 */
int synth_neyman_scott(double *xyz, int64_t n, int64_t per_parent, double sigma,
                       double L, uint64_t seed) {
    if (n < 0 || per_parent < 1 || !(L > 0) || !(sigma >= 0)) return -1;
    rng_t rp;
    rng_seed(&rp, seed);
    gauss_t g;
    memset(&g, 0, sizeof g);
    rng_seed(&g.r, seed ^ 0xA5A5A5A5DEADBEEFull);
    int64_t i = 0;
    while (i < n) {
        double c[3];
        for (int a = 0; a < 3; ++a) c[a] = ucoord(&rp, L);
        int64_t m = per_parent;
        if (n - i < m) m = n - i;
        for (int64_t k = 0; k < m; ++k, ++i)
            for (int a = 0; a < 3; ++a) xyz[3 * i + a] = wrap(c[a] + sigma * gauss(&g), L);
    }
    return 0;
}

/* periodic 1-D Gaussian smoothing along one axis of an m^3 mesh (x slowest) */
static void smooth_axis(double *f, double *tmp, int m, int axis, const double *k, int rad) {
    int64_t m2 = (int64_t)m * m;
    for (int64_t a = 0; a < m; ++a)
        for (int64_t b = 0; b < m; ++b)
            for (int64_t c = 0; c < m; ++c) {
                double acc = 0.0;
                for (int t = -rad; t <= rad; ++t) {
                    int64_t ia = a, ib = b, ic = c;
                    if (axis == 0) ia = ((a + t) % m + m) % m;
                    if (axis == 1) ib = ((b + t) % m + m) % m;
                    if (axis == 2) ic = ((c + t) % m + m) % m;
                    acc += k[t + rad] * f[ia * m2 + ib * m + ic];
                }
                tmp[a * m2 + b * m + c] = acc;
            }
    memcpy(f, tmp, sizeof(double) * (size_t)(m2 * m));
}

/*
 * Lognormal-like field: white noise on an m^3 mesh, smoothed with a Gaussian
 * of width sigma_s (separable, periodic, truncated at 5 sigma), rescaled to
 * standard deviation sigma_g; density rho ~ exp(G - sigma_g^2/2); n points
 * drawn over cells with probability proportional to rho, uniform inside the
 * chosen cell.
 */
int synth_lognormal(double *xyz, int64_t n, double L, int m, double sigma_s, double sigma_g,
                    uint64_t seed) {
    if (n < 0 || !(L > 0) || m < 1 || m > 512) return -1;
    int64_t nc = (int64_t)m * m * m;
    double *f = (double *)malloc(sizeof(double) * (size_t)nc);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)nc);
    if (!f || !tmp) { free(f); free(tmp); return -2; }
    gauss_t g;
    memset(&g, 0, sizeof g);
    rng_seed(&g.r, seed);
    for (int64_t c = 0; c < nc; ++c) f[c] = gauss(&g);
    double h = L / m, s = sigma_s / h;
    int rad = (int)ceil(5.0 * s);
    if (rad > m / 2) rad = m / 2;
    double *k = (double *)malloc(sizeof(double) * (size_t)(2 * rad + 1));
    double ks = 0.0;
    for (int t = -rad; t <= rad; ++t) { k[t + rad] = exp(-0.5 * (t / s) * (t / s)); ks += k[t + rad]; }
    for (int t = 0; t <= 2 * rad; ++t) k[t] /= ks;
    if (s > 0) for (int axis = 0; axis < 3; ++axis) smooth_axis(f, tmp, m, axis, k, rad);
    free(k);
    double mean = 0.0, var = 0.0;
    for (int64_t c = 0; c < nc; ++c) mean += f[c];
    mean /= (double)nc;
    for (int64_t c = 0; c < nc; ++c) var += (f[c] - mean) * (f[c] - mean);
    double sd = sqrt(var / (double)nc);
    /* cumulative weights into tmp */
    double tot = 0.0;
    for (int64_t c = 0; c < nc; ++c) {
        double G = (f[c] - mean) * (sigma_g / sd);
        tot += exp(G - 0.5 * sigma_g * sigma_g);
        tmp[c] = tot;
    }
    rng_t r;
    rng_seed(&r, seed ^ 0x5DEECE66Dull);
    for (int64_t i = 0; i < n; ++i) {
        double u = u01(&r) * tot;
        int64_t lo = 0, hi = nc - 1;
        while (lo < hi) { int64_t mid = (lo + hi) / 2; if (tmp[mid] > u) hi = mid; else lo = mid + 1; }
        int64_t a = lo / ((int64_t)m * m), b = (lo / m) % m, c = lo % m;
        int64_t cell[3] = {a, b, c};
        for (int ax = 0; ax < 3; ++ax) xyz[3 * i + ax] = wrap((cell[ax] + u01(&r)) * h, L);
    }
    free(f);
    free(tmp);
    return 0;
}

/* n values uniform in [lo, lo + width) */
int synth_uniform_values(double *out, int64_t n, double lo, double width, uint64_t seed) {
    if (n < 0) return -1;
    rng_t r;
    rng_seed(&r, seed);
    for (int64_t i = 0; i < n; ++i) out[i] = lo + u01(&r) * width;
    return 0;
}

/* n raw 64-bit draws (for Python-side derived inputs: permutations, dyadic grids) */
int synth_u64(uint64_t *out, int64_t n, uint64_t seed) {
    if (n < 0) return -1;
    rng_t r;
    rng_seed(&r, seed);
    for (int64_t i = 0; i < n; ++i) out[i] = rng_next(&r);
    return 0;
}
