/*
 * FP64 CPU oracle: 3-D neighborhood attention, literal definition.
 *
 * TEST INFRASTRUCTURE ONLY.  Built as liboracle_nat.so and called from the
 * Python oracle; the product library never links or calls it, and it shares
 * no code with the HIP path.
 *
 * Definition followed (WeatherMesh-3, Sec. 2.1 "NATTEN" and App. A.2):
 *   each query token attends to the Kz x Ky x Kx box of tokens around it
 *   over (level z, lat y, lon x).  Per axis of length N, odd K <= N,
 *   r = (K-1)/2:
 *     periodic axis (lon, circular padding):  key_t = (i - r + t) mod N,
 *                                             offset = t - r
 *     clamped axis (lat and level, the window keeps its size and slides
 *     inward at the border, NATTEN's border behaviour):
 *                                             start = min(max(i-r, 0), N-K)
 *                                             key_t = start + t,
 *                                             offset = key_t - i
 *   score(n, m) = q_h(n) . k_h(m) / sqrt(d) + rpb[h][oz+Kz-1][oy+Ky-1][ox+Kx-1]
 *   p = softmax over the Kvol keys of n (maximum subtracted first)
 *   out_h(n) = sum_m p(n, m) v_h(m)
 * Keys are enumerated (tz, ty, tx) with tx fastest.
 *
 * Layouts: q, k, v, out are [T][H][d] doubles with token
 * n = (z*Y + y)*X + x; rpb is [H][2Kz-1][2Ky-1][2Kx-1]; probs (optional,
 * may be NULL) is [T][H][Kvol].
 */
#include <math.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static void axis_window(int i, int N, int K, int periodic, int *key, int *off)
{
    int r = (K - 1) / 2;
    for (int t = 0; t < K; ++t) {
        if (periodic) {
            int j = i - r + t;
            j %= N;
            if (j < 0) j += N;
            key[t] = j;
            off[t] = t - r;
        } else {
            int s = i - r;
            if (s < 0) s = 0;
            if (s > N - K) s = N - K;
            key[t] = s + t;
            off[t] = s + t - i;
        }
    }
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Returns 0 on success, -1 on invalid arguments. */
int oracle_nat(int Z, int Y, int X, int H, int d, int Kz, int Ky, int Kx,
               unsigned periodic_mask, const double *q, const double *k,
               const double *v, const double *rpb, double *out, double *probs)
{
    if (Kz % 2 == 0 || Ky % 2 == 0 || Kx % 2 == 0) return -1;
    if (Kz > Z || Ky > Y || Kx > X || Kz < 1 || Ky < 1 || Kx < 1) return -1;
    const long T = (long)Z * Y * X;
    const int Kvol = Kz * Ky * Kx;
    const int Bz = 2 * Kz - 1, By = 2 * Ky - 1, Bx = 2 * Kx - 1;
    const double scale = 1.0 / sqrt((double)d);

#pragma omp parallel
    {
        int *kz = malloc(sizeof(int) * Kz), *oz = malloc(sizeof(int) * Kz);
        int *ky = malloc(sizeof(int) * Ky), *oy = malloc(sizeof(int) * Ky);
        int *kx = malloc(sizeof(int) * Kx), *ox = malloc(sizeof(int) * Kx);
        double *s = malloc(sizeof(double) * Kvol);
        long *kid = malloc(sizeof(long) * Kvol);
        int *bid = malloc(sizeof(int) * Kvol);
#pragma omp for schedule(static)
        for (long n = 0; n < T; ++n) {
            int z = (int)(n / ((long)Y * X));
            int y = (int)((n / X) % Y);
            int x = (int)(n % X);
            axis_window(z, Z, Kz, (periodic_mask >> 0) & 1, kz, oz);
            axis_window(y, Y, Ky, (periodic_mask >> 1) & 1, ky, oy);
            axis_window(x, X, Kx, (periodic_mask >> 2) & 1, kx, ox);
            int m = 0;
            for (int a = 0; a < Kz; ++a)
                for (int b = 0; b < Ky; ++b)
                    for (int c = 0; c < Kx; ++c, ++m) {
                        kid[m] = ((long)kz[a] * Y + ky[b]) * X + kx[c];
                        bid[m] = ((oz[a] + Kz - 1) * By + (oy[b] + Ky - 1)) * Bx
                                 + (ox[c] + Kx - 1);
                    }
            for (int h = 0; h < H; ++h) {
                const double *qv = q + (n * H + h) * d;
                const double *bias = rpb + (long)h * Bz * By * Bx;
                double mx = -INFINITY;
                for (int j = 0; j < Kvol; ++j) {
                    const double *kv = k + (kid[j] * H + h) * d;
                    double dot = 0.0;
                    for (int e = 0; e < d; ++e) dot += qv[e] * kv[e];
                    s[j] = dot * scale + bias[bid[j]];
                    if (s[j] > mx) mx = s[j];
                }
                double sum = 0.0;
                for (int j = 0; j < Kvol; ++j) {
                    s[j] = exp(s[j] - mx);
                    sum += s[j];
                }
                double *o = out + (n * H + h) * d;
                for (int e = 0; e < d; ++e) o[e] = 0.0;
                for (int j = 0; j < Kvol; ++j) {
                    double pj = s[j] / sum;
                    if (probs) probs[(n * H + h) * Kvol + j] = pj;
                    const double *vv = v + (kid[j] * H + h) * d;
                    for (int e = 0; e < d; ++e) o[e] += pj * vv[e];
                }
            }
        }
        free(kz); free(oz); free(ky); free(oy); free(kx); free(ox);
        free(s); free(kid); free(bid);
    }
    return 0;
}
