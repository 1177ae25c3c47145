/*
 * Seeded banded random matrices for batched products (input generation only:
 * nothing here multiplies matrices).
 *
 * Counter-based draws, the same definitions as gen.py:
 *   mix(z)         splitmix64 output function
 *   key(seed, s)   = mix(seed * GAMMA ^ mix(s + GAMMA))
 *   u64(seed,s,i)  = mix(key(seed, s) + (i + 1) * GAMMA)
 *   uniform        = (u64 >> 11) * 2^-53
 *   normal(i)      = sqrt(-2 log1p(-u(2i))) * cos(2 pi u(2i+1))   (Box-Muller)
 * Matrix t (stream st[t]) is n[t] x n[t]; row r has k_r = lo + u64(ROWLEN,
 * (st<<32) + r) mod (hi-lo+1) columns (capped at the window width), chosen
 * distinct and uniform in the window [r-bw, r+bw] cut to [0, n) by Floyd's
 * sampling algorithm with draw s of row r at COLS index ((st<<32)+r)*64 + s;
 * entry e of matrix t takes normal(VALUES, (st<<32) + e).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ull
#define TWO_PI 6.283185307179586476925286766559
enum { S_VALUES = 1, S_ROWLEN = 3, S_COLS = 4 };

static uint64_t mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint64_t key_of(uint64_t seed, uint64_t stream) { return mix((seed * GAMMA) ^ mix(stream + GAMMA)); }
static uint64_t draw(uint64_t key, uint64_t idx) { return mix(key + (idx + 1) * GAMMA); }
static double unif(uint64_t key, uint64_t idx) { return (double)(draw(key, idx) >> 11) * 0x1p-53; }

/* Row counts of every matrix (pass 1): cnt[sum n] and per-matrix nnz. */
static int64_t row_len(uint64_t krow, uint64_t st, int64_t r, int64_t n, int64_t bw, int lo, int hi) {
    int64_t lo_c = r - bw < 0 ? 0 : r - bw;
    int64_t hi_c = r + bw > n - 1 ? n - 1 : r + bw;
    int64_t w = hi_c - lo_c + 1;
    int64_t k = lo + (int64_t)(draw(krow, (st << 32) + (uint64_t)r) % (uint64_t)(hi - lo + 1));
    return k < w ? k : w;
}

/* nnz of each of the P matrices. */
void gen_banded_nnz(int32_t P, const int64_t* n, const int64_t* bw, uint64_t seed, const uint64_t* st, int lo,
                    int hi, int64_t* nnz_out) {
    uint64_t krow = key_of(seed, S_ROWLEN);
    for (int32_t t = 0; t < P; ++t) {
        int64_t s = 0;
        for (int64_t r = 0; r < n[t]; ++r) s += row_len(krow, st[t], r, n[t], bw[t], lo, hi);
        nnz_out[t] = s;
    }
}

/* Fills pools: rp[sum (n+1)] (per-matrix row pointers from 0), cols and vals
   (sum nnz).  Returns 0, or -1 if a window is wider than 192. */
int gen_banded_fill(int32_t P, const int64_t* n, const int64_t* bw, uint64_t seed, const uint64_t* st, int lo,
                    int hi, int32_t* rp, int32_t* cols, double* vals) {
    uint64_t krow = key_of(seed, S_ROWLEN), kcol = key_of(seed, S_COLS), kval = key_of(seed, S_VALUES);
    int64_t rpo = 0, eo = 0;
    for (int32_t t = 0; t < P; ++t) {
        const uint64_t sb = st[t] << 32;
        int64_t e = 0;
        rp[rpo] = 0;
        for (int64_t r = 0; r < n[t]; ++r) {
            int64_t lo_c = r - bw[t] < 0 ? 0 : r - bw[t];
            int64_t hi_c = r + bw[t] > n[t] - 1 ? n[t] - 1 : r + bw[t];
            int64_t w = hi_c - lo_c + 1;
            if (w > 192) return -1;
            int64_t k = row_len(krow, st[t], r, n[t], bw[t], lo, hi);
            uint64_t sel[3] = {0, 0, 0};
            const uint64_t base = (sb + (uint64_t)r) << 6;
            for (int64_t s = 0; s < k; ++s) {
                int64_t j = w - k + s;
                double u = unif(kcol, base + (uint64_t)s);
                int64_t pick = (int64_t)(u * (double)(j + 1));
                if (pick > j) pick = j;
                if (sel[pick >> 6] >> (pick & 63) & 1) pick = j;
                sel[pick >> 6] |= 1ull << (pick & 63);
            }
            for (int word = 0; word < 3; ++word) {
                uint64_t m = sel[word];
                while (m) {
                    int b = __builtin_ctzll(m);
                    cols[eo + e++] = (int32_t)(lo_c + word * 64 + b);
                    m &= m - 1;
                }
            }
            rp[rpo + r + 1] = (int32_t)e;
        }
        for (int64_t q = 0; q < e; ++q) {
            double u1 = unif(kval, (sb + (uint64_t)q) << 1);
            double u2 = unif(kval, ((sb + (uint64_t)q) << 1) + 1);
            vals[eo + q] = sqrt(-2.0 * log1p(-u1)) * cos(TWO_PI * u2);
        }
        rpo += n[t] + 1;
        eo += e;
    }
    return 0;
}
