/*
 * Counter-based random numbers (oracle side).
 *
 * Philox4x32-10 as published by Salmon et al. (SC'11, "Parallel random numbers:
 * as easy as 1, 2, 3"): each of ten rounds multiplies counter words 0 and 2 by
 * the two round multipliers, swaps the halves and XORs in the key; the key is
 * bumped by the two Weyl constants between rounds.
 *
 * Keying follows the paper's reproducibility scheme (Sec. 5.1): every track
 * owns its own stream, indexed by the event (high part) and a track id (low
 * part); here the stream index is the counter (event, tid, step, purpose) and
 * the run seed is the key, so no generator state is carried by the track.
 */
#include "or_internal.h"

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void or_stream(uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, uint32_t purpose,
               uint32_t out[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {event, (uint32_t)tid, (uint32_t)(tid >> 32),
                       ((nstep & 0xFFFFFFu) << 8) | (purpose & 0xFFu)};
    or_philox4x32_10(ctr, key, out);
}

/* 53-bit uniform in (0, 1] from two words (first word is the high half) */
double or_u53(uint32_t wa, uint32_t wb)
{
    uint64_t x = (((uint64_t)wa << 32) | (uint64_t)wb) >> 11;
    return (double)(x + 1) * 0x1p-53;
}

/* 32-bit uniform in (0, 1] from one word */
double or_u32(uint32_t w)
{
    return ((double)w + 1.0) * 0x1p-32;
}

/* Exponential variate: -log(u) for u <= 1/2, -log1p(-v) with v = 1-u taken
 * from the integer complement above, so both ends keep full precision. */
double or_expo(uint32_t wa, uint32_t wb)
{
    uint64_t x = (((uint64_t)wa << 32) | (uint64_t)wb) >> 11;
    if (x < (1ull << 52)) {
        double u = (double)(x + 1) * 0x1p-53;
        return -log(u);
    }
    double v = (double)((1ull << 53) - 1ull - x) * 0x1p-53;
    return -log1p(-v);
}

void or_box_muller(double ua, double ub, double* g1, double* g2)
{
    double r = sqrt(-2.0 * log(ua));
    double a = 2.0 * OR_PI * ub;
    *g1 = r * cos(a);
    *g2 = r * sin(a);
}
