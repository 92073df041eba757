// Host check of the device's FP64 -> BF16 rounding (vl_storage.h) against a
// plain definition: the two BF16 neighbours of |d| are found by truncating
// the FP64 bits to 8 significant bits, and the nearer one is taken, ties to
// the even one.  Values: random normal FP32-range doubles, exact BF16
// midpoints, midpoints plus and minus one FP64 ulp, and FP32 midpoints next to
// BF16 midpoints (where FP64 -> FP32 -> BF16 rounds twice).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>

#include "../../paper_2504_21450_amd/csrc/vl_storage.h"

static uint64_t dbits(double d) { uint64_t u; memcpy(&u, &d, 8); return u; }
static double bitsd(uint64_t u) { double d; memcpy(&d, &u, 8); return d; }

// reference: round |d| (normal, within the BF16 normal range) to 8 significant bits
static uint16_t ref_bf16(double d)
{
    const uint64_t u = dbits(d);
    const uint64_t sign = u >> 63, mag = u & 0x7FFFFFFFFFFFFFFFull;
    const uint64_t lo = mag & ~((1ull << 45) - 1);         // truncated to 8 significant bits
    const uint64_t hi = lo + (1ull << 45);                 // next BF16 value up
    const double a = bitsd(mag) - bitsd(lo), b = bitsd(hi) - bitsd(mag);
    uint64_t r;
    if (a < b) r = lo;
    else if (b < a) r = hi;
    else r = ((lo >> 45) & 1) ? hi : lo;
    const float f = (float)bitsd(r);                      // exact: r has 8 significant bits
    uint32_t fb;
    memcpy(&fb, &f, 4);
    return (uint16_t)((fb >> 16) | (sign << 15));
}

int main()
{
    std::mt19937_64 g(12345);
    std::uniform_real_distribution<double> ue(-120.0, 120.0), um(1.0, 2.0);
    long bad = 0, n = 0;
    auto check = [&](double d) {
        n++;
        if (vl::bf16_rne_f64(d) != ref_bf16(d)) {
            if (bad < 10) printf("mismatch %.17g: %04x vs %04x\n", d, vl::bf16_rne_f64(d), ref_bf16(d));
            bad++;
        }
    };
    for (int i = 0; i < 2000000; i++) {
        const double d = std::ldexp(um(g), (int)ue(g)) * ((i & 1) ? -1.0 : 1.0);
        check(d);
        // the BF16 midpoint above d's truncation, and its FP64 neighbours
        const uint64_t mag = dbits(std::fabs(d)) & ~((1ull << 45) - 1);
        const double mid = bitsd(mag + (1ull << 44));
        check(mid);
        check(std::nextafter(mid, 0.0));
        check(std::nextafter(mid, 1e300));
        // within half an FP32 ulp of the midpoint: FP32 rounding lands on it
        const double h = bitsd(mag + (1ull << 44) + (1ull << 28));
        const double l = bitsd(mag + (1ull << 44) - (1ull << 28));
        check(h);
        check(l);
        check(-h);
    }
    printf("%ld of %ld mismatched\n", bad, n);
    return bad != 0;
}
