// Host-side prime-field set-up for the NTT multiplication (Section 4.1).
//
// A prime p = k 2^n + 1 admits 2^n-th roots of unity.  The paper's search:
// for a = 2, 3, ..., take g = a^k; by Fermat's little theorem g^(2^n) = 1, and
// g is a primitive 2^n-th root exactly when g^(2^(n-1)) != 1.  A primitive
// L-th root for L = 2^l <= 2^n is then omega = g^(2^(n-l)).
//
// The library works with two primes below 2^31, so that sums of two residues
// fit in 32 bits and the Chinese remainder theorem recovers every product
// coefficient exactly (see bi_ntt_prime below).  Twiddle factors are stored
// with their Shoup companions w' = floor(w 2^32 / p), so a product by a fixed
// twiddle needs one high and two low 32-bit multiplies; the pointwise product
// of two transforms uses Montgomery reduction with R = 2^32.
//
// It also sets up the single 64-bit prime of Section 4.1 (PrimeField64):
// twiddles, the twist powers of a root of twice the transform order, and the
// output scales, all in Montgomery form with R = 2^64.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "bi_internal.hpp"

namespace bi {

namespace {

using u128 = unsigned __int128;

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p) { return uint64_t(u128(a) * b % p); }

uint64_t powmod(uint64_t a, uint64_t e, uint64_t p) {
    uint64_t r = 1 % p;
    a %= p;
    while (e) {
        if (e & 1) r = mulmod(r, a, p);
        a = mulmod(a, a, p);
        e >>= 1;
    }
    return r;
}

// Deterministic Miller-Rabin for 64-bit integers (the first 12 prime bases).
bool is_prime(uint64_t n) {
    if (n < 2) return false;
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t b : bases)
        if (n % b == 0) return n == b;
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; ++s; }
    for (uint64_t a : bases) {
        uint64_t x = powmod(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; ++r) {
            x = mulmod(x, x, n);
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

uint32_t shoup(uint32_t w, uint32_t p) { return uint32_t((uint64_t(w) << 32) / p); }

uint32_t neg_inv32(uint32_t p) {  // -p^-1 mod 2^32 (p odd), by Newton iteration
    uint32_t x = p;               // correct to 3 bits
    for (int i = 0; i < 5; ++i) x *= 2u - p * x;
    return 0u - x;
}

}  // namespace

bi_status field_info(uint64_t p, bi_ntt_field_info *out) {
    if (!out) return BI_EINVAL;
    std::memset(out, 0, sizeof *out);
    if (p < 3 || (p & 1) == 0 || p >= (uint64_t(1) << 63) || !is_prime(p)) return BI_EINVAL;
    uint64_t k = p - 1;
    uint32_t n = 0;
    while ((k & 1) == 0) { k >>= 1; ++n; }
    for (uint64_t a = 2; a < p; ++a) {
        const uint64_t g = powmod(a, k, p);
        if (powmod(g, uint64_t(1) << (n - 1), p) != 1) {
            out->p = p;
            out->k = k;
            out->two_adicity = n;
            out->a = a;
            out->g = g;
            return BI_OK;
        }
    }
    return BI_EINVAL;
}

// Primes of the form k 2^n + 1 below 2^31 (product ~2^61.9): every coefficient
// of a product of two integers of up to 2^18 bits split into 16-bit digits is
// below 2^14 (2^16 - 1)^2 < 2^46, so it is recovered exactly from its residues.
static const uint32_t kPrimes[kNttPrimes] = {2113929217u /* 63 2^25 + 1 */, 2130706433u /* 127 2^24 + 1 */};

bi_status ntt_setup(NttTables &t) {
    std::vector<uint2> host(size_t(kNttPrimes) * 2 * kNttTableWords);
    for (int i = 0; i < kNttPrimes; ++i) {
        bi_ntt_field_info fi;
        if (field_info(kPrimes[i], &fi) != BI_OK || fi.two_adicity < kNttLogLmax) return BI_EINVAL;
        const uint32_t p = kPrimes[i];
        const uint64_t w = powmod(fi.g, uint64_t(1) << (fi.two_adicity - kNttLogLmax), p);  // order Lmax
        const uint64_t wi = powmod(w, p - 2, p);
        t.c.p[i] = p;
        t.c.pneg[i] = neg_inv32(p);
        t.c.one_sh[i] = shoup(1u, p);
        uint64_t f = 1, g = 1;
        uint2 *fw = host.data() + size_t(2 * i) * kNttTableWords;
        uint2 *iw = fw + kNttTableWords;
        for (uint32_t e = 0; e < kNttLmax; ++e) {
            fw[e] = make_uint2(uint32_t(f), shoup(uint32_t(f), p));
            iw[e] = make_uint2(uint32_t(g), shoup(uint32_t(g), p));
            f = mulmod(f, w, p);
            g = mulmod(g, wi, p);
        }
        // Twiddles of the passes, laid out so a wave reads consecutive entries:
        // pass 1 (any length): T1[j][lo] = w_1024^(lo j), lo, j < 32;
        // pass 0 (length 2^M): T0[j][gidx] = w_L^(gidx j), gidx < 1024, j < 2^(M-10).
        for (int dir = 0; dir < 2; ++dir) {
            uint2 *base = dir ? iw : fw;  // base[e] = w_Lmax^(+-e)
            for (uint32_t j = 0; j < 32; ++j)
                for (uint32_t lo = 0; lo < 32; ++lo)
                    base[kNttT1 + 32 * j + lo] = base[((lo * j) % 1024) * (kNttLmax / 1024)];
            for (uint32_t m = kNttLogLmin; m <= kNttLogLmax; ++m) {
                uint2 *t0 = base + ntt_t0_offset(m);
                const uint32_t L = 1u << m;
                for (uint32_t j = 0; j < (L >> 10); ++j)
                    for (uint32_t gi = 0; gi < 1024; ++gi)
                        t0[1024 * j + gi] = base[(uint64_t(gi) * j % L) * (kNttLmax / L)];
            }
        }
        // Output scale for transform length 2^l: L^-1 * R mod p (R = 2^32 undoes
        // the R^-1 left by the Montgomery pointwise product).
        const uint64_t R = (uint64_t(1) << 32) % p;
        for (uint32_t l = 0; l <= uint32_t(kNttScaleMax); ++l) {
            const uint64_t linv = powmod(powmod(2, l, p), p - 2, p);
            const uint32_t s = uint32_t(mulmod(linv, R, p));
            t.c.scale[i][l] = s;
            t.c.scale_sh[i][l] = shoup(s, p);
        }
    }
    // Garner: c = r1 + p1 * ((r2 - r1) * p1^-1 mod p2)
    const uint32_t c12 = uint32_t(powmod(kPrimes[0], kPrimes[1] - 2, kPrimes[1]));
    t.c.crt = c12;
    t.c.crt_sh = shoup(c12, kPrimes[1]);

    const size_t bytes = host.size() * sizeof(uint2);
    void *d = nullptr;
    if (hipMalloc(&d, bytes) != hipSuccess) return BI_ENOMEM;
    if (hipMemcpy(d, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return BI_EHIP;
    }
    t.dev = static_cast<uint2 *>(d);
    for (int i = 0; i < kNttPrimes; ++i) {
        t.c.fwd[i] = t.dev + size_t(2 * i) * kNttTableWords;
        t.c.inv[i] = t.dev + size_t(2 * i + 1) * kNttTableWords;
    }
    return ntt64_setup(t);
}

// PrimeField64: w of order Hmax for the half-length transforms, psi of order
// 2 Hmax for the negacyclic twist (psi_H = psi^(Hmax/H) has order 2H, so
// psi_H^H = -1).  Montgomery form m(x) = x 2^64 mod p.
bi_status ntt64_setup(NttTables &t) {
    bi_ntt_field_info fi;
    if (field_info(kP64, &fi) != BI_OK || fi.two_adicity < kP64LogHmax + 1) return BI_EINVAL;
    const uint64_t p = kP64;
    const uint64_t R1 = uint64_t((u128(1) << 64) % p);
    auto mform = [&](uint64_t x) { return mulmod(x, R1, p); };
    const uint64_t w = powmod(fi.g, uint64_t(1) << (fi.two_adicity - kP64LogHmax), p);
    const uint64_t psi = powmod(fi.g, uint64_t(1) << (fi.two_adicity - kP64LogHmax - 1), p);
    const uint64_t wi = powmod(w, p - 2, p), psii = powmod(psi, p - 2, p);
    std::vector<uint64_t> host(size_t(2) * kP64TableWords + 2 * size_t(kP64Hmax));
    uint64_t *fw = host.data(), *iw = fw + kP64TableWords;
    uint64_t *tw = iw + kP64TableWords, *utw = tw + kP64Hmax;
    uint64_t f = 1, g = 1, x = 1, y = 1;
    for (uint32_t e = 0; e < kP64Hmax; ++e) {
        fw[e] = mform(f);
        iw[e] = mform(g);
        tw[e] = mform(x);
        utw[e] = mform(y);
        f = mulmod(f, w, p);
        g = mulmod(g, wi, p);
        x = mulmod(x, psi, p);
        y = mulmod(y, psii, p);
    }
    for (int dir = 0; dir < 2; ++dir) {
        uint64_t *base = dir ? iw : fw;
        for (uint32_t j = 0; j < 32; ++j)
            for (uint32_t lo = 0; lo < 32; ++lo)
                base[kP64T1 + 32 * j + lo] = base[((lo * j) % 1024) * (kP64Hmax / 1024)];
        for (uint32_t m = kP64LogHmin; m <= kP64LogHmax; ++m) {
            uint64_t *t0 = base + p64_t0_offset(m);
            const uint32_t H = 1u << m;
            for (uint32_t j = 0; j < (H >> 10); ++j)
                for (uint32_t gi = 0; gi < 1024; ++gi)
                    t0[1024 * j + gi] = base[(uint64_t(gi) * j % H) * (kP64Hmax / H)];
        }
    }
    for (uint32_t l = 0; l <= kP64LogHmax; ++l) {
        const uint64_t linv = powmod(uint64_t(1) << l, p - 2, p);
        t.c64.scale[l] = mform(mform(linv));
    }
    const size_t bytes = host.size() * sizeof(uint64_t);
    void *d = nullptr;
    if (hipMalloc(&d, bytes) != hipSuccess) return BI_ENOMEM;
    if (hipMemcpy(d, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return BI_EHIP;
    }
    t.dev64 = static_cast<uint64_t *>(d);
    t.c64.fwd = t.dev64;
    t.c64.inv = t.dev64 + kP64TableWords;
    t.c64.twist = t.dev64 + 2 * size_t(kP64TableWords);
    t.c64.untwist = t.c64.twist + kP64Hmax;
    return BI_OK;
}

void ntt_release(NttTables &t) {
    if (t.dev) (void)hipFree(t.dev);
    t.dev = nullptr;
    if (t.dev64) (void)hipFree(t.dev64);
    t.dev64 = nullptr;
}

}  // namespace bi

extern "C" bi_status bi_ntt_field(uint64_t p, bi_ntt_field_info *out) { return bi::field_info(p, out); }
