// atlas.cpp -- per-device constant tables of the HIP compressor, built once on the host.
//
// For every base B in [2, 2^16 + 1] and for B = 2^j + 1 (j = 17..31) the table holds the
// advanced-method schedule of Sec. 3.2 in cycle form. The series
//   p_i = max{p : R'_{i-1} B^p <= 2^64},  R_i = floor(2^64 / (R'_{i-1} B^{p_i})),
//   R'_i = ceil(B / R_i),  q_{i+1} = q_i + p_i + 1
// depends on B only, and the carried base s_i = R'_{i-1} takes few distinct values: the
// state sequence becomes periodic after mu words with period lam (at most a few hundred
// for every base here). Storing the mu + lam distinct words lets a GPU lane find the
// state of any word i, and the word count of any block length, in O(log) time.
// Also stored: digits per word k(B) (Sec. 3.1, Eq. (1), read with exact integers) and
// the Granlund-Montgomery magic numbers (PLDI 1994, Fig. 4.1) for dividing by B and R_i.
#include <hip/hip_runtime.h>

#include <mutex>
#include <unordered_map>
#include <vector>

#include "device_math.h"
#include "pcomp_internal.h"

namespace pcomp {
namespace {

typedef unsigned __int128 u128;
const u128 kTwo64 = ((u128)1) << 64;

// Magic numbers for any divisor 1 <= d < 2^64: m = floor(2^64 (2^l - d) / d) + 1, l = ceil(log2 d).
Magic magic_host(uint64_t d) {
    Magic mg;
    if (d <= 1) {
        mg.m = 1;
        mg.sh1 = 0;
        mg.sh2 = 0;
        return mg;
    }
    uint32_t l = 0;
    while ((((u128)1) << l) < d) l++;
    u128 num = ((((u128)1) << l) - d) << 64;
    mg.m = (uint64_t)(num / d) + 1;
    mg.sh1 = 1;
    mg.sh2 = l - 1;
    return mg;
}

uint32_t k_host(uint64_t B);

Chunk chunk_host(uint64_t B) {
    Chunk c{};
    c.rB = 1.0 / (double)B;  // IEEE division: correctly rounded
    const uint32_t k = k_host(B);
    c.h2 = k / 2 > 1 ? k / 2 : 1;
    uint64_t P2 = 1;
    for (uint32_t i = 0; i < c.h2; i++) P2 *= B;  // at most 2^32
    c.P2 = (double)P2;
    c.rP2 = 1.0 / (double)P2;
    if (B >= (1ull << 24)) return c;  // h = 0
    uint64_t P = 1;
    uint32_t h = 0;
    while (P * B < (1ull << 32) && P < (1ull << 24)) {  // keeps B^h < 2^32 and B^(h-1) < 2^24
        P *= B;
        h++;
    }
    c.h = h;
    c.P = (uint32_t)P;
    return c;
}

uint32_t k_host(uint64_t B) {
    u128 acc = 1;
    uint32_t k = 0;
    while (acc * B <= kTwo64) {
        acc *= B;
        k++;
    }
    return k;
}

void build_base(uint64_t B, BaseDesc &D, std::vector<AtlasEntry> &ent) {
    D.k = k_host(B);
    u128 bk = 1;
    for (uint32_t i = 0; i + 1 < D.k; i++) bk *= B;
    D.Qk1 = (uint64_t)(kTwo64 / bk);  // B^(k-1) >= 2, so the quotient fits
    D.mBp[0] = magic_host((uint64_t)bk);
    bk *= B;
    D.Qk = (uint64_t)(kTwo64 / bk);
    D.mBp[1] = magic_host(bk < kTwo64 ? (uint64_t)bk : 1);
    D.ch = chunk_host(B);
    D.off = (uint32_t)ent.size();
    std::unordered_map<uint64_t, uint32_t> seen;
    uint64_t s = 1;
    uint32_t q = 0, t = 0;
    for (;;) {
        auto it = seen.find(s);
        if (it != seen.end()) {
            D.mu = (uint16_t)it->second;
            D.lam = (uint16_t)(t - it->second);
            D.V = q - ent[D.off + it->second].q;
            return;
        }
        seen[s] = t;
        uint32_t p = (s <= D.Qk) ? D.k : D.k - 1;
        uint64_t Q = (p == D.k) ? D.Qk : D.Qk1;
        uint64_t R = Q / s;
        AtlasEntry e;
        e.s = (uint32_t)s;
        e.R = (uint32_t)R;
        e.q = q;
        e.p = p;
        e.mR = magic_host(R);
        ent.push_back(e);
        q += p + 1;
        s = (B + R - 1) / R;
        t++;
    }
}

// The same for 32-bit words (capacity 2^32): k, the two quotients, the cycle form, and binary64
// reciprocals of B and of every R_i.
const u128 kTwo32 = ((u128)1) << 32;

uint32_t k32_host(uint64_t B) {
    u128 acc = 1;
    uint32_t k = 0;
    while (acc * B <= kTwo32) {
        acc *= B;
        k++;
    }
    return k;
}

void build_base32(uint64_t B, BaseDesc32 &D, std::vector<AtlasEntry32> &ent) {
    D.rB = 1.0 / (double)B;  // IEEE division: correctly rounded
    D.k = k32_host(B);
    u128 bk = 1;
    for (uint32_t i = 0; i + 1 < D.k; i++) bk *= B;
    D.Qk1 = (uint64_t)(kTwo32 / bk);
    bk *= B;
    D.Qk = (uint64_t)(kTwo32 / bk);
    D.off = (uint32_t)ent.size();
    std::unordered_map<uint64_t, uint32_t> seen;
    uint64_t s = 1;
    uint32_t q = 0, t = 0;
    for (;;) {
        auto it = seen.find(s);
        if (it != seen.end()) {
            D.mu = (uint16_t)it->second;
            D.lam = (uint16_t)(t - it->second);
            D.V = q - ent[D.off + it->second].q;
            return;
        }
        seen[s] = t;
        const uint32_t p = (s <= D.Qk) ? D.k : D.k - 1;
        const uint64_t R = ((p == D.k) ? D.Qk : D.Qk1) / s;
        AtlasEntry32 e;
        e.rR = 1.0 / (double)R;
        e.s = (uint32_t)s;
        e.R = (uint32_t)R;
        e.q = q;
        e.p = p;
        ent.push_back(e);
        q += p + 1;
        s = (B + R - 1) / R;
        t++;
    }
}

struct DeviceTables {
    bool ready = false;
    DevTables t{};
};

std::mutex g_mu;
DeviceTables g_dev[64];
std::vector<BaseDesc> *g_desc = nullptr;
std::vector<AtlasEntry> *g_ent = nullptr;
std::vector<BaseDesc32> *g_desc32 = nullptr;
std::vector<AtlasEntry32> *g_ent32 = nullptr;
uint64_t g_kmax[65];

void build_host_tables() {
    if (g_desc) return;
    auto *desc = new std::vector<BaseDesc>(kAtlasBases);
    auto *ent = new std::vector<AtlasEntry>();
    ent->reserve(720000);
    for (uint32_t B = 2; B <= kAtlasDirect; B++) build_base(B, (*desc)[B], *ent);
    for (uint32_t j = 17; j <= 31; j++) build_base((1ull << j) + 1, (*desc)[kAtlasDirect + 1 + (j - 17)], *ent);
    g_kmax[0] = 0;
    g_kmax[1] = UINT64_MAX;
    for (int k = 2; k <= 64; k++) {
        // integer k-th root of 2^64
        uint64_t lo = 1, hi = 1ull << 33;
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo + 1) / 2;
            u128 acc = 1;
            bool ok = true;
            for (int i = 0; i < k && ok; i++) {
                acc *= mid;
                if (acc > kTwo64) ok = false;
            }
            if (ok)
                lo = mid;
            else
                hi = mid - 1;
        }
        g_kmax[k] = lo;
    }
    auto *desc32 = new std::vector<BaseDesc32>(kAtlasDirect + 1);
    auto *ent32 = new std::vector<AtlasEntry32>();
    ent32->reserve(400000);
    for (uint32_t B = 2; B <= kAtlasDirect; B++) build_base32(B, (*desc32)[B], *ent32);
    g_desc32 = desc32;
    g_ent32 = ent32;
    g_desc = desc;
    g_ent = ent;
}

}  // namespace

int tables_for_current_device(DevTables *out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return PCOMP_EHIP;
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceTables &D = g_dev[dev];
    if (!D.ready) {
        build_host_tables();
        void *pd = nullptr, *pe = nullptr, *pk = nullptr, *pt = nullptr;
        size_t bd = sizeof(BaseDesc) * g_desc->size(), be = sizeof(AtlasEntry) * g_ent->size();
        if (hipMalloc(&pd, bd) != hipSuccess) return PCOMP_EHIP;
        if (hipMalloc(&pe, be) != hipSuccess) return PCOMP_EHIP;
        if (hipMalloc(&pk, sizeof(g_kmax)) != hipSuccess) return PCOMP_EHIP;
        std::vector<uint8_t> ktab(kAtlasDirect + 1, 0);
        for (uint32_t B = 2; B <= kAtlasDirect; B++) ktab[B] = (uint8_t)(*g_desc)[B].k;
        if (hipMalloc(&pt, ktab.size()) != hipSuccess) return PCOMP_EHIP;
        if (hipMemcpy(pt, ktab.data(), ktab.size(), hipMemcpyHostToDevice) != hipSuccess) return PCOMP_EHIP;
        if (hipMemcpy(pd, g_desc->data(), bd, hipMemcpyHostToDevice) != hipSuccess) return PCOMP_EHIP;
        if (hipMemcpy(pe, g_ent->data(), be, hipMemcpyHostToDevice) != hipSuccess) return PCOMP_EHIP;
        if (hipMemcpy(pk, g_kmax, sizeof(g_kmax), hipMemcpyHostToDevice) != hipSuccess) return PCOMP_EHIP;
        void *pd32 = nullptr, *pe32 = nullptr;
        const size_t bd32 = sizeof(BaseDesc32) * g_desc32->size(), be32 = sizeof(AtlasEntry32) * g_ent32->size();
        if (hipMalloc(&pd32, bd32) != hipSuccess) return PCOMP_EHIP;
        if (hipMalloc(&pe32, be32) != hipSuccess) return PCOMP_EHIP;
        if (hipMemcpy(pd32, g_desc32->data(), bd32, hipMemcpyHostToDevice) != hipSuccess) return PCOMP_EHIP;
        if (hipMemcpy(pe32, g_ent32->data(), be32, hipMemcpyHostToDevice) != hipSuccess) return PCOMP_EHIP;
        D.t.desc32 = (const BaseDesc32 *)pd32;
        D.t.ent32 = (const AtlasEntry32 *)pe32;
        D.t.desc = (const BaseDesc *)pd;
        D.t.ent = (const AtlasEntry *)pe;
        D.t.kmax = (const uint64_t *)pk;
        D.t.ktab = (const uint8_t *)pt;
        D.ready = true;
    }
    *out = D.t;
    return PCOMP_OK;
}

bool tables_ready_for_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_dev[dev].ready;
}

}  // namespace pcomp

// Host-side introspection of the tables, for tests that need no GPU.
extern "C" int pcomp_atlas_info(uint64_t B, uint32_t *k, uint32_t *mu, uint32_t *lam, uint32_t *V) {
    using namespace pcomp;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        build_host_tables();
    }
    int idx = -1;
    if (B >= 2 && B <= kAtlasDirect) idx = (int)B;
    for (uint32_t j = 17; j <= 31; j++)
        if (B == (1ull << j) + 1) idx = (int)(kAtlasDirect + 1 + (j - 17));
    if (idx < 0) return PCOMP_EINVAL;
    const BaseDesc &D = (*g_desc)[idx];
    if (k) *k = D.k;
    if (mu) *mu = D.mu;
    if (lam) *lam = D.lam;
    if (V) *V = D.V;
    return PCOMP_OK;
}

// Host-side: state (R'_{i-1}), p_i, R_i, q_i of word i of base B from the cycle form.
extern "C" int pcomp_atlas_word(uint64_t B, uint32_t i, uint64_t *s, uint32_t *p, uint64_t *R, uint64_t *q) {
    using namespace pcomp;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        build_host_tables();
    }
    if (B < 2 || B > kAtlasDirect) return PCOMP_EINVAL;
    const BaseDesc &D = (*g_desc)[B];
    const AtlasEntry *E = g_ent->data() + D.off;
    uint32_t tot = D.mu + D.lam;
    uint64_t qq;
    const AtlasEntry *e;
    if (i < tot) {
        e = E + i;
        qq = e->q;
    } else {
        uint32_t c = (i - D.mu) / D.lam;
        e = E + D.mu + (i - D.mu) - c * D.lam;
        qq = (uint64_t)e->q + (uint64_t)c * D.V;
    }
    *s = e->s;
    *p = e->p;
    *R = e->R;
    *q = qq;
    return PCOMP_OK;
}

// Host-side: advanced word count of n digits of base B computed from the cycle form.
extern "C" int pcomp_atlas_words(uint64_t B, uint32_t n, uint32_t *words) {
    using namespace pcomp;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        build_host_tables();
    }
    int idx = -1;
    if (B >= 2 && B <= kAtlasDirect) idx = (int)B;
    for (uint32_t j = 17; j <= 31; j++)
        if (B == (1ull << j) + 1) idx = (int)(kAtlasDirect + 1 + (j - 17));
    if (idx < 0 || n == 0) return PCOMP_EINVAL;
    const BaseDesc &D = (*g_desc)[idx];
    *words = adv_words_cycle(g_ent->data() + D.off, D, n);
    return PCOMP_OK;
}

// Host-side: advanced word count of n digits of base B <= 2^16 + 1 in 32-bit words, from the
// cycle form of that word size.
extern "C" int pcomp_atlas32_words(uint64_t B, uint32_t n, uint32_t *words) {
    using namespace pcomp;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        build_host_tables();
    }
    if (B < 2 || B > kAtlasDirect || n == 0 || !words) return PCOMP_EINVAL;
    const BaseDesc32 &D = (*g_desc32)[B];
    *words = adv_words_cycle(g_ent32->data() + D.off, D, n);
    return PCOMP_OK;
}
