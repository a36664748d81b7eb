// Test-only helper: exposes rocRAND's own Philox4x32-10 block function (an
// independent implementation shipped with ROCm) so the oracle's generator can
// be checked word for word on the CPU.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>

namespace {
struct probe : public rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
}

extern "C" void rr_philox_block(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n)
{
    probe p;
    for (int64_t i = 0; i < n; ++i) {
        uint4 c{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
        uint2 k{key[2 * i], key[2 * i + 1]};
        uint4 r = p.block(c, k);
        out[4 * i] = r.x; out[4 * i + 1] = r.y; out[4 * i + 2] = r.z; out[4 * i + 3] = r.w;
    }
}
