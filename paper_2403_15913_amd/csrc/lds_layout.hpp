// LDS footprint of one front in the factor and sweep kernels. Shared by the
// symbolic analysis (which splits supernodes whose fronts do not fit) and
// the launch code (which sizes dynamic LDS).
#pragma once
#include <algorithm>
#include <cstdint>

namespace kkt {

// Panels use an odd leading dimension r|1 in LDS and in HBM (conflict-free
// strided LDS access; the HBM<->LDS copies are contiguous).
// factor: (r|1) x rup16(c) panel of doubles (columns padded to the 16-wide
// matrix-core tile) + r staged relative indices
inline int64_t factor_lds_bytes(int r, int c) {
    const int64_t cp = (c + 15) & ~15;
    return (int64_t)(r | 1) * cp * 8 + (int64_t)r * 4 + 16;
}

// sweeps: (r|1) x c panel (padded to an even count) + r vector entries + c pivot reciprocals
inline int64_t solve_lds_bytes(int r, int c) { return ((((int64_t)(r | 1) * c + 1) & ~(int64_t)1) + r + c) * 8; }

inline int64_t front_lds_bytes(int r, int c) { return std::max(factor_lds_bytes(r, c), solve_lds_bytes(r, c)); }

// A front too tall for the LDS budget even at one column is a large front:
// factored and solved in HBM, in chunks of at most this many columns (the
// sweeps stage its c x c triangle in LDS and solve it with one wave).
constexpr int kLargeFrontCols = 64;

}  // namespace kkt
