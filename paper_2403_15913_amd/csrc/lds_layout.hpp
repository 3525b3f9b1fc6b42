// LDS footprint of one front in the factor and sweep kernels. Shared by the
// symbolic analysis (which splits supernodes whose fronts do not fit) and
// the launch code (which sizes dynamic LDS).
#pragma once
#include <algorithm>
#include <cstdint>

namespace kkt {

// factor: (rup16(r)+1) x rup16(c) panel of doubles + r staged relative indices
inline int64_t factor_lds_bytes(int r, int c) {
    const int64_t rp = (r + 15) & ~15, cp = (c + 15) & ~15;
    return (rp + 1) * cp * 8 + (int64_t)r * 4;
}

// sweeps: (r|1) x c panel + r vector entries + c pivot reciprocals
inline int64_t solve_lds_bytes(int r, int c) { return ((int64_t)(r | 1) * c + r + c) * 8; }

inline int64_t front_lds_bytes(int r, int c) { return std::max(factor_lds_bytes(r, c), solve_lds_bytes(r, c)); }

}  // namespace kkt
