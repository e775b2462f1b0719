// Layout of the domain-labelling results shared by the union-find kernels and
// the host runtime.
#pragma once
#include <stdint.h>

#include <cmath>
#include <cstddef>

namespace xyl {

// launch_domains takes parent (N labels), size (N), hist (N + 1) and stats,
// which receives the number of distinct sizes in stats[0] and the (size,
// count) pairs, at most domain_size_cap(N) of them, from stats[kDomainPairs]
// on; hist and stats[0] must be zero on entry.
constexpr size_t kDomainPairs = 4;
inline uint32_t domain_size_cap(size_t N) {
    // k distinct sizes sum to at least k (k + 1) / 2 <= N
    uint32_t k = (uint32_t)std::sqrt(2.0 * (double)N) + 2u;
    while ((uint64_t)(k - 1) * k / 2 > N) --k;
    return k;
}

}  // namespace xyl
