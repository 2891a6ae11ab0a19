// cpu_sort.cpp -- std::sort / std::stable_sort on the host, the comparator
// the paper times SquareSort against (Section 4).  TEST INFRASTRUCTURE ONLY:
// used by the benchmark's CPU-baseline leg for context, never by the
// product path.
#include <algorithm>
#include <cstdint>
#include <numeric>
#include <vector>

extern "C" {

void orc_std_sort_u32(uint64_t n, uint32_t *keys) { std::sort(keys, keys + n); }

// (key, value) pairs stably sorted by key
int orc_std_stable_sort_kv(uint64_t n, uint64_t *keys, uint32_t *vals)
{
    std::vector<uint64_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](uint64_t a, uint64_t b) { return keys[a] < keys[b]; });
    std::vector<uint64_t> k(n);
    std::vector<uint32_t> v(n);
    for (uint64_t i = 0; i < n; ++i) { k[i] = keys[idx[i]]; v[i] = vals[idx[i]]; }
    std::copy(k.begin(), k.end(), keys);
    std::copy(v.begin(), v.end(), vals);
    return 0;
}

}  // extern "C"
