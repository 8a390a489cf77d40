// Host helpers shared by the library's translation units.
#pragma once

#include <stdint.h>

namespace degk {

// One autotuned launch setting for (dtype, dim, degree, pool-size bucket).
struct TuneEntry {
    int32_t dtype, dim, degree, kp_bucket;
    int32_t hash_slots;    // LDS visited-table slots
    int32_t waves_per_cu;  // resident waves per CU of the persistent grid (0 = occupancy limit)
};

// Returns the registered entry for the pool size's bucket, or nullptr.
const TuneEntry *tune_lookup(int dtype, int dim, int degree, int kp);
int kp_bucket_of(int kp);

}  // namespace degk
