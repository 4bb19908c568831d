// Instances of the persistent batch kernel for segment kinds: kBatchKindsCobg.
#include "batch_impl.h"

namespace bg {

template int batch_occupancy_kinds<kBatchKindsCobg>(bool, int, int, size_t);
template void batch_launch_kinds<kBatchKindsCobg>(bool, int, int, const BatchSegTable&,
                                                 const BatchTile*, unsigned, unsigned,
                                                 const unsigned*, unsigned*, double*, int64_t, int,
                                                 size_t, hipStream_t);

}  // namespace bg
