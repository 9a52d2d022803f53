// Local tile sort, low-phase path: phases k <= 64 in registers with DPP lane exchanges.
#include "local_sort.h"

namespace meld {

hipError_t launch_bitonic_sort_regs_xch(const SortArray &a, uint32_t log_t, uint32_t n_tiles,
                                        int32_t step_limit, bool meld_lo, bool meld_hi,
                                        int io_mode, hipStream_t stream) {
    return launch_sort_regs_path<true>(a, log_t, n_tiles, step_limit, meld_lo, meld_hi, io_mode,
                                        stream);
}

}  // namespace meld
