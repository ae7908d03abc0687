// Batch-cluster interaction kernels for TAGI_YUKAWA (all orbital blocks, proxy-grid
// widths and precisions), instantiated in a translation unit of their own.
#include "interact_impl.hpp"

namespace tagi {
namespace ik {
template void launch_interact_ob<TAGI_YUKAWA>(int, tagi_tree*, bool, const InteractArgs&, const OrbArg&,
                                        hipStream_t);
}  // namespace ik
}  // namespace tagi
