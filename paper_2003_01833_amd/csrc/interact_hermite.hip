// Batch-cluster interaction kernels with the Hermite far field, for every Green's
// function, instantiated in a translation unit of their own.
#include "interact_impl.hpp"

namespace tagi {
namespace ik {
template void launch_interact_herm_ob<TAGI_YUKAWA_SS>(int, const InteractArgs&, const OrbArg&,
                                                      hipStream_t);
template void launch_interact_herm_ob<TAGI_COULOMB_SS>(int, const InteractArgs&, const OrbArg&,
                                                       hipStream_t);
template void launch_interact_herm_ob<TAGI_YUKAWA>(int, const InteractArgs&, const OrbArg&,
                                                   hipStream_t);
template void launch_interact_herm_ob<TAGI_COULOMB>(int, const InteractArgs&, const OrbArg&,
                                                    hipStream_t);
}  // namespace ik
}  // namespace tagi
