// Persistent solve kernel for MR degree l = 2 (see persist_impl.h).
#include "persist_impl.h"

namespace msb {
MSB_PERSIST_INSTANTIATE(2)
}  // namespace msb
