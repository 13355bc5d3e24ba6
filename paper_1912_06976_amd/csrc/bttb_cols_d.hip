// bttb_cols_d.hip -- column kernels (cols_impl.h) of the transform lengths
// 2048, 4096, 2304, 3072.
#include "cols_impl.h"

namespace bttbk {
BTTB_COLS_INSTANTIATE(2048)
BTTB_COLS_INSTANTIATE(4096)
BTTB_COLS_INSTANTIATE(2304)
BTTB_COLS_INSTANTIATE(3072)
}  // namespace bttbk
