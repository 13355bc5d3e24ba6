// bttb_cols_c.hip -- column kernels (cols_impl.h) of the transform lengths
// 1024, 768, 1152, 1536.
#include "cols_impl.h"

namespace bttbk {
BTTB_COLS_INSTANTIATE(1024)
BTTB_COLS_INSTANTIATE(768)
BTTB_COLS_INSTANTIATE(1152)
BTTB_COLS_INSTANTIATE(1536)
}  // namespace bttbk
