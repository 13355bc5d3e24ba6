// bttb_cols_b.hip -- column kernels (cols_impl.h) of the transform lengths
// 256, 512, 384, 576.
#include "cols_impl.h"

namespace bttbk {
BTTB_COLS_INSTANTIATE(256)
BTTB_COLS_INSTANTIATE(512)
BTTB_COLS_INSTANTIATE(384)
BTTB_COLS_INSTANTIATE(576)
}  // namespace bttbk
