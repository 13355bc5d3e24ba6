// bttb_rows_a.hip -- row transforms and spectra column transforms
// (rows_impl.h) of the transform lengths 8, 16, 32, 64, 128, 96, 144, 192, 288.
#include "rows_impl.h"

namespace bttbk {
BTTB_ROWS_INSTANTIATE(8)
BTTB_ROWS_INSTANTIATE(16)
BTTB_ROWS_INSTANTIATE(32)
BTTB_ROWS_INSTANTIATE(64)
BTTB_ROWS_INSTANTIATE(128)
BTTB_ROWS_INSTANTIATE(96)
BTTB_ROWS_INSTANTIATE(144)
BTTB_ROWS_INSTANTIATE(192)
BTTB_ROWS_INSTANTIATE(288)
}  // namespace bttbk
