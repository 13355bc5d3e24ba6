// bttb_rows_b.hip -- row transforms and spectra column transforms
// (rows_impl.h) of the transform lengths 256, 512, 384, 576.
#include "rows_impl.h"

namespace bttbk {
BTTB_ROWS_INSTANTIATE(256)
BTTB_ROWS_INSTANTIATE(512)
BTTB_ROWS_INSTANTIATE(384)
BTTB_ROWS_INSTANTIATE(576)
}  // namespace bttbk
