// bttb_rows_c.hip -- row transforms and spectra column transforms
// (rows_impl.h) of the transform lengths 1024, 768, 1152, 1536.
#include "rows_impl.h"

namespace bttbk {
BTTB_ROWS_INSTANTIATE(1024)
BTTB_ROWS_INSTANTIATE(768)
BTTB_ROWS_INSTANTIATE(1152)
BTTB_ROWS_INSTANTIATE(1536)
}  // namespace bttbk
