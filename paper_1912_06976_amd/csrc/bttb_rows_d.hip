// bttb_rows_d.hip -- row transforms and spectra column transforms
// (rows_impl.h) of the transform lengths 2048, 4096, 2304, 3072.
#include "rows_impl.h"

namespace bttbk {
BTTB_ROWS_INSTANTIATE(2048)
BTTB_ROWS_INSTANTIATE(4096)
BTTB_ROWS_INSTANTIATE(2304)
BTTB_ROWS_INSTANTIATE(3072)
}  // namespace bttbk
