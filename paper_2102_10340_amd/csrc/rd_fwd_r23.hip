// Forward kernel instances: even-level recording (modes 2 and 3), one or two
// columns per lane, depth <= 8 (rd_fwd_kernel.h).
#include "rd_fwd_kernel.h"

namespace rd {
RD_STREAM_TABLE(stream_fn_r2c1, 2, 1, 8)
RD_STREAM_TABLE(stream_fn_r2c2, 2, 2, 8)
RD_STREAM_TABLE(stream_fn_r3c1, 3, 1, 8)
RD_STREAM_TABLE(stream_fn_r3c2, 3, 2, 8)
}  // namespace rd
