// Forward kernel instances: recording mode 1, 2 column(s) per lane (rd_fwd_kernel.h).
#include "rd_fwd_kernel.h"

namespace rd {
RD_STREAM_TABLE(stream_fn_r1c2, 1, 2, kMaxDepthCpl2)
}  // namespace rd
