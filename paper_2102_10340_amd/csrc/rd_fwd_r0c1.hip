// Forward kernel instances: recording mode 0, 1 column(s) per lane (rd_fwd_kernel.h).
#include "rd_fwd_kernel.h"

namespace rd {
RD_STREAM_TABLE(stream_fn_r0c1, 0, 1, kMaxDepthCpl1)
}  // namespace rd
