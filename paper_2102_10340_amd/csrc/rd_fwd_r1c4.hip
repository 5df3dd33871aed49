// Forward kernel instances: recording mode 1, 4 column(s) per lane (rd_fwd_kernel.h).
#include "rd_fwd_kernel.h"

namespace rd {
RD_STREAM_TABLE(stream_fn_r1c4, 1, 4, kMaxDepthCpl4)
}  // namespace rd
