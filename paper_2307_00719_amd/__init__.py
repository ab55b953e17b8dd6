"""MI355X (gfx950) streaming tensor-ring tracking: the per-batch STR / rSTR
update of Yu & Li (arXiv 2307.00719) as hand-written HIP kernels behind the
C ABI in include/tr_stream.h.

The compute lives in libtrstream.so (built by ``build.build()``); this
package only marshals arguments.  Importing it does not require a GPU, but
every compute call does, and a missing library raises ImportError.
"""

from ._lib import (LIB_PATH, TRError, declared_functions, load, tr_batch_als,  # noqa: F401
                   tr_fit_loss_bwd, tr_fit_loss_fwd, tr_gram_chain, tr_last_error, tr_mttkrp,
                   tr_mttkrp_noalloc, tr_mttkrp_noalloc_max_bytes,
                   tr_stream_get_stats,
                   tr_reconstruct_error, tr_stream_destroy, tr_stream_get_cores,
                   tr_stream_get_PQ, tr_stream_get_samples, tr_stream_init, tr_stream_load,
                   tr_stream_num_slices, tr_stream_profile, tr_stream_profile_read,
                   tr_stream_save, tr_stream_set_samples, tr_stream_sync,
                   tr_stream_update, tr_workspace_bytes)
from .stream import TRStream  # noqa: F401
