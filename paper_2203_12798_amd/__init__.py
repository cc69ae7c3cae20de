"""libdpar2: DPar2 (fast PARAFAC2 decomposition of irregular dense tensors)
on AMD Instinct MI355X.  The compute path is the HIP library libdpar2.so
(C ABI in include/dpar2.h); this package is its thin Python binding."""
from .binding import (Dpar2Error, Factors, Options, Tensor, alloc_append_workspace, alloc_batch_workspace,
                      alloc_plain_workspace, alloc_workspace, als_plain, als_step, append, append_workspace_size,
                      batch_report_read, batch_workspace_size, compress, compressed_view, decompose, decompose_batch,
                      decompose_noalloc, feature_pcc, fitness, load, output_A, output_U, release, release_all,
                      report_read, rwr, slice_similarity, top_k, workspace_size)

__all__ = ["Dpar2Error", "Factors", "Options", "Tensor", "alloc_append_workspace", "alloc_batch_workspace",
           "alloc_plain_workspace", "alloc_workspace", "als_plain", "als_step", "append", "append_workspace_size",
           "batch_report_read", "batch_workspace_size", "compress", "compressed_view", "decompose", "decompose_batch",
           "decompose_noalloc", "feature_pcc", "fitness", "load", "output_A", "output_U", "release", "release_all",
           "report_read", "rwr", "slice_similarity", "top_k", "workspace_size"]
