"""MI355X (gfx950) layered sparse-DNN inference and training.

The computation is the one that dominates the large sparse-DNN workload of the
Taskflow paper (section "Large Sparse Neural Network Inference"):
Y_{l+1} = min(32, max(0, Y_l W_l + b_l)) over many sparse layers.  The kernels
are hand-written HIP in ``csrc/`` behind the C ABI of ``include/sdnn.h``;
``sdnn`` is its ctypes binding and ``torch_fn`` an autograd wrapper.
"""
from .sdnn import (Net, SdnnError, lib, mse, sdnn_backward, sdnn_check_device, sdnn_ckpt_size, sdnn_create,
                   sdnn_inject_device_error,
                   sdnn_destroy, sdnn_forward, sdnn_get_plan, sdnn_set_plan, sdnn_layer, sdnn_layer_backward, sdnn_mse, sdnn_mse_noalloc, sdnn_schedule_host, sdnn_set_exec, sdnn_tune, sdnn_set_timing, sdnn_kernel_time,
                   sdnn_version, sdnn_workspace_size, make_desc, LIB_PATH)

__all__ = ["Net", "SdnnError", "lib", "mse", "sdnn_backward", "sdnn_check_device", "sdnn_inject_device_error", "sdnn_ckpt_size", "sdnn_create",
           "sdnn_destroy", "sdnn_forward", "sdnn_get_plan", "sdnn_set_plan", "sdnn_layer", "sdnn_layer_backward", "sdnn_mse", "sdnn_mse_noalloc", "sdnn_schedule_host", "sdnn_set_exec", "sdnn_tune", "sdnn_set_timing", "sdnn_kernel_time",
           "sdnn_version", "sdnn_workspace_size", "make_desc", "LIB_PATH"]
