"""ctypes signatures of the libmd entry points beyond the core step
(surrogate network, data generation, judge, autotuner, graphs)."""
import ctypes

_VP = ctypes.c_void_p
_FP = ctypes.POINTER(ctypes.c_float)
_I32 = ctypes.c_int32


def signatures():
    return {
        "md_mlp_create": (_I32, [ctypes.c_int, ctypes.POINTER(_VP)]),
        "md_mlp_destroy": (None, [_VP]),
        "md_mlp_last_error": (ctypes.c_char_p, [_VP]),
        "md_mlp_set_params": (_I32, [_VP, _FP]),
        "md_mlp_get_params": (_I32, [_VP, _FP]),
        "md_mlp_set_norm": (_I32, [_VP, _FP]),
        "md_mlp_get_norm": (_I32, [_VP, _FP]),
        "md_mlp_forward": (_I32, [_VP, _VP, ctypes.c_int, _VP, _VP]),
        "md_mlp_forward_noalloc": (_I32, [_VP, _VP, ctypes.c_int, _VP, _VP]),
        "md_mlp_backward": (_I32, [_VP, _VP, ctypes.c_int, _VP]),
        "md_mlp_get_grads": (_I32, [_VP, _FP]),
        "md_mlp_loss": (_I32, [_VP, ctypes.POINTER(ctypes.c_double)]),
        "md_mlp_adam": (_I32, [_VP, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _VP]),
        "md_load_surrogate": (_I32, [_VP, _FP, _FP, ctypes.c_float, ctypes.c_int]),
        "md_load_surrogate_mlp": (_I32, [_VP, _VP, ctypes.c_float, ctypes.c_int]),
        "md_datagen": (_I32, [_VP, _VP, ctypes.c_uint32, _VP, _VP, _VP, _VP]),
        "md_judge_stats": (_I32, [_VP, _VP]),
        "md_judge_reset": (_I32, [_VP]),
        "md_set_surrogate_knn_reuse": (_I32, [_VP, ctypes.c_int]),
        "md_set_surrogate_region": (_I32, [_VP, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
        "md_set_surrogate_ood": (_I32, [_VP, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
        "md_set_integrator": (_I32, [_VP, ctypes.c_int]),
        "md_set_domain_randomization": (_I32, [_VP, _VP]),
        "md_set_wind": (_I32, [_VP, _VP]),
        "md_get_integrator": (_I32, [_VP, ctypes.POINTER(ctypes.c_int)]),
        "md_get_launch_config": (_I32, [_VP, _VP]),
        "md_set_launch_config": (_I32, [_VP, _VP]),
        "md_autotune": (_I32, [_VP, _VP, _VP, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _VP,
                               ctypes.c_char_p, ctypes.c_int]),
        "md_autotune_obs": (_I32, [_VP, _VP, _VP, ctypes.c_int, _VP, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int64, _VP, ctypes.c_char_p, ctypes.c_int]),
        "md_rollout_graph_create": (_I32, [_VP, _VP, _VP, ctypes.c_int, _VP, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int64, _VP, ctypes.POINTER(_VP)]),
        "md_graph_launch": (_I32, [_VP, _VP]),
        "md_graph_destroy": (None, [_VP]),
    }
