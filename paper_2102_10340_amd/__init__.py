"""MI355X-native RD-CNN simulator (arXiv 2102.10340): hand-written HIP kernels
for the FitzHugh-Nagumo reaction-diffusion cellular nonlinear network step,
behind the C ABI of include/rdcnn.h.

The library is loaded on first use of any public name; that raises ImportError
if librdcnn.so has not been built (``python -m paper_2102_10340_amd.build``).
There is no fallback implementation.
"""
import importlib

_EXPORTS = {
    "BC": "._lib", "PARAM_FIELDS": "._lib", "Params": "._lib", "RDCNNError": "._lib",
    "LIB_PATH": "._lib", "Simulation": ".sim", "init_backward": ".sim",
    "RDCNNFunction": ".autograd", "RDCNNStateFunction": ".autograd", "simulate": ".autograd",
    "simulate_state": ".autograd", "default_segment": ".autograd", "Batch": ".batch",
    "RDCNNBatchFunction": ".autograd", "simulate_batch": ".autograd", "tune": ".tune",
    "atlas": ".atlas",
}

__all__ = sorted(_EXPORTS)


def __getattr__(name):
    mod = _EXPORTS.get(name)
    if mod is None:
        raise AttributeError(name)
    m = importlib.import_module(mod, __name__)
    return m if mod == "." + name else getattr(m, name)
