"""MI355X-native FP64 ELBO hot path of Celeste (Regier et al., 2018).

Submodules are imported on demand: ``synth`` (seeded synthetic fields) needs only numpy,
``binding`` loads the HIP library ``libceleste.so`` and ``torch_fn`` adds the PyTorch
autograd wrapper.
"""
__all__ = ["synth", "binding", "torch_fn"]
