"""FP64 CPU oracle for the Cool-chic 5.0 encoding step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import it.  It shares no code with the
GPU library and never imports it.

Parity status by function (see the tests under tests/test_oracle_*.py):
  philox4x32_10, box_muller      pinned (published known-answer vectors,
                                 closed forms, moments)
  softround, q_train, q_hard     pinned (closed forms, limits, continuity)
  spatial_context, ifce_input    pinned (brute-force loops, causality)
  hyperlatent grids              pinned (nearest upsampling of the extra IFCE
                                 inputs, reduction to the model without them
                                 at zero weights, no distortion gradient,
                                 central finite differences, all-zero rate)
  arm_mlp                        pinned (special cases, explicit loops)
  laplace_bin_prob, latent_bits  pinned (sum to one, closed forms)
  upsample                       pinned (bicubic interpolation routine,
                                 constants, explicit loops)
  upsampling Conv refinement     pinned (scipy 1-D convolution with
  (conv_taps, conv1d)            replicated edges, identity taps equal the
                                 plain upsampling, constants, central finite
                                 differences)
  synthesis                      pinned (scipy correlation, explicit loops)
  forward, loss_and_grad         pinned (closed-form totals, central finite
                                 differences)
  adam                           pinned (first- and second-step closed forms)
  soap (SoapState)               pinned (eigenbases at the first call,
                                 constant-gradient closed form, reduction to
                                 elementwise Adam for diagonal gradients,
                                 equivariance under orthogonal changes of
                                 basis, refresh as power iteration, einsum)
  nnq (quantisation, Exp-Golomb) pinned (explicit encoder/decoder, bijection,
                                 exact grouping, per-choice minimality)
  multi-step trajectories        parity unpinned beyond the per-step pins
"""
from .coolchic_ref import *  # noqa: F401,F403
from .philox import philox4x32_10, box_muller, latent_noise  # noqa: F401
