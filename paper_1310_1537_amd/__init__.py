"""MI355X (gfx950) library for the Bayesian logistic-regression log-posterior
and its gradient, evaluated in one fused pass over a tall design matrix.

The compute lives in the HIP shared library ``libglm_hip.so`` (C interface in
``include/glm.h``); ``paper_1310_1537_amd.glm`` is its Python binding.  This
package file imports nothing so that building does not need a GPU.
"""

__all__ = ["glm"]
