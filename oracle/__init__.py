"""FP64 CPU oracle (test infrastructure only; the library never imports it)."""
from .ssoct_oracle import *  # noqa: F401,F403
from .ssoct_oracle import (render, render_columns, cuts, sharpness, sharpness_grad, vjp,  # noqa: F401
                           forward_linear, adjoint_linear)
