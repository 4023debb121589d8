"""MI355X-native engine for the hot path of the FE-DMN method.

Batched online evaluation of direct deep material networks at Gauss points
(J2 leaves, Newton on the laminate jumps with a tree block-Cholesky), the
linear DMN homogenisation used in offline training, its hand-written
backward, the training objective, optimiser and stiffness sampler, and the
adjoint of a Newton-converged load path.  All computation
runs in the HIP kernels of libdmn.so; this package only marshals arguments
(and captures sequences of calls into HIP graphs).
"""
from .api import (AdjointGroup, Orientation, PointGroup, dmn_homogenize_backward,  # noqa: F401
                  dmn_homogenize_backward_groups, dmn_homogenize_linear,
                  dmn_homogenize_linear_groups, dmn_update_adjoint, dmn_update_gauss_points,
                  dmn_update_gauss_points_noalloc, error_word, workspace)
from ._lib import DmnError, STATUS  # noqa: F401
from .graph import LinearStepGraph, LoadStepGraph  # noqa: F401
from .training import (AmsgradOpts, OrientedTrainingStepGraph, OrientedTrainParams,  # noqa: F401
                       TrainingStepGraph, TrainParams, dmn_orientation_group_chain,
                       dmn_orientation_group_normals, dmn_sample_stiffness, dmn_training_loss,
                       dmn_training_refresh, dmn_training_update, dmn_training_update_oriented)
