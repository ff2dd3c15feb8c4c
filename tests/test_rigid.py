"""Host chain of the rigid-transform optimisation (Sec. 3.3.2): the exponential map against
scipy, the pose parametrisation against the stack generator's rigid placement, and the
tangent gradient against central differences of a linear functional of the affine."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2603_00145_amd import inputs, rigid


@pytest.mark.parametrize("w", [[0.1, -0.2, 0.3], [1e-10, 0, 2e-10], [0.0, 0.0, 0.0], [2.0, 1.0, -1.5]])
def test_rotvec_matches_scipy(w):
    np.testing.assert_allclose(rigid.rotvec_to_matrix(w), Rotation.from_rotvec(w).as_matrix(),
                               atol=1e-14)


def test_pose_affine_is_the_stack_placement():
    rng = np.random.default_rng(0)
    R, sh = inputs.random_rigid(rng, 3.0, 2.0, 64)
    placed = inputs.stack_grid("coronal", 64, 16, 1.0, R, sh)
    pose = rigid.StackPose(inputs.stack_grid("coronal", 64, 16, 1.0), R, sh)
    np.testing.assert_allclose(pose.affine(), placed.world_to_index, atol=1e-12)


@pytest.mark.parametrize("centred", [False, True])
def test_tangent_gradient_vs_central_differences(centred):
    rng = np.random.default_rng(1)
    R, sh = inputs.random_rigid(rng, 5.0, 3.0, 32)
    c = rng.normal(size=3) * 0.5 if centred else None
    base = rigid.StackPose(inputs.stack_grid("sagittal", 32, 8, 1.0), R, sh, c)
    G = rng.normal(size=(3, 4))
    f = lambda pose: float((G * pose.affine()).sum())
    ana = base.tangent_grad(G)
    h = 1e-6
    for j in range(6):
        d = np.zeros(6)
        d[j] = h
        pp = rigid.StackPose(base.nominal, base.R.copy(), base.tau.copy(), c)
        pm = rigid.StackPose(base.nominal, base.R.copy(), base.tau.copy(), c)
        pp.apply(d)
        pm.apply(-d)
        fd = (f(pp) - f(pm)) / (2 * h)
        assert abs(fd - ana[j]) <= 1e-7 * max(1.0, np.abs(ana).max()), j


def test_centred_pose_is_the_same_motion():
    """A rotation about a centre c with translation tau moves c to c + tau and is the origin
    form with tau' = tau + c - R c."""
    rng = np.random.default_rng(2)
    R, sh = inputs.random_rigid(rng, 4.0, 2.0, 32)
    c = rng.normal(size=3) * 0.4
    g = inputs.stack_grid("axial", 32, 8, 1.0)
    centred = rigid.StackPose(g, R, sh, c)
    origin = rigid.StackPose(g, R, sh + c - R @ c)
    np.testing.assert_allclose(centred.affine(), origin.affine(), atol=1e-13)
    # the nominal index of the moved centre is the nominal index of c
    A = centred.affine()
    A0 = np.asarray(g.world_to_index)
    moved = R @ (c - c) + c + sh
    np.testing.assert_allclose(A[:, :3] @ moved + A[:, 3], A0[:, :3] @ c + A0[:, 3], atol=1e-12)


def test_pose_adam_frozen_and_first_step():
    nom = [inputs.stack_grid("axial", 16, 4, 1.0), inputs.stack_grid("coronal", 16, 4, 1.0)]
    poses = [rigid.StackPose(g) for g in nom]
    opt = rigid.PoseAdam(poses, lr_rot=1e-2, lr_trans=2e-2, frozen=(0,))
    G = [np.ones((3, 4)), np.ones((3, 4))]
    steps = opt.step(G)
    assert np.all(steps[0] == 0) and np.allclose(poses[0].R, np.eye(3))
    g1 = rigid.StackPose(nom[1]).tangent_grad(G[1])
    # Adam's first step is -lr sign(g) (for |g| >> eps)
    np.testing.assert_allclose(steps[1], -np.array([1e-2] * 3 + [2e-2] * 3) * np.sign(g1),
                               rtol=1e-6)


def test_slice_grids_reproduce_the_stack():
    """A stack split into one-slice grids (inputs.slice_grids) gives, slice by slice, the
    stack's own values in the oracle: same voxel positions, slice profile and affine up to the
    integer z shift."""
    from oracle import gauss
    w = inputs.workload("small", with_data=False)
    for st in w.stacks:
        ref = gauss.render_all(w.gauss, [st])[0]
        rows = gauss.render_all(w.gauss, inputs.slice_grids(st))
        got = np.concatenate(rows, 0)
        assert got.shape == ref.shape
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
