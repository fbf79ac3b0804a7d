"""Pose front-end (Sec. 3.1.2 residual composition, Rodrigues rotations;
Sec. 3.3 volume prior) pinned to scipy's rotation routines and to finite
differences."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from paper_2103_01954_amd import pose


def test_rodrigues_matches_scipy():
    rng = np.random.default_rng(0)
    r = np.concatenate([rng.normal(size=(50, 3)), rng.normal(size=(5, 3)) * 1e-6, np.zeros((1, 3)),
                        np.array([[np.pi, 0, 0], [0, 0, -np.pi + 1e-3]])])
    got = pose.rodrigues(torch.from_numpy(r)).numpy()
    want = Rotation.from_rotvec(r).as_matrix()
    np.testing.assert_allclose(got, want, atol=1e-12)


def test_quaternion_matches_scipy():
    q = np.random.default_rng(1).normal(size=(40, 4))
    got = pose.quaternion_to_matrix(torch.from_numpy(q)).numpy()
    want = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()   # scipy uses (x, y, z, w)
    np.testing.assert_allclose(got, want, atol=1e-12)


def test_gradients_against_finite_differences():
    rng = np.random.default_rng(2)
    r = torch.from_numpy(rng.normal(size=(4, 3))).requires_grad_(True)
    tiny = torch.from_numpy(rng.normal(size=(2, 3)) * 1e-7).requires_grad_(True)
    q = torch.from_numpy(rng.normal(size=(3, 4))).requires_grad_(True)
    assert torch.autograd.gradcheck(pose.rodrigues, (r,), eps=1e-6, atol=1e-7)
    assert torch.autograd.gradcheck(pose.rodrigues, (tiny,), eps=1e-9, atol=1e-6)
    assert torch.autograd.gradcheck(pose.quaternion_to_matrix, (q,), eps=1e-6, atol=1e-7)


def test_compose_and_volume_prior():
    rng = np.random.default_rng(3)
    t_hat = torch.from_numpy(rng.normal(size=(5, 3)))
    R_hat = torch.from_numpy(Rotation.random(5, random_state=4).as_matrix())
    s_hat = torch.from_numpy(rng.uniform(0.1, 0.2, size=(5, 3)))
    dt, dr, ds = (torch.from_numpy(rng.normal(size=(5, 3)) * 0.01) for _ in range(3))
    t, R, s = pose.compose(t_hat, R_hat, s_hat, dt, dr, ds)
    np.testing.assert_allclose(t.numpy(), (t_hat + dt).numpy())
    want = Rotation.from_rotvec(dr.numpy()).as_matrix() @ R_hat.numpy()
    np.testing.assert_allclose(R.numpy(), want, atol=1e-12)
    np.testing.assert_allclose(torch.linalg.det(R).numpy(), 1.0, atol=1e-12)
    assert pose.volume_prior(s).item() == pytest.approx(0.01 * np.prod(s.numpy(), axis=1).sum(), rel=1e-12)
