"""Trajectory error used to report results (Sec. V: ATE RMSE after SE(3) alignment).

The alignment is Horn's closed form with orthonormal matrices: the rotation is the
orthonormal factor of the cross-covariance (via its singular value decomposition,
with the determinant fixed to +1), the translation aligns the centroids.  Positions
are associated by index (keyframe k with keyframe k).
"""
import numpy as np


def align_rigid(P, Q):
    """(R, t) minimising sum_k |R P_k + t - Q_k|^2 over rotations R and translations t."""
    P = np.asarray(P, np.float64)
    Q = np.asarray(Q, np.float64)
    mp, mq = P.mean(0), Q.mean(0)
    M = (Q - mq).T @ (P - mp)
    U, _, Vt = np.linalg.svd(M)
    S = np.eye(3)
    S[2, 2] = np.sign(np.linalg.det(U @ Vt)) or 1.0
    R = U @ S @ Vt
    return R, mq - R @ mp


def ate_rmse(est_poses, ref_poses):
    """RMSE of the translational differences after aligning est to ref (poses: N x 12, R then t)."""
    P = np.asarray(est_poses, np.float64)[:, 9:12]
    Q = np.asarray(ref_poses, np.float64)[:, 9:12]
    R, t = align_rigid(P, Q)
    d = P @ R.T + t - Q
    return float(np.sqrt(np.mean(np.sum(d * d, axis=1))))
