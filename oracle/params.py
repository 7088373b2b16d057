"""Method parameters (the globals of the paper's Table I). Test infrastructure only."""
from dataclasses import dataclass, asdict


@dataclass
class Params:
    d_min: int = 0          # smallest disparity searched (N_D = d_max - d_min + 1, Table I)
    d_max: int = 63         # largest disparity searched
    census_w: int = 5       # census window width (5x5 in the cost-evaluation section)
    census_h: int = 5       # census window height
    support_step: int = 10  # pitch of the initial support-candidate grid, px
    n_iters: int = 1        # n_iters of Alg. 1
    t_hi: int = 8           # upper cost threshold t_hi (Table I), raw Hamming distance
    t_lo: int = 4           # lower cost threshold t_lo (Table I), raw Hamming distance
    grad_thr: int = 16      # threshold of the high-gradient set Omega_I
    lr_tol: int = 1         # allowed |d_LR - d| in the left-right check
    uniqueness: int = 1     # margin: reject if a disparity >= 2 away costs < best + margin
    sz_occ0: int = 32       # initial occupancy-grid size (Alg. 1 initialisation)
    support_mode: int = 0   # 0: candidate grid; 1: FAST keypoints from spatial bins (Sec. III-A)
    fast_threshold: int = 16  # FAST: corner when the arc contrast exceeds this
    fast_bins_x: int = 12   # FAST spatial bins across (12 x 10 in Sec. III-A)
    fast_bins_y: int = 10   # FAST spatial bins down
    fast_per_bin: int = 25  # at most this many keypoints per bin
    levels: int = 1         # disparity levels tested by cost evaluation (1 = Alg. 2; 3 or 5)

    @classmethod
    def from_dict(cls, d):
        return cls(**{k: int(v) for k, v in d.items() if k in cls.__dataclass_fields__})

    def as_dict(self):
        return asdict(self)

    @property
    def rx(self):
        return (self.census_w - 1) // 2

    @property
    def ry(self):
        return (self.census_h - 1) // 2
