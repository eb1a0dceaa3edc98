"""Annealing schedules beta(t), eta(t) as float64 arrays of length T.

* linear beta from beta0 to beta1 over t = 0..T-1, the workload's stated ramp;
* eta(t) = sqrt(beta(t) / 5), the PIMI noise rule for Max-Cut and SK-1
  (Suppl. "PIMI FPGA implementation for Max-cut and SK-1", noise schedule);
* beta(t) = beta_scale * tanh(beta_init + dbeta * t) (same section, the paper's
  inverse-temperature shape; its constants are not printed, so they are
  arguments here);
* the conventional PIM's constant beta with eta(t) = max(eta_scale / sqrt(t+1),
  eta_floor) (Suppl. "Conventional PIM FPGA implementation for Max-cut and SK-1");
* MIMO detection (Suppl. "PIMI FPGA implementation for MIMO detection", update
  schedule): constant beta = 1 and eta(t) = sqrt(1 / (5 gamma(t))) with gamma
  linear from gamma_init to gamma_final over the T steps (the two constants
  are not printed, so they are arguments); the conventional PIM for MIMO uses
  eta(t) = 1 / sqrt((t + 1) / 5).
"""
import numpy as np


def linear_beta(steps, beta0=0.1, beta1=3.0):
    t = np.arange(steps, dtype=np.float64)
    if steps == 1:
        return np.array([beta0], dtype=np.float64)
    return beta0 + ((beta1 - beta0) * t) / (steps - 1)


def eta_sqrt_beta_over_5(beta):
    return np.sqrt(np.asarray(beta, dtype=np.float64) / 5.0)


def paper_tanh_beta(steps, beta_scale, beta_init, dbeta):
    t = np.arange(steps, dtype=np.float64)
    return beta_scale * np.tanh(beta_init + dbeta * t)


def conventional_eta(steps, eta_scale, eta_floor):
    t = np.arange(steps, dtype=np.float64)
    return np.maximum(eta_scale / np.sqrt(t + 1.0), eta_floor)


def constant(steps, value):
    return np.full(steps, float(value), dtype=np.float64)


def mimo_eta(steps, gamma_init, gamma_final):
    if steps == 1:
        gamma = np.array([float(gamma_init)], dtype=np.float64)
    else:
        t = np.arange(steps, dtype=np.float64)
        gamma = gamma_init + ((gamma_final - gamma_init) * t) / (steps - 1)
    return np.sqrt(1.0 / (5.0 * gamma))


def mimo_conventional_eta(steps):
    t = np.arange(steps, dtype=np.float64)
    return 1.0 / np.sqrt((t + 1.0) / 5.0)
