# A CPU program with three calls of library matrix products (a small
# multilayer perceptron's forward pass): the function blocks the front end
# finds by the called routine's name and may replace with the GPU routine.
import numpy as np


def mlp(x, w1, w2, w3):
    h = np.maximum(np.matmul(x, w1), 0.0)
    h = np.maximum(h @ w2, 0.0)
    return np.dot(h, w3)
